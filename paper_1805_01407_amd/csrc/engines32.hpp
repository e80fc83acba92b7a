// The 32-bit generators of Blackman & Vigna, Section "The 32-bit case":
// engines xoroshiro64 (two words, A/B/C = 26/9/13) and xoshiro128 (four
// words, A/B = 9/11) of table tab:par32, scramblers of table tab:scr32.  The
// paper notes that the words each scrambler reads are those of the 64-bit
// two-word xoroshiro (fig:xoroshiro128) and of xoshiro256 (fig:xoshiro256), so
// the update and output follow those figures with 32-bit words:
//
//  * xoroshiro64*:  s0 * 0x9E3779BB           xoroshiro64**: rotl(s0 * 0x9E3779BB, 5) * 5
//  * xoshiro128+:   s0 + s3                   xoshiro128++:  rotl(s0 + s3, 7) + s0
//  * xoshiro128**:  rotl(s1 * 5, 7) * 9
//
// Seeding (the paper only says a 32-bit SplitMix is immediate to define):
// the state array is filled with the output stream of SplitMix64, each
// 64-bit output giving two 32-bit words, low half first.
#pragma once
#include <stdint.h>

#include "engines.hpp"

namespace slrng {

typedef uint32_t u32;

// Variant ids 14..18 of slrng_variant.
constexpr int kFirstVariant32 = 14;
constexpr int kEndVariant32 = 19;
constexpr u32 kStarMul32 = 0x9E3779BBu;  // tab:scr32

template <int V> struct Params32;

#define SL_VARIANT32(ID, FAM, K, A, B, C, SCR, R, MS, MT)                 \
  template <> struct Params32<ID> {                                       \
    static constexpr int family = FAM, k = K, a = A, b = B, c = C;        \
    static constexpr int scr = SCR, r = R;                                \
    static constexpr u32 ms = MS, mt = MT;                                \
  };
SL_VARIANT32(14, XOROSHIRO, 2, 26, 9, 13, SCR_STAR, 0, kStarMul32, 0)
SL_VARIANT32(15, XOROSHIRO, 2, 26, 9, 13, SCR_STARSTAR, 5, kStarMul32, 5)
SL_VARIANT32(16, XOSHIRO, 4, 9, 11, 0, SCR_PLUS, 0, 0, 0)
SL_VARIANT32(17, XOSHIRO, 4, 9, 11, 0, SCR_PLUSPLUS, 7, 0, 0)
SL_VARIANT32(18, XOSHIRO, 4, 9, 11, 0, SCR_STARSTAR, 7, 5, 9)
#undef SL_VARIANT32

// Engine ids continue those of the 64-bit engines.
template <int V>
constexpr int engine_id32() { return Params32<V>::k == 2 ? 5 : 6; }
constexpr int kNumEngines32 = 2;

template <int R>
SL_HD u32 rotl32(u32 x) {
  static_assert(R > 0 && R < 32, "rotation amount");
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_alignbit(x, x, 32 - R);
#else
  return (x << R) | (x >> (32 - R));
#endif
}

SL_HD u32 xor3_32(u32 a, u32 b, u32 c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
  return a ^ b ^ c;
#endif
}

// Multiplication by a constant; 5 and 9 as a shift and a sum (the paper's
// remark on the ** constants), the * multiplier as a plain multiply.
template <u32 M>
SL_HD u32 mul32(u32 x) {
  if constexpr (M == 5) return (x << 2) + x;
  else if constexpr (M == 9) return (x << 3) + x;
  else return x * M;
}

template <int V>
SL_HD u32 output32(const u32 (&s)[Params32<V>::k]) {
  using Q = Params32<V>;
  if constexpr (Q::family == XOROSHIRO) {
    if constexpr (Q::scr == SCR_STAR) return mul32<Q::ms>(s[0]);
    else return mul32<Q::mt>(rotl32<Q::r>(mul32<Q::ms>(s[0])));
  } else {
    if constexpr (Q::scr == SCR_PLUS) return s[0] + s[3];
    else if constexpr (Q::scr == SCR_PLUSPLUS) return rotl32<Q::r>(s[0] + s[3]) + s[0];
    else return mul32<Q::mt>(rotl32<Q::r>(mul32<Q::ms>(s[1])));
  }
}

template <int V>
SL_HD void step32(u32 (&s)[Params32<V>::k]) {
  using Q = Params32<V>;
  if constexpr (Q::family == XOROSHIRO) {
    const u32 s0 = s[0];
    const u32 t = s[1] ^ s0;
    s[0] = xor3_32(rotl32<Q::a>(s0), t, t << Q::b);
    s[1] = rotl32<Q::c>(t);
  } else {
    // s2 ^= s0; s3 ^= s1; s1 ^= s2; s0 ^= s3; s2 ^= t; rotate s3, each word
    // written once from the old values
    const u32 t = s[1] << Q::a;
    const u32 n0 = xor3_32(s[0], s[3], s[1]);
    const u32 n1 = xor3_32(s[1], s[2], s[0]);
    const u32 n2 = xor3_32(s[2], s[0], t);
    const u32 n3 = rotl32<Q::b>(s[3] ^ s[1]);
    s[0] = n0;
    s[1] = n1;
    s[2] = n2;
    s[3] = n3;
  }
}

// The seeded state: SplitMix64 outputs cut into 32-bit words, low half first.
template <int K>
SL_HD void splitmix64_fill32(u64 seed, u32 (&s)[K]) {
#pragma unroll
  for (int j = 0; j < K; j += 2) {
    const u64 o = splitmix64_mix(seed + (u64)(j / 2 + 1) * kGoldenGamma);
    s[j] = (u32)o;
    if (j + 1 < K) s[j + 1] = (u32)(o >> 32);
  }
}

template <int V>
inline void host_step32(u64 *x) {
  constexpr int K = Params32<V>::k;
  u32 s[K];
  for (int j = 0; j < K; j++) s[j] = (u32)x[j];
  step32<V>(s);
  for (int j = 0; j < K; j++) x[j] = s[j];
}

}  // namespace slrng

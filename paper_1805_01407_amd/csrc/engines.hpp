// Linear engines and scramblers of Blackman & Vigna, "Scrambled Linear
// Pseudorandom Number Generators", as compile-time templates usable on the GPU
// (per-lane state in VGPRs) and on the host (the planner derives each engine's
// characteristic polynomial from them).
//
//  * xoroshiro, 2 words: Section "Linear engines", figure fig:xoroshiro128.
//  * xoroshiro, 16 words: figure fig:xoroshiro1024.  The figure's cyclic index
//    p is kept as a compile-time phase P in 0..15 so every register index is
//    static; a block of 16 steps brings the registers back to logical order
//    x_j = s[j] (logical order: the row vector of the block matrix eq:M).
//  * xoshiro, 4 and 8 words: figures fig:xoshiro256 and fig:xoshiro512.
//  * scramblers +, ++, *, **: Section "Scramblers", applied to the state
//    before it is advanced; parameters from tables tab:par64 and tab:scr64.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define SL_HD __host__ __device__ __forceinline__
#else
#define SL_HD inline
#endif

namespace slrng {

typedef uint64_t u64;

enum Family { XOROSHIRO = 0, XOSHIRO = 1 };
enum Scrambler { SCR_PLUS = 0, SCR_PLUSPLUS = 1, SCR_STAR = 2, SCR_STARSTAR = 3 };

// Left rotation of a 64-bit word.  On the GPU it is two v_alignbit_b32 (a
// funnel shift of the two 32-bit halves) instead of two 64-bit shifts and an or.
template <int R>
SL_HD u64 rotl(u64 x) {
  static_assert(R > 0 && R < 64, "rotation amount");
#if defined(__HIP_DEVICE_COMPILE__)
  const unsigned lo = (unsigned)x, hi = (unsigned)(x >> 32);
  unsigned nlo, nhi;
  if constexpr (R == 32) {
    nlo = hi;
    nhi = lo;
  } else if constexpr (R < 32) {
    nhi = __builtin_amdgcn_alignbit(hi, lo, 32 - R);
    nlo = __builtin_amdgcn_alignbit(lo, hi, 32 - R);
  } else {
    nhi = __builtin_amdgcn_alignbit(lo, hi, 64 - R);
    nlo = __builtin_amdgcn_alignbit(hi, lo, 64 - R);
  }
  return ((u64)nhi << 32) | nlo;
#else
  return (x << R) | (x >> (64 - R));
#endif
}

// Three-input bitwise functions.  On gfx950 each 32-bit half is one
// v_bitop3_b32, whose 8-bit immediate is the truth table indexed by
// 4 a + 2 b + c for input bits (a, b, c): 0x96 is a ^ b ^ c and 0x6a is
// c ^ (a & b).
SL_HD u64 xor3(u64 a, u64 b, u64 c) {
#if defined(__HIP_DEVICE_COMPILE__)
  const unsigned lo = __builtin_amdgcn_bitop3_b32((unsigned)a, (unsigned)b, (unsigned)c, 0x96);
  const unsigned hi =
      __builtin_amdgcn_bitop3_b32((unsigned)(a >> 32), (unsigned)(b >> 32), (unsigned)(c >> 32), 0x96);
  return ((u64)hi << 32) | lo;
#else
  return a ^ b ^ c;
#endif
}

// acc ^ (s & m) with the same 32-bit mask m (0 or all ones) for both halves.
SL_HD u64 xor_and(u64 acc, u64 s, unsigned m) {
#if defined(__HIP_DEVICE_COMPILE__)
  const unsigned lo = __builtin_amdgcn_bitop3_b32((unsigned)s, m, (unsigned)acc, 0x6a);
  const unsigned hi = __builtin_amdgcn_bitop3_b32((unsigned)(s >> 32), m, (unsigned)(acc >> 32), 0x6a);
  return ((u64)hi << 32) | lo;
#else
  return acc ^ (s & (((u64)m << 32) | m));
#endif
}

// ** multiplies by 2^s + 1 (S = 5, T = 9 in tab:scr64), which the paper notes
// can be computed as a shift and a sum.  On the GPU that is one
// v_lshl_add_u64 (the compiler would otherwise turn it back into 32-bit
// multiply-adds).
template <u64 M>
SL_HD u64 mul_const(u64 x) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (M == 5 || M == 9) {
    u64 r;
    if constexpr (M == 5) asm("v_lshl_add_u64 %0, %1, 2, %1" : "=v"(r) : "v"(x));
    else asm("v_lshl_add_u64 %0, %1, 3, %1" : "=v"(r) : "v"(x));
    return r;
  } else {
    return x * M;
  }
#else
  if constexpr (M == 5) return x + (x << 2);
  else if constexpr (M == 9) return x + (x << 3);
  else return x * M;
#endif
}

// Parameters per variant id (the ids of slrng_variant in include/slrng.h).
template <int V> struct Params;

#define SL_VARIANT(ID, FAM, K, A, B, C, SCR, R)                           \
  template <> struct Params<ID> {                                          \
    static constexpr int family = FAM, k = K, a = A, b = B, c = C;         \
    static constexpr int scr = SCR, r = R;                                 \
  };

// tab:par64: xoroshiro128 24/16/37 (for +, *, **); xoroshiro128++ 49/21/28;
// xoshiro256 17/45; xoshiro512 11/21; xoroshiro1024 25/27/36.
// tab:scr64: ++ rotation 17 / 23 / 17 / 23; ** is (5, 7, 9).
SL_VARIANT(0, XOROSHIRO, 2, 24, 16, 37, SCR_PLUS, 0)
SL_VARIANT(1, XOROSHIRO, 2, 49, 21, 28, SCR_PLUSPLUS, 17)
SL_VARIANT(2, XOROSHIRO, 2, 24, 16, 37, SCR_STARSTAR, 7)
SL_VARIANT(3, XOSHIRO, 4, 17, 45, 0, SCR_PLUS, 0)
SL_VARIANT(4, XOSHIRO, 4, 17, 45, 0, SCR_PLUSPLUS, 23)
SL_VARIANT(5, XOSHIRO, 4, 17, 45, 0, SCR_STARSTAR, 7)
SL_VARIANT(6, XOSHIRO, 8, 11, 21, 0, SCR_PLUS, 0)
SL_VARIANT(7, XOSHIRO, 8, 11, 21, 0, SCR_PLUSPLUS, 17)
SL_VARIANT(8, XOSHIRO, 8, 11, 21, 0, SCR_STARSTAR, 7)
SL_VARIANT(9, XOROSHIRO, 16, 25, 27, 36, SCR_PLUS, 0)
SL_VARIANT(10, XOROSHIRO, 16, 25, 27, 36, SCR_PLUSPLUS, 23)
SL_VARIANT(11, XOROSHIRO, 16, 25, 27, 36, SCR_STARSTAR, 7)
SL_VARIANT(12, XOROSHIRO, 2, 24, 16, 37, SCR_STAR, 0)
SL_VARIANT(13, XOROSHIRO, 16, 25, 27, 36, SCR_STAR, 0)
#undef SL_VARIANT

constexpr int kNumVariants = 14;
constexpr u64 kStarMul = 0x9e3779b97f4a7c13ull;  // tab:scr64, the * multiplier

// Engine id: variants that share an engine (same transition matrix) share
// characteristic polynomial and jump tables.
template <int V>
constexpr int engine_id() {
  using P = Params<V>;
  return P::k == 2 ? (P::a == 24 ? 0 : 1) : (P::k == 4 ? 2 : (P::k == 8 ? 3 : 4));
}
constexpr int kNumEngines = 5;

// Steps per static block: 16 for the cyclic 16-word xoroshiro, 1 otherwise.
template <int V>
constexpr int block_steps() { return Params<V>::k == 16 ? 16 : 1; }

// ---------------------------------------------------------------- output

// Scrambled output of the current state.  P is the step's phase inside a
// block (only meaningful for 16 words: the figure's s0 is s[P] and its s15
// is s[(P + 15) & 15]).
template <int V, int P>
SL_HD u64 output(const u64 (&s)[Params<V>::k]) {
  using Q = Params<V>;
  constexpr int K = Q::k;
  if constexpr (Q::family == XOROSHIRO) {
    constexpr int i0 = K == 2 ? 0 : (P & 15);
    constexpr int il = K == 2 ? 1 : ((P + 15) & 15);
    const u64 s0 = s[i0], sl = s[il];
    if constexpr (Q::scr == SCR_PLUS) return s0 + sl;
    else if constexpr (Q::scr == SCR_PLUSPLUS) {
      // fig:xoroshiro128 adds s0 after the rotation, fig:xoroshiro1024 s15
      if constexpr (K == 2) return rotl<Q::r>(s0 + sl) + s0;
      else return rotl<Q::r>(s0 + sl) + sl;
    } else if constexpr (Q::scr == SCR_STAR) return s0 * kStarMul;
    else return mul_const<9>(rotl<7>(mul_const<5>(s0)));
  } else {
    if constexpr (Q::scr == SCR_STARSTAR) return mul_const<9>(rotl<7>(mul_const<5>(s[1])));
    else if constexpr (K == 4) {
      if constexpr (Q::scr == SCR_PLUS) return s[0] + s[3];
      else return rotl<Q::r>(s[0] + s[3]) + s[0];      // fig:xoshiro256
    } else {
      if constexpr (Q::scr == SCR_PLUS) return s[0] + s[2];
      else return rotl<Q::r>(s[0] + s[2]) + s[2];      // fig:xoshiro512
    }
  }
}

// ---------------------------------------------------------------- step

// The step's rotations and three-way xors, either as the VALU forms above or
// (SCALAR) as plain shifts and xors, which the compiler can keep on the
// scalar unit when the state is the same in every lane.
template <int R, bool SCALAR>
SL_HD u64 rot_sel(u64 x) {
  if constexpr (SCALAR) return (x << R) | (x >> (64 - R));
  else return rotl<R>(x);
}

template <bool SCALAR>
SL_HD u64 xor3_sel(u64 a, u64 b, u64 c) {
  if constexpr (SCALAR) return a ^ b ^ c;
  else return xor3(a, b, c);
}

template <int V, int P, bool SCALAR = false>
SL_HD void step(u64 (&s)[Params<V>::k]) {
  using Q = Params<V>;
  constexpr int K = Q::k;
  if constexpr (Q::family == XOROSHIRO) {
    constexpr int i0 = K == 2 ? 0 : (P & 15);
    constexpr int il = K == 2 ? 1 : ((P + 15) & 15);
    const u64 s0 = s[i0];
    const u64 t = s[il] ^ s0;
    // the updated pair lands in the slots of s[q] and s[p] of the figure:
    // for two words that is s[0] and s[1]; for 16 words s[P+15] and s[P]
    if constexpr (K == 2) {
      s[0] = xor3_sel<SCALAR>(rot_sel<Q::a, SCALAR>(s0), t, t << Q::b);
      s[1] = rot_sel<Q::c, SCALAR>(t);
    } else {
      s[il] = xor3_sel<SCALAR>(rot_sel<Q::a, SCALAR>(s0), t, t << Q::b);
      s[i0] = rot_sel<Q::c, SCALAR>(t);
    }
  } else if constexpr (K == 4) {
    // the figure's six in-place updates, each word written once from the
    // old values: s2 ^= s0; s3 ^= s1; s1 ^= s2; s0 ^= s3; s2 ^= t; rotate s3
    const u64 t = s[1] << Q::a;
    const u64 n0 = xor3_sel<SCALAR>(s[0], s[3], s[1]);
    const u64 n1 = xor3_sel<SCALAR>(s[1], s[2], s[0]);
    const u64 n2 = xor3_sel<SCALAR>(s[2], s[0], t);
    const u64 n3 = rot_sel<Q::b, SCALAR>(s[3] ^ s[1]);
    s[0] = n0;
    s[1] = n1;
    s[2] = n2;
    s[3] = n3;
  } else {
    // likewise for the eight-word figure: s2 ^= s0; s5 ^= s1; s1 ^= s2;
    // s7 ^= s3; s3 ^= s4; s4 ^= s5; s0 ^= s6; s6 ^= s7; s6 ^= t; rotate s7
    const u64 t = s[1] << Q::a;
    const u64 n0 = s[0] ^ s[6];
    const u64 n1 = xor3_sel<SCALAR>(s[1], s[2], s[0]);
    const u64 n2 = s[2] ^ s[0];
    const u64 n3 = s[3] ^ s[4];
    const u64 n4 = xor3_sel<SCALAR>(s[4], s[5], s[1]);
    const u64 n5 = s[5] ^ s[1];
    // s7 ^ s3 feeds both the new s6 and the rotation (one xor, not two)
    const u64 m7 = s[7] ^ s[3];
    const u64 n6 = xor3_sel<SCALAR>(s[6], m7, t);
    const u64 n7 = rot_sel<Q::b, SCALAR>(m7);
    s[0] = n0;
    s[1] = n1;
    s[2] = n2;
    s[3] = n3;
    s[4] = n4;
    s[5] = n5;
    s[6] = n6;
    s[7] = n7;
  }
}

// Logical word j of a 16-word state whose registers have run `ph` steps past
// logical alignment: s[(ph + j) & 15].
template <int V>
SL_HD void rotate_to_logical(u64 (&s)[Params<V>::k], int ph) {
  constexpr int K = Params<V>::k;
  if constexpr (K == 16) {
    // rotate left by ph in four static passes (ph is uniform across a wave)
    if (ph & 1) { u64 t = s[0]; for (int j = 0; j < 15; j++) s[j] = s[j + 1]; s[15] = t; }
    if (ph & 2) { u64 t0 = s[0], t1 = s[1]; for (int j = 0; j < 14; j++) s[j] = s[j + 2]; s[14] = t0; s[15] = t1; }
    if (ph & 4) { u64 t[4]; for (int j = 0; j < 4; j++) t[j] = s[j]; for (int j = 0; j < 12; j++) s[j] = s[j + 4]; for (int j = 0; j < 4; j++) s[12 + j] = t[j]; }
    if (ph & 8) { u64 t[8]; for (int j = 0; j < 8; j++) t[j] = s[j]; for (int j = 0; j < 8; j++) s[j] = s[j + 8]; for (int j = 0; j < 8; j++) s[8 + j] = t[j]; }
  } else {
    (void)s; (void)ph;
  }
}

// Host-side single step on a logical-order state (slow path for the planner).
template <int V>
inline void host_step_logical(u64 *x) {
  constexpr int K = Params<V>::k;
  u64 s[K];
  for (int j = 0; j < K; j++) s[j] = x[j];
  step<V, 0>(s);
  if constexpr (K == 16) rotate_to_logical<V>(s, 1);
  for (int j = 0; j < K; j++) x[j] = s[j];
}

template <int V>
inline u64 host_output_logical(const u64 *x) {
  constexpr int K = Params<V>::k;
  u64 s[K];
  for (int j = 0; j < K; j++) s[j] = x[j];
  return output<V, 0>(s);
}

// ---------------------------------------------------------------- SplitMix64

// Seeding (Section "Choosing a generator"): the state is filled with
// consecutive outputs of SplitMix64 seeded with the 64-bit seed.  SplitMix64
// (Steele, Lea, Flood, OOPSLA 2014): counter += golden gamma, then the mix64
// finalizer.
constexpr u64 kGoldenGamma = 0x9e3779b97f4a7c15ull;

SL_HD u64 splitmix64_mix(u64 z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <int K>
SL_HD void splitmix64_fill(u64 seed, u64 (&s)[K]) {
#pragma unroll
  for (int j = 0; j < K; j++) s[j] = splitmix64_mix(seed + (u64)(j + 1) * kGoldenGamma);
}

}  // namespace slrng

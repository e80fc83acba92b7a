// Device building blocks shared by the generation kernels: jump application,
// LDS-staged tiles, stores.  See kernels.hip for the design notes.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "engines.hpp"
#include "kernels.hpp"

namespace slrng {

typedef u64 u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exact 53-bit double of the upper 53 bits: (x >> 11) * 2^-53 as
// hi * 2^-32 + lo * 2^-64 with hi = the upper word of x and lo = the lower
// word with its low 11 bits cleared.  Both terms are exact (32-bit integers
// scaled by powers of two) and their sum has at most 53 significant bits, so
// the fused multiply-add rounds nothing; no 64-bit shift is needed.
__device__ __forceinline__ u64 to_f64_bits(u64 x) {
  unsigned hi = (unsigned)(x >> 32);
  // opaque to the optimiser, which would otherwise widen the conversion of
  // hi to a 64-bit one (an extra f64 add); emits no instruction
  asm("" : "+v"(hi));
  const unsigned lo = (unsigned)x & 0xFFFFF800u;
  const double d = __fma_rn((double)hi, 0x1p-32, (double)lo * 0x1p-64);
  return (u64)__double_as_longlong(d);
}

template <int KIND>
__device__ __forceinline__ u64 emit(u64 x) {
  if constexpr (KIND == 1) return to_f64_bits(x);
  else return x;
}

// compile-time loop
template <int N, typename F, int I = 0>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<N, F, I + 1>(static_cast<F &&>(f));
  }
}

// ---------------------------------------------------------------- jumps

// acc ^= logical(s) at phase P (16 words: logical word j is s[(P+j)&15])
template <int V, int P>
__device__ __forceinline__ void acc_xor(u64 (&acc)[Params<V>::k], const u64 (&s)[Params<V>::k]) {
  constexpr int K = Params<V>::k;
#pragma unroll
  for (int j = 0; j < K; j++) acc[j] ^= s[K == 16 ? ((P + j) & 15) : j];
}

template <int V, int P>
__device__ __forceinline__ void acc_xor_masked(u64 (&acc)[Params<V>::k], const u64 (&s)[Params<V>::k],
                                               unsigned m) {
  constexpr int K = Params<V>::k;
#pragma unroll
  for (int j = 0; j < K; j++) acc[j] = xor_and(acc[j], s[K == 16 ? ((P + j) & 15) : j], m);
}

// s <- s * M^J where the uniform polynomial r(x) = x^J mod p has its 64-bit
// words at r[0 .. n/64) (same address in every lane).
template <int V>
__device__ __forceinline__ void jump_uniform(u64 (&s)[Params<V>::k], const u64 *__restrict__ r) {
  constexpr int K = Params<V>::k;
  constexpr int BLK = block_steps<V>();
  u64 acc[K];
#pragma unroll
  for (int j = 0; j < K; j++) acc[j] = 0;
  for (int wi = 0; wi < K; wi++) {  // n/64 = K words
    // readfirstlane returns int: widen through unsigned so the low half is
    // not sign-extended into the high half
    const u64 lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)r[wi]);
    const u64 hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(r[wi] >> 32));
    const u64 word = lo | (hi << 32);
    for (int b = 0; b < 64; b += BLK) {
      static_for<BLK>([&](auto P) {
        if ((word >> (b + P)) & 1) acc_xor<V, P>(acc, s);
        step<V, P>(s);
      });
    }
  }
#pragma unroll
  for (int j = 0; j < K; j++) s[j] = acc[j];
}

// The same with a per-lane polynomial read word by word from r_words(wi).
template <int V, typename GetWord>
__device__ __forceinline__ void jump_lane(u64 (&s)[Params<V>::k], GetWord &&r_word) {
  constexpr int K = Params<V>::k;
  constexpr int BLK = block_steps<V>();
  u64 acc[K];
#pragma unroll
  for (int j = 0; j < K; j++) acc[j] = 0;
  for (int wi = 0; wi < K; wi++) {
    const u64 word = r_word(wi);
    const unsigned half[2] = {(unsigned)word, (unsigned)(word >> 32)};
#pragma unroll
    for (int h = 0; h < 2; h++) {
      for (int b = 0; b < 32; b += BLK) {
        static_for<BLK>([&](auto P) {
          // sign-extended one-bit field: 0 or all ones
          const unsigned m = (unsigned)__builtin_amdgcn_sbfe((int)half[h], b + P, 1);
          acc_xor_masked<V, P>(acc, s, m);
          step<V, P>(s);
        });
      }
    }
  }
#pragma unroll
  for (int j = 0; j < K; j++) s[j] = acc[j];
}

// The same when the start state s is the same in every lane (the chunks of
// one request in a run tile), each lane with its own polynomial: the state
// sequence s M^i is common to the wave, so it advances once, on the scalar
// unit, and each lane only accumulates its own selection of it.
__device__ __forceinline__ u64 uniform64(u64 x) {
  const u64 lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)x);
  const u64 hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(x >> 32));
  return lo | (hi << 32);
}

template <int V, typename GetWord>
__device__ __forceinline__ void jump_lane_from_uniform(u64 (&s)[Params<V>::k], GetWord &&r_word) {
  constexpr int K = Params<V>::k;
  constexpr int BLK = block_steps<V>();
  u64 su[K], acc[K];
#pragma unroll
  for (int j = 0; j < K; j++) {
    su[j] = uniform64(s[j]);
    acc[j] = 0;
  }
  for (int wi = 0; wi < K; wi++) {
    const u64 word = r_word(wi);
    const unsigned half[2] = {(unsigned)word, (unsigned)(word >> 32)};
#pragma unroll
    for (int h = 0; h < 2; h++) {
      for (int b = 0; b < 32; b += BLK) {
        static_for<BLK>([&](auto P) {
          const unsigned m = (unsigned)__builtin_amdgcn_sbfe((int)half[h], b + P, 1);
          acc_xor_masked<V, P>(acc, su, m);
          step<V, P, true>(su);
        });
      }
    }
  }
#pragma unroll
  for (int j = 0; j < K; j++) s[j] = acc[j];
}

// ---------------------------------------------------------------- generation tiles

template <int T>
struct TileGeom {
  static constexpr int kPad = 2;            // u64 of padding per LDS row
  static constexpr int kStride = T + kPad;  // LDS row stride (u64), even
  static constexpr int kWaveLds = kWave * kStride;
};

// T outputs of one lane into its LDS row (row pointer `row`), as pairs.
template <int V, int KIND, int T>
__device__ __forceinline__ void gen_tile_full(u64 (&s)[Params<V>::k], u64 *row) {
  constexpr int BLK = block_steps<V>();
  static_assert(T % BLK == 0 && T % 2 == 0, "tile");
#pragma unroll
  for (int t0 = 0; t0 < T; t0 += (BLK > 2 ? BLK : 2)) {
    static_for<(BLK > 2 ? BLK : 2) / 2>([&](auto H) {
      constexpr int P0 = (2 * H.value) % BLK;
      constexpr int P1 = (2 * H.value + 1) % BLK;
      u64x2 v;
      v.x = emit<KIND>(output<V, P0>(s));
      step<V, P0>(s);
      v.y = emit<KIND>(output<V, P1>(s));
      step<V, P1>(s);
      *reinterpret_cast<u64x2 *>(row + t0 + 2 * H.value) = v;
    });
  }
}

// m < T outputs (the last, partial tile of a chunk).  Returns the number of
// steps past the last 16-step block boundary (for the 16-word engine).
template <int V, int KIND, int T>
__device__ __forceinline__ int gen_tile_partial(u64 (&s)[Params<V>::k], u64 *row, int m) {
  constexpr int BLK = block_steps<V>();
  for (int t0 = 0; t0 < T; t0 += BLK) {
    if (t0 >= m) break;
    static_for<BLK>([&](auto P) {
      if (t0 + P < m) {
        row[t0 + P] = emit<KIND>(output<V, P>(s));
        step<V, P>(s);
      }
    });
  }
  return m % BLK;
}

// Output stores of the generation kernels: plain (write-back) or
// nontemporal (the nt cache policy), chosen per launch.  Which is faster
// depends on where the output's physical pages lie: in one compact range plain
// stores measured faster, in memory whose pages are spread over the HBM
// nontemporal ones did; the autotuner measures both per generator and kind.
template <typename VT>
__device__ __forceinline__ void out_store(VT *p, VT v) {
  *p = v;
}

template <typename VT>
__device__ __forceinline__ void out_store_nt(VT *p, VT v) {
  __builtin_nontemporal_store(v, p);
}

template <bool NT, typename VT>
__device__ __forceinline__ void out_store_as(VT *p, VT v) {
  if constexpr (NT) out_store_nt(p, v);
  else out_store(p, v);
}

// Store with the device-scope cache policy (sc1): the line is written through
// the XCD's L2 instead of staying dirty there.  For the batched kernel, whose
// rows are consecutive chunks of one request, this measured about 10% faster
// than plain stores; for the stream-major generation kernel about 2% slower.
//  * The compiler cannot see that the asm is a store, so it does not insert the
//    wait states that a VALU write of a store's data registers needs right
//    after a store of more than 8 bytes (two on this family); the asm carries
//    them itself (s_nop 1 = two wait states).
//  * No memory clobber: the outputs are never read back by the kernel, and
//    the stores must not become scheduling barriers for the LDS reads that
//    feed them.
template <typename VT>
__device__ __forceinline__ void out_store_wt(VT *p, VT v) {
  static_assert(sizeof(VT) == 16 || sizeof(VT) == 8, "16- or 8-byte stores");
  if constexpr (sizeof(VT) == 16)
    asm volatile("global_store_dwordx4 %0, %1, off sc1\n\ts_nop 1" ::"v"(p), "v"(v));
  else
    asm volatile("global_store_dwordx2 %0, %1, off sc1\n\ts_nop 1" ::"v"(p), "v"(v));
}

// Store a staged tile: rows 0..rows_live of the wave, m outputs each, to
// base + r*ld + c.  A16: every row start is 16-byte aligned (dwordx4 path).
// A full tile (all 64 rows, T outputs) takes the unpredicated path.
template <int T, bool A16, bool NT>
__device__ __forceinline__ void store_tile(const u64 *lds, int lane, u64 *base, u64 ld,
                                           int rows_live, int m) {
  constexpr int S = TileGeom<T>::kStride;
  if constexpr (A16) {
    constexpr int LPR = T / 2;         // lanes per row, 16 bytes each
    constexpr int RPI = kWave / LPR;   // rows per store instruction
    const int r0 = lane / LPR;
    const int c = 2 * (lane % LPR);
    const u64x2 *src = reinterpret_cast<const u64x2 *>(lds + r0 * S + c);
    u64 *dst = base + (u64)r0 * ld + c;
    const u64 step = (u64)RPI * ld;
    if (rows_live == kWave && m == T) {
      // all LDS reads of the tile first, then the stores: the reads overlap
      // each other instead of each waiting for the previous store (LDS
      // already limits occupancy to two waves per SIMD, so the registers
      // are free)
      u64x2 v[T / 2];
#pragma unroll
      for (int q = 0; q < T / 2; q++) v[q] = src[q * RPI * S / 2];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < T / 2; q++) out_store_as<NT>(reinterpret_cast<u64x2 *>(dst + q * step), v[q]);
      return;
    }
#pragma unroll
    for (int q = 0; q < T / 2; q++) {
      const int r = q * RPI + r0;
      if (r < rows_live && c < m) {
        const u64x2 v = src[q * RPI * S / 2];
        if (c + 1 < m) out_store_as<NT>(reinterpret_cast<u64x2 *>(dst + q * step), v);
        else out_store_as<NT>(dst + q * step, v.x);
      }
    }
  } else {
    constexpr int LPR = T;
    constexpr int RPI = kWave / LPR;
    const int r0 = lane / LPR;
    const int c = lane % LPR;
    u64 *dst = base + (u64)r0 * ld + c;
    const u64 step = (u64)RPI * ld;
#pragma unroll
    for (int q = 0; q < T; q++) {
      const int r = q * RPI + r0;
      if (r < rows_live && c < m) out_store_as<NT>(dst + q * step, lds[r * S + c]);
    }
  }
}

}  // namespace slrng

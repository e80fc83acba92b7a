// gfx950 kernels of the 32-bit generators (Section "The 32-bit case":
// xoroshiro64*, xoroshiro64**, xoshiro128+, xoshiro128++, xoshiro128**).
//
// Same design as the 64-bit kernels: one stream per lane with its k 32-bit
// words in VGPRs (native 32-bit xor / shift / v_alignbit rotations), streams
// split into jumped slots with staggered boundaries, a per-wave LDS transpose
// of a 64 x 64 tile of 32-bit outputs and 16-byte stores that each write four
// 256-byte row runs.  States stay in the handle's 64-bit word-major buffers
// (one 32-bit word per 64-bit slot, upper half zero), so the host side of the
// handles is shared with the 64-bit generators.  Jump polynomials are n = 64
// or 128 bits, one or two 64-bit words.
#include <hip/hip_runtime.h>

#include "engines32.hpp"
#include "gen_device.hpp"
#include "kernels.hpp"
#include "kernels32.hpp"

namespace slrng {

typedef u32 u32x4 __attribute__((ext_vector_type(4)));

constexpr int kT32 = 64;          // outputs per lane per tile
constexpr int kPad32 = 4;         // u32 of padding per LDS row (keeps rows 16-byte aligned)
constexpr int kStride32 = kT32 + kPad32;
constexpr int kWaveLds32 = kWave * kStride32;

// ---------------------------------------------------------------- jumps

// s <- s * M^J, r(x) = x^J mod p in r[0 .. n/64), the same in every lane.
template <int V>
__device__ __forceinline__ void jump_uniform32(u32 (&s)[Params32<V>::k], const u64 *__restrict__ r) {
  constexpr int K = Params32<V>::k;
  constexpr int NW = K / 2;  // n / 64
  u32 acc[K];
#pragma unroll
  for (int j = 0; j < K; j++) acc[j] = 0;
  for (int wi = 0; wi < NW; wi++) {
    const u64 lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)r[wi]);
    const u64 hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(r[wi] >> 32));
    const u64 word = lo | (hi << 32);
    for (int b = 0; b < 64; b++) {
      if ((word >> b) & 1) {
#pragma unroll
        for (int j = 0; j < K; j++) acc[j] ^= s[j];
      }
      step32<V>(s);
    }
  }
#pragma unroll
  for (int j = 0; j < K; j++) s[j] = acc[j];
}

// The same with a per-lane polynomial read word by word from r_word(wi).
template <int V, typename GetWord>
__device__ __forceinline__ void jump_lane32(u32 (&s)[Params32<V>::k], GetWord &&r_word) {
  constexpr int K = Params32<V>::k;
  constexpr int NW = K / 2;
  u32 acc[K];
#pragma unroll
  for (int j = 0; j < K; j++) acc[j] = 0;
  for (int wi = 0; wi < NW; wi++) {
    const u64 word = r_word(wi);
    const unsigned half[2] = {(unsigned)word, (unsigned)(word >> 32)};
#pragma unroll
    for (int h = 0; h < 2; h++) {
      for (int b = 0; b < 32; b++) {
        // sign-extended one-bit field: 0 or all ones; acc ^= s & m
        const unsigned m = (unsigned)__builtin_amdgcn_sbfe((int)half[h], b, 1);
#pragma unroll
        for (int j = 0; j < K; j++) acc[j] = __builtin_amdgcn_bitop3_b32(s[j], m, acc[j], 0x6a);
        step32<V>(s);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < K; j++) s[j] = acc[j];
}

// ---------------------------------------------------------------- tiles

// Upper 24 bits as a float in [0, 1): (x >> 8) * 2^-24, exact.
__device__ __forceinline__ u32 to_f32_bits(u32 x) {
  return __float_as_uint((float)(x >> 8) * 0x1p-24f);
}

template <int KIND>
__device__ __forceinline__ u32 emit32(u32 x) {
  if constexpr (KIND == 1) return to_f32_bits(x);
  else return x;
}

template <int V, int KIND>
__device__ __forceinline__ void gen_tile32_full(u32 (&s)[Params32<V>::k], u32 *row) {
#pragma unroll
  for (int t = 0; t < kT32; t += 4) {
    u32x4 v;
    v.x = emit32<KIND>(output32<V>(s));
    step32<V>(s);
    v.y = emit32<KIND>(output32<V>(s));
    step32<V>(s);
    v.z = emit32<KIND>(output32<V>(s));
    step32<V>(s);
    v.w = emit32<KIND>(output32<V>(s));
    step32<V>(s);
    *reinterpret_cast<u32x4 *>(row + t) = v;
  }
}

template <int V, int KIND>
__device__ __forceinline__ void gen_tile32_partial(u32 (&s)[Params32<V>::k], u32 *row, int m) {
  for (int t = 0; t < m; t++) {
    row[t] = emit32<KIND>(output32<V>(s));
    step32<V>(s);
  }
}

// Store a staged tile: rows 0..rows_live of the wave, m outputs each, to
// base + r*ld + c.  A16: every row start is 16-byte aligned (4 outputs per
// lane and store, 16 lanes per row); else one output per lane and store.
template <bool A16, bool NT>
__device__ __forceinline__ void store_tile32(const u32 *lds, int lane, u32 *base, u64 ld,
                                             int rows_live, int m) {
  if constexpr (A16) {
    constexpr int LPR = kT32 / 4;
    constexpr int RPI = kWave / LPR;
    const int r0 = lane / LPR;
    const int c = 4 * (lane % LPR);
    const u32x4 *src = reinterpret_cast<const u32x4 *>(lds + r0 * kStride32 + c);
    u32 *dst = base + (u64)r0 * ld + c;
    const u64 step = (u64)RPI * ld;
    if (rows_live == kWave && m == kT32) {
      u32x4 v[kT32 / 4];
#pragma unroll
      for (int q = 0; q < kT32 / 4; q++) v[q] = src[q * RPI * kStride32 / 4];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < kT32 / 4; q++) out_store_as<NT>(reinterpret_cast<u32x4 *>(dst + q * step), v[q]);
      return;
    }
#pragma unroll
    for (int q = 0; q < kT32 / 4; q++) {
      const int r = q * RPI + r0;
      if (r < rows_live && c < m) {
        const u32x4 v = src[q * RPI * kStride32 / 4];
        u32 *d = dst + q * step;
        if (c + 3 < m) {
          out_store_as<NT>(reinterpret_cast<u32x4 *>(d), v);
        } else {
          d[0] = v.x;
          if (c + 1 < m) d[1] = v.y;
          if (c + 2 < m) d[2] = v.z;
        }
      }
    }
  } else {
    u32 *dst = base + lane;
    for (int r = 0; r < rows_live; r++)
      if (lane < m) dst[(u64)r * ld] = lds[r * kStride32 + lane];
  }
}

// ---------------------------------------------------------------- kernels

// Generation (see GenArgs for the slot and skew plan; outputs are 32-bit).
template <int V, int KIND, bool A16, bool NT>
__global__ __launch_bounds__(kBlock) void k_generate32(GenArgs a) {
  constexpr int K = Params32<V>::k;
  __shared__ __attribute__((aligned(16))) u32 lds_all[(kBlock / kWave) * kWaveLds32];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const u64 g = (u64)blockIdx.x * (kBlock / kWave) + wave;
  const u64 row0 = g * kWave;
  if (row0 >= a.S) return;  // uniform per wave
  const u64 i = row0 + lane;
  const bool live = i < a.S;
  const u64 d = g % a.D;
  const u64 delta = d * (a.C / a.D);
  const u64 j = blockIdx.y;
  auto bound = [&](u64 jj) -> u64 {
    if (jj == 0) return 0;
    if (jj >= a.nslots) return a.n;
    const u64 p = jj * a.C - delta;
    return p < a.n ? p : a.n;
  };
  const u64 t_begin = bound(j), t_end = bound(j + 1);
  if (t_begin >= t_end) return;  // empty slot
  const u64 cnt = t_end - t_begin;

  u32 s[K];
#pragma unroll
  for (int w = 0; w < K; w++) s[w] = live ? (u32)a.state_in[(u64)w * a.S + i] : 0u;
  if (j > 0) jump_uniform32<V>(s, a.slot_polys + (d * kMaxSlots + j) * 16);

  u32 *lds = lds_all + wave * kWaveLds32;
  u32 *myrow = lds + lane * kStride32;
  const int rows_live = (a.S - row0 < (u64)kWave) ? (int)(a.S - row0) : kWave;
  u32 *base = reinterpret_cast<u32 *>(a.out) + row0 * a.ld + t_begin;
  for (u64 t0 = 0; t0 < cnt; t0 += kT32) {
    const int m = (cnt - t0 < (u64)kT32) ? (int)(cnt - t0) : kT32;
    if (m == kT32) gen_tile32_full<V, KIND>(s, myrow);
    else gen_tile32_partial<V, KIND>(s, myrow, m);
    wave_sync();
    store_tile32<A16, NT>(lds, lane, base + t0, a.ld, rows_live, m);
    wave_sync();
  }
  if (t_end == a.n && live) {
#pragma unroll
    for (int w = 0; w < K; w++) a.state_out[(u64)w * a.S + i] = s[w];
  }
}

// Stream i = seeded base * M^(i J): a per-lane jump by x^((i mod 1024) J)
// and wave-uniform jumps for the upper radix-1024 digits of i.
template <int V>
__global__ __launch_bounds__(kBlock) void k_position32(u64 seed, u64 S, const u64 *__restrict__ tab0,
                                                       const u64 *__restrict__ up, int levels,
                                                       u64 *__restrict__ state_out) {
  constexpr int K = Params32<V>::k;
  const u64 i = (u64)blockIdx.x * kBlock + threadIdx.x;
  const u64 first = i - (threadIdx.x % kWave);
  if (first >= S) return;  // uniform per wave
  u32 s[K];
  splitmix64_fill32<K>(seed, s);
  const unsigned d0 = (unsigned)(i % kTabRadix);
  jump_lane32<V>(s, [&](int wi) { return tab0[(u64)wi * kTabRadix + d0]; });
  for (int l = 1; l < levels; l++) {
    const unsigned d = (unsigned)((first >> (10 * l)) % kTabRadix);
    if (d) jump_uniform32<V>(s, up + ((u64)(l - 1) * kTabRadix + d) * 16);
  }
  if (i < S) {
#pragma unroll
    for (int w = 0; w < K; w++) state_out[(u64)w * S + i] = s[w];
  }
}

template <int V>
__global__ __launch_bounds__(kBlock) void k_jump32(u64 *__restrict__ state, u64 S, UPoly r) {
  constexpr int K = Params32<V>::k;
  const u64 i = (u64)blockIdx.x * kBlock + threadIdx.x;
  const u64 first = i - (threadIdx.x % kWave);
  if (first >= S) return;
  const bool live = i < S;
  u32 s[K];
#pragma unroll
  for (int w = 0; w < K; w++) s[w] = live ? (u32)state[(u64)w * S + i] : 0u;
  jump_uniform32<V>(s, r.w);
  if (live) {
#pragma unroll
    for (int w = 0; w < K; w++) state[(u64)w * S + i] = s[w];
  }
}

// Stream i advances by its own 128-bit distance (digit tables as for the
// 64-bit generators: word w of entry d of level l at tab[(l*W + w)*1024 + d]
// with W = n/64 words).
template <int V>
__global__ __launch_bounds__(kBlock) void k_advance_each32(u64 *__restrict__ state, u64 S,
                                                           const u64 *__restrict__ steps,
                                                           const u64 *__restrict__ tab) {
  constexpr int K = Params32<V>::k;
  constexpr int NW = K / 2;
  const u64 i = (u64)blockIdx.x * kBlock + threadIdx.x;
  const u64 first = i - (threadIdx.x % kWave);
  if (first >= S) return;
  const bool live = i < S;
  u32 s[K];
#pragma unroll
  for (int w = 0; w < K; w++) s[w] = live ? (u32)state[(u64)w * S + i] : 0u;
  const u64 lo = live ? steps[2 * i] : 0;
  const u64 hi = live ? steps[2 * i + 1] : 0;
  for (int l = 0; l < kDigitLevels; l++) {
    const int sh = 10 * l;
    u64 bits;
    if (sh + 10 <= 64) bits = lo >> sh;
    else if (sh >= 64) bits = hi >> (sh - 64);
    else bits = (lo >> sh) | (hi << (64 - sh));
    const unsigned d = (unsigned)(bits & (kTabRadix - 1));
    if (!__any(d != 0)) continue;
    const u64 *t = tab + (u64)l * NW * kTabRadix;
    jump_lane32<V>(s, [&](int wi) { return t[(u64)wi * kTabRadix + d]; });
  }
  if (live) {
#pragma unroll
    for (int w = 0; w < K; w++) state[(u64)w * S + i] = s[w];
  }
}

// ---------------------------------------------------------------- launchers

#define SL_DISPATCH32(v, EXPR_T)     \
  switch (v) {                       \
    case 14: return EXPR_T(14);      \
    case 15: return EXPR_T(15);      \
    case 16: return EXPR_T(16);      \
    case 17: return EXPR_T(17);      \
    case 18: return EXPR_T(18);      \
    default: return hipErrorInvalidValue; \
  }

template <int V, int KIND>
static hipError_t gen32_k(const GenArgs &a, bool nt, dim3 grid, bool a16, hipStream_t st) {
  // nontemporal stores on the 16-byte path only
  if (a16 && nt) hipLaunchKernelGGL((k_generate32<V, KIND, true, true>), grid, dim3(kBlock), 0, st, a);
  else if (a16) hipLaunchKernelGGL((k_generate32<V, KIND, true, false>), grid, dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_generate32<V, KIND, false, false>), grid, dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <int V>
static hipError_t gen32_v(int kind, const GenArgs &a, bool nt, hipStream_t st) {
  const u64 waves = (a.S + kWave - 1) / kWave;
  dim3 grid((unsigned)((waves + (kBlock / kWave) - 1) / (kBlock / kWave)), (unsigned)a.nslots);
  // slot starts are multiples of C/D, a multiple of the tile, so rows start
  // 16-byte aligned when the buffer is and the row stride is a multiple of 4
  const bool a16 = ((uintptr_t)a.out % 16 == 0) && (a.ld % 4 == 0) && ((a.C / a.D) % 4 == 0);
  return kind ? gen32_k<V, 1>(a, nt, grid, a16, st) : gen32_k<V, 0>(a, nt, grid, a16, st);
}

hipError_t launch_generate32(int variant, int kind, const GenArgs &a, bool nt, hipStream_t st) {
#define SL_GEN32(V) gen32_v<V>(kind, a, nt, st)
  SL_DISPATCH32(variant, SL_GEN32)
#undef SL_GEN32
}

template <int V>
static hipError_t pos32_v(u64 seed, u64 S, const u64 *tab0, const u64 *up, int levels, u64 *out,
                          hipStream_t st) {
  dim3 grid((unsigned)((S + kBlock - 1) / kBlock));
  hipLaunchKernelGGL((k_position32<V>), grid, dim3(kBlock), 0, st, seed, S, tab0, up, levels, out);
  return hipGetLastError();
}

hipError_t launch_position32(int variant, uint64_t seed, uint64_t S, const uint64_t *tab0,
                             const uint64_t *up, int levels, uint64_t *state_out, hipStream_t st) {
#define SL_POS32(V) pos32_v<V>(seed, S, tab0, up, levels, state_out, st)
  SL_DISPATCH32(variant, SL_POS32)
#undef SL_POS32
}

template <int V>
static hipError_t jump32_v(u64 *state, u64 S, const UPoly &r, hipStream_t st) {
  dim3 grid((unsigned)((S + kBlock - 1) / kBlock));
  hipLaunchKernelGGL((k_jump32<V>), grid, dim3(kBlock), 0, st, state, S, r);
  return hipGetLastError();
}

hipError_t launch_jump32(int variant, uint64_t *state, uint64_t S, const UPoly &r, hipStream_t st) {
#define SL_JMP32(V) jump32_v<V>(state, S, r, st)
  SL_DISPATCH32(variant, SL_JMP32)
#undef SL_JMP32
}

template <int V>
static hipError_t adv32_v(u64 *state, u64 S, const u64 *steps, const u64 *tab, hipStream_t st) {
  dim3 grid((unsigned)((S + kBlock - 1) / kBlock));
  hipLaunchKernelGGL((k_advance_each32<V>), grid, dim3(kBlock), 0, st, state, S, steps, tab);
  return hipGetLastError();
}

hipError_t launch_advance_each32(int variant, uint64_t *state, uint64_t S, const uint64_t *steps,
                                 const uint64_t *tab, hipStream_t st) {
#define SL_ADV32(V) adv32_v<V>(state, S, steps, tab, st)
  SL_DISPATCH32(variant, SL_ADV32)
#undef SL_ADV32
}

}  // namespace slrng

// gfx950 kernels for bulk generation from scrambled linear generators
// (Blackman & Vigna, "Scrambled Linear Pseudorandom Number Generators").
//
// Design for CDNA4:
//  * one stream per lane; the k-word engine state lives in VGPRs and every
//    step is a handful of 64-bit VALU xor / shift / rotate operations (the
//    code figures of Section "Linear engines");
//  * outputs are stream-major (out[i*ld + t]), so a lane's consecutive outputs
//    are contiguous.  Each wave stages a tile of T outputs per lane in LDS
//    (row = lane) and then reads it back column-wise so that each
//    global_store_dwordx4 writes whole 128/256-byte runs of a few rows:
//    fully coalesced; plain or nontemporal stores as the launch shape says
//    (write-through stores measured slower for this stream-major pattern);
//  * waves never wait on each other: every wave owns its LDS rows and the
//    LDS exchange inside a wave is ordered by the in-order LDS queue plus
//    a wavefront-scope fence (no workgroup barrier);
//  * positioning uses the jump polynomials of the planner (Cayley-Hamilton
//    reading of the paper's jump functions): acc ^= s for every set
//    coefficient while the engine steps.
#include <hip/hip_runtime.h>

#include "engines.hpp"
#include "gen_device.hpp"
#include "kernels.hpp"

namespace slrng {

template <int V, int KIND, int T, bool A16, bool NT>
__global__ __launch_bounds__(kBlock) void k_generate(GenArgs a) {
  constexpr int K = Params<V>::k;
  __shared__ __attribute__((aligned(16))) u64 lds_all[(kBlock / kWave) * TileGeom<T>::kWaveLds];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const u64 g = (u64)blockIdx.x * (kBlock / kWave) + wave;  // stream group
  const u64 row0 = g * kWave;
  if (row0 >= a.S) return;  // uniform per wave
  const u64 i = row0 + lane;
  const bool live = i < a.S;
  // slot boundaries of this group (uniform per wave)
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

  u64 s[K];
#pragma unroll
  for (int w = 0; w < K; w++) s[w] = live ? a.state_in[(u64)w * a.S + i] : 0;
  if (j > 0) jump_uniform<V>(s, a.slot_polys + (d * kMaxSlots + j) * 16);

  u64 *lds = lds_all + wave * TileGeom<T>::kWaveLds;
  u64 *myrow = lds + lane * TileGeom<T>::kStride;
  const int rows_live = (a.S - row0 < (u64)kWave) ? (int)(a.S - row0) : kWave;
  u64 *base = reinterpret_cast<u64 *>(a.out) + row0 * a.ld + t_begin;
  int ph = 0;
  for (u64 t0 = 0; t0 < cnt; t0 += T) {
    const int m = (cnt - t0 < (u64)T) ? (int)(cnt - t0) : T;
    if (m == T) gen_tile_full<V, KIND, T>(s, myrow);
    else ph = gen_tile_partial<V, KIND, T>(s, myrow, m);
    wave_sync();
    store_tile<T, A16, NT>(lds, lane, base + t0, a.ld, rows_live, m);
    wave_sync();
  }
  if constexpr (K == 16) rotate_to_logical<V>(s, ph);
  if (t_end == a.n && live) {
#pragma unroll
    for (int w = 0; w < K; w++) a.state_out[(u64)w * a.S + i] = s[w];
  }
}

// ---------------------------------------------------------------- positioning

template <int V>
__global__ __launch_bounds__(kBlock) void k_position(u64 seed, u64 S, const u64 *__restrict__ tab0,
                                                     const u64 *__restrict__ up, int levels,
                                                     u64 *__restrict__ state_out) {
  constexpr int K = Params<V>::k;
  const u64 i = (u64)blockIdx.x * kBlock + threadIdx.x;
  const u64 first = i - (threadIdx.x % kWave);
  if (first >= S) return;  // uniform per wave
  u64 s[K];
  splitmix64_fill<K>(seed, s);
  const unsigned d0 = (unsigned)(i % kTabRadix);
  jump_lane<V>(s, [&](int wi) { return tab0[(u64)wi * kTabRadix + d0]; });
  for (int l = 1; l < levels; l++) {
    // (i >> 10l) is the same in every lane of a wave (64 divides 1024)
    const unsigned d = (unsigned)((first >> (10 * l)) % kTabRadix);
    if (d) jump_uniform<V>(s, up + ((u64)(l - 1) * kTabRadix + d) * 16);
  }
  if (i < S) {
#pragma unroll
    for (int w = 0; w < K; w++) state_out[(u64)w * S + i] = s[w];
  }
}

template <int V>
__global__ __launch_bounds__(kBlock) void k_jump(u64 *__restrict__ state, u64 S, UPoly r) {
  constexpr int K = Params<V>::k;
  const u64 i = (u64)blockIdx.x * kBlock + threadIdx.x;
  const u64 first = i - (threadIdx.x % kWave);
  if (first >= S) return;
  const bool live = i < S;
  u64 s[K];
#pragma unroll
  for (int w = 0; w < K; w++) s[w] = live ? state[(u64)w * S + i] : 0;
  jump_uniform<V>(s, r.w);
  if (live) {
#pragma unroll
    for (int w = 0; w < K; w++) state[(u64)w * S + i] = s[w];
  }
}

// Stream i advances by J_i = steps[2i] + 2^64 steps[2i+1]: for each
// radix-1024 digit d_l of J_i, one per-lane jump by x^(d_l 2^(10 l)) mod p
// (entry 0 is the polynomial 1, the identity, for lanes whose digit is 0).
// A level is skipped when the digit is 0 in every lane of the wave.
template <int V>
__global__ __launch_bounds__(kBlock) void k_advance_each(u64 *__restrict__ state, u64 S,
                                                         const u64 *__restrict__ steps,
                                                         const u64 *__restrict__ tab) {
  constexpr int K = Params<V>::k;
  const u64 i = (u64)blockIdx.x * kBlock + threadIdx.x;
  const u64 first = i - (threadIdx.x % kWave);
  if (first >= S) return;  // uniform per wave
  const bool live = i < S;
  u64 s[K];
#pragma unroll
  for (int w = 0; w < K; w++) s[w] = live ? state[(u64)w * S + i] : 0;
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
    const u64 *t = tab + (u64)l * K * kTabRadix;
    jump_lane<V>(s, [&](int wi) { return t[(u64)wi * kTabRadix + d]; });
  }
  if (live) {
#pragma unroll
    for (int w = 0; w < K; w++) state[(u64)w * S + i] = s[w];
  }
}

// ---------------------------------------------------------------- calibration

__global__ __launch_bounds__(kBlock) void k_write_ceiling(u64x2 *out, u64 n16) {
  const u64 stride = (u64)gridDim.x * kBlock;
  const u64x2 v = {0x0123456789abcdefull, 0xfedcba9876543210ull};
  for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride) out_store(out + i, v);
}

__global__ __launch_bounds__(kBlock) void k_copy(u64x2 *dst, const u64x2 *src, u64 n16) {
  const u64 stride = (u64)gridDim.x * kBlock;
  for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

// ---------------------------------------------------------------- launchers

template <int V, int KIND, int T>
static hipError_t gen_t(const GenArgs &a, bool nt, hipStream_t st) {
  const u64 waves = (a.S + kWave - 1) / kWave;
  dim3 grid((unsigned)((waves + (kBlock / kWave) - 1) / (kBlock / kWave)), (unsigned)a.nslots);
  // slot starts are multiples of C/D (even), so rows start 16-byte aligned
  // when the buffer and the row stride are
  const bool a16 = ((uintptr_t)a.out % 16 == 0) && (a.ld % 2 == 0) && ((a.C / a.D) % 2 == 0);
  // nontemporal stores on the 16-byte path only (the 8-byte path is the
  // rare misaligned case)
  if (a16 && nt) hipLaunchKernelGGL((k_generate<V, KIND, T, true, true>), grid, dim3(kBlock), 0, st, a);
  else if (a16) hipLaunchKernelGGL((k_generate<V, KIND, T, true, false>), grid, dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_generate<V, KIND, T, false, false>), grid, dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <int V>
static hipError_t gen_v(int kind, const GenArgs &a, const GenConfig &cfg, hipStream_t st) {
  if (cfg.tile == 32) return kind ? gen_t<V, 1, 32>(a, cfg.nt, st) : gen_t<V, 0, 32>(a, cfg.nt, st);
  return kind ? gen_t<V, 1, 16>(a, cfg.nt, st) : gen_t<V, 0, 16>(a, cfg.nt, st);
}

#define SL_DISPATCH(v, EXPR_T)      \
  switch (v) {                      \
    case 0: return EXPR_T(0);       \
    case 1: return EXPR_T(1);       \
    case 2: return EXPR_T(2);       \
    case 3: return EXPR_T(3);       \
    case 4: return EXPR_T(4);       \
    case 5: return EXPR_T(5);       \
    case 6: return EXPR_T(6);       \
    case 7: return EXPR_T(7);       \
    case 8: return EXPR_T(8);       \
    case 9: return EXPR_T(9);       \
    case 10: return EXPR_T(10);     \
    case 11: return EXPR_T(11);     \
    case 12: return EXPR_T(12);     \
    case 13: return EXPR_T(13);     \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_generate(int variant, int kind, const GenArgs &a, const GenConfig &cfg,
                           hipStream_t st) {
#define SL_GEN(V) gen_v<V>(kind, a, cfg, st)
  SL_DISPATCH(variant, SL_GEN)
#undef SL_GEN
}

template <int V>
static hipError_t pos_v(u64 seed, u64 S, const u64 *tab0, const u64 *up, int levels, u64 *out,
                        hipStream_t st) {
  dim3 grid((unsigned)((S + kBlock - 1) / kBlock));
  hipLaunchKernelGGL((k_position<V>), grid, dim3(kBlock), 0, st, seed, S, tab0, up, levels, out);
  return hipGetLastError();
}

hipError_t launch_position(int variant, uint64_t seed, uint64_t S, const uint64_t *tab0,
                           const uint64_t *up, int levels, uint64_t *state_out, hipStream_t st) {
#define SL_POS(V) pos_v<V>(seed, S, tab0, up, levels, state_out, st)
  SL_DISPATCH(variant, SL_POS)
#undef SL_POS
}

template <int V>
static hipError_t jump_v(u64 *state, u64 S, const UPoly &r, hipStream_t st) {
  dim3 grid((unsigned)((S + kBlock - 1) / kBlock));
  hipLaunchKernelGGL((k_jump<V>), grid, dim3(kBlock), 0, st, state, S, r);
  return hipGetLastError();
}

hipError_t launch_jump(int variant, uint64_t *state, uint64_t S, const UPoly &r, hipStream_t st) {
#define SL_JMP(V) jump_v<V>(state, S, r, st)
  SL_DISPATCH(variant, SL_JMP)
#undef SL_JMP
}

template <int V>
static hipError_t advance_each_v(u64 *state, u64 S, const u64 *steps, const u64 *tab,
                                 hipStream_t st) {
  dim3 grid((unsigned)((S + kBlock - 1) / kBlock));
  hipLaunchKernelGGL((k_advance_each<V>), grid, dim3(kBlock), 0, st, state, S, steps, tab);
  return hipGetLastError();
}

hipError_t launch_advance_each(int variant, uint64_t *state, uint64_t S, const uint64_t *steps,
                               const uint64_t *tab, hipStream_t st) {
#define SL_ADV(V) advance_each_v<V>(state, S, steps, tab, st)
  SL_DISPATCH(variant, SL_ADV)
#undef SL_ADV
}

hipError_t launch_write_ceiling(void *out, uint64_t bytes, hipStream_t st) {
  const u64 n16 = bytes / 16;
  hipLaunchKernelGGL(k_write_ceiling, dim3(256 * 32), dim3(kBlock), 0, st,
                     reinterpret_cast<u64x2 *>(out), n16);
  return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t st) {
  const u64 n16 = bytes / 16;
  hipLaunchKernelGGL(k_copy, dim3(256 * 32), dim3(kBlock), 0, st, reinterpret_cast<u64x2 *>(dst),
                     reinterpret_cast<const u64x2 *>(src), n16);
  return hipGetLastError();
}

}  // namespace slrng

// Persistent batched generation kernel (see batch.hpp for the work split).
//
// Each wave repeatedly claims one tile (64 lane-chunks of one variant and
// kind) from an atomic counter, switches on the tile's variant and kind (the
// switch is uniform per wave: the tile index is read through readfirstlane, so
// the branch is a scalar one), positions its lanes (SplitMix64 origin or a
// precomputed request state, then one per-lane jump by the chunk offset), and
// generates with the same LDS-staged tile and store code as k_generate, with a
// destination pointer and a length per row.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "gen_device.hpp"

namespace slrng {

// Output store of the batched kernels by policy: 0 write-through (sc1, the
// default: rows of a tile are consecutive chunks of one request), 1 plain,
// 2 nontemporal.
template <int ST, typename VT>
__device__ __forceinline__ void out_store_pol(VT *p, VT v) {
  if constexpr (ST == 0) out_store_wt(p, v);
  else if constexpr (ST == 1) out_store(p, v);
  else out_store_nt(p, v);
}

// Store a staged tile with per-row destinations and lengths: row r writes
// outputs t0 + c for c < m and t0 + c < len[r].
template <int T, bool A16, int ST>
__device__ __forceinline__ void store_tile_rows(const u64 *lds, int lane, const u64 *rowptr,
                                                const unsigned *rowlen, int nrows, unsigned t0,
                                                int m) {
  constexpr int S = TileGeom<T>::kStride;
  if constexpr (A16) {
    constexpr int LPR = T / 2;
    constexpr int RPI = kWave / LPR;
#pragma unroll
    for (int q = 0; q < T / 2; q++) {
      const int r = q * RPI + lane / LPR;
      const int c = 2 * (lane % LPR);
      if (r < nrows && c < m) {
        const unsigned len = rowlen[r];
        const unsigned col = t0 + (unsigned)c;
        if (col < len) {
          const u64x2 v = *reinterpret_cast<const u64x2 *>(lds + r * S + c);
          u64 *dst = reinterpret_cast<u64 *>(rowptr[r]) + col;
          if (col + 1 < len && c + 1 < m) out_store_pol<ST>(reinterpret_cast<u64x2 *>(dst), v);
          else out_store_pol<ST>(dst, v.x);
        }
      }
    }
  } else {
    constexpr int LPR = T;
    constexpr int RPI = kWave / LPR;
#pragma unroll
    for (int q = 0; q < T; q++) {
      const int r = q * RPI + lane / LPR;
      const int c = lane % LPR;
      if (r < nrows && c < m) {
        const unsigned col = t0 + (unsigned)c;
        if (col < rowlen[r]) out_store_pol<ST>(reinterpret_cast<u64 *>(rowptr[r]) + col, lds[r * S + c]);
      }
    }
  }
}

// The unpredicated store of a full tile (all 64 rows have T more outputs,
// 16-byte aligned rows): lane (r0, c) of the 16-byte layout writes rows
// q*RPI + r0, whose destinations (column c) it holds in dst[q].  All LDS reads
// first, then the stores, so that the reads overlap.
template <int T, int ST>
__device__ __forceinline__ void store_tile_full(const u64 *lds, int lane, const u64 (&dst)[T / 2],
                                                unsigned t0) {
  constexpr int S = TileGeom<T>::kStride;
  constexpr int LPR = T / 2;
  constexpr int RPI = kWave / LPR;
  const int r0 = lane / LPR;
  const int c = 2 * (lane % LPR);
  u64x2 v[T / 2];
#pragma unroll
  for (int q = 0; q < T / 2; q++) v[q] = *reinterpret_cast<const u64x2 *>(lds + (q * RPI + r0) * S + c);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < T / 2; q++) out_store_pol<ST>(reinterpret_cast<u64x2 *>(dst[q] + (u64)t0 * 8), v[q]);
}

template <int V, int KIND, int T, int ST = 0>
__device__ __forceinline__ void batch_tile(const BatchArgs &a, const TileDesc &td, u64 *lds,
                                           u64 *rowptr, unsigned *rowlen, int lane) {
  constexpr int K = Params<V>::k;
  const bool active = lane < (int)td.nlanes;
  LaneDesc ld;
  if (td.flags & kTileRun) {
    const RunDesc rd = a.runs[td.lane0];  // uniform
    const u64 off = (u64)lane * rd.c;
    ld.seed = rd.seed;
    ld.out = rd.out0 + off * 8;
    ld.len = active ? (unsigned)((rd.n_rem - off < (u64)rd.c) ? rd.n_rem - off : rd.c) : 0u;
    ld.jidx = rd.j0 + (unsigned)lane;
    ld.req = rd.req;
    ld.pad = 0;
  } else if (active) {
    ld = a.lanes[td.lane0 + lane];
  } else {
    ld.seed = 0;
    ld.out = 0;
    ld.len = 0;
    ld.jidx = 0;
    ld.req = kNoReqState;
    ld.pad = 0;
  }
  u64 s[K];
  if (ld.req != kNoReqState) {
#pragma unroll
    for (int w = 0; w < K; w++) s[w] = a.req_state[(u64)ld.req * 16 + w];
  } else {
    splitmix64_fill<K>(ld.seed, s);
  }
  if (td.flags & kTileJump) {
    const u64 *tab = a.tab[V];
    const u64 tn = a.tab_n[V];
    const u64 jj = ld.jidx;
    auto word = [&](int wi) { return tab[(u64)wi * tn + jj]; };
    // a run tile's lanes all start from the request's start state
    if (td.flags & kTileRun) jump_lane_from_uniform<V>(s, word);
    else jump_lane<V>(s, word);
  }
  rowptr[lane] = ld.out;
  rowlen[lane] = ld.len;
  const bool a16 = __all((ld.out & 15) == 0);
  wave_sync();
  // destinations of the unpredicated path (16-byte layout), loaded once
  u64 dst[T / 2];
  {
    constexpr int LPR = T / 2;
    constexpr int RPI = kWave / LPR;
    const int r0 = lane / LPR;
    const u64 c8 = 16 * (u64)(lane % LPR);
#pragma unroll
    for (int q = 0; q < T / 2; q++) dst[q] = rowptr[q * RPI + r0] + c8;
  }
  u64 *myrow = lds + lane * TileGeom<T>::kStride;
  const int nrows = td.nlanes;
  for (unsigned t0 = 0; t0 < td.max_len; t0 += T) {
    const int m = (td.max_len - t0 < (unsigned)T) ? (int)(td.max_len - t0) : T;
    if (m == T) gen_tile_full<V, KIND, T>(s, myrow);
    else gen_tile_partial<V, KIND, T>(s, myrow, m);
    wave_sync();
    const bool full = nrows == kWave && m == T && t0 + T <= td.min_len;
    if (a16 && full) store_tile_full<T, ST>(lds, lane, dst, t0);
    else if (a16) store_tile_rows<T, true, ST>(lds, lane, rowptr, rowlen, nrows, t0, m);
    else store_tile_rows<T, false, ST>(lds, lane, rowptr, rowlen, nrows, t0, m);
    wave_sync();
  }
}

// Tile claims.  Wave w of the grid's W waves takes tile w first, with no
// atomic (tiles are ordered heaviest first, so the W heaviest go one to a
// wave); further tiles come from the claim counter, as W plus its old value,
// and only when there are more tiles than waves.  A device-wide atomic on
// one address from every wave of a full grid measurably delays the start of
// every wave (on MI355X a one-tile-per-wave launch over all 256 CUs took
// twice as long as over 64).  When a block's waves are done, one atomic per
// block counts it finished; the last block returns both counters to zero for
// the next launch, so no reset kernel is needed between launches.  With a
// completion signal (a.sig), every wave makes its output stores visible
// device-wide before the block counts itself finished, and the last block
// then signals the host (see BatchArgs).  WT: the kernel's output stores are
// written through the L2 (sc1), so a wave's stores are visible device-wide
// once they have completed, and waiting for the wave's vector-memory counter
// is enough (s_waitcnt vmcnt(0), the other counters left at their maximum);
// other stores also need the L2 written back (an agent-scope release fence).
__device__ __forceinline__ void sig_store(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The wave's next tile into t (uniform); false when none is left.  `first`
// starts true for each wave.
__device__ __forceinline__ bool next_tile(const BatchArgs &a, int lane, unsigned &t, bool &first) {
  const unsigned W = gridDim.x * (kBlock / kWave);
  if (first) {
    first = false;
    t = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (t >= a.ntiles) return false;
    if (t == 0 && a.sig && lane == 0) sig_store(a.sig + 2, (uint64_t)wall_clock64());
    return true;
  }
  if (a.ntiles <= W) return false;
  unsigned v = 0;
  if (lane == 0) v = atomicAdd(a.counter, 1u);
  t = W + (unsigned)__builtin_amdgcn_readfirstlane((int)v);
  return t < a.ntiles;
}

// After the block's waves have claimed their last tile (every wave of the
// block calls it).
template <bool WT>
__device__ __forceinline__ void finish_block(const BatchArgs &a) {
  if (a.sig) {  // uniform
    if constexpr (WT) __builtin_amdgcn_s_waitcnt(0x0F70);
    else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (atomicAdd(a.counter + 1, 1u) == gridDim.x - 1) {
      atomicExch(a.counter, 0u);
      atomicExch(a.counter + 1, 0u);
      if (a.sig) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        sig_store(a.sig + 3, (uint64_t)wall_clock64());
        __hip_atomic_store(a.sig, a.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

// Every variant and kind: the switch on the tile's (variant, kind) is uniform
// per wave (the tile index is read through readfirstlane).
template <int T>
__global__ __launch_bounds__(kBlock) void k_batch(BatchArgs a) {
  __shared__ __attribute__((aligned(16))) u64 lds_all[(kBlock / kWave) * TileGeom<T>::kWaveLds];
  __shared__ u64 rowptr_all[kBlock];
  __shared__ unsigned rowlen_all[kBlock];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  u64 *lds = lds_all + wave * TileGeom<T>::kWaveLds;
  u64 *rowptr = rowptr_all + wave * kWave;
  unsigned *rowlen = rowlen_all + wave * kWave;
  unsigned t = 0;
  bool first = true;
  while (next_tile(a, lane, t, first)) {
    const TileDesc td = a.tiles[t];
    switch (td.variant * 2 + td.kind) {
#define SL_CASE(V)                                                  \
  case 2 * V: batch_tile<V, 0, T>(a, td, lds, rowptr, rowlen, lane); break; \
  case 2 * V + 1: batch_tile<V, 1, T>(a, td, lds, rowptr, rowlen, lane); break;
      SL_CASE(0) SL_CASE(1) SL_CASE(2) SL_CASE(3) SL_CASE(4) SL_CASE(5) SL_CASE(6)
      SL_CASE(7) SL_CASE(8) SL_CASE(9) SL_CASE(10) SL_CASE(11) SL_CASE(12) SL_CASE(13)
#undef SL_CASE
      default: break;
    }
    wave_sync();
  }
  finish_block<true>(a);
}

// The same loop for tiles of one variant (the server's): the registers of
// the other variants' code do not count, so more waves fit on a CU.
template <int V, int T, int ST>
__global__ __launch_bounds__(kBlock) void k_batch1(BatchArgs a) {
  __shared__ __attribute__((aligned(16))) u64 lds_all[(kBlock / kWave) * TileGeom<T>::kWaveLds];
  __shared__ u64 rowptr_all[kBlock];
  __shared__ unsigned rowlen_all[kBlock];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  u64 *lds = lds_all + wave * TileGeom<T>::kWaveLds;
  u64 *rowptr = rowptr_all + wave * kWave;
  unsigned *rowlen = rowlen_all + wave * kWave;
  unsigned t = 0;
  bool first = true;
  while (next_tile(a, lane, t, first)) {
    const TileDesc td = a.tiles[t];
    if (td.kind) batch_tile<V, 1, T, ST>(a, td, lds, rowptr, rowlen, lane);
    else batch_tile<V, 0, T, ST>(a, td, lds, rowptr, rowlen, lane);
    wave_sync();
  }
  finish_block<ST == 0>(a);
}

template <int V>
__global__ __launch_bounds__(kBlock) void k_req_state(ReqArgs a) {
  constexpr int K = Params<V>::k;
  const unsigned i = blockIdx.x * kBlock + threadIdx.x;
  const unsigned first = i - (threadIdx.x % kWave);
  if (first >= a.m) return;
  const bool live = i < a.m;
  u64 s[K];
  if (a.origin_state) {
    const u64 j = live ? a.origin_idx[i] : 0;
#pragma unroll
    for (int w = 0; w < K; w++) s[w] = live ? a.origin_state[(u64)w * a.origin_stride + j] : 0;
  } else {
    splitmix64_fill<K>(live ? a.seeds[i] : 0, s);
  }
  const unsigned pi = live ? i : 0;
  jump_lane<V>(s, [&](int wi) { return a.polys[(u64)pi * 16 + wi]; });
  if (live) {
#pragma unroll
    for (int w = 0; w < K; w++) a.req_state[(u64)a.slot[i] * 16 + w] = s[w];
  }
}

// Columns of the digit matrices.  Matrix e is M^(J_e) with x^(J_e) mod p =
// polys[e * 16 ..]; its row i is e_i M^(J_e), e_i the state whose only set
// bit is bit i (word i / 64, bit i % 64, logical order), and its column b is
// stored as k words: bit r of word w is bit b of row 64 w + r, at
// cols[(e n + b) k + w].  One lane per row: the lane steps e_i through the
// jump, then each wave turns its 64 rows into one word of every column with
// one ballot per bit.
template <int V>
__global__ __launch_bounds__(kBlock) void k_digit_cols(const u64 *__restrict__ polys,
                                                       u64 *__restrict__ cols) {
  constexpr int K = Params<V>::k;
  constexpr int N = 64 * K;
  const unsigned i = blockIdx.x * kBlock + threadIdx.x;
  if (i - (threadIdx.x % kWave) >= (unsigned)N) return;  // uniform per wave (64 divides N)
  const int lane = threadIdx.x % kWave;
  const unsigned w = i / 64;  // this wave's word of every column
  const u64 e = blockIdx.y;
  u64 s[K];
#pragma unroll
  for (int q = 0; q < K; q++) s[q] = (q == (int)w) ? (u64)1 << (i % 64) : 0;
  jump_uniform<V>(s, polys + e * 16);
  u64 *out = cols + e * N * K;
#pragma unroll
  for (int q = 0; q < K; q++) {
    for (int r = 0; r < 64; r++) {
      const u64 m = __ballot((int)((s[q] >> r) & 1));
      if (lane == r) out[(u64)(64 * q + r) * K + w] = m;
    }
  }
}

// Request start states from a 128-bit position, all on the device: s M^pos is
// the origin s multiplied, for every nonzero digit d_l of pos in radix 2^bits,
// by the matrix M^(d_l 2^(bits l)) (entry l 2^bits + d_l of `cols`).  One
// wave per request; bit b of s M^J is the parity of s AND column b: lane
// `lane` takes bits lane, lane + 64, ... (consecutive lanes read consecutive
// columns), and one ballot per state word gathers the product, the same in
// every lane, for the next digit.  The columns a digit needs do not depend on
// the state, so the next nonzero digit's are loaded while the current one is
// applied (two-, four-word engines).
template <int V>
__device__ __forceinline__ void req_state_digits_wave(const ReqArgs &a, const u64 *__restrict__ cols,
                                                      int bits, int levels, unsigned r, int lane) {
  constexpr int K = Params<V>::k;
  constexpr int N = 64 * K;
  constexpr bool kAhead = K <= 4;
  // every input of the request read up front (they may be in host memory:
  // one round trip instead of one per use)
  const u64 pos[2] = {a.pos[2 * (u64)r], a.pos[2 * (u64)r + 1]};
  const u64 slot = a.slot[r];
  u64 s[K];
  if (a.origin_state) {
    const u64 j = a.origin_idx[r];
#pragma unroll
    for (int w = 0; w < K; w++) s[w] = a.origin_state[(u64)w * a.origin_stride + j];
  } else {
    splitmix64_fill<K>(a.seeds[r], s);
  }
  const u64 dmask = ((u64)1 << bits) - 1;
  auto digit = [&](int l) -> unsigned {
    const int b0 = l * bits;  // bits divides 64: a digit never straddles the two words
    return (unsigned)((pos[b0 >> 6] >> (b0 & 63)) & dmask);
  };
  auto next_level = [&](int l) {
    while (l < levels && !digit(l)) l++;
    return l;
  };
  // this lane's columns of one matrix: K columns of K words
  auto load = [&](int l, u64 (&c)[K][K]) {
    const u64 *C = cols + ((((u64)l << bits) + digit(l)) * N) * K;
#pragma unroll
    for (int q = 0; q < K; q++) {
#pragma unroll
      for (int w = 0; w < K; w++) c[q][w] = C[(u64)(64 * q + lane) * K + w];
    }
  };
  auto apply = [&](const u64 (&c)[K][K]) {
    u64 t[K];
#pragma unroll
    for (int q = 0; q < K; q++) {
      unsigned cnt = 0;
#pragma unroll
      for (int w = 0; w < K; w++) {
        const u64 v = s[w] & c[q][w];
        cnt += __popc((unsigned)v) + __popc((unsigned)(v >> 32));
      }
      t[q] = __ballot((int)(cnt & 1));
    }
#pragma unroll
    for (int q = 0; q < K; q++) s[q] = t[q];
  };
  int l = next_level(0);
  if constexpr (kAhead) {
    u64 cur[K][K], nxt[K][K];
    if (l < levels) load(l, cur);
    while (l < levels) {
      const int ln = next_level(l + 1);
      if (ln < levels) load(ln, nxt);
      apply(cur);
#pragma unroll
      for (int q = 0; q < K; q++) {
#pragma unroll
        for (int w = 0; w < K; w++) cur[q][w] = nxt[q][w];
      }
      l = ln;
    }
  } else {
    while (l < levels) {
      u64 cur[K][K];
      load(l, cur);
      apply(cur);
      l = next_level(l + 1);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int w = 0; w < K; w++) a.req_state[slot * 16 + w] = s[w];
  }
}

template <int V>
__global__ __launch_bounds__(kBlock) void k_req_state_digits(ReqArgs a, const u64 *__restrict__ cols,
                                                             int bits, int levels) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const unsigned r = blockIdx.x * (kBlock / kWave) + wave;
  if (r >= a.m) return;  // uniform per wave
  req_state_digits_wave<V>(a, cols, bits, levels, r, lane);
}

// A served iteration's prologue in one launch: blocks [0, up_blocks) copy
// the descriptor pack (n16 16-byte words) from pinned host memory, through
// its device mapping, to device memory, block 0 first stamping the device
// clock; the other blocks compute the request start states as
// k_req_state_digits does, one wave per request, reading positions, origins
// and slots from the same pinned memory, so the two parts do not wait for
// each other and the generation kernel follows one launch instead of two.
template <int V>
__global__ __launch_bounds__(kBlock) void k_prologue(ReqArgs a, const u64 *__restrict__ cols, int bits,
                                                     int levels, const uint4 *__restrict__ src,
                                                     uint4 *__restrict__ dst, u64 n16,
                                                     unsigned up_blocks, u64 *stamp) {
  if (blockIdx.x < up_blocks) {
    if (stamp && blockIdx.x == 0 && threadIdx.x == 0)
      __hip_atomic_store(stamp, (u64)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const u64 stride = (u64)up_blocks * kBlock;
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
    return;
  }
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const unsigned r = (blockIdx.x - up_blocks) * (kBlock / kWave) + wave;
  if (r >= a.m) return;  // uniform per wave
  req_state_digits_wave<V>(a, cols, bits, levels, r, lane);
}

template <int V, int ST>
static hipError_t batch1_vs(const BatchArgs &a, int tile, unsigned blocks, hipStream_t st) {
  if (tile == 16) hipLaunchKernelGGL((k_batch1<V, 16, ST>), dim3(blocks), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_batch1<V, 32, ST>), dim3(blocks), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <int V>
static hipError_t batch1_v(const BatchArgs &a, int tile, unsigned blocks, hipStream_t st, int store) {
  if (store == 1) return batch1_vs<V, 1>(a, tile, blocks, st);
  if (store == 2) return batch1_vs<V, 2>(a, tile, blocks, st);
  return batch1_vs<V, 0>(a, tile, blocks, st);
}

template <int V>
static hipError_t batch1_occupancy_v(int tile, int *blocks) {
  return tile == 16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch1<V, 16, 0>, kBlock, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch1<V, 32, 0>, kBlock, 0);
}

#define SL_DISPATCH64(v, EXPR)           \
  switch (v) {                           \
    case 0: return EXPR(0);              \
    case 1: return EXPR(1);              \
    case 2: return EXPR(2);              \
    case 3: return EXPR(3);              \
    case 4: return EXPR(4);              \
    case 5: return EXPR(5);              \
    case 6: return EXPR(6);              \
    case 7: return EXPR(7);              \
    case 8: return EXPR(8);              \
    case 9: return EXPR(9);              \
    case 10: return EXPR(10);            \
    case 11: return EXPR(11);            \
    case 12: return EXPR(12);            \
    case 13: return EXPR(13);            \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_batch(const BatchArgs &a, int tile, unsigned blocks, hipStream_t st, int variant,
                        int store) {
  if (variant >= 0) {
#define SL_B1(V) batch1_v<V>(a, tile, blocks, st, store)
    SL_DISPATCH64(variant, SL_B1)
#undef SL_B1
  }
  if (tile == 16) hipLaunchKernelGGL(k_batch<16>, dim3(blocks), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL(k_batch<32>, dim3(blocks), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t batch_resident_blocks_per_cu(int tile, int *blocks, int variant) {
  if (variant >= 0) {
#define SL_O1(V) batch1_occupancy_v<V>(tile, blocks)
    SL_DISPATCH64(variant, SL_O1)
#undef SL_O1
  }
  return tile == 16
             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch<16>, kBlock, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch<32>, kBlock, 0);
}

template <int V>
static hipError_t req_v(const ReqArgs &a, hipStream_t st) {
  dim3 grid((a.m + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_req_state<V>), grid, dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <int V>
static hipError_t digit_cols_v(const u64 *polys, unsigned entries, u64 *cols, hipStream_t st) {
  constexpr int N = 64 * Params<V>::k;
  dim3 grid((N + kBlock - 1) / kBlock, entries);
  hipLaunchKernelGGL((k_digit_cols<V>), grid, dim3(kBlock), 0, st, polys, cols);
  return hipGetLastError();
}

template <int V>
static hipError_t req_digits_v(const ReqArgs &a, const u64 *cols, int bits, int levels, hipStream_t st) {
  dim3 grid((a.m + (kBlock / kWave) - 1) / (kBlock / kWave));
  hipLaunchKernelGGL((k_req_state_digits<V>), grid, dim3(kBlock), 0, st, a, cols, bits, levels);
  return hipGetLastError();
}

hipError_t launch_digit_cols(int variant, const uint64_t *polys, unsigned entries, uint64_t *cols,
                             hipStream_t st) {
#define SL_DR(V) digit_cols_v<V>(polys, entries, cols, st)
  SL_DISPATCH64(variant, SL_DR)
#undef SL_DR
}

template <int V>
static hipError_t prologue_v(const ReqArgs &a, const u64 *cols, int bits, int levels, const uint4 *src,
                             uint4 *dst, u64 n16, u64 *stamp, hipStream_t st) {
  const u64 ub = (n16 + kBlock - 1) / kBlock;
  const unsigned up_blocks = (unsigned)(ub == 0 ? 1 : ub < 1024 ? ub : 1024);
  const unsigned req_blocks = (a.m + (kBlock / kWave) - 1) / (kBlock / kWave);
  hipLaunchKernelGGL((k_prologue<V>), dim3(up_blocks + req_blocks), dim3(kBlock), 0, st, a, cols, bits,
                     levels, src, dst, n16, up_blocks, stamp);
  return hipGetLastError();
}

hipError_t launch_prologue(int variant, const ReqArgs &a, const uint64_t *cols, int bits, int levels,
                           void *dst, const void *src, size_t bytes, uint64_t *stamp, hipStream_t st) {
  if ((bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15)) return hipErrorInvalidValue;
  const uint4 *s16 = static_cast<const uint4 *>(src);
  uint4 *d16 = static_cast<uint4 *>(dst);
  const u64 n16 = bytes / 16;
#define SL_PR(V) prologue_v<V>(a, cols, bits, levels, s16, d16, n16, stamp, st)
  SL_DISPATCH64(variant, SL_PR)
#undef SL_PR
}

hipError_t launch_req_state_digits(int variant, const ReqArgs &a, const uint64_t *cols, int bits,
                                   int levels, hipStream_t st) {
  if (a.m == 0) return hipSuccess;
#define SL_RD(V) req_digits_v<V>(a, cols, bits, levels, st)
  SL_DISPATCH64(variant, SL_RD)
#undef SL_RD
}

hipError_t launch_req_state(int variant, const ReqArgs &a, hipStream_t st) {
  switch (variant) {
    case 0: return req_v<0>(a, st);
    case 1: return req_v<1>(a, st);
    case 2: return req_v<2>(a, st);
    case 3: return req_v<3>(a, st);
    case 4: return req_v<4>(a, st);
    case 5: return req_v<5>(a, st);
    case 6: return req_v<6>(a, st);
    case 7: return req_v<7>(a, st);
    case 8: return req_v<8>(a, st);
    case 9: return req_v<9>(a, st);
    case 10: return req_v<10>(a, st);
    case 11: return req_v<11>(a, st);
    case 12: return req_v<12>(a, st);
    case 13: return req_v<13>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace slrng

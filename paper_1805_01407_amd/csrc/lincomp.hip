// On-device linearity check: the linear complexity of one output bit of
// every stream, by Berlekamp-Massey over Z/2Z -- the measurement the paper
// uses in Section "A theoretical analysis of scramblers" (subsection on
// representing scramblers by polynomials, and the + and * scrambler
// subsections with table tab:plusdeg) to see how far a scrambler lifts the
// linear complexity of the low bits above the engine's n.
//
// One wave per workgroup, one stream per lane, the streams are not advanced.
// Each lane keeps three bit arrays in LDS, word-interleaved across the lanes
// ([array][word][lane]) so that every LDS access of the wave is
// conflict-free:
//   R  the nbits sequence bits in reverse order (s_t at bit nbits - 1 - t),
//      so that the window s_N, s_{N-1}, ... of step N is R shifted right by
//      nbits - 1 - N (a funnel shift per word, v_alignbit);
//   C  the current connection polynomial (C_0 = 1);
//   B  the connection polynomial before the last length change.
// Massey's iteration: the discrepancy d = parity(C & window); if d = 1,
// C <- C + x^m B; when 2L <= N the length changes to N + 1 - L and B takes
// the old C (the two arrays swap roles instead of being copied).
#include <hip/hip_runtime.h>

#include "engines.hpp"
#include "engines32.hpp"
#include "gen_device.hpp"
#include "kernels.hpp"
#include "lincomp.hpp"

namespace slrng {

// 32 consecutive outputs of a 64-bit generator, bit `bit` of output j at bit
// 31 - j of the result (so that later outputs sit at lower positions).
template <int V>
__device__ __forceinline__ unsigned next32_bits(u64 (&s)[Params<V>::k], int bit) {
  constexpr int BLK = block_steps<V>();
  unsigned v = 0;
  static_for<32>([&](auto J) {
    constexpr int P = J.value % BLK;
    v |= (unsigned)((output<V, P>(s) >> bit) & 1) << (31 - J.value);
    step<V, P>(s);
  });
  return v;
}

template <int V>
__device__ __forceinline__ unsigned next32_bits32(u32 (&s)[Params32<V>::k], int bit) {
  unsigned v = 0;
#pragma unroll
  for (int j = 0; j < 32; j++) {
    v |= ((output32<V>(s) >> bit) & 1u) << (31 - j);
    step32<V>(s);
  }
  return v;
}

// Berlekamp-Massey on the lane's sequence held in R (nbits bits, reversed).
__device__ __forceinline__ unsigned massey(unsigned *lds, int lane, unsigned nbits, unsigned nwa) {
  auto at = [&](int arr, unsigned w) -> unsigned & { return lds[((unsigned)arr * nwa + w) * kWave + lane]; };
  unsigned L = 0, m = 1;
  int cidx = 1;  // array holding C (1 or 2); the other holds B
  for (unsigned N = 0; N < nbits; N++) {
    const unsigned base = nbits - 1 - N;
    const unsigned q = base >> 5, r = base & 31;
    unsigned W = (N + 1) / 32 + 1;  // C has degree <= N + 1
    if (W > nwa - 2) W = nwa - 2;
    unsigned acc = 0;
    for (unsigned w = 0; w < W; w++) {
      const unsigned lo = at(0, q + w), hi = at(0, q + w + 1);
      const unsigned win = r ? __builtin_amdgcn_alignbit(hi, lo, r) : lo;
      acc ^= at(cidx, w) & win;
    }
    const unsigned d = __popc(acc) & 1u;
    if (d) {
      const int bidx = 3 - cidx;
      const bool swap = 2 * L <= N;
      const unsigned qm = m >> 5, rm = m & 31;
      unsigned W2 = (N + 1) / 32 + 2;
      if (W2 > nwa) W2 = nwa;
      // high words first: B[w - qm] and B[w - qm - 1] are read before any
      // lower word of the destination is written
      for (unsigned w = W2; w-- > 0;) {
        const unsigned b1 = w >= qm ? at(bidx, w - qm) : 0u;
        const unsigned b0 = w >= qm + 1 ? at(bidx, w - qm - 1) : 0u;
        const unsigned bs = rm ? __builtin_amdgcn_alignbit(b1, b0, 32 - rm) : b1;
        const unsigned nv = at(cidx, w) ^ bs;
        at(swap ? bidx : cidx, w) = nv;
      }
      if (swap) {
        L = N + 1 - L;
        cidx = bidx;  // the B array now holds the new C; the old C is B
        m = 1;
      } else {
        m++;
      }
    } else {
      m++;
    }
  }
  return L;
}

template <int V, bool W32>
__global__ __launch_bounds__(kWave) void k_lincomp(const u64 *__restrict__ state, u64 S, int bit,
                                                   unsigned nbits, unsigned nwa,
                                                   unsigned *__restrict__ out) {
  extern __shared__ unsigned lds[];
  const int lane = threadIdx.x;
  const u64 i = (u64)blockIdx.x * kWave + lane;
  const bool live = i < S;
  for (unsigned w = 0; w < 3 * nwa; w++) lds[w * kWave + lane] = 0u;
  lds[(1 * nwa) * kWave + lane] = 1u;  // C = 1
  lds[(2 * nwa) * kWave + lane] = 1u;  // B = 1
  const unsigned nw = nbits / 32;
  if constexpr (W32) {
    constexpr int K = Params32<V>::k;
    u32 s[K];
#pragma unroll
    for (int w = 0; w < K; w++) s[w] = live ? (u32)state[(u64)w * S + i] : 0u;
    for (unsigned k = 0; k < nw; k++) lds[(nw - 1 - k) * kWave + lane] = next32_bits32<V>(s, bit);
  } else {
    constexpr int K = Params<V>::k;
    u64 s[K];
#pragma unroll
    for (int w = 0; w < K; w++) s[w] = live ? state[(u64)w * S + i] : 0;
    for (unsigned k = 0; k < nw; k++) lds[(nw - 1 - k) * kWave + lane] = next32_bits<V>(s, bit);
  }
  const unsigned L = massey(lds, lane, nbits, nwa);
  if (live) out[i] = L;
}

// ---------------------------------------------------------------- rank over Z/2Z
//
// Gaussian elimination of an nrows x ncols bit matrix (both <= 1024) held in
// LDS by one workgroup of 1024 threads, one row per thread.  Storage is
// word-major, rows[q * nrows + r] = columns 64q .. 64q+63 of row r (bit b =
// column 64q + b), so the threads of a wave touch consecutive words.  For each
// column: the lowest unused row with that bit set is the pivot (one ballot per
// wave, an LDS atomic minimum across waves); every other unused row with the
// bit set adds the pivot row.  The rank is the number of pivots.  Two
// barriers per column; the pivot slot alternates between two LDS words so
// that clearing the next one needs no third.
__device__ unsigned eliminate(u64 *rows, unsigned nrows, unsigned ncols, unsigned *piv) {
  const unsigned tid = threadIdx.x;
  const unsigned lane = tid % kWave;
  const unsigned nwords = (ncols + 63) / 64;
  bool used = tid >= nrows;  // threads past the last row never take part
  unsigned rank = 0;
  if (tid == 0) {
    piv[0] = nrows;
    piv[1] = nrows;
  }
  __syncthreads();
  for (unsigned c = 0; c < ncols; c++) {
    const unsigned q = c / 64, b = c % 64;
    const bool cand = !used && ((rows[q * nrows + tid] >> b) & 1);
    const u64 mask = __ballot(cand);
    if (mask && lane == 0) atomicMin(&piv[c & 1], tid + (unsigned)__builtin_ctzll(mask));
    if (tid == 0) piv[(c + 1) & 1] = nrows;
    __syncthreads();
    const unsigned p = piv[c & 1];
    if (p < nrows) {
      rank++;
      if (tid == p) used = true;
      else if (cand) {
        for (unsigned w = q; w < nwords; w++) rows[w * nrows + tid] ^= rows[w * nrows + p];
      }
    }
    __syncthreads();
  }
  return rank;
}

constexpr unsigned kRankMax = 1024;  // rows and columns

__global__ __launch_bounds__(kRankMax) void k_gf2_rank(const u64 *__restrict__ in, unsigned nrows,
                                                       unsigned ncols, unsigned *__restrict__ out) {
  __shared__ u64 rows[kRankMax * (kRankMax / 64)];
  __shared__ unsigned piv[2];
  const unsigned tid = threadIdx.x;
  const unsigned nwords = (ncols + 63) / 64;
  if (tid < nrows)
    for (unsigned w = 0; w < nwords; w++) rows[w * nrows + tid] = in[(u64)tid * nwords + w];
  // columns past ncols in the last word are ignored by eliminate()
  const unsigned r = eliminate(rows, nrows, ncols, piv);
  if (tid == 0) *out = r;
}

// Row i of the equidistribution matrix: word `word` of e_i M^t for t < dims
// (e_i = the state with logical bit i set: word i / w, bit i % w), word t at
// columns t w .. t w + w - 1.
template <int V>
__device__ void equidist_row64(u64 *rows, unsigned n, int word, int dims) {
  constexpr int K = Params<V>::k;
  const unsigned i = threadIdx.x;
  u64 s[K];
#pragma unroll
  for (int w = 0; w < K; w++) s[w] = (unsigned)w == i / 64 ? (1ull << (i % 64)) : 0ull;
  for (int t = 0; t < dims; t++) {
    u64 x = 0;
#pragma unroll
    for (int w = 0; w < K; w++)
      if (w == word) x = s[w];
    rows[(unsigned)t * n + i] = x;
    step<V, 0>(s);
    if constexpr (K == 16) rotate_to_logical<V>(s, 1);  // back to logical order
  }
}

template <int V>
__device__ void equidist_row32(u64 *rows, unsigned n, int word, int dims) {
  constexpr int K = Params32<V>::k;
  const unsigned i = threadIdx.x;
  u32 s[K];
#pragma unroll
  for (int w = 0; w < K; w++) s[w] = (unsigned)w == i / 32 ? (1u << (i % 32)) : 0u;
  const unsigned nwords = ((unsigned)dims * 32 + 63) / 64;
  for (unsigned q = 0; q < nwords; q++) rows[q * n + i] = 0;
  for (int t = 0; t < dims; t++) {
    u32 x = 0;
#pragma unroll
    for (int w = 0; w < K; w++)
      if (w == word) x = s[w];
    rows[(unsigned)(t / 2) * n + i] |= (u64)x << (32 * (t % 2));
    step32<V>(s);
  }
}

template <int V, bool W32>
constexpr unsigned state_bits() {
  if constexpr (W32) return 32u * Params32<V>::k;
  else return 64u * Params<V>::k;
}

template <int V, bool W32>
__global__ __launch_bounds__(kRankMax) void k_equidist_rank(int word, int dims, unsigned *__restrict__ out) {
  __shared__ u64 rows[kRankMax * (kRankMax / 64)];
  __shared__ unsigned piv[2];
  constexpr unsigned n = state_bits<V, W32>();
  if (threadIdx.x < n) {
    if constexpr (W32) equidist_row32<V>(rows, n, word, dims);
    else equidist_row64<V>(rows, n, word, dims);
  }
  const unsigned r = eliminate(rows, n, (unsigned)dims * (W32 ? 32u : 64u), piv);
  if (threadIdx.x == 0) *out = r;
}

#define SL_DISPATCH_ALL(v, EXPR64, EXPR32) \
  switch (v) {                             \
    case 0: return EXPR64(0);              \
    case 1: return EXPR64(1);              \
    case 2: return EXPR64(2);              \
    case 3: return EXPR64(3);              \
    case 4: return EXPR64(4);              \
    case 5: return EXPR64(5);              \
    case 6: return EXPR64(6);              \
    case 7: return EXPR64(7);              \
    case 8: return EXPR64(8);              \
    case 9: return EXPR64(9);              \
    case 10: return EXPR64(10);            \
    case 11: return EXPR64(11);            \
    case 12: return EXPR64(12);            \
    case 13: return EXPR64(13);            \
    case 14: return EXPR32(14);            \
    case 15: return EXPR32(15);            \
    case 16: return EXPR32(16);            \
    case 17: return EXPR32(17);            \
    case 18: return EXPR32(18);            \
    default: return hipErrorInvalidValue;  \
  }

template <int V, bool W32>
static hipError_t lincomp_v(const u64 *state, u64 S, int bit, unsigned nbits, unsigned *out,
                            hipStream_t st) {
  const unsigned nwa = lincomp_words(nbits);
  const size_t lds = (size_t)3 * nwa * kWave * 4;
  dim3 grid((unsigned)((S + kWave - 1) / kWave));
  hipLaunchKernelGGL((k_lincomp<V, W32>), grid, dim3(kWave), lds, st, state, S, bit, nbits, nwa, out);
  return hipGetLastError();
}

hipError_t launch_lincomp(int variant, const uint64_t *state, uint64_t S, int bit, unsigned nbits,
                          unsigned *out, hipStream_t st) {
#define SL_LC64(V) lincomp_v<V, false>(state, S, bit, nbits, out, st)
#define SL_LC32(V) lincomp_v<V, true>(state, S, bit, nbits, out, st)
  SL_DISPATCH_ALL(variant, SL_LC64, SL_LC32)
#undef SL_LC64
#undef SL_LC32
}

hipError_t launch_gf2_rank(const uint64_t *rows, unsigned nrows, unsigned ncols, unsigned *out,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_gf2_rank, dim3(1), dim3(kRankMax), 0, st, rows, nrows, ncols, out);
  return hipGetLastError();
}

template <int V, bool W32>
static hipError_t equidist_v(int word, int dims, unsigned *out, hipStream_t st) {
  hipLaunchKernelGGL((k_equidist_rank<V, W32>), dim3(1), dim3(kRankMax), 0, st, word, dims, out);
  return hipGetLastError();
}

hipError_t launch_equidist_rank(int variant, int word, int dims, unsigned *out, hipStream_t st) {
#define SL_ED64(V) equidist_v<V, false>(word, dims, out, st)
#define SL_ED32(V) equidist_v<V, true>(word, dims, out, st)
  SL_DISPATCH_ALL(variant, SL_ED64, SL_ED32)
#undef SL_ED64
#undef SL_ED32
}

}  // namespace slrng

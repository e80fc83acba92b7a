// F2[x] arithmetic modulo an engine's characteristic polynomial on the
// device: tables of jump polynomials and x^J mod p for arbitrary distances.
//
// A polynomial of degree < n = 64 K is K little-endian words (bit i of word
// i/64 is the coefficient of x^i).  By Cayley-Hamilton, x^J mod p gives the
// jump of J steps (Section "Combining linear engines and scramblers"):
// state M^J = sum_i r_i state M^i for r = x^J mod p.
//
//  * a b mod p is the sum of x^i b mod p over the set bits i of a, the
//    factor x^i b built by repeated multiplication by x (a shift, then p
//    subtracted when the degree reaches n): one lane per product.
//  * Squaring is linear over Z/2Z: (sum a_i x^i)^2 = sum a_i x^(2i), so a^2
//    mod p is the sum of the rows x^(2i) mod p selected by the bits of a;
//    a wave squares by letting each lane sum the rows of its bits and
//    xor-reducing across the wave.  The chain x^(2^m) mod p of a table's
//    bases is a sequence of such squarings.
//  * Table entry (l, d) = x^(d 2^(e0 + b l)) mod p is the product of the
//    bases x^(2^(e0 + b l + j)) of the set bits j of d: entry d is entry
//    d - 2^h times one base (h the highest set bit of d), built in rounds of
//    increasing popcount(d), one launch per round.
#include <hip/hip_runtime.h>

#include "xpow.hpp"

namespace slrng {
namespace {

template <int K>
struct PLow {
  uint64_t w[K];  // p(x) - x^n
};

// c = c x mod p
template <int K>
__device__ __forceinline__ void mulx(uint64_t (&c)[K], const PLow<K> &p) {
  const uint64_t top = 0 - (c[K - 1] >> 63);
#pragma unroll
  for (int v = K - 1; v > 0; v--) c[v] = (c[v] << 1) | (c[v - 1] >> 63);
  c[0] <<= 1;
#pragma unroll
  for (int v = 0; v < K; v++) c[v] ^= p.w[v] & top;
}

// r = a b mod p
template <int K>
__device__ void mulmod(const uint64_t (&a)[K], const uint64_t (&b)[K], const PLow<K> &p,
                       uint64_t (&r)[K]) {
  uint64_t acc[K], cur[K];
#pragma unroll
  for (int v = 0; v < K; v++) {
    acc[v] = 0;
    cur[v] = b[v];
  }
#pragma unroll
  for (int w = 0; w < K; w++) {
    uint64_t aw = a[w];
#pragma unroll 2
    for (int i = 0; i < 64; i++) {
      const uint64_t m = 0 - (aw & 1);
      aw >>= 1;
#pragma unroll
      for (int v = 0; v < K; v++) acc[v] ^= cur[v] & m;
      mulx<K>(cur, p);
    }
  }
#pragma unroll
  for (int v = 0; v < K; v++) r[v] = acc[v];
}

__device__ __forceinline__ uint64_t wave_xor(uint64_t v) {
  int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo ^= __shfl_xor(lo, o);
    hi ^= __shfl_xor(hi, o);
  }
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Rows x^(2i) mod p for i < n, X2[i K + w]: one lane, two multiplications by
// x per row.
template <int K>
__global__ __launch_bounds__(64) void k_xpow_sq_rows(PLow<K> p, uint64_t *X2) {
  if (threadIdx.x != 0) return;
  uint64_t cur[K];
#pragma unroll
  for (int v = 0; v < K; v++) cur[v] = v == 0 ? 1 : 0;
  for (int i = 0; i < 64 * K; i++) {
#pragma unroll
    for (int v = 0; v < K; v++) X2[(size_t)i * K + v] = cur[v];
    mulx<K>(cur, p);
    mulx<K>(cur, p);
  }
}

// bases[m K + w] = x^(2^(e0 + m)) mod p for m < M: one wave squaring from x.
template <int K>
__global__ __launch_bounds__(64) void k_xpow_bases(const uint64_t *__restrict__ X2, int e0, int M,
                                                   uint64_t *bases) {
  const int lane = threadIdx.x;
  uint64_t cur[K];
#pragma unroll
  for (int v = 0; v < K; v++) cur[v] = v == 0 ? 2 : 0;  // x (n >= 64)
  for (int s = 0;; s++) {
    if (s >= e0 && lane == 0) {
#pragma unroll
      for (int v = 0; v < K; v++) bases[(size_t)(s - e0) * K + v] = cur[v];
    }
    if (s + 1 >= e0 + M) break;
    uint64_t acc[K];
#pragma unroll
    for (int v = 0; v < K; v++) acc[v] = 0;
#pragma unroll
    for (int w = 0; w < K; w++) {
      if ((cur[w] >> lane) & 1) {
        const uint64_t *row = X2 + (size_t)(64 * w + lane) * K;
#pragma unroll
        for (int v = 0; v < K; v++) acc[v] ^= row[v];
      }
    }
#pragma unroll
    for (int v = 0; v < K; v++) cur[v] = wave_xor(acc[v]);
  }
}

// Round r of a table: the entries whose digit d has r set bits.
template <int K>
__global__ __launch_bounds__(256) void k_xpow_digits(PLow<K> p, const uint64_t *__restrict__ bases,
                                                     int bits, int levels, int r, uint64_t *out,
                                                     XpowLayout lay) {
  const unsigned per = 1u << bits;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)levels * per) return;
  const unsigned l = (unsigned)(idx / per), d = (unsigned)(idx % per);
  if (__popc(d) != r) return;
  uint64_t *o = out + l * lay.ls + d * lay.ds;
  if (r == 0) {
#pragma unroll
    for (int v = 0; v < K; v++) o[v * lay.ws] = v == 0 ? 1 : 0;
    return;
  }
  const int h = 31 - __clz(d);
  const uint64_t *b = bases + (size_t)(bits * l + h) * K;
  uint64_t bv[K];
#pragma unroll
  for (int v = 0; v < K; v++) bv[v] = b[v];
  if (r == 1) {
#pragma unroll
    for (int v = 0; v < K; v++) o[v * lay.ws] = bv[v];
    return;
  }
  const uint64_t *a = out + l * lay.ls + (d ^ (1u << h)) * lay.ds;
  uint64_t av[K], rv[K];
#pragma unroll
  for (int v = 0; v < K; v++) av[v] = a[v * lay.ws];
  mulmod<K>(av, bv, p, rv);
#pragma unroll
  for (int v = 0; v < K; v++) o[v * lay.ws] = rv[v];
}

// x^J mod p for m distances: the product of the radix-1024 digit entries.
// J_j from the array J, or, when J is null, J_j = j0 + j step (mod 2^128);
// word w of result j at out[j es + w ws].
template <int K>
__global__ __launch_bounds__(256) void k_xpow_batch(PLow<K> p, const uint64_t *__restrict__ digits,
                                                    const uint64_t *__restrict__ J, uint64_t j0_lo,
                                                    uint64_t j0_hi, uint64_t step, uint64_t m,
                                                    uint64_t *out, uint64_t es, uint64_t ws) {
  const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= m) return;
  uint64_t lo, hi;
  if (J) {
    lo = J[2 * j];
    hi = J[2 * j + 1];
  } else {
    const uint64_t plo = j * step, phi = __umul64hi(j, step);
    lo = j0_lo + plo;
    hi = j0_hi + phi + (lo < plo ? 1 : 0);
  }
  uint64_t acc[K];
#pragma unroll
  for (int v = 0; v < K; v++) acc[v] = v == 0 ? 1 : 0;
  bool unit = true;  // acc is still 1
  for (int l = 0; l < 13; l++) {
    const int sh = 10 * l;
    uint64_t bitsv;
    if (sh + 10 <= 64) bitsv = lo >> sh;
    else if (sh >= 64) bitsv = hi >> (sh - 64);
    else bitsv = (lo >> sh) | (hi << (64 - sh));
    const unsigned d = (unsigned)(bitsv & 1023);
    if (!d) continue;
    uint64_t e[K];
#pragma unroll
    for (int v = 0; v < K; v++) e[v] = digits[((size_t)l * K + v) * 1024 + d];
    if (unit) {
#pragma unroll
      for (int v = 0; v < K; v++) acc[v] = e[v];
      unit = false;
    } else {
      uint64_t r[K];
      mulmod<K>(acc, e, p, r);
#pragma unroll
      for (int v = 0; v < K; v++) acc[v] = r[v];
    }
  }
#pragma unroll
  for (int v = 0; v < K; v++) out[j * es + v * ws] = acc[v];
}

template <int K>
hipError_t table_k(const uint64_t *p_low, int e0, int bits, int levels, uint64_t *out,
                   XpowLayout lay, hipStream_t st) {
  PLow<K> p;
  for (int v = 0; v < K; v++) p.w[v] = p_low[v];
  const int M = bits * levels;
  uint64_t *X2 = nullptr, *bases = nullptr;
  hipError_t e = hipMalloc(&X2, (size_t)64 * K * K * 8);
  if (e == hipSuccess) e = hipMalloc(&bases, (size_t)M * K * 8);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_xpow_sq_rows<K>, dim3(1), dim3(64), 0, st, p, X2);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_xpow_bases<K>, dim3(1), dim3(64), 0, st, X2, e0, M, bases);
    e = hipGetLastError();
  }
  const size_t total = (size_t)levels << bits;
  const unsigned grid = (unsigned)((total + 255) / 256);
  for (int r = 0; r <= bits && e == hipSuccess; r++) {
    hipLaunchKernelGGL(k_xpow_digits<K>, dim3(grid), dim3(256), 0, st, p, bases, bits, levels, r, out, lay);
    e = hipGetLastError();
  }
  const hipError_t es = hipStreamSynchronize(st);
  if (X2) (void)hipFree(X2);
  if (bases) (void)hipFree(bases);
  return e != hipSuccess ? e : es;
}

template <int K>
hipError_t batch_k(const uint64_t *p_low, const uint64_t *digits, const uint64_t *J, uint64_t j0_lo,
                   uint64_t j0_hi, uint64_t step, uint64_t m, uint64_t *out, uint64_t es,
                   uint64_t ws, hipStream_t st) {
  PLow<K> p;
  for (int v = 0; v < K; v++) p.w[v] = p_low[v];
  const uint64_t grid = (m + 255) / 256;
  if (grid > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_xpow_batch<K>, dim3((unsigned)grid), dim3(256), 0, st, p, digits, J, j0_lo, j0_hi,
                     step, m, out, es, ws);
  return hipGetLastError();
}

hipError_t batch_any(int K, const uint64_t *p_low, const uint64_t *digits, const uint64_t *J,
                     uint64_t j0_lo, uint64_t j0_hi, uint64_t step, uint64_t m, uint64_t *out,
                     uint64_t es, uint64_t ws, hipStream_t st) {
  if (m == 0) return hipSuccess;
  if (!p_low || !digits || !out) return hipErrorInvalidValue;
  switch (K) {
    case 1: return batch_k<1>(p_low, digits, J, j0_lo, j0_hi, step, m, out, es, ws, st);
    case 2: return batch_k<2>(p_low, digits, J, j0_lo, j0_hi, step, m, out, es, ws, st);
    case 4: return batch_k<4>(p_low, digits, J, j0_lo, j0_hi, step, m, out, es, ws, st);
    case 8: return batch_k<8>(p_low, digits, J, j0_lo, j0_hi, step, m, out, es, ws, st);
    case 16: return batch_k<16>(p_low, digits, J, j0_lo, j0_hi, step, m, out, es, ws, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t xpow_table_device(int K, const uint64_t *p_low, int e0, int bits, int levels,
                             uint64_t *out, XpowLayout lay, hipStream_t st) {
  if (bits < 1 || bits > 10 || levels < 1 || e0 < 0 || !out || !p_low) return hipErrorInvalidValue;
  switch (K) {
    case 1: return table_k<1>(p_low, e0, bits, levels, out, lay, st);
    case 2: return table_k<2>(p_low, e0, bits, levels, out, lay, st);
    case 4: return table_k<4>(p_low, e0, bits, levels, out, lay, st);
    case 8: return table_k<8>(p_low, e0, bits, levels, out, lay, st);
    case 16: return table_k<16>(p_low, e0, bits, levels, out, lay, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_xpow_batch(int K, const uint64_t *p_low, const uint64_t *digits, const uint64_t *J,
                             uint64_t m, uint64_t *out, hipStream_t st) {
  if (m && !J) return hipErrorInvalidValue;
  return batch_any(K, p_low, digits, J, 0, 0, 0, m, out, (uint64_t)K, 1, st);
}

hipError_t launch_xpow_seq(int K, const uint64_t *p_low, const uint64_t *digits, uint64_t j0_lo,
                           uint64_t j0_hi, uint64_t step, uint64_t m, uint64_t *out, uint64_t es,
                           uint64_t ws, hipStream_t st) {
  return batch_any(K, p_low, digits, nullptr, j0_lo, j0_hi, step, m, out, es, ws, st);
}

}  // namespace slrng

// Jump polynomials computed on the device: F2[x] arithmetic modulo an
// engine's characteristic polynomial p(x) (degree n = 64 K), for the tables
// of jump polynomials x^(d 2^(e0 + b l)) mod p that positioning, per-stream
// advances and the request server read, and for x^J mod p of arbitrary
// 128-bit distances J (jump functions, Section "Combining linear engines and
// scramblers").  The host supplies p only.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace slrng {

// Layout of a table of polynomials: word w of entry d of level l is at
// out[l ls + d ds + w ws].
struct XpowLayout {
  size_t ls, ds, ws;
};

// Entry (l, d) = x^(d 2^(e0 + bits l)) mod p for l < levels, d < 2^bits
// (bits <= 10), p = x^n + sum_i p_low[i] (K = n/64 words of p_low, K in
// {1, 2, 4, 8, 16}).  Temporary device memory is allocated and freed here;
// the call returns once the table is written (it synchronizes `st`).
hipError_t xpow_table_device(int K, const uint64_t *p_low, int e0, int bits, int levels,
                             uint64_t *out, XpowLayout lay, hipStream_t st);

// out[j K + w] = word w of x^(J_j) mod p for m distances J_j = J[2j] +
// 2^64 J[2j+1], as the product of the table entries x^(d 2^(10 l)) mod p
// (`digits`, 13 levels of 1,024 entries in the layout ls = 1024 K, ds = 1,
// ws = 1024) selected by J's radix-1024 digits; asynchronous on `st`.
hipError_t launch_xpow_batch(int K, const uint64_t *p_low, const uint64_t *digits,
                             const uint64_t *J, uint64_t m, uint64_t *out, hipStream_t st);

// The same for the arithmetic sequence J_j = j0 + j step (mod 2^128, j0 =
// j0_lo + 2^64 j0_hi), word w of result j at out[j es + w ws].
hipError_t launch_xpow_seq(int K, const uint64_t *p_low, const uint64_t *digits, uint64_t j0_lo,
                           uint64_t j0_hi, uint64_t step, uint64_t m, uint64_t *out, uint64_t es,
                           uint64_t ws, hipStream_t st);

}  // namespace slrng

// On-device linear complexity of one output bit per stream (internal).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace slrng {

// Longest sequence per stream: three bit arrays of nbits/32 + 4 words per
// lane for a wave of 64 lanes stay within 64 KiB of LDS.
constexpr unsigned kLincompMaxBits = 2560;

// 32-bit words per LDS array for a sequence of nbits bits (nbits % 32 == 0).
inline unsigned lincomp_words(unsigned nbits) { return nbits / 32 + 4; }

// out[i] = linear complexity of bit `bit` of outputs 0 .. nbits-1 of stream i
// (states word-major as in the handles; the states are not modified).
hipError_t launch_lincomp(int variant, const uint64_t *state, uint64_t S, int bit, unsigned nbits,
                          unsigned *out, hipStream_t st);

// Rank over Z/2Z of an nrows x ncols bit matrix (both in [1, 1024]); row r
// at rows[r * ceil(ncols / 64) + q], bit b = column 64 q + b.  One
// workgroup; *out on the device.
hipError_t launch_gf2_rank(const uint64_t *rows, unsigned nrows, unsigned ncols, unsigned *out,
                           hipStream_t st);

// Rank of the equidistribution matrix of one engine word: rows e_i (i < n),
// columns word `word` of e_i M^t for t < dims (the engine of `variant`,
// logical word order; word < k, 1 <= dims <= k).
hipError_t launch_equidist_rank(int variant, int word, int dims, unsigned *out, hipStream_t st);

}  // namespace slrng

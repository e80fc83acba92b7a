// Launch interface of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace slrng {

constexpr int kWave = 64;        // lanes per wavefront on CDNA
constexpr int kBlock = 256;      // 4 waves per workgroup, each wave independent
constexpr int kTabRadix = 1024;  // entries per positioning table level
constexpr int kMaxLevels = 4;    // up to 2^40 streams
constexpr int kMaxChunks = 16;   // chunks per stream in one generate launch
constexpr int kMaxSkew = 16;     // skew classes of chunk boundaries
constexpr int kMaxSlots = kMaxChunks + 1;

// A polynomial of degree < 1024 passed by value (jump by one uniform distance).
struct UPoly {
  uint64_t w[16];
};

// Generation of n outputs per stream for S streams whose states are stored
// word-major (word w of stream i at state[w*S + i]).
//
// Each stream may be split into slots that start from the stream state jumped
// ahead, so that short, wide workloads still fill the GPU.  Streams are taken
// 64 at a time (one wave, "group" g); group g has skew class d = g mod D and
// offset delta_d = d*C/D, and slot j covers outputs [b_j, b_{j+1}) with
// b_0 = 0, b_j = min(n, j*C - delta_d) for 0 < j < nslots and b_nslots = n.
// Staggering the boundaries keeps concurrent waves off the same low address
// bits when the row stride is a power of two.  The start polynomial of slot
// j > 0 is x^(j*C - delta_d) mod p, at slot_polys[(d*kMaxSlots + j)*16].
struct GenArgs {
  const uint64_t *state_in;
  uint64_t *state_out;
  uint64_t S;
  uint64_t n;
  uint64_t C;
  uint64_t nslots;
  uint64_t D;
  void *out;
  uint64_t ld;
  const uint64_t *slot_polys;
};

struct GenConfig {
  int tile;  // outputs per lane staged through LDS per round: 16 or 32
  bool nt;   // nontemporal output stores (else plain write-back stores)
};

// All return hipError_t of the launch.
hipError_t launch_generate(int variant, int kind, const GenArgs &a, const GenConfig &cfg,
                           hipStream_t st);

// Stream positioning: stream i = splitmix(seed) * M^(i*J).  tab0 is the
// per-lane level (word-major: word w of entry d at tab0[w*1024 + d]); upper
// levels hold entry d of level l at up[((l-1)*1024 + d)*16].
hipError_t launch_position(int variant, uint64_t seed, uint64_t S, const uint64_t *tab0,
                           const uint64_t *up, int levels, uint64_t *state_out, hipStream_t st);

// In-place jump of S word-major states by one polynomial.
hipError_t launch_jump(int variant, uint64_t *state, uint64_t S, const UPoly &r, hipStream_t st);

// In-place advance of stream i by its own 128-bit distance (steps[2i] +
// 2^64 steps[2i+1]) with the radix-1024 digit tables: word w of entry d of
// level l at tab[(l*W + w)*1024 + d], W = k words, kDigitLevels levels.
constexpr int kDigitLevels = 13;  // ceil(128 / 10)
hipError_t launch_advance_each(int variant, uint64_t *state, uint64_t S, const uint64_t *steps,
                               const uint64_t *tab, hipStream_t st);

// Calibration: write `bytes` of a constant with the same store path, and a
// plain copy kernel.
hipError_t launch_write_ceiling(void *out, uint64_t bytes, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t st);

}  // namespace slrng

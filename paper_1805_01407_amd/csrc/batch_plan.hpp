// Host planner of batched generation (internal): turns requests into tiles of
// lane-chunks, shared by the batch API and the server.
#pragma once
#include <stdint.h>

#include <vector>

#include "../../include/slrng.h"
#include "batch.hpp"

namespace slrng {

// One request as the planner sees it.  The origin is either SplitMix64(seed)
// or the resident state `origin_idx` of a stream array (from_state).
struct PlanReq {
  int variant;
  int kind;
  uint64_t n;
  uint64_t out;  // device address of the first output
  uint64_t start;
  bool from_state;
  uint64_t seed;
  uint32_t origin_idx;
  uint64_t tag;  // caller's request index (the plain form's unit)
  uint64_t start_hi = 0;  // state origins: upper word of the 128-bit start position
};

struct PlanUnit {
  uint32_t tile0 = 0, ntiles = 0;
  int64_t req = -1;               // plain form: the request index
  int variant = -1;               // plain form: the request's variant
  const uint64_t *tab = nullptr;  // plain form: its chunk table
  uint32_t tab_n = 0;
};

// Requests whose start state is computed by the request-state kernel.
struct PlanReqStates {
  std::vector<uint64_t> seeds;       // per entry (seed origins)
  std::vector<uint32_t> origin_idx;  // per entry (state origins)
  std::vector<uint64_t> polys;       // 16 words per entry (seed origins: x^start mod p)
  std::vector<uint64_t> pos;         // 2 words per entry (state origins: the 128-bit start)
  std::vector<uint32_t> slot;        // request-state slot per entry
  std::vector<std::pair<int, uint32_t>> runs;  // (variant, entries) in order
  uint32_t nslots = 0;
};

struct PlanHost {
  std::vector<TileDesc> tiles;
  std::vector<LaneDesc> lanes;
  std::vector<RunDesc> runs;
  std::vector<PlanUnit> units;
  PlanReqStates rs;
  const uint64_t *tab[kNumVariants] = {nullptr};
  uint32_t tab_n[kNumVariants] = {0};
  std::vector<uint64_t> host_tab[kNumVariants];  // with host_tables: the tables themselves
  uint64_t total_outputs = 0;
};

// Builds the plan.  `grid_lanes` is the persistent grid size in lanes (used to
// size the plain form's chunks, and with `fit` those of the whole batch: the
// chunk length shrinks until the batch's lane-chunks cover the grid about
// four times over, down to `fit_floor` outputs, by default the larger of 64
// and n/2); `from_state`
// requests always get a request state.  With `host_tables` the chunk tables
// are computed into host_tab (tab_n entries each, word-major; tab stays null)
// instead of being taken from the device cache, so that planning allocates no
// device memory (not for the plain form: EINVAL).  Returns SLRNG_OK or an
// error code.
int build_plan(const PlanReq *reqs, size_t n, const slrng_batch_opts &o, int device,
               uint64_t grid_lanes, PlanHost &out, bool fit = false, uint64_t fit_floor = 0,
               bool host_tables = false);

// Builds ahead of time the chunk tables (x^(jC) mod p, all entries) of every
// chunk length that fitting can choose for `variant`, so that no iteration
// pays for building one.
int warm_fit_tables(int device, int variant, const slrng_batch_opts &o, uint64_t fit_floor);

// Digit matrices of one engine on one device, for positioning requests from a
// 128-bit position entirely on the device: entry l 2^bits + d holds the n
// columns (k words each) of M^(d 2^(bits l)), l < levels = 128 / bits.  Built
// once per (device, engine) with a kernel, kept until the process ends: 8-bit
// digits for n <= 256 (32 MiB for n = 256), 4-bit digits above (64 MiB for
// n = 1024).
struct DigitMatrices {
  const uint64_t *dev = nullptr;
  int bits = 0, levels = 0;
};
int digit_matrices(int device, int variant, DigitMatrices *out);

// The persistent grid (blocks of 4 waves) for the options on `device`, for
// the kernel of all variants or (variant >= 0) the one specialised to it.
int batch_grid_blocks(const slrng_batch_opts &o, int device, unsigned *blocks, int variant = -1);

}  // namespace slrng

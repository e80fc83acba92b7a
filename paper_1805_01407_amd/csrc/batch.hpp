// Batched generation: descriptors shared by the host planner and the
// persistent kernel (internal to the library).
//
// A request asks for n outputs of one generator, starting `start` steps after
// the SplitMix64-seeded origin state of `seed`.  The planner cuts every
// request into lane-chunks of at most C_v outputs (C_v per variant); chunk j
// starts from the request's start state jumped by j*C_v steps (one per-lane
// jump with the table entry x^(j C_v) mod p).  Every 64 consecutive chunks of
// a request form a run tile, described by one RunDesc (each lane derives its
// chunk); the remaining chunks of all requests are grouped by variant and
// kind, sorted by length and packed 64 to a list tile of LaneDescs.  One wave
// processes a tile.  A persistent kernel hands the first tiles out one to a
// wave and the rest through an atomic counter, heaviest tiles first, and
// switches on the (wave-uniform) variant and kind.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "engines.hpp"

namespace slrng {

constexpr uint32_t kNoReqState = 0xffffffffu;

enum : uint8_t { kTileJump = 1, kTileRun = 2 };

struct TileDesc {
  uint8_t variant;
  uint8_t kind;
  uint8_t nlanes;     // 1..64
  uint8_t flags;      // kTileJump: some lane has a chunk index > 0; kTileRun: see RunDesc
  uint32_t max_len;   // longest lane-chunk of the tile
  uint32_t min_len;   // shortest lane-chunk of the tile
  uint32_t lane0;     // first lane descriptor, or the RunDesc of a run tile
};

// A run tile: lane l takes chunk j0 + l of one request, i.e. outputs
// [l c, min((l+1) c, n_rem)) counted from out0 (the address of chunk j0).
struct RunDesc {
  uint64_t seed;
  uint64_t out0;
  uint64_t n_rem;     // outputs of the request from chunk j0 on
  uint32_t c;         // chunk length
  uint32_t j0;
  uint32_t req;       // request-state index, or kNoReqState
  uint32_t pad;
};

struct LaneDesc {
  uint64_t seed;      // origin seed (used when req == kNoReqState)
  uint64_t out;       // device address of the chunk's first output
  uint32_t len;       // outputs of this chunk
  uint32_t jidx;      // chunk index j (table entry x^(j C) mod p)
  uint32_t req;       // request-state index, or kNoReqState
  uint32_t pad;
};

struct BatchArgs {
  const TileDesc *tiles;
  uint32_t ntiles;
  uint32_t pad;
  const LaneDesc *lanes;
  const RunDesc *runs;
  const uint64_t *req_state;          // [r][16] start states of requests with start > 0
  const uint64_t *tab[kNumVariants];  // chunk tables, word-major: word w of entry j at [w*tab_n + j]
  uint32_t tab_n[kNumVariants];
  unsigned *counter;                  // [0] tiles claimed beyond the first one per wave,
                                      // [1] blocks finished: both zero at launch; the
                                      // last block to finish zeroes them
  // Completion signal in host-mapped memory, or null: the wave that takes
  // tile 0 writes the device clock to sig[2]; the last block to finish, once
  // the output stores of every wave are visible device-wide, writes the clock
  // to sig[3] and then seq to sig[0].
  uint64_t *sig = nullptr;
  uint64_t seq = 0;
};

// Request start states: the origin of request i (SplitMix64(seeds[i]), or, when
// origin_state is set, word w of resident stream origin_idx[i] at
// origin_state[w*origin_stride + origin_idx[i]]) jumped by its start position
// (per-request polynomial, 16 words), written to req_state[slot[i]].
struct ReqArgs {
  const uint64_t *seeds;         // [m] (seed origins)
  const uint64_t *origin_state;  // resident states, word-major, or null
  uint64_t origin_stride;
  const uint32_t *origin_idx;    // [m] (state origins)
  const uint64_t *polys;         // [m][16] (host-computed jump polynomials)
  const uint64_t *pos;           // [m][2] 128-bit positions, low word first (digit kernel)
  const uint32_t *slot;          // [m] index into req_state
  uint64_t *req_state;           // [..][16]
  uint32_t m;
};

// The persistent kernel over all tiles: any variant (variant < 0), or the
// kernel specialised to one variant when every tile is of that variant, with
// its output stores write-through (store 0), plain (1) or nontemporal (2);
// the kernel of all variants always writes through.
hipError_t launch_batch(const BatchArgs &a, int tile, unsigned blocks, hipStream_t st, int variant = -1,
                        int store = 0);
// Workgroups of that kernel that fit on one CU at once (LDS and registers
// decide).
hipError_t batch_resident_blocks_per_cu(int tile, int *blocks, int variant = -1);
hipError_t launch_req_state(int variant, const ReqArgs &a, hipStream_t st);

// Columns of digit matrices: entry e of `polys` (16 words each, x^(J_e) mod
// p) gives the matrix M^(J_e); its column b at cols[(e n + b) k + w], bit r of
// word w being bit b of row 64 w + r (row i = e_i M^(J_e)).
hipError_t launch_digit_cols(int variant, const uint64_t *polys, unsigned entries, uint64_t *cols,
                             hipStream_t st);
// Request states s M^pos from 128-bit positions (a.pos) with the digit
// matrices of radix 2^bits (`levels` digits; entry l 2^bits + d holds
// M^(d 2^(bits l))), one wave per request; origins from origin_state or seeds.
hipError_t launch_req_state_digits(int variant, const ReqArgs &a, const uint64_t *cols, int bits,
                                   int levels, hipStream_t st);
// The two in one launch for a served iteration: `bytes` (a multiple of 16)
// copied from `src`, the device mapping of coherent pinned host memory, to
// device memory `dst` (16-byte aligned), the device clock stamped to `stamp`
// (host-mapped, or null) when the copy starts, and the request states of
// `a` computed as above, its pos, origin_idx and slot read from that pinned
// memory (a.m may be 0).
hipError_t launch_prologue(int variant, const ReqArgs &a, const uint64_t *cols, int bits, int levels,
                           void *dst, const void *src, size_t bytes, uint64_t *stamp, hipStream_t st);
}  // namespace slrng

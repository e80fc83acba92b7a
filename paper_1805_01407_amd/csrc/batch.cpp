// Batched generation: host planner and C ABI (slrng_batch_*).
//
// Planning (host): validate requests; for requests that do not start at the
// SplitMix64 origin compute the start polynomial x^start mod p (applied by the
// request-state kernel); cut requests into lane-chunks; group by (variant,
// kind); sort by length; pack into tiles of 64; order tiles heaviest first;
// upload descriptors.  Launch: either one persistent kernel over all tiles
// (optionally captured once into a hipGraph and replayed), or — the plain form
// used for comparison — one launch of the same kernel per request.
#include <hip/hip_runtime_api.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/slrng.h"
#include "api_internal.hpp"
#include "batch.hpp"
#include "batch_plan.hpp"
#include "engines.hpp"
#include "f2poly.hpp"
#include "kernels.hpp"
#include "xpow.hpp"

using namespace slrng;

#define HIPCHK(call)                              \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(e_);    \
  } while (0)

namespace {

constexpr uint32_t kMaxTable = 65536;  // chunk-table entries per variant

// Chunk tables x^(j C) mod p for j < entries, word-major, per (device, engine, C).
struct ChunkTable {
  uint64_t *dev = nullptr;
  uint32_t n = 0;
};
std::mutex g_ct_mu;
std::map<std::tuple<int, int, uint64_t>, ChunkTable> g_ct;

int chunk_table(int device, int engine, uint64_t C, uint32_t need, ChunkTable *out) {
  std::lock_guard<std::mutex> g(g_ct_mu);
  ChunkTable &t = g_ct[std::make_tuple(device, engine, C)];
  if (t.n >= need) {
    *out = t;
    return SLRNG_OK;
  }
  uint32_t n = std::max<uint32_t>(need, 64);
  n = std::min<uint32_t>(std::max<uint32_t>(n, t.n * 2), kMaxTable);
  // entries x^(j C) mod p on the device: products of the digit tables' entries
  const uint64_t *digits = nullptr;
  const int rc = get_digit_tables(device, engine, &digits);
  if (rc) return rc;
  const Field &f = engine_field(engine);
  const int W = f.n / 64;
  uint64_t *d = nullptr;
  HIPCHK(hipMalloc(&d, (size_t)W * n * 8));
  hipError_t e = launch_xpow_seq(W, f.p.w, digits, 0, 0, C, n, d, 1, n, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e);
  }
  // a smaller table may still be in use by queued work: it is kept
  t.dev = d;
  t.n = n;
  *out = t;
  return SLRNG_OK;
}

// The same entries computed into host memory (word-major, n entries).
void chunk_table_host(int engine, uint64_t C, uint32_t n, std::vector<uint64_t> &h) {
  const Field &f = engine_field(engine);
  const int W = f.n / 64;
  Poly step, cur;
  uint64_t J[1] = {C};
  f.xpow(J, 1, step);
  cur.clear();
  cur.w[0] = 1;
  h.assign((size_t)W * n, 0);
  for (uint32_t j = 0; j < n; j++) {
    for (int w = 0; w < W; w++) h[(size_t)w * n + j] = cur.w[w];
    Poly nx;
    f.mulmod(cur, step, nx);
    cur = nx;
  }
}

std::mutex g_dr_mu;
std::map<std::pair<int, int>, DigitMatrices> g_dr;  // (device, engine)

// Relative cost of one output per variant (engine and scrambler work), for
// ordering tiles heaviest first.
uint64_t output_cost(int v) { return (v >= 6 && v <= 8) ? 3 : 2; }

}  // namespace

namespace slrng {

int digit_matrices(int device, int variant, DigitMatrices *out) {
  std::lock_guard<std::mutex> g(g_dr_mu);
  const int engine = variant_engine(variant);
  DigitMatrices &t = g_dr[std::make_pair(device, engine)];
  if (t.dev) {
    *out = t;
    return SLRNG_OK;
  }
  const Field &f = engine_field(engine);
  const int K = f.n / 64;
  const int bits = K <= 4 ? 8 : 4;
  const int levels = 128 / bits;
  const unsigned per = 1u << bits, entries = (unsigned)levels * per;
  // entry l 2^bits + d: x^(d 2^(bits l)) mod p (16 words, the first K used),
  // built on the device from p alone
  const size_t pwords = (size_t)entries * 16;
  uint64_t *polys = nullptr, *cols = nullptr;
  HIPCHK(hipMalloc(&polys, pwords * 8));
  hipError_t e = hipMalloc(&cols, (size_t)entries * f.n * K * 8);
  if (e == hipSuccess) e = hipMemset(polys, 0, pwords * 8);
  if (e == hipSuccess)
    e = xpow_table_device(K, f.p.w, 0, bits, levels, polys, XpowLayout{(size_t)per * 16, 16, 1}, nullptr);
  if (e == hipSuccess) e = launch_digit_cols(variant, polys, entries, cols, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  (void)hipFree(polys);
  if (e != hipSuccess) {
    if (cols) (void)hipFree(cols);
    return e == hipErrorOutOfMemory ? SLRNG_ENOMEM : hip_fail(e);
  }
  t.dev = cols;
  t.bits = bits;
  t.levels = levels;
  *out = t;
  return SLRNG_OK;
}

int batch_grid_blocks(const slrng_batch_opts &o, int device, unsigned *blocks, int variant) {
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return hip_fail(e);
  const int wpc = o.waves_per_cu ? o.waves_per_cu : 12;
  // a persistent grid larger than what is resident at once only adds blocks
  // that start after the tiles are gone
  int per_cu = 0;
  e = batch_resident_blocks_per_cu(o.tile, &per_cu, variant);
  if (e != hipSuccess) return hip_fail(e);
  const int want = cus * wpc / (kBlock / kWave);
  const int cap = per_cu > 0 ? cus * per_cu : want;
  *blocks = (unsigned)std::max(1, std::min(want, cap));
  return SLRNG_OK;
}

constexpr uint64_t kFitTilesPerWave = 4;

static uint64_t option_chunk(const slrng_batch_opts &o, int v) {
  uint64_t c = o.chunk[v] ? o.chunk[v] : 16384;
  if (c > 0xffffffffull) c = 0xffffffffull & ~(uint64_t)63;
  return c;
}

// Smallest fitted chunk: the option, else the larger of 64 and n/2 (128 for
// xoshiro256: short requests spread over more lanes; the run tiles' jumps
// from the request's common start state are cheap enough for that).
static uint64_t fit_floor_for(int v, uint64_t fit_floor) {
  return fit_floor ? fit_floor : std::max<uint64_t>(64, 32 * (uint64_t)variant_words(v));
}

int warm_fit_tables(int device, int variant, const slrng_batch_opts &o, uint64_t fit_floor) {
  const uint64_t c = option_chunk(o, variant);
  for (uint64_t want = fit_floor_for(variant, fit_floor);; want *= 2) {
    const uint64_t cc = (std::min(c, want) + o.tile - 1) / o.tile * o.tile;
    ChunkTable t;
    int rc = chunk_table(device, variant_engine(variant), cc, kMaxTable, &t);
    if (rc) return rc;
    if (want >= c) break;
  }
  return SLRNG_OK;
}

int build_plan(const PlanReq *reqs, size_t n_reqs, const slrng_batch_opts &o, int device,
               uint64_t grid_lanes, PlanHost &P, bool fit, uint64_t fit_floor, bool host_tables) {
  const bool plain = o.mode == SLRNG_BATCH_PLAIN;
  if (plain && host_tables) return SLRNG_EINVAL;
  // chunk length per variant: the option value, rounded up to the tile and
  // raised if a request would need more than kMaxTable chunks
  uint64_t C[kNumVariants];
  uint64_t maxn[kNumVariants] = {0};
  for (size_t r = 0; r < n_reqs; r++) maxn[reqs[r].variant] = std::max(maxn[reqs[r].variant], reqs[r].n);
  uint64_t total[kNumVariants] = {0};
  for (size_t r = 0; r < n_reqs; r++) total[reqs[r].variant] += reqs[r].n;
  for (int v = 0; v < kNumVariants; v++) {
    uint64_t c = option_chunk(o, v);
    if (fit) {
      uint64_t want = fit_floor_for(v, fit_floor);
      // about kFitTilesPerWave tiles per resident wave, so that waves that
      // finish early take more work instead of idling until the slowest ends
      while (want < c && want * grid_lanes * kFitTilesPerWave < total[v]) want *= 2;
      c = std::min(c, want);
    }
    c = (c + o.tile - 1) / o.tile * o.tile;
    const uint64_t need = (maxn[v] + kMaxTable - 1) / kMaxTable;
    if (c < need) {
      // a power of two, so that the chunk lengths stay within the set whose
      // tables warm_fit_tables builds ahead of time
      uint64_t p2 = c;
      while (p2 < need) p2 *= 2;
      c = (p2 + o.tile - 1) / o.tile * o.tile;
    }
    if (c > 0xffffffffull) return SLRNG_ERANGE;
    C[v] = c;
  }
  // request states: requests that start past their origin, and every request
  // whose origin is a resident state (those are positioned on the device from
  // their 128-bit start, no polynomial here)
  std::vector<uint32_t> req_slot(n_reqs, kNoReqState);
  std::vector<std::vector<uint32_t>> by_var(kNumVariants);
  uint32_t nslots = 0;
  for (size_t r = 0; r < n_reqs; r++)
    if ((reqs[r].start || reqs[r].from_state) && reqs[r].n) {
      req_slot[r] = nslots++;
      by_var[reqs[r].variant].push_back((uint32_t)r);
    }
  // The plain form runs each request alone, so each request is cut finely
  // enough to fill the GPU by itself: chunk = the smallest power of two >= 1024
  // giving at most one chunk per lane of the persistent grid (capped by C_v).
  //
  // Every 64 consecutive chunks of a request form one run tile, described by a
  // single RunDesc (the lanes derive their chunk on the device).  The request's
  // remaining chunks (fewer than 64) go to buckets keyed by (unit, variant,
  // kind) as explicit lane descriptors: full-length chunks first, then the
  // partial last chunks by decreasing length, 64 to a tile.
  struct Bucket {
    uint64_t unit;
    int variant, kind;
    std::vector<LaneDesc> full, part;
  };
  std::map<std::tuple<uint64_t, int, int>, size_t> bucket_of;
  std::vector<Bucket> buckets;
  std::map<uint64_t, std::vector<std::pair<uint64_t, TileDesc>>> unit_tiles;
  std::vector<uint64_t> req_chunk(n_reqs, 0);
  uint32_t tab_need[kNumVariants] = {0};
  P.total_outputs = 0;
  P.tiles.clear();
  P.lanes.clear();
  P.runs.clear();
  P.units.clear();
  for (size_t r = 0; r < n_reqs; r++) {
    const PlanReq &q = reqs[r];
    if (!q.n) continue;
    P.total_outputs += q.n;
    uint64_t c = C[q.variant];
    if (plain) {
      uint64_t want = 1024;
      while (want < c && want * grid_lanes < q.n) want *= 2;
      c = std::min<uint64_t>(c, std::max<uint64_t>(want, (q.n + kMaxTable - 1) / kMaxTable));
      c = (c + o.tile - 1) / o.tile * o.tile;
      req_chunk[r] = c;
    }
    const uint64_t nch = (q.n + c - 1) / c;
    if (!plain) tab_need[q.variant] = std::max<uint32_t>(tab_need[q.variant], (uint32_t)nch);
    const uint64_t unit = plain ? (uint64_t)r : 0ull;
    auto &ut = unit_tiles[unit];
    const uint64_t nrun = nch / kWave;
    for (uint64_t k = 0; k < nrun; k++) {
      const uint64_t j0 = k * kWave;
      RunDesc rd;
      rd.seed = q.seed;
      rd.out0 = q.out + j0 * c * 8;
      rd.n_rem = q.n - j0 * c;
      rd.c = (uint32_t)c;
      rd.j0 = (uint32_t)j0;
      rd.req = req_slot[r];
      rd.pad = 0;
      TileDesc td;
      td.variant = (uint8_t)q.variant;
      td.kind = (uint8_t)q.kind;
      td.nlanes = (uint8_t)kWave;
      td.flags = kTileRun | kTileJump;
      td.max_len = (uint32_t)c;
      td.min_len = (uint32_t)std::min<uint64_t>(c, q.n - (j0 + kWave - 1) * c);
      td.lane0 = (uint32_t)P.runs.size();
      P.runs.push_back(rd);
      ut.push_back({(uint64_t)td.max_len * output_cost(td.variant), td});
    }
    if (nrun * kWave == nch) continue;
    const auto key = std::make_tuple(unit, q.variant, q.kind);
    auto it = bucket_of.find(key);
    if (it == bucket_of.end()) {
      it = bucket_of.emplace(key, buckets.size()).first;
      buckets.push_back(Bucket{unit, q.variant, q.kind, {}, {}});
    }
    Bucket &bk = buckets[it->second];
    for (uint64_t j = nrun * kWave; j < nch; j++) {
      LaneDesc d;
      d.seed = q.seed;
      d.out = q.out + j * c * 8;
      d.len = (uint32_t)std::min<uint64_t>(c, q.n - j * c);
      d.jidx = (uint32_t)j;
      d.req = req_slot[r];
      d.pad = 0;
      if (d.len == c) bk.full.push_back(d);
      else bk.part.push_back(d);
    }
  }
  for (int v = 0; v < kNumVariants; v++) {
    P.tab[v] = nullptr;
    P.tab_n[v] = 0;
    P.host_tab[v].clear();
    if (!tab_need[v]) continue;
    if (host_tables) {
      chunk_table_host(variant_engine(v), C[v], tab_need[v], P.host_tab[v]);
      P.tab_n[v] = tab_need[v];
      continue;
    }
    ChunkTable t;
    int rc = chunk_table(device, variant_engine(v), C[v], tab_need[v], &t);
    if (rc) return rc;
    P.tab[v] = t.dev;
    P.tab_n[v] = t.n;
  }
  // list tiles from the buckets
  for (auto &kv : bucket_of) {
    Bucket &bk = buckets[kv.second];
    auto &ut = unit_tiles[bk.unit];
    std::stable_sort(bk.part.begin(), bk.part.end(),
                     [](const LaneDesc &x, const LaneDesc &y) { return x.len > y.len; });
    const size_t nf = bk.full.size(), nl = nf + bk.part.size();
    auto lane_at = [&](size_t k) -> const LaneDesc & { return k < nf ? bk.full[k] : bk.part[k - nf]; };
    for (size_t s0 = 0; s0 < nl; s0 += kWave) {
      const size_t cnt = std::min<size_t>(kWave, nl - s0);
      TileDesc td;
      td.variant = (uint8_t)bk.variant;
      td.kind = (uint8_t)bk.kind;
      td.nlanes = (uint8_t)cnt;
      td.flags = 0;
      td.max_len = lane_at(s0).len;  // lanes are in decreasing length
      td.min_len = lane_at(s0 + cnt - 1).len;
      td.lane0 = (uint32_t)P.lanes.size();
      for (size_t k = s0; k < s0 + cnt; k++) {
        const LaneDesc &d = lane_at(k);
        if (d.jidx) td.flags |= kTileJump;
        P.lanes.push_back(d);
      }
      ut.push_back({(uint64_t)td.max_len * output_cost(td.variant), td});
    }
  }
  // units in order; tiles heaviest first within a unit (room for all tiles
  // at once: the plain form has one unit per request)
  size_t ntiles_all = 0;
  for (auto &kv : unit_tiles) ntiles_all += kv.second.size();
  P.tiles.reserve(ntiles_all);
  for (auto &kv : unit_tiles) {
    auto &tiles = kv.second;
    const auto heavier = [](const std::pair<uint64_t, TileDesc> &x, const std::pair<uint64_t, TileDesc> &y) {
      return x.first > y.first;
    };
    // one request's tiles come out in order already (its run tiles, then its
    // list tiles by decreasing length): a check in linear time spares the
    // sort (about 20 us for 1,000 tiles on the request server's path)
    if (!std::is_sorted(tiles.begin(), tiles.end(), heavier))
      std::stable_sort(tiles.begin(), tiles.end(), heavier);
    PlanUnit u;
    u.tile0 = (uint32_t)P.tiles.size();
    for (auto &t : tiles) P.tiles.push_back(t.second);
    u.ntiles = (uint32_t)tiles.size();
    if (plain) {
      const uint64_t unit = kv.first;
      const uint64_t c = req_chunk[unit];
      ChunkTable t;
      int rc = chunk_table(device, variant_engine(reqs[unit].variant), c,
                           (uint32_t)((reqs[unit].n + c - 1) / c), &t);
      if (rc) return rc;
      u.req = (int64_t)reqs[unit].tag;
      u.variant = reqs[unit].variant;
      u.tab = t.dev;
      u.tab_n = t.n;
    }
    P.units.push_back(u);
  }
  if (P.units.empty()) P.units.push_back(PlanUnit());
  // request states, grouped by variant (one kernel launch per variant)
  PlanReqStates &rs = P.rs;
  rs = PlanReqStates();
  rs.nslots = nslots;
  for (int v = 0; v < kNumVariants; v++) {
    if (by_var[v].empty()) continue;
    const Field &f = engine_field(variant_engine(v));
    for (uint32_t r : by_var[v]) {
      rs.seeds.push_back(reqs[r].seed);
      rs.origin_idx.push_back(reqs[r].origin_idx);
      rs.slot.push_back(req_slot[r]);
      if (reqs[r].from_state || !host_tables) {
        // positioned on the device from the digits of its 128-bit start
        rs.pos.push_back(reqs[r].start);
        rs.pos.push_back(reqs[r].start_hi);
        continue;
      }
      Poly pr;
      if (reqs[r].start) {
        uint64_t J[1] = {reqs[r].start};
        f.xpow(J, 1, pr);
      } else {
        pr.clear();
        pr.w[0] = 1;
      }
      for (int w = 0; w < 16; w++) rs.polys.push_back(pr.w[w]);
    }
    rs.runs.push_back({v, (uint32_t)by_var[v].size()});
  }
  return SLRNG_OK;
}

}  // namespace slrng

// ---------------------------------------------------------------- the batch object

struct slrng_batch {
  int device = 0;
  slrng_batch_opts opts;
  uint64_t n_requests = 0;
  PlanHost plan;
  TileDesc *d_tiles = nullptr;
  LaneDesc *d_lanes = nullptr;
  RunDesc *d_runs = nullptr;
  uint64_t *d_req_state = nullptr;
  uint64_t *d_req_seed = nullptr, *d_req_pos = nullptr;
  uint32_t *d_req_slot = nullptr;
  unsigned *d_counter = nullptr;  // two counters per unit (claims, finished waves)
  struct ReqLaunch {
    int variant;
    ReqArgs args;
    DigitMatrices digits;
  };
  std::vector<ReqLaunch> req_launches;
  BatchArgs args;
  unsigned blocks = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void free_batch(slrng_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  void *ptrs[] = {b->d_tiles, b->d_lanes, b->d_runs, b->d_req_state, b->d_req_seed, b->d_req_pos,
                  b->d_req_slot, b->d_counter};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete b;
}

extern "C" int slrng_batch_default_opts(slrng_batch_opts *o) {
  return guarded([&]() -> int {
    if (!o) return SLRNG_EINVAL;
    memset(o, 0, sizeof(*o));
    o->mode = SLRNG_BATCH_GRAPH;
    o->tile = 32;
    o->waves_per_cu = 8;
    for (int v = 0; v < SLRNG_NUM_VARIANTS; v++)
      o->chunk[v] = (v == 9 || v == 10 || v == 11 || v == 13) ? 65536 : 8192;
    return SLRNG_OK;
  });
}

namespace slrng {
int check_batch_opts(const slrng_batch_opts &o) {
  if (o.mode != SLRNG_BATCH_GRAPH && o.mode != SLRNG_BATCH_PERSISTENT && o.mode != SLRNG_BATCH_PLAIN)
    return SLRNG_EINVAL;
  if (o.tile != 16 && o.tile != 32) return SLRNG_EINVAL;
  if (o.waves_per_cu < 0 || o.waves_per_cu > 64) return SLRNG_EINVAL;
  return SLRNG_OK;
}
}  // namespace slrng

static int enqueue_unit(slrng_batch *b, const PlanUnit &u, unsigned *counter, hipStream_t st) {
  if (u.ntiles == 0) return SLRNG_OK;
  BatchArgs a = b->args;
  if (u.variant >= 0) {
    a.tab[u.variant] = u.tab;
    a.tab_n[u.variant] = u.tab_n;
  }
  a.tiles = b->d_tiles + u.tile0;
  a.ntiles = u.ntiles;
  a.counter = counter;  // zero: from the upload, then reset by each launch's last wave
  const unsigned blocks = std::min<unsigned>(b->blocks, (u.ntiles + 3) / 4);
  hipError_t e = launch_batch(a, b->opts.tile, blocks, st);
  return e == hipSuccess ? SLRNG_OK : hip_fail(e);
}

static int enqueue_req_states(slrng_batch *b, hipStream_t st) {
  for (auto &rl : b->req_launches) {
    hipError_t e = launch_req_state_digits(rl.variant, rl.args, rl.digits.dev, rl.digits.bits,
                                           rl.digits.levels, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  return SLRNG_OK;
}

// Enqueue the whole batch on `st` (no graph).
static int enqueue_all(slrng_batch *b, hipStream_t st) {
  int rc = enqueue_req_states(b, st);
  for (size_t i = 0; i < b->plan.units.size() && !rc; i++)
    rc = enqueue_unit(b, b->plan.units[i], b->d_counter + 2 * i, st);
  return rc;
}

extern "C" int slrng_batch_plan(const slrng_request *reqs, size_t n_reqs,
                                const slrng_batch_opts *opts, slrng_batch **out) {
  return guarded([&]() -> int {
    if (!out || (n_reqs && !reqs)) return SLRNG_EINVAL;
    *out = nullptr;
    slrng_batch_opts o;
    if (opts) o = *opts;
    else slrng_batch_default_opts(&o);
    int rc = check_batch_opts(o);
    if (rc) return rc;
    if (n_reqs > (1u << 24)) return SLRNG_ERANGE;
    std::vector<PlanReq> pr(n_reqs);
    for (size_t r = 0; r < n_reqs; r++) {
      const slrng_request &q = reqs[r];
      if (!valid_variant64(q.variant) || (q.kind != SLRNG_U64 && q.kind != SLRNG_F64)) return SLRNG_EINVAL;
      if (q.n && (!q.dev_out || ((uintptr_t)q.dev_out & 7))) return SLRNG_EINVAL;
      if (q.n > UINT64_MAX / 8) return SLRNG_ERANGE;
      pr[r] = PlanReq{q.variant, q.kind, q.n, (uint64_t)(uintptr_t)q.dev_out, q.start, false, q.seed, 0,
                      (uint64_t)r};
    }
    slrng_batch *b = new (std::nothrow) slrng_batch();
    if (!b) return SLRNG_ENOMEM;
    b->opts = o;
    b->n_requests = n_reqs;
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
      free_batch(b);
      return hip_fail(e);
    }
    rc = batch_grid_blocks(o, b->device, &b->blocks);
    if (!rc) rc = build_plan(pr.data(), n_reqs, o, b->device, (uint64_t)b->blocks * kBlock, b->plan);
    if (rc) {
      free_batch(b);
      return rc;
    }
    const PlanHost &P = b->plan;
    auto upload = [&](void **dst, const void *src, size_t bytes) -> int {
      if (!bytes) return SLRNG_OK;
      hipError_t e3 = hipMalloc(dst, bytes);
      if (e3 != hipSuccess) return e3 == hipErrorOutOfMemory ? SLRNG_ENOMEM : hip_fail(e3);
      e3 = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
      return e3 == hipSuccess ? SLRNG_OK : hip_fail(e3);
    };
    rc = upload((void **)&b->d_tiles, P.tiles.data(), P.tiles.size() * sizeof(TileDesc));
    if (!rc) rc = upload((void **)&b->d_lanes, P.lanes.data(), P.lanes.size() * sizeof(LaneDesc));
    if (!rc) rc = upload((void **)&b->d_runs, P.runs.data(), P.runs.size() * sizeof(RunDesc));
    if (!rc) {
      std::vector<unsigned> zeros(2 * P.units.size(), 0);  // two counters per unit
      rc = upload((void **)&b->d_counter, zeros.data(), zeros.size() * sizeof(unsigned));
    }
    if (!rc && P.rs.nslots) {
      e = hipMalloc(&b->d_req_state, (size_t)P.rs.nslots * 16 * 8);
      if (e != hipSuccess) rc = hip_fail(e);
      if (!rc) rc = upload((void **)&b->d_req_seed, P.rs.seeds.data(), P.rs.seeds.size() * 8);
      if (!rc) rc = upload((void **)&b->d_req_pos, P.rs.pos.data(), P.rs.pos.size() * 8);
      if (!rc) rc = upload((void **)&b->d_req_slot, P.rs.slot.data(), P.rs.slot.size() * 4);
      // start states s M^start from the digits of start, on the device (the
      // engine's digit matrices, built once per device)
      uint32_t off = 0;
      for (size_t k = 0; k < P.rs.runs.size() && !rc; k++) {
        slrng_batch::ReqLaunch rl;
        rl.variant = P.rs.runs[k].first;
        rc = digit_matrices(b->device, rl.variant, &rl.digits);
        if (rc) break;
        ReqArgs &ra = rl.args;
        ra.seeds = b->d_req_seed + off;
        ra.origin_state = nullptr;
        ra.origin_stride = 0;
        ra.origin_idx = nullptr;
        ra.polys = nullptr;
        ra.pos = b->d_req_pos + (size_t)off * 2;
        ra.slot = b->d_req_slot + off;
        ra.req_state = b->d_req_state;
        ra.m = P.rs.runs[k].second;
        b->req_launches.push_back(rl);
        off += ra.m;
      }
    }
    if (rc) {
      free_batch(b);
      return rc;
    }
    b->args.tiles = b->d_tiles;
    b->args.ntiles = (uint32_t)P.tiles.size();
    b->args.pad = 0;
    b->args.lanes = b->d_lanes;
    b->args.runs = b->d_runs;
    b->args.req_state = b->d_req_state;
    b->args.counter = b->d_counter;
    for (int v = 0; v < kNumVariants; v++) {
      b->args.tab[v] = P.tab[v];
      b->args.tab_n[v] = P.tab_n[v];
    }
    // graph: capture the whole enqueue sequence once
    if (o.mode == SLRNG_BATCH_GRAPH) {
      hipStream_t cs = nullptr;
      e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
      if (e != hipSuccess) {
        free_batch(b);
        return hip_fail(e);
      }
      e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        rc = enqueue_all(b, cs);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (!rc && e2 != hipSuccess) rc = hip_fail(e2);
        b->graph = g;
        if (!rc) {
          e2 = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
          if (e2 != hipSuccess) rc = hip_fail(e2);
        }
      } else {
        rc = hip_fail(e);
      }
      (void)hipStreamDestroy(cs);
      if (rc) {
        free_batch(b);
        return rc;
      }
    }
    *out = b;
    return SLRNG_OK;
  });
}

extern "C" int slrng_batch_launch(slrng_batch *b, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!b) return SLRNG_EINVAL;
    if (b->exec) {
      hipError_t e = hipGraphLaunch(b->exec, stream);
      return e == hipSuccess ? SLRNG_OK : hip_fail(e);
    }
    return enqueue_all(b, stream);
  });
}

extern "C" int slrng_batch_latencies(slrng_batch *b, hipStream_t stream, double *done_ms) {
  return guarded([&]() -> int {
    if (!b || !done_ms) return SLRNG_EINVAL;
    for (uint64_t r = 0; r < b->n_requests; r++) done_ms[r] = 0.0;
    const bool per_unit = b->opts.mode == SLRNG_BATCH_PLAIN;
    const auto &units = b->plan.units;
    std::vector<hipEvent_t> ev(per_unit ? units.size() + 1 : 2, nullptr);
    int rc = SLRNG_OK;
    for (auto &x : ev) {
      hipError_t e = hipEventCreate(&x);
      if (e != hipSuccess) {
        rc = hip_fail(e);
        break;
      }
    }
    if (!rc) {
      hipError_t e = hipEventRecord(ev[0], stream);
      if (e != hipSuccess) rc = hip_fail(e);
    }
    if (!rc && !per_unit) {
      rc = slrng_batch_launch(b, stream);
      if (!rc) {
        hipError_t e = hipEventRecord(ev[1], stream);
        if (e != hipSuccess) rc = hip_fail(e);
      }
    } else if (!rc) {
      rc = enqueue_req_states(b, stream);
      for (size_t i = 0; i < units.size() && !rc; i++) {
        rc = enqueue_unit(b, units[i], b->d_counter + 2 * i, stream);
        if (!rc) {
          hipError_t e = hipEventRecord(ev[i + 1], stream);
          if (e != hipSuccess) rc = hip_fail(e);
        }
      }
    }
    if (!rc) {
      hipError_t e = hipStreamSynchronize(stream);
      if (e != hipSuccess) rc = hip_fail(e);
    }
    if (!rc) {
      if (!per_unit) {
        float ms = 0;
        hipError_t e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e != hipSuccess) rc = hip_fail(e);
        for (uint64_t r = 0; r < b->n_requests && !rc; r++) done_ms[r] = ms;
      } else {
        for (size_t i = 0; i < units.size() && !rc; i++) {
          float ms = 0;
          hipError_t e = hipEventElapsedTime(&ms, ev[0], ev[i + 1]);
          if (e != hipSuccess) rc = hip_fail(e);
          else if (units[i].req >= 0) done_ms[units[i].req] = ms;
        }
      }
    }
    for (auto &x : ev)
      if (x) (void)hipEventDestroy(x);
    return rc;
  });
}

extern "C" int slrng_batch_info(const slrng_batch *b, uint64_t *n_tiles, uint64_t *n_lanes,
                                uint64_t *total_outputs) {
  return guarded([&]() -> int {
    if (!b) return SLRNG_EINVAL;
    if (n_tiles) *n_tiles = b->plan.tiles.size();
    if (n_lanes) *n_lanes = b->plan.lanes.size() + (uint64_t)b->plan.runs.size() * kWave;
    if (total_outputs) *total_outputs = b->plan.total_outputs;
    return SLRNG_OK;
  });
}

extern "C" int slrng_batch_destroy(slrng_batch *b) {
  return guarded([&]() -> int {
    if (!b) return SLRNG_EINVAL;
    free_batch(b);
    return SLRNG_OK;
  });
}

extern "C" int slrng_batch_run(const slrng_request *reqs, size_t n_reqs, const slrng_batch_opts *opts,
                               hipStream_t stream) {
  return guarded([&]() -> int {
    slrng_batch *b = nullptr;
    int rc = slrng_batch_plan(reqs, n_reqs, opts, &b);
    if (rc) return rc;
    rc = slrng_batch_launch(b, stream);
    hipError_t e = hipStreamSynchronize(stream);
    free_batch(b);
    if (rc) return rc;
    return e == hipSuccess ? SLRNG_OK : hip_fail(e);
  });
}

// slrng_batch_run_static: batched generation that allocates no device memory.
//
// The same plan and kernels as slrng_batch_run (persistent form), but every
// byte the kernels need besides the caller's outputs — tile, run and lane
// descriptors, the claim counters, request start states and the chunk tables
// x^(jC) mod p — is staged in `scratch`, a fixed array in device memory that
// the library holds on every device it runs on until the process ends.  For
// callers that cannot allocate device memory.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/slrng.h"
#include "api_internal.hpp"
#include "batch.hpp"
#include "batch_plan.hpp"
#include "kernels.hpp"

using namespace slrng;

namespace {

constexpr size_t kScratchBytes = SLRNG_BATCH_STATIC_SCRATCH_BYTES;

// Device-side staging area of slrng_batch_run_static.  In host code this name
// only stands for the array: its device address on the current device comes
// from hipGetSymbolAddress (each device holds its own copy), and only that
// address is ever passed to copies and kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DevScratch {
  unsigned char *ptr = nullptr;  // this device's copy of `scratch`
  std::mutex mu;                 // one call at a time per device
};

std::mutex g_scratch_mu;
std::map<int, DevScratch> g_scratch;  // by device; nodes never move

// The device address of `scratch` on `device` (the current device), taken
// once per device.
int scratch_of(int device, DevScratch **out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  DevScratch &d = g_scratch[device];
  if (!d.ptr) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (!p) return SLRNG_EHIP;
    d.ptr = static_cast<unsigned char *>(p);
  }
  *out = &d;
  return SLRNG_OK;
}

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" int slrng_batch_run_static(const slrng_request *reqs, size_t n_reqs,
                                      const slrng_batch_opts *opts, hipStream_t stream) {
  return guarded([&]() -> int {
    if (n_reqs && !reqs) return SLRNG_EINVAL;
    slrng_batch_opts o;
    if (opts) o = *opts;
    else slrng_batch_default_opts(&o);
    int rc = check_batch_opts(o);
    if (rc) return rc;
    if (o.mode == SLRNG_BATCH_PLAIN) return SLRNG_EINVAL;
    o.mode = SLRNG_BATCH_PERSISTENT;  // no graph: instantiating one allocates
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
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e);
    unsigned blocks = 0;
    rc = batch_grid_blocks(o, device, &blocks);
    if (rc) return rc;
    PlanHost P;
    rc = build_plan(pr.data(), n_reqs, o, device, (uint64_t)blocks * kBlock, P, false, 0,
                    /*host_tables=*/true);
    if (rc) return rc;
    if (P.tiles.empty()) return SLRNG_OK;

    // layout of the staged bytes (each part 256-byte aligned); the request
    // states are written by the request-state kernel, not uploaded
    const size_t nreq = P.rs.seeds.size();
    size_t off = 256;  // [0, 256): the two claim counters, zero
    const size_t o_tiles = off;
    off = up256(off + P.tiles.size() * sizeof(TileDesc));
    const size_t o_lanes = off;
    off = up256(off + P.lanes.size() * sizeof(LaneDesc));
    const size_t o_runs = off;
    off = up256(off + P.runs.size() * sizeof(RunDesc));
    const size_t o_seeds = off;
    off = up256(off + nreq * 8);
    const size_t o_polys = off;
    off = up256(off + nreq * 16 * 8);
    const size_t o_slot = off;
    off = up256(off + nreq * 4);
    size_t o_tab[kNumVariants];
    for (int v = 0; v < kNumVariants; v++) {
      o_tab[v] = off;
      off = up256(off + P.host_tab[v].size() * 8);
    }
    const size_t upload = off;
    const size_t o_state = off;
    off = up256(off + (size_t)P.rs.nslots * 16 * 8);
    if (off > kScratchBytes) return SLRNG_ERANGE;

    std::vector<unsigned char> h(upload, 0);
    memcpy(h.data() + o_tiles, P.tiles.data(), P.tiles.size() * sizeof(TileDesc));
    if (!P.lanes.empty()) memcpy(h.data() + o_lanes, P.lanes.data(), P.lanes.size() * sizeof(LaneDesc));
    if (!P.runs.empty()) memcpy(h.data() + o_runs, P.runs.data(), P.runs.size() * sizeof(RunDesc));
    if (nreq) {
      memcpy(h.data() + o_seeds, P.rs.seeds.data(), nreq * 8);
      memcpy(h.data() + o_polys, P.rs.polys.data(), nreq * 16 * 8);
      memcpy(h.data() + o_slot, P.rs.slot.data(), nreq * 4);
    }
    for (int v = 0; v < kNumVariants; v++)
      if (!P.host_tab[v].empty()) memcpy(h.data() + o_tab[v], P.host_tab[v].data(), P.host_tab[v].size() * 8);

    DevScratch *ds = nullptr;
    rc = scratch_of(device, &ds);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(ds->mu);
    unsigned char *d = ds->ptr;
    e = hipMemcpyAsync(d, h.data(), upload, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e);
    uint64_t *d_state = reinterpret_cast<uint64_t *>(d + o_state);
    uint32_t at = 0;
    for (auto &run : P.rs.runs) {
      ReqArgs ra;
      ra.seeds = reinterpret_cast<const uint64_t *>(d + o_seeds) + at;
      ra.origin_state = nullptr;
      ra.origin_stride = 0;
      ra.origin_idx = nullptr;
      ra.polys = reinterpret_cast<const uint64_t *>(d + o_polys) + (size_t)at * 16;
      ra.pos = nullptr;
      ra.slot = reinterpret_cast<const uint32_t *>(d + o_slot) + at;
      ra.req_state = d_state;
      ra.m = run.second;
      e = launch_req_state(run.first, ra, stream);
      if (e != hipSuccess) break;
      at += run.second;
    }
    if (e == hipSuccess) {
      BatchArgs a{};
      a.tiles = reinterpret_cast<const TileDesc *>(d + o_tiles);
      a.ntiles = (uint32_t)P.tiles.size();
      a.lanes = reinterpret_cast<const LaneDesc *>(d + o_lanes);
      a.runs = reinterpret_cast<const RunDesc *>(d + o_runs);
      a.req_state = d_state;
      for (int v = 0; v < kNumVariants; v++) {
        a.tab[v] = P.host_tab[v].empty() ? nullptr : reinterpret_cast<const uint64_t *>(d + o_tab[v]);
        a.tab_n[v] = P.tab_n[v];
      }
      a.counter = reinterpret_cast<unsigned *>(d);  // zeroed by the upload
      e = launch_batch(a, o.tile, std::min<unsigned>(blocks, ((unsigned)P.tiles.size() + 3) / 4), stream);
    }
    // the host staging buffer and the scratch contents must outlive the work
    const hipError_t es = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e);
    return es == hipSuccess ? SLRNG_OK : hip_fail(es);
  });
}

// Serving loop with continuous batching (slrng_server_*).
//
// The server keeps S streams resident on the device (positioned like
// slrng_streams_create) and a device output arena of a fixed budget.
//  * submit: admission reserves the request's output bytes in the arena (or
//    returns EAGAIN / waits when the budget is full) and assigns it the next
//    positions of its stream: pos = head[stream], head[stream] += n (128-bit
//    positions).  A request is thus fully defined by (stream, pos, n): its
//    values are the stream's outputs pos .. pos+n-1, whatever else is in
//    flight.  Its latency counts from the moment it arrived (the call, or the
//    scheduled arrival of a replayed trace), admission wait included.
//  * iteration thread: takes every pending request (up to max_batch), plans
//    them as one batch (lane-chunks, tiles; no polynomial arithmetic per
//    request: the start state s M^pos is computed on the device from the
//    digits of pos), copies the descriptors into one of `inflight`
//    preallocated slots with one upload and launches [request-state kernel ->
//    persistent generation kernel] on that slot's HIP stream.  Requests that
//    arrive while earlier iterations run join the next iteration, which runs
//    concurrently on another slot.
//  * completion: one thread per slot waits for that slot's iteration (so
//    iterations complete in any order), stamps the completion time of its
//    requests, frees auto-released arena ranges and the slot.
#include <hip/hip_runtime_api.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/slrng.h"
#include "api_internal.hpp"
#include "batch.hpp"
#include "batch_plan.hpp"
#include "kernels.hpp"
#include "memory.hpp"

using namespace slrng;

namespace {

typedef std::chrono::steady_clock Clock;

double secs(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

constexpr uint64_t kAlign = 256;  // arena allocation granularity (bytes)
constexpr size_t kInitialPackBytes = 4u << 20;    // per-slot upload buffer at creation
constexpr size_t kInitialReqs = 1024;             // per-slot request states at creation

// First-fit allocator over [0, size) with coalescing.
struct Arena {
  std::map<uint64_t, uint64_t> free_;  // offset -> length
  uint64_t size = 0, used = 0;
  void init(uint64_t sz) {
    size = sz;
    free_.clear();
    free_[0] = sz;
    used = 0;
  }
  bool alloc(uint64_t bytes, uint64_t *off) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used += bytes;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

enum ReqState { R_PENDING = 0, R_INFLIGHT = 1, R_DONE = 2, R_FAILED = 3 };

struct Req {
  uint32_t stream;
  int kind;
  uint64_t n, pos, pos_hi, off;  // position pos_hi 2^64 + pos
  bool auto_release;
  int state;
  Clock::time_point t_arrival;   // latency origin
};

// One in-flight slot: a HIP stream, an end event, a completion signal and
// reusable buffers.  Everything an iteration reads (the tile claim counter,
// already zero, then the tile, lane and run descriptors and the request-state
// inputs) is packed into one pinned buffer, which the iteration's first
// kernel copies to device memory while it computes the request states.
//
// The signal is four words of coherent pinned memory that the iteration's
// kernels write: [1] the device clock when the upload starts, [2] when the
// generation kernel claims its first tile, [3] when its last wave finishes,
// then [0] the iteration's sequence number, once its outputs are visible
// device-wide.  The completer watches [0] (the end event only as a fallback),
// and the busy and kernel intervals come from the clock words, so no timing
// event sits between the kernels.
struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev1 = nullptr;  // after the iteration's last kernel
  uint64_t *h_sig = nullptr;  // the signal words (host address)
  uint64_t *d_sig = nullptr;  // their device mapping
  uint64_t seq = 0;           // iterations launched on the slot
  bool signals = false;       // the in-flight iteration runs the generation kernel
  bool busy = false;      // taken by the worker until its iteration has completed
  bool launched = false;  // an iteration is in flight (the slot's completer waits for it)
  std::vector<uint64_t> tickets;  // that iteration's requests
  std::condition_variable cv;     // wakes the slot's completer
  std::thread completer;
  size_t cap_pack = 0, cap_req = 0;
  uint8_t *d_pack = nullptr, *h_pack = nullptr;
  const uint8_t *h_pack_dev = nullptr;  // h_pack's device mapping, read by the prologue kernel
  uint64_t *d_req_state = nullptr;
};

// Byte offsets of the parts of a packed upload (each 256-byte aligned).
struct PackLayout {
  size_t counter = 0, tiles, lanes, runs, pos, idx, slot, total;
  PackLayout(size_t nt, size_t nl, size_t nr, size_t nreq) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    tiles = 256;
    lanes = up(tiles + nt * sizeof(TileDesc));
    runs = up(lanes + nl * sizeof(LaneDesc));
    pos = up(runs + nr * sizeof(RunDesc));
    idx = up(pos + nreq * 2 * 8);
    slot = up(idx + nreq * 4);
    total = up(slot + nreq * 4);
  }
};

// 128-bit position arithmetic: (hi, lo) += (bhi, blo) modulo 2^128.
void add128(uint64_t &hi, uint64_t &lo, uint64_t bhi, uint64_t blo) {
  const uint64_t s = lo + blo;
  hi += bhi + (s < lo ? 1 : 0);
  lo = s;
}

}  // namespace

struct slrng_server {
  slrng_server_opts o;
  slrng_batch_opts bo;
  int device = 0;
  unsigned blocks = 0;
  slrng_streams *streams = nullptr;
  uint8_t *arena_dev = nullptr;
  DigitMatrices digits;  // the engine's digit matrices (positioning from 128-bit positions)
  Arena arena;
  std::vector<uint64_t> head, head_hi;  // next position of each stream (128-bit)

  std::mutex mu;
  std::condition_variable cv_work, cv_space, cv_done;
  std::deque<uint64_t> pending;
  uint64_t pending_bytes = 0;
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next_ticket = 1;
  std::unique_ptr<Slot[]> slots;
  int nslots = 0;
  int launched = 0;  // slots with an iteration in flight
  bool stop = false, worker_done = false;
  int error = 0;
  uint64_t clock_origin = 0;  // device clock at creation: origin of the intervals
  double clock_khz = 1;       // device clock rate
  std::vector<std::pair<double, double>> busy_ivals;    // device [start, end) ms per iteration
  std::vector<std::pair<double, double>> kernel_ivals;  // generation kernel [start, end) ms
  std::thread worker;

  // statistics
  Clock::time_point t0;
  std::vector<double> lat_us;
  uint64_t submitted = 0, completed = 0, failed = 0, rejected = 0, outputs = 0;
  uint64_t iterations = 0, max_inflight = 0, peak_reserved = 0, max_batch_seen = 0, batch_sum = 0;
};

// Make the slot's buffers hold a packed upload of `bytes` and `nreq` request
// states (the slot is idle: its previous iteration has completed, so the
// pinned buffer is no longer being copied from).
static int slot_reserve(Slot &s, size_t bytes, size_t nreq) {
  if (bytes > s.cap_pack) {
    const size_t n = std::max<size_t>({bytes, s.cap_pack * 2, (size_t)1 << 16});
    if (s.d_pack) (void)hipFree(s.d_pack);
    if (s.h_pack) (void)hipHostFree(s.h_pack);
    s.d_pack = s.h_pack = nullptr;
    s.h_pack_dev = nullptr;
    s.cap_pack = 0;
    hipError_t e = hipMalloc((void **)&s.d_pack, n);
    // coherent: the prologue kernel reads what the host wrote just before its
    // launch, never a copy cached from the slot's previous iteration
    if (e == hipSuccess) e = hipHostMalloc((void **)&s.h_pack, n, hipHostMallocCoherent);
    void *mapped = nullptr;
    if (e == hipSuccess) e = hipHostGetDevicePointer(&mapped, s.h_pack, 0);
    if (e != hipSuccess) return hip_fail(e);
    s.h_pack_dev = static_cast<const uint8_t *>(mapped);
    s.cap_pack = n;
  }
  if (nreq > s.cap_req) {
    const size_t n = std::max<size_t>({nreq, s.cap_req * 2, 64});
    if (s.d_req_state) (void)hipFree(s.d_req_state);
    s.d_req_state = nullptr;
    s.cap_req = 0;
    hipError_t e = hipMalloc(&s.d_req_state, n * 16 * 8);
    if (e != hipSuccess) return hip_fail(e);
    s.cap_req = n;
  }
  return SLRNG_OK;
}

static void free_slot(Slot &s) {
  if (s.d_pack) (void)hipFree(s.d_pack);
  if (s.d_req_state) (void)hipFree(s.d_req_state);
  if (s.h_pack) (void)hipHostFree(s.h_pack);
  if (s.h_sig) (void)hipHostFree(s.h_sig);
  if (s.ev1) (void)hipEventDestroy(s.ev1);
  if (s.st) (void)hipStreamDestroy(s.st);
}

// Plan and launch one iteration on slot `si` (called by the worker without the lock).
static int launch_iteration(slrng_server *sv, int si, const std::vector<PlanReq> &pr) {
  Slot &s = sv->slots[si];
  PlanHost P;
  int rc = build_plan(pr.data(), pr.size(), sv->bo, sv->device, (uint64_t)sv->blocks * kBlock, P,
                      /*fit=*/true, (uint64_t)sv->o.min_chunk);
  if (rc) return rc;
  const size_t nreq = P.rs.origin_idx.size();
  const PackLayout L(P.tiles.size(), P.lanes.size(), P.runs.size(), nreq);
  rc = slot_reserve(s, L.total, nreq);
  if (rc) return rc;
  uint8_t *h = s.h_pack;
  memset(h + L.counter, 0, 256);  // the claim counters start at zero
  if (!P.tiles.empty()) memcpy(h + L.tiles, P.tiles.data(), P.tiles.size() * sizeof(TileDesc));
  if (!P.lanes.empty()) memcpy(h + L.lanes, P.lanes.data(), P.lanes.size() * sizeof(LaneDesc));
  if (!P.runs.empty()) memcpy(h + L.runs, P.runs.data(), P.runs.size() * sizeof(RunDesc));
  if (nreq) {
    memcpy(h + L.pos, P.rs.pos.data(), P.rs.pos.size() * 8);
    memcpy(h + L.idx, P.rs.origin_idx.data(), P.rs.origin_idx.size() * 4);
    memcpy(h + L.slot, P.rs.slot.data(), P.rs.slot.size() * 4);
  }
  uint8_t *d = s.d_pack;
  const TileDesc *d_tiles = reinterpret_cast<const TileDesc *>(d + L.tiles);
  const LaneDesc *d_lanes = reinterpret_cast<const LaneDesc *>(d + L.lanes);
  const RunDesc *d_runs = reinterpret_cast<const RunDesc *>(d + L.runs);
  unsigned *d_counter = reinterpret_cast<unsigned *>(d + L.counter);
  hipStream_t st = s.st;
  // the upload is done by a kernel on the slot's stream (reading the pinned
  // buffer), not a copy-engine transfer, so that the generation kernel does
  // not wait for a hand-off between engines; it stamps the iteration's start
  s.seq++;
  __atomic_store_n(s.h_sig + 2, 0, __ATOMIC_RELAXED);
  __atomic_store_n(s.h_sig + 3, 0, __ATOMIC_RELAXED);
  s.signals = false;
  // the request states are computed in the same launch as the upload (the
  // server has one variant: at most one run), reading positions, origins
  // and slots from the pinned buffer
  const uint8_t *hd = s.h_pack_dev;
  ReqArgs ra;
  ra.seeds = nullptr;
  ra.origin_state = streams_state_ptr(sv->streams);
  ra.origin_stride = sv->o.n_streams;
  ra.origin_idx = reinterpret_cast<const uint32_t *>(hd + L.idx);
  ra.polys = nullptr;
  ra.pos = reinterpret_cast<const uint64_t *>(hd + L.pos);
  ra.slot = reinterpret_cast<const uint32_t *>(hd + L.slot);
  ra.req_state = s.d_req_state;
  ra.m = 0;
  for (auto &run : P.rs.runs) {
    if (run.first != sv->o.variant) return SLRNG_EINVAL;  // not reached: requests carry the server's variant
    ra.m += run.second;
  }
  hipError_t e = launch_prologue(sv->o.variant, ra, sv->digits.dev, sv->digits.bits, sv->digits.levels, d,
                                 hd, L.total, s.d_sig + 1, st);
  if (e != hipSuccess) return hip_fail(e);
  if (!P.tiles.empty()) {
    BatchArgs a{};
    a.tiles = d_tiles;
    a.ntiles = (uint32_t)P.tiles.size();
    a.lanes = d_lanes;
    a.runs = d_runs;
    a.req_state = s.d_req_state;
    for (int v = 0; v < kNumVariants; v++) {
      a.tab[v] = P.tab[v];
      a.tab_n[v] = P.tab_n[v];
    }
    a.counter = d_counter;  // zeroed by the upload
    a.sig = s.d_sig;
    a.seq = s.seq;
    const unsigned blocks = std::min<unsigned>(sv->blocks, ((unsigned)P.tiles.size() + 3) / 4);
    e = launch_batch(a, sv->bo.tile, blocks, st, sv->o.variant, sv->o.store);
    if (e != hipSuccess) return hip_fail(e);
    s.signals = true;
  }
  e = hipEventRecord(s.ev1, st);
  return e == hipSuccess ? SLRNG_OK : hip_fail(e);
}

static int free_slot_index(slrng_server *sv) {
  for (int i = 0; i < sv->nslots; i++)
    if (!sv->slots[i].busy) return i;
  return -1;
}

static void worker_main(slrng_server *sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    sv->cv_work.wait(lk, [&] {
      if (sv->pending.empty()) return sv->stop;
      return free_slot_index(sv) >= 0;
    });
    if (sv->pending.empty()) {  // stop requested and nothing left to launch
      sv->worker_done = true;
      for (int i = 0; i < sv->nslots; i++) sv->slots[i].cv.notify_all();
      sv->cv_done.notify_all();
      return;
    }
    // batching window: hold the iteration until the oldest pending request
    // has waited window_us, unless enough bytes are pending already
    if (sv->o.window_us > 0 && !sv->stop) {
      const auto due = sv->reqs[sv->pending.front()].t_arrival + std::chrono::microseconds(sv->o.window_us);
      if (Clock::now() < due && sv->pending_bytes < sv->o.window_bytes) {
        sv->cv_work.wait_until(lk, due, [&] { return sv->stop || sv->pending_bytes >= sv->o.window_bytes; });
        continue;  // re-check slots and pending
      }
    }
    const int si = free_slot_index(sv);
    if (si < 0) continue;
    Slot &slot = sv->slots[si];
    slot.tickets.clear();
    std::vector<PlanReq> pr;
    const size_t take = std::min<size_t>(sv->pending.size(), (size_t)sv->o.max_batch);
    for (size_t k = 0; k < take; k++) {
      const uint64_t t = sv->pending.front();
      sv->pending.pop_front();
      Req &q = sv->reqs[t];
      sv->pending_bytes -= q.n * 8;
      q.state = R_INFLIGHT;
      slot.tickets.push_back(t);
      PlanReq p{sv->o.variant, q.kind, q.n, (uint64_t)(uintptr_t)(sv->arena_dev + q.off), q.pos,
                true, 0, q.stream, (uint64_t)k};
      p.start_hi = q.pos_hi;
      pr.push_back(p);
    }
    slot.busy = true;
    lk.unlock();
    const int rc = launch_iteration(sv, si, pr);
    // after a failed launch, let whatever was queued on the slot's stream
    // (the upload reads the slot's pinned buffer) finish before the slot is
    // handed out again
    if (rc) (void)hipStreamSynchronize(slot.st);
    lk.lock();
    if (rc) {
      // the launch failed: fail exactly these requests and free the slot
      sv->error = rc;
      for (uint64_t t : slot.tickets) {
        auto f = sv->reqs.find(t);
        if (f == sv->reqs.end()) continue;
        f->second.state = R_FAILED;
        sv->failed++;
        if (f->second.auto_release) {
          sv->arena.release(f->second.off, f->second.n * 8);
          sv->reqs.erase(f);
        }
      }
      slot.tickets.clear();
      slot.busy = false;
      sv->cv_done.notify_all();
      sv->cv_space.notify_all();
      continue;
    }
    sv->iterations++;
    sv->batch_sum += slot.tickets.size();
    sv->max_batch_seen = std::max<uint64_t>(sv->max_batch_seen, slot.tickets.size());
    slot.launched = true;
    sv->launched++;
    sv->max_inflight = std::max<uint64_t>(sv->max_inflight, (uint64_t)sv->launched);
    slot.cv.notify_all();  // wakes the slot's completer
  }
}

// Waits for the slot's in-flight iteration: for its signal when the
// generation kernel writes one (polled, with the end event queried now and
// then for errors), else, and after kSpinLimit of polling, for the end event.
constexpr std::chrono::microseconds kSpinLimit(2000);

static hipError_t wait_iteration(const Slot &s) {
  if (s.signals) {
    const Clock::time_point t0 = Clock::now();
    for (unsigned i = 1;; i++) {
      if (__atomic_load_n(s.h_sig, __ATOMIC_ACQUIRE) == s.seq) return hipSuccess;
      if ((i & 255) == 0) {
        const hipError_t q = hipEventQuery(s.ev1);
        if (q != hipErrorNotReady) return q;  // complete (the signal is then written) or failed
        if (Clock::now() - t0 > kSpinLimit) break;
      }
      __builtin_ia32_pause();
    }
  }
  return hipEventSynchronize(s.ev1);
}

// Completion of the iterations of one slot, whatever the other slots are
// doing.
static void completer_main(slrng_server *sv, int si) {
  (void)hipSetDevice(sv->device);
  Slot &s = sv->slots[si];
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    s.cv.wait(lk, [&] { return s.launched || sv->worker_done; });
    if (!s.launched) return;  // the worker has exited and this slot is idle
    lk.unlock();
    const hipError_t e = wait_iteration(s);
    const Clock::time_point now = Clock::now();
    lk.lock();
    if (e == hipSuccess && s.signals) {
      uint64_t t[4];
      for (int w = 1; w < 4; w++) t[w] = __atomic_load_n(s.h_sig + w, __ATOMIC_RELAXED);
      auto ms = [&](uint64_t c) { return (double)(int64_t)(c - sv->clock_origin) / sv->clock_khz; };
      // the end stamp precedes the signal in the last wave; a start stamp
      // that reads 0 or out of order (not expected) is replaced by the other
      // one, the kernel interval then widening to the whole iteration
      const bool ok1 = t[1] && t[1] <= t[3], ok2 = t[2] && t[2] <= t[3];
      if (ok1 || ok2) {
        const uint64_t k0 = ok2 ? t[2] : t[1];
        const uint64_t b0 = ok1 ? std::min(t[1], k0) : k0;
        sv->busy_ivals.push_back({ms(b0), ms(t[3])});
        sv->kernel_ivals.push_back({ms(k0), ms(t[3])});
      }
    }
    for (uint64_t t : s.tickets) {
      auto f = sv->reqs.find(t);
      if (f == sv->reqs.end()) continue;
      Req &q = f->second;
      if (e == hipSuccess) {
        q.state = R_DONE;
        sv->completed++;
        sv->outputs += q.n;
        sv->lat_us.push_back(secs(q.t_arrival, now) * 1e6);
      } else {
        q.state = R_FAILED;
        sv->failed++;
        sv->error = hip_fail(e);
      }
      if (q.auto_release) {
        sv->arena.release(q.off, q.n * 8);
        sv->reqs.erase(f);
      }
    }
    s.tickets.clear();
    s.launched = false;
    s.busy = false;
    sv->launched--;
    sv->cv_work.notify_all();
    sv->cv_space.notify_all();
    sv->cv_done.notify_all();
  }
}

extern "C" int slrng_server_default_opts(slrng_server_opts *o) {
  return guarded([&]() -> int {
    if (!o) return SLRNG_EINVAL;
    memset(o, 0, sizeof(*o));
    o->budget_bytes = 16ull << 30;
    o->n_streams = 4096;
    o->variant = SLRNG_XOSHIRO256_STARSTAR;
    o->seed = 42;
    o->max_batch = 4096;
    o->inflight = 3;
    o->tile = 32;
    o->waves_per_cu = 8;
    o->chunk = 0;
    o->window_us = 0;
    o->window_bytes = 256ull << 20;
    return SLRNG_OK;
  });
}

static void destroy_server(slrng_server *sv) {
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  sv->cv_done.notify_all();
  sv->cv_space.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  // the worker has launched everything it took; the completers finish those
  // iterations and exit
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->worker_done = true;
    for (int i = 0; i < sv->nslots; i++) sv->slots[i].cv.notify_all();
  }
  for (int i = 0; i < sv->nslots; i++)
    if (sv->slots[i].completer.joinable()) sv->slots[i].completer.join();
  for (int i = 0; i < sv->nslots; i++) {
    Slot &s = sv->slots[i];
    if (s.st) (void)hipStreamSynchronize(s.st);
    free_slot(s);
  }
  if (sv->arena_dev) {
    if (sv->o.arena_plain) (void)hipFree(sv->arena_dev);
    else (void)spread_free(sv->arena_dev);
  }
  if (sv->streams) slrng_streams_destroy(sv->streams);
  delete sv;
}

extern "C" int slrng_server_create(const slrng_server_opts *opts, slrng_server **out) {
  return guarded([&]() -> int {
    if (!out) return SLRNG_EINVAL;
    *out = nullptr;
    slrng_server_opts o;
    if (opts) o = *opts;
    else slrng_server_default_opts(&o);
    if (!valid_variant64(o.variant) || o.n_streams == 0 || o.budget_bytes < kAlign) return SLRNG_EINVAL;
    if (o.max_batch <= 0) o.max_batch = 4096;
    if (o.inflight <= 0) o.inflight = 3;
    if (o.inflight > 8 || o.min_chunk < 0 || o.window_us < 0 || o.store < 0 || o.store > 2)
      return SLRNG_EINVAL;
    if (o.tile == 0) o.tile = 32;
    slrng_batch_opts bo;
    slrng_batch_default_opts(&bo);
    bo.mode = SLRNG_BATCH_PERSISTENT;
    bo.tile = o.tile;
    bo.waves_per_cu = o.waves_per_cu;
    if (o.chunk) bo.chunk[o.variant] = o.chunk;
    int rc = check_batch_opts(bo);
    if (rc) return rc;
    slrng_server *sv = new (std::nothrow) slrng_server();
    if (!sv) return SLRNG_ENOMEM;
    sv->o = o;
    sv->bo = bo;
    hipError_t e = hipGetDevice(&sv->device);
    if (e != hipSuccess) {
      delete sv;
      return hip_fail(e);
    }
    rc = batch_grid_blocks(bo, sv->device, &sv->blocks, o.variant);
    // every chunk table an iteration can pick, built now rather than in the
    // middle of serving (one table of 65,536 polynomials takes milliseconds)
    if (!rc) rc = warm_fit_tables(sv->device, o.variant, bo, (uint64_t)o.min_chunk);
    if (!rc) rc = slrng_streams_create(o.variant, o.seed, o.n_streams, nullptr, &sv->streams);
    // the engine's digit matrices: a request's start state s_j M^pos is then
    // computed on the device from the digits of pos (built once per device
    // and engine)
    if (!rc) rc = digit_matrices(sv->device, o.variant, &sv->digits);
    if (!rc) {
      e = hipDeviceSynchronize();
      if (e != hipSuccess) rc = hip_fail(e);
    }
    if (!rc) {
      // spread physical pages by default: iterations of hundreds of MB and
      // more write measurably faster there (creation briefly holds a few
      // times the budget); a plain allocation on request
      e = o.arena_plain ? hipMalloc(&sv->arena_dev, o.budget_bytes)
                        : spread_alloc(o.budget_bytes, (void **)&sv->arena_dev);
      if (e != hipSuccess) rc = e == hipErrorOutOfMemory ? SLRNG_ENOMEM : hip_fail(e);
    }
    if (!rc) {
      sv->arena.init(o.budget_bytes / kAlign * kAlign);
      sv->head.assign(o.n_streams, 0);
      sv->head_hi.assign(o.n_streams, 0);
      sv->slots.reset(new Slot[o.inflight]);
      sv->nslots = o.inflight;
      for (int i = 0; i < sv->nslots; i++) {
        Slot &s = sv->slots[i];
        e = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ev1, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s.h_sig, 4 * sizeof(uint64_t), hipHostMallocCoherent);
        void *mapped = nullptr;
        if (e == hipSuccess) e = hipHostGetDevicePointer(&mapped, s.h_sig, 0);
        if (e == hipSuccess) {
          s.d_sig = static_cast<uint64_t *>(mapped);
          for (int w = 0; w < 4; w++) s.h_sig[w] = 0;
        }
        if (e != hipSuccess) {
          rc = hip_fail(e);
          break;
        }
        // buffers for typical iterations now: pinned allocations take
        // milliseconds, which the first iterations would otherwise wait for
        rc = slot_reserve(s, kInitialPackBytes, kInitialReqs);
        if (rc) break;
      }
    }
    if (!rc) {
      // the interval origin: the device clock now, stamped by an empty upload
      int khz = 0;
      e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, sv->device);
      Slot &s = sv->slots[0];
      if (e == hipSuccess) {
        ReqArgs none{};
        e = launch_prologue(o.variant, none, nullptr, 0, 0, nullptr, nullptr, 0, s.d_sig + 1, s.st);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(s.st);
      if (e == hipSuccess && khz <= 0) e = hipErrorInvalidValue;
      if (e != hipSuccess) rc = hip_fail(e);
      else {
        sv->clock_khz = khz;
        sv->clock_origin = __atomic_load_n(s.h_sig + 1, __ATOMIC_ACQUIRE);
      }
    }
    if (rc) {
      sv->worker_done = true;
      destroy_server(sv);
      return rc;
    }
    sv->t0 = Clock::now();
    for (int i = 0; i < sv->nslots; i++) sv->slots[i].completer = std::thread(completer_main, sv, i);
    sv->worker = std::thread(worker_main, sv);
    *out = sv;
    return SLRNG_OK;
  });
}

extern "C" int slrng_server_destroy(slrng_server *sv) {
  return guarded([&]() -> int {
    if (!sv) return SLRNG_EINVAL;
    destroy_server(sv);
    return SLRNG_OK;
  });
}

// Admission of one request that arrived at `arrival` (the latency origin).
static int submit_at(slrng_server *sv, uint32_t stream_id, uint64_t n, int kind, int flags,
                     uint64_t *ticket, Clock::time_point arrival) {
  if (!sv || !ticket || (kind != SLRNG_U64 && kind != SLRNG_F64)) return SLRNG_EINVAL;
  if (stream_id >= sv->o.n_streams || n == 0) return SLRNG_EINVAL;
  if (n > sv->arena.size / 8) return SLRNG_ERANGE;
  std::unique_lock<std::mutex> lk(sv->mu);
  uint64_t off = 0;
  for (;;) {
    if (sv->stop) return SLRNG_EINVAL;
    if (sv->arena.alloc(n * 8, &off)) break;
    if (flags & SLRNG_SUBMIT_NONBLOCK) {
      sv->rejected++;
      return SLRNG_EAGAIN;
    }
    sv->cv_space.wait(lk);
  }
  sv->peak_reserved = std::max(sv->peak_reserved, sv->arena.used);
  Req q;
  q.stream = stream_id;
  q.kind = kind;
  q.n = n;
  q.pos = sv->head[stream_id];
  q.pos_hi = sv->head_hi[stream_id];
  add128(sv->head_hi[stream_id], sv->head[stream_id], 0, n);
  q.off = off;
  q.auto_release = (flags & SLRNG_SUBMIT_AUTORELEASE) != 0;
  q.state = R_PENDING;
  q.t_arrival = arrival;
  const uint64_t t = sv->next_ticket++;
  sv->reqs.emplace(t, q);
  sv->pending.push_back(t);
  sv->pending_bytes += n * 8;
  sv->submitted++;
  *ticket = t;
  sv->cv_work.notify_one();
  return SLRNG_OK;
}

extern "C" int slrng_server_submit(slrng_server *sv, uint32_t stream_id, uint64_t n, int kind,
                                   int flags, uint64_t *ticket) {
  return guarded([&]() -> int {
    // the request arrives now: a wait for arena space counts in its latency
    return submit_at(sv, stream_id, n, kind, flags, ticket, Clock::now());
  });
}

extern "C" int slrng_server_advance(slrng_server *sv, uint32_t stream_id, uint64_t steps_hi,
                                    uint64_t steps_lo) {
  return guarded([&]() -> int {
    if (!sv || stream_id >= sv->o.n_streams) return SLRNG_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    add128(sv->head_hi[stream_id], sv->head[stream_id], steps_hi, steps_lo);
    return SLRNG_OK;
  });
}

extern "C" int slrng_server_intervals(slrng_server *sv, double *kernel_start_ms, double *kernel_end_ms,
                                      uint64_t cap, uint64_t *count) {
  return guarded([&]() -> int {
    if (!sv || !count || (cap && (!kernel_start_ms || !kernel_end_ms))) return SLRNG_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    const uint64_t n = sv->kernel_ivals.size();
    for (uint64_t i = 0; i < n && i < cap; i++) {
      kernel_start_ms[i] = sv->kernel_ivals[i].first;
      kernel_end_ms[i] = sv->kernel_ivals[i].second;
    }
    *count = n;
    return SLRNG_OK;
  });
}

extern "C" int slrng_server_poll(slrng_server *sv, uint64_t ticket, void **dev_ptr, uint64_t *pos) {
  return guarded([&]() -> int {
    if (!sv) return SLRNG_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    auto f = sv->reqs.find(ticket);
    if (f == sv->reqs.end()) return SLRNG_EINVAL;
    if (dev_ptr) *dev_ptr = sv->arena_dev + f->second.off;
    if (pos) *pos = f->second.pos;
    if (f->second.state == R_FAILED) return SLRNG_EHIP;
    return f->second.state == R_DONE ? 1 : 0;
  });
}

extern "C" int slrng_server_wait(slrng_server *sv, uint64_t ticket, void **dev_ptr, uint64_t *pos) {
  return guarded([&]() -> int {
    if (!sv) return SLRNG_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
      auto f = sv->reqs.find(ticket);
      if (f == sv->reqs.end()) return SLRNG_EINVAL;
      if (dev_ptr) *dev_ptr = sv->arena_dev + f->second.off;
      if (pos) *pos = f->second.pos;
      if (f->second.state == R_FAILED) return SLRNG_EHIP;
      if (f->second.state == R_DONE) return SLRNG_OK;
      sv->cv_done.wait(lk);
    }
  });
}

extern "C" int slrng_server_release(slrng_server *sv, uint64_t ticket) {
  return guarded([&]() -> int {
    if (!sv) return SLRNG_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    auto f = sv->reqs.find(ticket);
    if (f == sv->reqs.end() || f->second.auto_release) return SLRNG_EINVAL;
    if (f->second.state != R_DONE && f->second.state != R_FAILED) return SLRNG_EAGAIN;
    sv->arena.release(f->second.off, f->second.n * 8);
    sv->reqs.erase(f);
    sv->cv_space.notify_all();
    return SLRNG_OK;
  });
}

extern "C" int slrng_server_drain(slrng_server *sv) {
  return guarded([&]() -> int {
    if (!sv) return SLRNG_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] {
      if (!sv->pending.empty()) return false;
      for (int i = 0; i < sv->nslots; i++)
        if (sv->slots[i].busy) return false;
      return true;
    });
    return sv->error ? sv->error : SLRNG_OK;
  });
}

extern "C" int slrng_server_get_stats(slrng_server *sv, slrng_server_stats *out) {
  return guarded([&]() -> int {
    if (!sv || !out) return SLRNG_EINVAL;
    std::vector<double> lat;
    {
      std::lock_guard<std::mutex> g(sv->mu);
      memset(out, 0, sizeof(*out));
      out->submitted = sv->submitted;
      out->completed = sv->completed;
      out->failed = sv->failed;
      out->rejected = sv->rejected;
      out->outputs = sv->outputs;
      out->wall_s = secs(sv->t0, Clock::now());
      // unions of the iterations' device intervals (iterations may overlap)
      auto union_ms = [](std::vector<std::pair<double, double>> iv) {
        std::sort(iv.begin(), iv.end());
        double tot = 0, cs = 0, ce = -1;
        for (auto &x : iv) {
          if (x.first > ce) {
            if (ce > cs) tot += ce - cs;
            cs = x.first;
            ce = x.second;
          } else {
            ce = std::max(ce, x.second);
          }
        }
        if (ce > cs) tot += ce - cs;
        return tot;
      };
      out->busy_s = union_ms(sv->busy_ivals) * 1e-3;
      out->kernel_s = union_ms(sv->kernel_ivals) * 1e-3;
      out->iterations = sv->iterations;
      out->max_inflight = sv->max_inflight;
      out->peak_reserved_bytes = sv->peak_reserved;
      out->reserved_bytes = sv->arena.used;
      out->max_batch = sv->max_batch_seen;
      out->mean_batch = sv->iterations ? (double)sv->batch_sum / sv->iterations : 0.0;
      lat = sv->lat_us;
    }
    if (!lat.empty()) {
      std::sort(lat.begin(), lat.end());
      auto q = [&](double p) { return lat[std::min(lat.size() - 1, (size_t)(p * (lat.size() - 1) + 0.5))]; };
      out->p50_us = q(0.50);
      out->p99_us = q(0.99);
      out->max_us = lat.back();
    }
    return SLRNG_OK;
  });
}

extern "C" int slrng_server_reset_stats(slrng_server *sv) {
  return guarded([&]() -> int {
    if (!sv) return SLRNG_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    sv->t0 = Clock::now();
    sv->lat_us.clear();
    sv->submitted = sv->completed = sv->failed = sv->rejected = sv->outputs = 0;
    sv->iterations = sv->max_inflight = sv->max_batch_seen = sv->batch_sum = 0;
    sv->peak_reserved = sv->arena.used;
    sv->busy_ivals.clear();
    sv->kernel_ivals.clear();
    return SLRNG_OK;
  });
}

extern "C" int slrng_server_replay(slrng_server *sv, const double *t_arrival_s, const uint32_t *stream_ids,
                                   const uint64_t *n, const int32_t *kinds, size_t count) {
  return guarded([&]() -> int {
    if (!sv || (count && (!t_arrival_s || !stream_ids || !n || !kinds))) return SLRNG_EINVAL;
    const Clock::time_point start = Clock::now();
    for (size_t i = 0; i < count; i++) {
      const auto due = start + std::chrono::duration_cast<Clock::duration>(
                                   std::chrono::duration<double>(t_arrival_s[i]));
      // sleep until close to the arrival, then spin for the last stretch
      while (true) {
        const auto now = Clock::now();
        if (now >= due) break;
        if (due - now > std::chrono::microseconds(200))
          std::this_thread::sleep_for(due - now - std::chrono::microseconds(100));
      }
      // the latency of a replayed request counts from its scheduled arrival,
      // so that a late submission (the replay falling behind, a wait for
      // arena space) shows in the statistics
      uint64_t t = 0;
      int rc = submit_at(sv, stream_ids[i], n[i], kinds[i], SLRNG_SUBMIT_AUTORELEASE, &t, due);
      if (rc) return rc;
    }
    return slrng_server_drain(sv);
  });
}

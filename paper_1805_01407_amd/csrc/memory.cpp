// Device memory for large outputs, laid out for HBM write bandwidth.
//
// On MI355X the store bandwidth that one buffer sees depends on how widely
// its physical pages are spread over the HBM: a large allocation made early
// in a process sits in one compact physical range and caps a stream of
// 16-byte stores near 5.5 TB/s, while the same bytes spread over about four
// times that span reach 6.5-6.9 TB/s (the same fill kernel, measured).  The
// allocator below keeps the buffer virtually contiguous (the output layout
// out[i*ld + t] does not change) and spreads its physical backing with the
// HIP virtual memory API:
//   * the buffer is cut into M pieces of P bytes (P a power of two in
//     [256 MiB, 1 GiB], about 1/64 of the buffer: few enough mappings that a
//     launch stays cheap, large enough that address translation does not
//     slow the stores);
//   * gap x M physical pieces are created in order, every gap-th one is kept
//     and the others are released at once, so the kept pieces lie about
//     gap x P apart (gap = 16, lower when free memory is short: the full
//     gap x M x P bytes are held during the call, so a 32 GiB buffer gets a
//     gap of about 8 on an otherwise empty 288 GB device, 16 GiB one of 16;
//     measured: a 32 GiB buffer at gap 8 fills at 7.0 TB/s and takes
//     k_generate at 6.7, against 6.5 and 6.5 at gap 4; a 16 GiB server arena
//     at gap 16 lifted 2 GB served iterations from 0.60 to 0.70 of peak);
//   * the kept pieces are mapped into one reserved virtual range aligned to
//     P, read-write for the current device, in bit-reversed order of their
//     creation (virtual piece v holds kept piece rev(v)): a contiguous part of
//     the buffer is then spread over the whole physical span too, not only
//     the buffer as a whole (measured: 1-17 GB written into the first pieces
//     of a 32 GiB buffer mapped in creation order ran at 5.3-5.5 TB/s, the
//     whole buffer at 6.4).
// Requests below 1 GiB are a plain device allocation, and so is any request
// on a device without the virtual memory API or whose pieces cannot be mapped
// (placement changes speed only, never values).
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/slrng.h"
#include "api_internal.hpp"
#include "memory.hpp"

namespace slrng {
namespace {

constexpr uint64_t kMiB = 1ull << 20, kGiB = 1ull << 30;
constexpr uint64_t kSpreadMin = kGiB;  // smaller requests: plain allocation
constexpr int kMaxGap = 16;
constexpr uint64_t kFreeMargin = 2 * kGiB;  // left free while the spare pieces exist

struct Block {
  bool spread = false;
  uint64_t reserved = 0;  // bytes of virtual range (M x P)
  std::vector<hipMemGenericAllocationHandle_t> pieces;
};

std::mutex g_mu;
std::unordered_map<void *, Block> g_blocks;

uint64_t piece_bytes(uint64_t bytes) {
  uint64_t p = 256 * kMiB;
  while (p < kGiB && p * 64 < bytes) p <<= 1;
  return p;
}

hipMemAllocationProp device_prop(int dev) {
  hipMemAllocationProp p = {};
  p.type = hipMemAllocationTypePinned;
  p.location.type = hipMemLocationTypeDevice;
  p.location.id = dev;
  return p;
}

void release_all(std::vector<hipMemGenericAllocationHandle_t> &v) {
  for (auto h : v) (void)hipMemRelease(h);
  v.clear();
}

// Creates gap x M pieces and keeps every gap-th; hipErrorOutOfMemory if the
// device cannot hold them all at once.
hipError_t take_pieces(int dev, uint64_t P, uint64_t M, int gap,
                       std::vector<hipMemGenericAllocationHandle_t> &keep) {
  const hipMemAllocationProp prop = device_prop(dev);
  std::vector<hipMemGenericAllocationHandle_t> all;
  all.reserve(M * gap);
  hipError_t e = hipSuccess;
  for (uint64_t j = 0; j < M * (uint64_t)gap; j++) {
    hipMemGenericAllocationHandle_t h;
    e = hipMemCreate(&h, P, &prop, 0);
    if (e != hipSuccess) break;
    all.push_back(h);
  }
  if (e != hipSuccess) {
    release_all(all);
    return e;
  }
  keep.clear();
  for (uint64_t j = 0; j < all.size(); j++) {
    if (j % gap == 0) keep.push_back(all[j]);
    else (void)hipMemRelease(all[j]);
  }
  return hipSuccess;
}

// The indices 0 .. M-1 in bit-reversed order (of ceil(log2 M) bits, the
// values >= M skipped): every run of consecutive entries is spread over the
// whole range.
std::vector<uint64_t> bit_reversed_order(uint64_t M) {
  int bits = 0;
  while ((1ull << bits) < M) bits++;
  std::vector<uint64_t> order;
  order.reserve(M);
  for (uint64_t i = 0; i < (1ull << bits); i++) {
    uint64_t r = 0;
    for (int b = 0; b < bits; b++) r |= ((i >> b) & 1) << (bits - 1 - b);
    if (r < M) order.push_back(r);
  }
  return order;
}

hipError_t map_pieces(int dev, uint64_t P, std::vector<hipMemGenericAllocationHandle_t> &keep,
                      void **out) {
  const uint64_t span = P * keep.size();
  void *va = nullptr;
  hipError_t e = hipMemAddressReserve(&va, span, P, nullptr, 0);
  if (e != hipSuccess) return e;
  const std::vector<uint64_t> order = bit_reversed_order(keep.size());
  uint64_t mapped = 0;
  for (; mapped < keep.size(); mapped++) {
    e = hipMemMap(static_cast<char *>(va) + mapped * P, P, 0, keep[order[mapped]], 0);
    if (e != hipSuccess) break;
  }
  if (e == hipSuccess) {
    hipMemAccessDesc d = {};
    d.location.type = hipMemLocationTypeDevice;
    d.location.id = dev;
    d.flags = hipMemAccessFlagsProtReadWrite;
    e = hipMemSetAccess(va, span, &d, 1);
  }
  if (e != hipSuccess) {
    if (mapped) (void)hipMemUnmap(va, mapped * P);
    (void)hipMemAddressFree(va, span);
    return e;
  }
  *out = va;
  return hipSuccess;
}

// Spread placement for `bytes` on device `dev` (hipErrorNotSupported when
// the device has no virtual memory API).
hipError_t spread_pieces(int dev, uint64_t bytes, Block &b, void **out) {
  int vmm = 0;
  hipError_t e = hipDeviceGetAttribute(&vmm, hipDeviceAttributeVirtualMemoryManagementSupported, dev);
  if (e != hipSuccess) return e;
  if (!vmm) return hipErrorNotSupported;
  const uint64_t P = piece_bytes(bytes);
  const uint64_t M = (bytes + P - 1) / P;
  size_t free_b = 0, total_b = 0;
  e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) return e;
  const uint64_t usable = free_b > kFreeMargin ? free_b - kFreeMargin : 0;
  int gap = (int)std::min<uint64_t>(kMaxGap, usable / (M * P));
  if (gap < 1) gap = 1;
  for (;; gap--) {
    e = take_pieces(dev, P, M, gap, b.pieces);
    if (e == hipSuccess || gap == 1) break;
  }
  if (e != hipSuccess) return e;
  e = map_pieces(dev, P, b.pieces, out);
  if (e != hipSuccess) {
    release_all(b.pieces);
    return e;
  }
  b.spread = true;
  b.reserved = M * P;
  return hipSuccess;
}

}  // namespace

hipError_t spread_alloc(uint64_t bytes, void **out) {
  *out = nullptr;
  Block b;
  hipError_t e = hipErrorNotSupported;
  if (bytes >= kSpreadMin) {
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = spread_pieces(dev, bytes, b, out);
    if (e == hipErrorOutOfMemory) return e;
    if (e != hipSuccess) {  // no virtual memory API, or a mapping failed
      (void)hipGetLastError();
      b = Block();
      *out = nullptr;
    }
  }
  if (e != hipSuccess) {
    e = hipMalloc(out, bytes);
    if (e != hipSuccess) return e;
  }
  std::lock_guard<std::mutex> g(g_mu);
  g_blocks.emplace(*out, std::move(b));
  return hipSuccess;
}

int spread_free(void *p) {
  Block b;
  {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_blocks.find(p);
    if (it == g_blocks.end()) return SLRNG_EINVAL;
    b = std::move(it->second);
    g_blocks.erase(it);
  }
  // unmapping memory that queued work still writes would fault: wait first
  hipError_t e = hipDeviceSynchronize();
  if (!b.spread) {
    hipError_t e2 = hipFree(p);
    if (e == hipSuccess) e = e2;
  } else {
    hipError_t e2 = hipMemUnmap(p, b.reserved);
    if (e == hipSuccess) e = e2;
    e2 = hipMemAddressFree(p, b.reserved);
    if (e == hipSuccess) e = e2;
    release_all(b.pieces);
  }
  return e == hipSuccess ? SLRNG_OK : hip_fail(e);
}

}  // namespace slrng

extern "C" int slrng_output_alloc(uint64_t bytes, void **dev_ptr) {
  return slrng::guarded([&]() -> int {
    if (!dev_ptr) return SLRNG_EINVAL;
    *dev_ptr = nullptr;
    if (bytes == 0) return SLRNG_EINVAL;
    hipError_t e = slrng::spread_alloc(bytes, dev_ptr);
    if (e == hipErrorOutOfMemory) {
      (void)slrng::hip_fail(e);
      return SLRNG_ENOMEM;
    }
    return e == hipSuccess ? SLRNG_OK : slrng::hip_fail(e);
  });
}

extern "C" int slrng_output_free(void *dev_ptr) {
  return slrng::guarded([&]() -> int {
    if (!dev_ptr) return SLRNG_OK;
    return slrng::spread_free(dev_ptr);
  });
}

// Host-to-device upload of small packed buffers by a kernel on the caller's
// stream.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stddef.h>

namespace slrng {
// Copies `bytes` (a multiple of 16) from `src`, the device mapping of pinned
// host memory allocated coherent (hipHostMallocCoherent, pointer from
// hipHostGetDevicePointer), to device memory `dst` (16-byte aligned), with a
// kernel on `st`.  The host writes to `src` must be complete before the call;
// `src` must stay unchanged until the kernel has run.  With `stamp` non-null
// (host-mapped memory too) the kernel writes the device clock
// (wall_clock64) there when it starts; bytes may then be 0.
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t st,
                         uint64_t *stamp = nullptr);
}  // namespace slrng

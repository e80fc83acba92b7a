// Device memory for large outputs whose physical pages are spread over HBM.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace slrng {

// Virtually contiguous device memory of at least `bytes`; from 1 GiB up its
// physical pieces are spread (plain hipMalloc below).  Thread-safe.
hipError_t spread_alloc(uint64_t bytes, void **out);
// Frees a pointer from spread_alloc after the device is idle; SLRNG_OK,
// SLRNG_EINVAL for an unknown pointer, SLRNG_EHIP for a failed HIP call.
int spread_free(void *p);

}  // namespace slrng

/*
 * Measurement aids shipped with slrng (not part of the generators' method).
 *
 * slrng_calib_write: writes `bytes` (a multiple of 16) of a constant pattern
 *   to dev_out with the same 16-byte stores as the generation kernel, in a
 *   contiguous grid-stride sweep: a write ceiling of this store path.
 * slrng_calib_copy: copies `bytes` (a multiple of 16) from dev_src to dev_dst:
 *   a kernel of known traffic (bytes read + bytes written) against which the
 *   hardware memory counters are scaled.
 * Both are asynchronous on `stream`; EINVAL for null pointers or a size that is
 * not a multiple of 16, SLRNG_EHIP if the launch fails.
 */
#ifndef SLRNG_CALIB_H
#define SLRNG_CALIB_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

int slrng_calib_write(void *dev_out, uint64_t bytes, hipStream_t stream);
int slrng_calib_copy(void *dev_dst, const void *dev_src, uint64_t bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SLRNG_CALIB_H */

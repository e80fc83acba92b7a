// Launch interface of the 32-bit generators' kernels (internal): the same
// arguments as the 64-bit launchers; states stay in 64-bit word-major
// buffers, one 32-bit word per 64-bit slot; outputs are 32-bit.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "kernels.hpp"

namespace slrng {

hipError_t launch_generate32(int variant, int kind, const GenArgs &a, bool nt, hipStream_t st);
hipError_t launch_position32(int variant, uint64_t seed, uint64_t S, const uint64_t *tab0,
                             const uint64_t *up, int levels, uint64_t *state_out, hipStream_t st);
hipError_t launch_jump32(int variant, uint64_t *state, uint64_t S, const UPoly &r, hipStream_t st);
hipError_t launch_advance_each32(int variant, uint64_t *state, uint64_t S, const uint64_t *steps,
                                 const uint64_t *tab, hipStream_t st);

}  // namespace slrng

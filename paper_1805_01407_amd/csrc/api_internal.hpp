// Internal helpers shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <new>

#include "../../include/slrng.h"
#include "f2poly.hpp"

namespace slrng {

int hip_fail(hipError_t e);  // records the HIP error, returns SLRNG_EHIP
bool valid_variant(int v);    // any generator (64- and 32-bit)
bool valid_variant64(int v);  // the 64-bit generators (batches, server)
bool is_variant32(int v);
int variant_words(int v);
int variant_engine(int v);
const Poly &jump_kind_poly(int engine, int jump_kind);
int levels_for(uint64_t S);
int get_slot_polys(int device, int engine, uint64_t C, uint64_t D, const uint64_t **out);
int get_digit_tables(int device, int engine, const uint64_t **out);
slrng_tuning tuning_for(int v, int kind);
const uint64_t *streams_state_ptr(const slrng_streams *h);
int check_batch_opts(const slrng_batch_opts &o);
void plan_slots(uint64_t S, uint64_t n, const slrng_tuning &t, uint64_t &C, uint64_t &nslots,
                uint64_t &D);

// Every C entry point runs its body through guarded(): a C++ exception
// (allocation failure, thread creation) becomes a return code instead of
// crossing the C ABI.
template <typename F>
int guarded(F &&f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    return SLRNG_ENOMEM;
  } catch (...) {
    return SLRNG_ENOMEM;
  }
}

}  // namespace slrng

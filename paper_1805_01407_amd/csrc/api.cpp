// C ABI of slrng (include/slrng.h): stream handles, jump planning and launch
// shapes.  The kernels are in kernels.hip; the polynomial arithmetic that turns
// a jump distance into a jump polynomial is in f2poly.cpp.
#include <hip/hip_runtime_api.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/slrng.h"
#include "../../include/slrng_calib.h"
#include "api_internal.hpp"
#include "engines.hpp"
#include "engines32.hpp"
#include "f2poly.hpp"
#include "kernels.hpp"
#include "kernels32.hpp"
#include "lincomp.hpp"
#include "xpow.hpp"

using namespace slrng;

// ---------------------------------------------------------------- errors

static thread_local int g_last_hip = 0;

namespace slrng {
int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return SLRNG_EHIP;
}
}  // namespace slrng

#define HIPCHK(call)                              \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(e_);    \
  } while (0)

extern "C" int slrng_version(void) { return SLRNG_ABI_VERSION; }

extern "C" const char *slrng_strerror(int err) {
  switch (err) {
    case SLRNG_OK: return "SLRNG_OK";
    case SLRNG_EINVAL: return "SLRNG_EINVAL: invalid argument";
    case SLRNG_ERANGE: return "SLRNG_ERANGE: size out of range";
    case SLRNG_ENOMEM: return "SLRNG_ENOMEM: out of memory";
    case SLRNG_EZEROSTATE: return "SLRNG_EZEROSTATE: all-zero state";
    case SLRNG_EAGAIN: return "SLRNG_EAGAIN: resource temporarily unavailable";
    case SLRNG_EHIP: return "SLRNG_EHIP: HIP call failed";
    case SLRNG_ENOTIMPL: return "SLRNG_ENOTIMPL: not implemented";
    default: return "SLRNG: unknown error";
  }
}

extern "C" int slrng_last_hip_error(void) { return g_last_hip; }

// ---------------------------------------------------------------- variants

namespace slrng {

static const int kK[kEndVariant32] = {2, 2, 2, 4, 4, 4, 8, 8, 8, 16, 16, 16, 2, 16,
                                      2, 2, 4, 4, 4};
static const int kEngine[kEndVariant32] = {0, 1, 0, 2, 2, 2, 3, 3, 3, 4, 4, 4, 0, 4,
                                           5, 5, 6, 6, 6};

bool valid_variant(int v) { return v >= 0 && v < kEndVariant32; }
bool valid_variant64(int v) { return v >= 0 && v < kNumVariants; }
bool is_variant32(int v) { return v >= kFirstVariant32 && v < kEndVariant32; }

// Kinds a generator accepts, and the index of the kind in its tuning row.
static bool valid_kind(int v, int kind) {
  return is_variant32(v) ? (kind == SLRNG_U32 || kind == SLRNG_F32)
                         : (kind == SLRNG_U64 || kind == SLRNG_F64);
}
static int kind_index(int kind) { return kind & 1; }
int variant_words(int v) { return kK[v]; }
int variant_engine(int v) { return kEngine[v]; }

// ---------------------------------------------------------------- polynomials

// x^J mod p for a jump kind (2^(n/2) or 2^(3n/4)), cached per engine.
const Poly &jump_kind_poly(int engine, int jump_kind) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, Poly> cache;
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_pair(engine, jump_kind);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const Field &f = engine_field(engine);
  Poly r;
  f.xpow2(jump_kind == SLRNG_LONG_JUMP ? 3 * f.n / 4 : f.n / 2, r);
  return cache.emplace(key, r).first->second;
}

// ---------------------------------------------------------------- device tables

// Positioning tables of one engine on one device.
struct PosTables {
  int levels = 0;
  uint64_t *tab0 = nullptr;  // word-major: word w of entry d at [w*1024 + d]
  uint64_t *up = nullptr;    // (levels-1) x 1024 x 16
};

static std::mutex g_tab_mu;
static std::map<std::pair<int, int>, PosTables> g_pos;             // (device, engine)
static std::map<std::tuple<int, int, uint64_t, uint64_t>, uint64_t *> g_slot;  // (device, engine, C, D)

int levels_for(uint64_t S) {
  int l = 1;
  uint64_t cap = kTabRadix;
  while (cap < S && l < kMaxLevels) {
    cap *= kTabRadix;
    l++;
  }
  return l;
}

// Tables x^(d 2^(e0 + 10 l)) mod p of one engine, built on the device from
// p alone (xpow.hip).
static hipError_t engine_table(const Field &f, int e0, int levels, uint64_t *out, XpowLayout lay) {
  return xpow_table_device(f.n / 64, f.p.w, e0, 10, levels, out, lay, nullptr);
}

int get_pos_tables(int device, int engine, int levels, PosTables **out) {
  std::lock_guard<std::mutex> g(g_tab_mu);
  PosTables &t = g_pos[std::make_pair(device, engine)];
  if (t.levels >= levels) {
    *out = &t;
    return SLRNG_OK;
  }
  const Field &f = engine_field(engine);
  const int W = f.n / 64;
  // level 0: jump distance J = 2^(n/2), entry d at [w 1024 + d]; level l >= 1:
  // 1024^l J = 2^(10 l + n/2), entry d at [((l-1) 1024 + d) 16 + w]
  const size_t nu = (size_t)(levels > 1 ? levels - 1 : 1) * kTabRadix * 16;
  uint64_t *d0 = nullptr, *du = nullptr;
  HIPCHK(hipMalloc(&d0, (size_t)W * kTabRadix * 8));
  hipError_t e = hipMalloc(&du, nu * 8);
  if (e == hipSuccess) e = hipMemset(du, 0, nu * 8);
  if (e == hipSuccess) e = engine_table(f, f.n / 2, 1, d0, XpowLayout{0, 1, (size_t)kTabRadix});
  if (e == hipSuccess && levels > 1)
    e = engine_table(f, f.n / 2 + 10, levels - 1, du, XpowLayout{(size_t)kTabRadix * 16, 16, 1});
  if (e != hipSuccess) {
    (void)hipFree(d0);
    if (du) (void)hipFree(du);
    return hip_fail(e);
  }
  // tables of fewer levels may still be in use by queued kernels: keep them
  t.tab0 = d0;
  t.up = du;
  t.levels = levels;
  *out = &t;
  return SLRNG_OK;
}

// Digit tables of slrng_streams_advance_each: entry d of level l is
// x^(d 2^(10 l)) mod p, word w at [(l W + w) 1024 + d] (W = n/64 words).
static std::map<std::pair<int, int>, uint64_t *> g_digit;  // (device, engine)

int get_digit_tables(int device, int engine, const uint64_t **out) {
  std::lock_guard<std::mutex> g(g_tab_mu);
  auto key = std::make_pair(device, engine);
  auto it = g_digit.find(key);
  if (it != g_digit.end()) {
    *out = it->second;
    return SLRNG_OK;
  }
  const Field &f = engine_field(engine);
  const int W = f.n / 64;
  uint64_t *dev = nullptr;
  HIPCHK(hipMalloc(&dev, (size_t)kDigitLevels * W * kTabRadix * 8));
  const hipError_t e = engine_table(f, 0, kDigitLevels, dev, XpowLayout{(size_t)W * kTabRadix, 1, (size_t)kTabRadix});
  if (e != hipSuccess) {
    (void)hipFree(dev);
    return hip_fail(e);
  }
  g_digit[key] = dev;
  *out = dev;
  return SLRNG_OK;
}

// Slot start polynomials x^(j C - delta_d) mod p with delta_d = d C / D, for
// skew class d < D and slot j < kMaxSlots (entry (d kMaxSlots + j), 16 words;
// entries with j C < delta_d are unused).
int get_slot_polys(int device, int engine, uint64_t C, uint64_t D, const uint64_t **out) {
  // the products of the digit tables' entries, on the device (taken before
  // the lock: get_digit_tables takes it too)
  const uint64_t *digits = nullptr;
  const int rc = get_digit_tables(device, engine, &digits);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(g_tab_mu);
  auto key = std::make_tuple(device, engine, C, D);
  auto it = g_slot.find(key);
  if (it != g_slot.end()) {
    *out = it->second;
    return SLRNG_OK;
  }
  const Field &f = engine_field(engine);
  const size_t words = (size_t)D * kMaxSlots * 16;
  uint64_t *dev = nullptr;
  HIPCHK(hipMalloc(&dev, words * 8));
  hipError_t e = hipMemset(dev, 0, words * 8);
  // class d: entries j = 1 .. kMaxSlots-1 at x^(j C - delta_d), delta_d < C
  for (uint64_t d = 0; d < D && e == hipSuccess; d++) {
    const uint64_t delta = d * (C / D);
    e = launch_xpow_seq(f.n / 64, f.p.w, digits, C - delta, 0, C, kMaxSlots - 1,
                        dev + ((size_t)d * kMaxSlots + 1) * 16, 16, 1, nullptr);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    (void)hipFree(dev);
    return hip_fail(e);
  }
  g_slot[key] = dev;
  *out = dev;
  return SLRNG_OK;
}

// ---------------------------------------------------------------- tuning

// Launch shapes per (variant, kind), read by every generate call and written
// by slrng_set_tuning, possibly from other threads: guarded by a mutex.
static slrng_tuning g_tune[kEndVariant32][2];
static std::once_flag g_tune_once;
static std::mutex g_tune_mu;

static void init_tuning() {
  for (int v = 0; v < kEndVariant32; v++)
    for (int k = 0; k < 2; k++)
      g_tune[v][k] = slrng_tuning{is_variant32(v) ? 64 : 32, 8192, 4, 0, 4096};
}

slrng_tuning tuning_for(int v, int kind) {
  std::call_once(g_tune_once, init_tuning);
  std::lock_guard<std::mutex> g(g_tune_mu);
  return g_tune[v][kind_index(kind)];
}

// Slot plan of a generate call: chunks of C outputs (C a multiple of D times
// the tile, so every slot boundary is tile aligned), nslots = chunks + 1 when
// the boundaries are staggered.
void plan_slots(uint64_t S, uint64_t n, const slrng_tuning &t, uint64_t &C, uint64_t &nslots,
                uint64_t &D) {
  const uint64_t waves = (S + kWave - 1) / kWave;
  uint64_t want = 1;
  if (waves < (uint64_t)t.target_waves) want = ((uint64_t)t.target_waves + waves - 1) / waves;
  if (want > (uint64_t)kMaxChunks) want = kMaxChunks;
  C = (n + want - 1) / want;
  if (C < t.min_chunk) C = t.min_chunk;
  // staggered boundaries pay only for long slots (the shift C/D spans at
  // least 8 tiles); short, latency-bound slots go without, so that their
  // length is not rounded up to a multiple of tile x D
  D = (uint64_t)t.skew;
  if (D > 1 && C < D * (uint64_t)t.tile * 8) D = 1;
  const uint64_t unit = (uint64_t)t.tile * D;
  C = (C + unit - 1) / unit * unit;
  uint64_t nchunks = (n + C - 1) / C;
  if (nchunks == 0) nchunks = 1;
  nslots = nchunks + (D > 1 ? 1 : 0);
}

}  // namespace slrng

// ---------------------------------------------------------------- handles

struct slrng_streams {
  int variant;
  int k;
  int engine;
  int device;
  uint64_t S;
  uint64_t *state[2];
  int cur;
};

extern "C" int slrng_state_words(int variant) {
  return guarded([&]() -> int {
    if (!valid_variant(variant)) return SLRNG_EINVAL;
    return variant_words(variant);
  });
}

extern "C" int slrng_charpoly(int variant, uint64_t *out, int out_words) {
  return guarded([&]() -> int {
    if (!valid_variant(variant) || !out) return SLRNG_EINVAL;
    const Field &f = engine_field(variant_engine(variant));
    if (out_words < f.n / 64 + 1) return SLRNG_EINVAL;
    for (int i = 0; i <= f.n / 64; i++) out[i] = f.p.w[i];
    return SLRNG_OK;
  });
}

extern "C" int slrng_jump_poly(int variant, const uint64_t *J, int nj, uint64_t *out,
                               int out_words) {
  return guarded([&]() -> int {
    if (!valid_variant(variant) || !out || nj < 0 || (nj > 0 && !J)) return SLRNG_EINVAL;
    const Field &f = engine_field(variant_engine(variant));
    if (out_words < f.n / 64) return SLRNG_EINVAL;
    Poly r;
    if (nj == 0) {
      r.clear();
      r.w[0] = 1;
    } else {
      f.xpow(J, nj, r);
    }
    for (int i = 0; i < f.n / 64; i++) out[i] = r.w[i];
    return SLRNG_OK;
  });
}

extern "C" int slrng_jump_poly_device(int variant, const uint64_t *dev_J, uint64_t m, uint64_t *dev_out,
                                      hipStream_t stream) {
  return guarded([&]() -> int {
    if (!valid_variant(variant)) return SLRNG_EINVAL;
    if (m == 0) return SLRNG_OK;
    if (!dev_J || !dev_out || ((uintptr_t)dev_J & 7) || ((uintptr_t)dev_out & 7)) return SLRNG_EINVAL;
    if (m > (1ull << 32)) return SLRNG_ERANGE;
    int device = 0;
    HIPCHK(hipGetDevice(&device));
    const int engine = variant_engine(variant);
    const uint64_t *tab = nullptr;
    const int rc = get_digit_tables(device, engine, &tab);
    if (rc) return rc;
    const Field &f = engine_field(engine);
    HIPCHK(launch_xpow_batch(f.n / 64, f.p.w, tab, dev_J, m, dev_out, stream));
    return SLRNG_OK;
  });
}

static int alloc_handle(int variant, uint64_t S, slrng_streams **out) {
  if (!valid_variant(variant) || !out) return SLRNG_EINVAL;
  if (S == 0 || S > (1ull << 31)) return SLRNG_ERANGE;
  slrng_streams *h = new (std::nothrow) slrng_streams();
  if (!h) return SLRNG_ENOMEM;
  h->variant = variant;
  h->k = variant_words(variant);
  h->engine = variant_engine(variant);
  h->S = S;
  h->cur = 0;
  h->state[0] = h->state[1] = nullptr;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e);
  }
  const size_t bytes = (size_t)S * h->k * 8;
  for (int b = 0; b < 2; b++) {
    e = hipMalloc(&h->state[b], bytes);
    if (e != hipSuccess) {
      if (h->state[0]) (void)hipFree(h->state[0]);
      delete h;
      return e == hipErrorOutOfMemory ? SLRNG_ENOMEM : hip_fail(e);
    }
  }
  *out = h;
  return SLRNG_OK;
}

extern "C" int slrng_streams_destroy(slrng_streams *h) {
  return guarded([&]() -> int {
    if (!h) return SLRNG_EINVAL;
    for (int b = 0; b < 2; b++)
      if (h->state[b]) (void)hipFree(h->state[b]);
    delete h;
    return SLRNG_OK;
  });
}

static int position(slrng_streams *h, uint64_t seed, hipStream_t stream) {
  // the base state must not be all zero: only a one-output fill (xoroshiro64)
  // can be, for one seed
  uint64_t any = 0;
  for (int j = 0; j < (is_variant32(h->variant) ? (h->k + 1) / 2 : h->k); j++)
    any |= splitmix64_mix(seed + (uint64_t)(j + 1) * kGoldenGamma);
  if (!any) return SLRNG_EZEROSTATE;
  PosTables *t = nullptr;
  const int levels = levels_for(h->S);
  int rc = get_pos_tables(h->device, h->engine, levels, &t);
  if (rc) return rc;
  hipError_t e =
      is_variant32(h->variant)
          ? launch_position32(h->variant, seed, h->S, t->tab0, t->up, levels, h->state[h->cur], stream)
          : launch_position(h->variant, seed, h->S, t->tab0, t->up, levels, h->state[h->cur], stream);
  return e == hipSuccess ? SLRNG_OK : hip_fail(e);
}

extern "C" int slrng_streams_create(int variant, uint64_t seed, uint64_t S, hipStream_t stream,
                                    slrng_streams **out) {
  return guarded([&]() -> int {
    if (!out) return SLRNG_EINVAL;
    *out = nullptr;
    slrng_streams *h = nullptr;
    int rc = alloc_handle(variant, S, &h);
    if (rc) return rc;
    rc = position(h, seed, stream);
    if (rc) {
      slrng_streams_destroy(h);
      return rc;
    }
    *out = h;
    return SLRNG_OK;
  });
}

extern "C" int slrng_streams_seed(slrng_streams *h, uint64_t seed, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h) return SLRNG_EINVAL;
    return position(h, seed, stream);
  });
}

// 32-bit generators: every word must fit in 32 bits.
static bool words_fit(int variant, const uint64_t *w, uint64_t S, int k) {
  if (!is_variant32(variant)) return true;
  for (uint64_t i = 0; i < S * (uint64_t)k; i++)
    if (w[i] >> 32) return false;
  return true;
}

static bool any_zero_state(const uint64_t *w, uint64_t S, int k) {
  for (uint64_t i = 0; i < S; i++) {
    uint64_t acc = 0;
    for (int j = 0; j < k; j++) acc |= w[i * k + j];
    if (!acc) return true;
  }
  return false;
}

extern "C" int slrng_set_state(slrng_streams *h, const uint64_t *host_words, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h || !host_words) return SLRNG_EINVAL;
    if (!words_fit(h->variant, host_words, h->S, h->k)) return SLRNG_EINVAL;
    if (any_zero_state(host_words, h->S, h->k)) return SLRNG_EZEROSTATE;
    std::vector<uint64_t> soa((size_t)h->S * h->k);
    for (uint64_t i = 0; i < h->S; i++)
      for (int j = 0; j < h->k; j++) soa[(size_t)j * h->S + i] = host_words[i * h->k + j];
    HIPCHK(hipMemcpyAsync(h->state[h->cur], soa.data(), soa.size() * 8, hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
    return SLRNG_OK;
  });
}

extern "C" int slrng_get_state(const slrng_streams *h, uint64_t *host_words, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h || !host_words) return SLRNG_EINVAL;
    std::vector<uint64_t> soa((size_t)h->S * h->k);
    HIPCHK(hipMemcpyAsync(soa.data(), h->state[h->cur], soa.size() * 8, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (uint64_t i = 0; i < h->S; i++)
      for (int j = 0; j < h->k; j++) host_words[i * h->k + j] = soa[(size_t)j * h->S + i];
    return SLRNG_OK;
  });
}

extern "C" int slrng_streams_create_from_states(int variant, const uint64_t *host_words, uint64_t S,
                                                hipStream_t stream, slrng_streams **out) {
  return guarded([&]() -> int {
    if (!out || !host_words) return SLRNG_EINVAL;
    *out = nullptr;
    if (valid_variant(variant) && S > 0 && S <= (1ull << 31) &&
        !words_fit(variant, host_words, S, variant_words(variant)))
      return SLRNG_EINVAL;
    if (valid_variant(variant) && S > 0 && S <= (1ull << 31) &&
        any_zero_state(host_words, S, variant_words(variant)))
      return SLRNG_EZEROSTATE;
    slrng_streams *h = nullptr;
    int rc = alloc_handle(variant, S, &h);
    if (rc) return rc;
    rc = slrng_set_state(h, host_words, stream);
    if (rc) {
      slrng_streams_destroy(h);
      return rc;
    }
    *out = h;
    return SLRNG_OK;
  });
}

extern "C" int slrng_streams_count(const slrng_streams *h, uint64_t *n) {
  return guarded([&]() -> int {
    if (!h || !n) return SLRNG_EINVAL;
    *n = h->S;
    return SLRNG_OK;
  });
}

namespace slrng {
// Current word-major state buffer of a handle (S words per state word).
const uint64_t *streams_state_ptr(const slrng_streams *h) { return h->state[h->cur]; }
}  // namespace slrng

extern "C" int slrng_streams_variant(const slrng_streams *h, int *v) {
  return guarded([&]() -> int {
    if (!h || !v) return SLRNG_EINVAL;
    *v = h->variant;
    return SLRNG_OK;
  });
}

static int apply_uniform(slrng_streams *h, const Poly &r, hipStream_t stream) {
  UPoly u;
  for (int i = 0; i < 16; i++) u.w[i] = r.w[i];
  hipError_t e = is_variant32(h->variant) ? launch_jump32(h->variant, h->state[h->cur], h->S, u, stream)
                                          : launch_jump(h->variant, h->state[h->cur], h->S, u, stream);
  return e == hipSuccess ? SLRNG_OK : hip_fail(e);
}

extern "C" int slrng_streams_jump(slrng_streams *h, int jump_kind, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h || (jump_kind != SLRNG_JUMP && jump_kind != SLRNG_LONG_JUMP)) return SLRNG_EINVAL;
    return apply_uniform(h, jump_kind_poly(h->engine, jump_kind), stream);
  });
}

extern "C" int slrng_streams_advance(slrng_streams *h, uint64_t hi, uint64_t lo, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h) return SLRNG_EINVAL;
    if (hi == 0 && lo == 0) return SLRNG_OK;
    const Field &f = engine_field(h->engine);
    uint64_t J[2] = {lo, hi};
    Poly r;
    f.xpow(J, 2, r);
    return apply_uniform(h, r, stream);
  });
}

extern "C" int slrng_streams_advance_each(slrng_streams *h, const uint64_t *dev_steps,
                                          hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h || !dev_steps || ((uintptr_t)dev_steps & 7)) return SLRNG_EINVAL;
    const uint64_t *tab = nullptr;
    int rc = get_digit_tables(h->device, h->engine, &tab);
    if (rc) return rc;
    hipError_t e =
        is_variant32(h->variant)
            ? launch_advance_each32(h->variant, h->state[h->cur], h->S, dev_steps, tab, stream)
            : launch_advance_each(h->variant, h->state[h->cur], h->S, dev_steps, tab, stream);
    return e == hipSuccess ? SLRNG_OK : hip_fail(e);
  });
}

extern "C" int slrng_linear_complexity(const slrng_streams *h, int bit, uint32_t nbits,
                                       uint32_t *dev_lc, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h || !dev_lc || ((uintptr_t)dev_lc & 3)) return SLRNG_EINVAL;
    const int wbits = is_variant32(h->variant) ? 32 : 64;
    if (bit < 0 || bit >= wbits) return SLRNG_EINVAL;
    if (nbits < 32 || nbits > kLincompMaxBits || nbits % 32) return SLRNG_EINVAL;
    hipError_t e = launch_lincomp(h->variant, h->state[h->cur], h->S, bit, nbits, dev_lc, stream);
    return e == hipSuccess ? SLRNG_OK : hip_fail(e);
  });
}

extern "C" int slrng_equidistribution_rank(int variant, int word, int dims, uint32_t *dev_rank,
                                           hipStream_t stream) {
  return guarded([&]() -> int {
    if (!valid_variant(variant) || !dev_rank || ((uintptr_t)dev_rank & 3)) return SLRNG_EINVAL;
    const int k = variant_words(variant);
    if (word < 0 || word >= k || dims < 1 || dims > k) return SLRNG_EINVAL;
    hipError_t e = launch_equidist_rank(variant, word, dims, dev_rank, stream);
    return e == hipSuccess ? SLRNG_OK : hip_fail(e);
  });
}

extern "C" int slrng_gf2_rank(const uint64_t *dev_rows, uint32_t nrows, uint32_t ncols,
                              uint32_t *dev_rank, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dev_rows || ((uintptr_t)dev_rows & 7) || !dev_rank || ((uintptr_t)dev_rank & 3))
      return SLRNG_EINVAL;
    if (nrows < 1 || nrows > 1024 || ncols < 1 || ncols > 1024) return SLRNG_EINVAL;
    hipError_t e = launch_gf2_rank(dev_rows, nrows, ncols, dev_rank, stream);
    return e == hipSuccess ? SLRNG_OK : hip_fail(e);
  });
}

constexpr uint64_t kNtMinRow = 2048;

extern "C" int slrng_generate(slrng_streams *h, int kind, uint64_t n, void *dev_out, uint64_t ld,
                              hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h || !valid_kind(h->variant, kind)) return SLRNG_EINVAL;
    if (n == 0) return SLRNG_OK;
    const uint64_t elem = is_variant32(h->variant) ? 4 : 8;
    if (!dev_out || ((uintptr_t)dev_out & (elem - 1))) return SLRNG_EINVAL;
    if (ld < n) return SLRNG_EINVAL;
    // extent (S-1) ld + n elements, in bytes, must fit in 64 bits
    const uint64_t S1 = h->S - 1;
    if (S1 && ld > (UINT64_MAX - n) / S1) return SLRNG_ERANGE;
    const uint64_t extent = S1 * ld + n;
    if (extent > UINT64_MAX / elem) return SLRNG_ERANGE;
    const slrng_tuning t = tuning_for(h->variant, kind);
    uint64_t C = 0, nslots = 1, D = 1;
    plan_slots(h->S, n, t, C, nslots, D);
    const uint64_t *sp = nullptr;
    if (nslots > 1) {
      int rc = get_slot_polys(h->device, h->engine, C, D, &sp);
      if (rc) return rc;
    }
    GenArgs a;
    a.state_in = h->state[h->cur];
    // with several slots, other waves still read the start states while the
    // last slot finishes: the final states go to the other buffer
    a.state_out = nslots > 1 ? h->state[1 - h->cur] : h->state[h->cur];
    a.S = h->S;
    a.n = n;
    a.C = C;
    a.nslots = nslots;
    a.D = D;
    a.out = dev_out;
    a.ld = ld;
    a.slot_polys = sp;
    // nontemporal stores only for rows of at least kNtMinRow outputs: with
    // rows of 1,024 outputs, plain stores measured 2-10% faster for nine of
    // ten (64-bit generator, kind) pairs on MI355X (8 GiB launches)
    const bool nt = t.store == 1 && (is_variant32(h->variant) || n >= kNtMinRow);
    GenConfig cfg{t.tile, nt};
    hipError_t e = is_variant32(h->variant)
                       ? launch_generate32(h->variant, kind_index(kind), a, cfg.nt, stream)
                       : launch_generate(h->variant, kind, a, cfg, stream);
    if (e != hipSuccess) return hip_fail(e);
    if (nslots > 1) h->cur = 1 - h->cur;
    return SLRNG_OK;
  });
}

// ---------------------------------------------------------------- tuning ABI

extern "C" int slrng_get_tuning(int variant, int kind, slrng_tuning *out) {
  return guarded([&]() -> int {
    if (!valid_variant(variant) || !valid_kind(variant, kind) || !out) return SLRNG_EINVAL;
    *out = tuning_for(variant, kind);
    return SLRNG_OK;
  });
}

extern "C" int slrng_set_tuning(int variant, int kind, const slrng_tuning *t) {
  return guarded([&]() -> int {
    if (!valid_variant(variant) || !valid_kind(variant, kind) || !t) return SLRNG_EINVAL;
    // the 32-bit kernels stage tiles of 64 outputs; the 64-bit ones 16 or 32
    const bool tile_ok = is_variant32(variant) ? t->tile == 64 : (t->tile == 16 || t->tile == 32);
    if (!tile_ok || t->target_waves < 1 || t->target_waves > (1 << 20) ||
        t->min_chunk < 1 || t->min_chunk > (1ull << 40) || (t->store != 0 && t->store != 1))
      return SLRNG_EINVAL;
    if (t->skew != 1 && t->skew != 2 && t->skew != 4 && t->skew != 8 && t->skew != 16)
      return SLRNG_EINVAL;
    std::call_once(g_tune_once, init_tuning);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[variant][kind_index(kind)] = *t;
    return SLRNG_OK;
  });
}

// ---------------------------------------------------------------- calibration

extern "C" int slrng_calib_write(void *dev_out, uint64_t bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dev_out || bytes % 16 || ((uintptr_t)dev_out & 15)) return SLRNG_EINVAL;
    hipError_t e = launch_write_ceiling(dev_out, bytes, stream);
    return e == hipSuccess ? SLRNG_OK : hip_fail(e);
  });
}

extern "C" int slrng_calib_copy(void *dst, const void *src, uint64_t bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dst || !src || bytes % 16 || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
      return SLRNG_EINVAL;
    hipError_t e = launch_copy(dst, src, bytes, stream);
    return e == hipSuccess ? SLRNG_OK : hip_fail(e);
  });
}

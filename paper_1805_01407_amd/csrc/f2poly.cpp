// Polynomial arithmetic over Z/2Z for the jump planner (see f2poly.hpp).
#include "f2poly.hpp"

#include <mutex>
#include <vector>

#include "engines.hpp"
#include "engines32.hpp"

#if defined(__x86_64__)
#include <immintrin.h>
#endif

namespace slrng {

// ---------------------------------------------------------------- carry-less multiply

static inline void clmul_portable(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi) {
  uint64_t l = 0, h = 0;
  for (int i = 0; i < 64; i++) {
    if ((b >> i) & 1) {
      l ^= a << i;
      if (i) h ^= a >> (64 - i);
    }
  }
  lo = l;
  hi = h;
}

#if defined(__x86_64__)
__attribute__((target("pclmul,sse2"))) static inline void clmul_hw(uint64_t a, uint64_t b, uint64_t &lo,
                                                                   uint64_t &hi) {
  __m128i va = _mm_set_epi64x(0, (long long)a), vb = _mm_set_epi64x(0, (long long)b);
  __m128i r = _mm_clmulepi64_si128(va, vb, 0x00);
  lo = (uint64_t)_mm_cvtsi128_si64(r);
  hi = (uint64_t)_mm_cvtsi128_si64(_mm_unpackhi_epi64(r, r));
}
#endif

static bool has_pclmul() {
#if defined(__x86_64__)
  __builtin_cpu_init();
  return __builtin_cpu_supports("pclmul");
#else
  return false;
#endif
}

static const bool g_hw = has_pclmul();

// ---------------------------------------------------------------- reduction tables

// X[i] = x^(n+i) mod p for i < n: a product of degree <= 2n-2 reduces by
// xoring X[i] for every set coefficient of x^(n+i).  R groups them by bytes.
static void build_reducer(Field &f) {
  std::vector<Poly> &X = f.X;
  X.resize(f.n);
  // x^n mod p = p - x^n
  Poly cur = f.p;
  cur.flip(f.n);
  for (int i = 0; i < f.n; i++) {
    X[i] = cur;
    // multiply by x: shift left one bit, reduce the x^n term
    uint64_t carry = 0;
    for (int j = 0; j < kPolyWords; j++) {
      uint64_t nc = cur.w[j] >> 63;
      cur.w[j] = (cur.w[j] << 1) | carry;
      carry = nc;
    }
    if (cur.bit(f.n)) {
      // x^n = p - x^n: xoring p clears the x^n coefficient
      for (int j = 0; j < kPolyWords; j++) cur.w[j] ^= f.p.w[j];
    }
  }
  const int W = f.n / 64, nb = f.n / 8;
  f.R.assign((size_t)nb * 256 * W, 0);
  for (int b = 0; b < nb; b++)
    for (int v = 1; v < 256; v++) {
      const int low = __builtin_ctz(v);
      uint64_t *dst = &f.R[((size_t)b * 256 + v) * W];
      const uint64_t *prev = &f.R[((size_t)b * 256 + (v & (v - 1))) * W];
      const Poly &x = X[8 * b + low];
      for (int w = 0; w < W; w++) dst[w] = prev[w] ^ x.w[w];
    }
}

// prod: 2W words, coefficients of degree < 2n; result: W words (degree < n)
static inline void reduce(const Field &f, const uint64_t *prod, Poly &r) {
  const int W = f.n / 64, nb = f.n / 8;
  uint64_t acc[kPolyWords] = {0};
  for (int w = 0; w < W; w++) acc[w] = prod[w];
  const uint8_t *hb = reinterpret_cast<const uint8_t *>(prod + W);  // little endian
  for (int b = 0; b < nb; b++) {
    const unsigned v = hb[b];
    if (!v) continue;
    const uint64_t *t = &f.R[((size_t)b * 256 + v) * W];
    for (int w = 0; w < W; w++) acc[w] ^= t[w];
  }
  r.clear();
  for (int w = 0; w < W; w++) r.w[w] = acc[w];
}

#if defined(__x86_64__)
__attribute__((target("pclmul,sse2"))) static void mul_words_hw(const uint64_t *a, const uint64_t *b, int W,
                                                                uint64_t *prod) {
  for (int i = 0; i < 2 * W; i++) prod[i] = 0;
  for (int i = 0; i < W; i++) {
    if (!a[i]) continue;
    for (int j = 0; j < W; j++) {
      uint64_t lo, hi;
      clmul_hw(a[i], b[j], lo, hi);
      prod[i + j] ^= lo;
      prod[i + j + 1] ^= hi;
    }
  }
}

__attribute__((target("pclmul,sse2"))) static void sqr_words_hw(const uint64_t *a, int W, uint64_t *prod) {
  // over Z/2Z the cross terms of a square cancel: (sum a_i X^i)^2 = sum a_i^2 X^2i
  for (int i = 0; i < W; i++) clmul_hw(a[i], a[i], prod[2 * i], prod[2 * i + 1]);
}
#endif

static void mul_words_sw(const uint64_t *a, const uint64_t *b, int W, uint64_t *prod) {
  for (int i = 0; i < 2 * W; i++) prod[i] = 0;
  for (int i = 0; i < W; i++) {
    if (!a[i]) continue;
    for (int j = 0; j < W; j++) {
      uint64_t lo, hi;
      clmul_portable(a[i], b[j], lo, hi);
      prod[i + j] ^= lo;
      prod[i + j + 1] ^= hi;
    }
  }
}

void Field::mulmod(const Poly &a, const Poly &b, Poly &r) const {
  const int W = n / 64;
  uint64_t prod[2 * kPolyWords];
#if defined(__x86_64__)
  if (g_hw) mul_words_hw(a.w, b.w, W, prod);
  else mul_words_sw(a.w, b.w, W, prod);
#else
  mul_words_sw(a.w, b.w, W, prod);
#endif
  reduce(*this, prod, r);
}

void Field::sqrmod(const Poly &a, Poly &r) const {
  const int W = n / 64;
  uint64_t prod[2 * kPolyWords];
#if defined(__x86_64__)
  if (g_hw) sqr_words_hw(a.w, W, prod);
  else mul_words_sw(a.w, a.w, W, prod);
#else
  mul_words_sw(a.w, a.w, W, prod);
#endif
  reduce(*this, prod, r);
}

void Field::xpow(const uint64_t *J, int nwords, Poly &r) const {
  int top = nwords * 64 - 1;
  while (top >= 0 && !((J[top >> 6] >> (top & 63)) & 1)) top--;
  Poly acc;
  acc.clear();
  acc.w[0] = 1;
  // left to right: square, then multiply by x (a shift) for a set bit
  for (int i = top; i >= 0; i--) {
    Poly t;
    sqrmod(acc, t);
    acc = t;
    if ((J[i >> 6] >> (i & 63)) & 1) {
      uint64_t carry = 0;
      for (int j = 0; j < kPolyWords; j++) {
        uint64_t nc = acc.w[j] >> 63;
        acc.w[j] = (acc.w[j] << 1) | carry;
        carry = nc;
      }
      if (acc.bit(n)) {
        for (int j = 0; j < kPolyWords; j++) acc.w[j] ^= p.w[j];
      }
    }
  }
  r = acc;
}

void Field::xpow2(int e, Poly &r) const {
  // x^(2^e): the exponent has a single bit
  std::vector<uint64_t> J((size_t)e / 64 + 1, 0);
  J[(size_t)e / 64] = 1ull << (e & 63);
  xpow(J.data(), (int)J.size(), r);
}

// ---------------------------------------------------------------- Berlekamp-Massey

int berlekamp_massey(const uint8_t *s, int N, Poly &out) {
  // connection polynomials C (current) and B (before the last length change),
  // one byte per coefficient
  std::vector<uint8_t> C((size_t)N + 1, 0), B((size_t)N + 1, 0), T;
  C[0] = B[0] = 1;
  int L = 0, m = 1;
  for (int i = 0; i < N; i++) {
    int d = s[i];
    for (int j = 1; j <= L; j++) d ^= C[j] & s[i - j];
    if (!d) {
      m++;
      continue;
    }
    if (2 * L <= i) {
      T = C;
      for (int j = 0; j + m <= N; j++) C[j + m] ^= B[j];
      L = i + 1 - L;
      B = T;
      m = 1;
    } else {
      for (int j = 0; j + m <= N; j++) C[j + m] ^= B[j];
      m++;
    }
  }
  out.clear();
  if (L > kMaxN) return -1;
  // characteristic polynomial x^L C(1/x): coefficient of x^(L-j) is c_j
  for (int j = 0; j <= L; j++)
    if (C[j]) out.flip(L - j);
  return L;
}

// ---------------------------------------------------------------- per-engine fields

template <int V>
static Field derive_field() {
  constexpr int K = Params<V>::k;
  constexpr int n = 64 * K;
  u64 x[K];
  u64 seed_state[K];
  splitmix64_fill<K>(0x5eedull, seed_state);
  for (int j = 0; j < K; j++) x[j] = seed_state[j];
  std::vector<uint8_t> bits(2 * n);
  for (int t = 0; t < 2 * n; t++) {
    bits[t] = (uint8_t)(x[0] & 1);
    host_step_logical<V>(x);
  }
  Field f;
  f.n = berlekamp_massey(bits.data(), 2 * n, f.p);
  return f;
}

// The same for a 32-bit engine (states of 32-bit words held in u64).
template <int V>
static Field derive_field32() {
  constexpr int K = Params32<V>::k;
  constexpr int n = 32 * K;
  u32 s[K];
  splitmix64_fill32<K>(0x5eedull, s);
  u64 x[K];
  for (int j = 0; j < K; j++) x[j] = s[j];
  std::vector<uint8_t> bits(2 * n);
  for (int t = 0; t < 2 * n; t++) {
    bits[t] = (uint8_t)(x[0] & 1);
    host_step32<V>(x);
  }
  Field f;
  f.n = berlekamp_massey(bits.data(), 2 * n, f.p);
  return f;
}

constexpr int kNumEnginesAll = kNumEngines + kNumEngines32;
static std::once_flag g_once[kNumEnginesAll];
static Field g_fields[kNumEnginesAll];

static void init_engine(int e) {
  switch (e) {
    case 0: g_fields[0] = derive_field<0>(); break;
    case 1: g_fields[1] = derive_field<1>(); break;
    case 2: g_fields[2] = derive_field<3>(); break;
    case 3: g_fields[3] = derive_field<6>(); break;
    case 4: g_fields[4] = derive_field<9>(); break;
    case 5: g_fields[5] = derive_field32<14>(); break;
    default: g_fields[6] = derive_field32<16>(); break;
  }
  build_reducer(g_fields[e]);
}

const Field &engine_field(int e) {
  std::call_once(g_once[e], init_engine, e);
  return g_fields[e];
}

}  // namespace slrng

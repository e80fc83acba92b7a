// Host-side polynomial arithmetic over Z/2Z for the jump functions.
//
// Every generator of the paper is linear, so it has jump functions (Section
// "Combining linear engines and scramblers").  The planner derives them from
// the engine's characteristic polynomial p(x) (Section "Polynomials and full
// period"): by Cayley-Hamilton, s * M^J = sum_i r_i (s * M^i) where
// r(x) = x^J mod p(x).  p(x) is obtained with Berlekamp-Massey on 2n values
// of one state bit, which is valid because p is irreducible for every engine
// used here.
#pragma once
#include <stdint.h>
#include <string.h>

#include <vector>

namespace slrng {

constexpr int kMaxN = 1024;                 // largest state (xoroshiro1024); n is a multiple of 64
constexpr int kPolyWords = kMaxN / 64 + 1;  // degree n needs n+1 bits

// Polynomial of degree <= kMaxN; bit i of w[i/64] is the coefficient of x^i.
struct Poly {
  uint64_t w[kPolyWords];
  void clear() { memset(w, 0, sizeof(w)); }
  bool bit(int i) const { return (w[i >> 6] >> (i & 63)) & 1; }
  void flip(int i) { w[i >> 6] ^= 1ull << (i & 63); }
};

// Characteristic polynomial of one engine, with helpers bound to its degree.
struct Field {
  int n = 0;  // degree of p
  Poly p;     // monic, degree n
  std::vector<Poly> X;  // X[i] = x^(n+i) mod p, i < n
  // byte-window reduction: R[(b*256 + v)*W .. +W) = sum of X[8b+i] over the set
  // bits i of v, W = n/64 words
  std::vector<uint64_t> R;
  // r = a * b mod p (a, b of degree < n)
  void mulmod(const Poly &a, const Poly &b, Poly &r) const;
  void sqrmod(const Poly &a, Poly &r) const;
  // r = x^J mod p for J given as little-endian 64-bit words
  void xpow(const uint64_t *J, int nwords, Poly &r) const;
  // r = x^(2^e) mod p
  void xpow2(int e, Poly &r) const;
};

// Berlekamp-Massey over Z/2Z on bits[0..N): returns the linear complexity L
// and the characteristic polynomial x^L C(1/x) in `out`.
int berlekamp_massey(const uint8_t *bits, int N, Poly &out);

// The engine's field, derived once per engine (thread-safe, cached).
const Field &engine_field(int engine);

}  // namespace slrng

"""Pins of the oracle's F2 tools: Berlekamp-Massey, characteristic polynomials,
full period, and the linear complexity of the weak scramblers' low bits."""
import itertools
import math
import random

import numpy as np
import pytest

import oracle as O
from conftest import read_golden


# ---------------------------------------------------------------- helpers

def series_bits(num, den, N):
    """Power-series coefficients of num(z)/den(z) over Z/2Z (den(0) = 1)."""
    assert den & 1
    out = []
    rem = num
    for t in range(N):
        b = rem & 1
        out.append(b)
        if b:
            rem ^= den
        rem >>= 1
    return out


def poly_from_exps(exps):
    v = 0
    for e in exps:
        v |= 1 << e
    return v


def pgcd(a, b):
    while b:
        while a and a.bit_length() >= b.bit_length():
            a ^= b << (a.bit_length() - b.bit_length())
        a, b = b, a
    return a


def is_probable_prime(n):
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def pollard_rho(n):
    if n % 2 == 0:
        return 2
    rnd = random.Random(n)
    while True:
        c = rnd.randrange(1, n)
        x = y = rnd.randrange(2, n)
        d = 1
        while d == 1:
            x = (x * x + c) % n
            y = (y * y + c) % n
            y = (y * y + c) % n
            d = math.gcd(abs(x - y), n)
        if d != n:
            return d


def prime_factors(n):
    out = set()
    stack = [n]
    while stack:
        m = stack.pop()
        if m == 1:
            continue
        for p in (2, 3, 5, 7, 11, 13):
            while m % p == 0:
                out.add(p)
                m //= p
        if m == 1:
            continue
        if is_probable_prime(m):
            out.add(m)
            continue
        d = pollard_rho(m)
        stack += [d, m // d]
    return sorted(out)


def is_primitive(p):
    """x has order 2^n - 1 modulo p (p of degree n, irreducibility implied)."""
    n = p.bit_length() - 1
    order = (1 << n) - 1
    if O.xpow_mod(order, p) != 1:
        return False
    return all(O.xpow_mod(order // q, p) != 1 for q in prime_factors(order))


def rabin_irreducible_pow2(p):
    """Rabin's test for degree n a power of two: x^(2^n) = x mod p and
    gcd(x^(2^(n/2)) - x, p) = 1."""
    n = p.bit_length() - 1
    assert n & (n - 1) == 0
    if O.xpow_mod(1 << n, p) != 0b10:
        return False
    h = O.xpow_mod(1 << (n // 2), p) ^ 0b10
    return pgcd(p, h) == 1


# ---------------------------------------------------------------- BM

def brute_lc(bits):
    """Smallest L for which some connection polynomial of degree <= L
    generates the sequence (exhaustive search)."""
    N = len(bits)
    for L in range(0, N + 1):
        for coeffs in itertools.product((0, 1), repeat=L):
            if all(bits[t] == (sum(coeffs[i] * bits[t - 1 - i] for i in range(L)) & 1)
                   for t in range(L, N)):
                return L
    return N


def test_bm_matches_exhaustive_search_on_short_sequences():
    rng = random.Random(5)
    for _ in range(300):
        N = rng.randint(1, 11)
        bits = [rng.randint(0, 1) for _ in range(N)]
        L, conn = O.berlekamp_massey(bits)
        assert L == brute_lc(bits), bits
        assert conn[0] == 1
        for t in range(L, N):
            assert (sum(conn[i] * bits[t - i] for i in range(L + 1)) & 1) == 0


def test_bm_on_the_papers_generating_functions():
    rows = read_golden("fig_sumgf.txt")
    num, den, expect = {}, {}, {}
    for r in rows:
        if r[0] == "expected_lc":
            expect[int(r[1])] = int(r[2])
        elif r[1] == "num":
            num[int(r[0])] = poly_from_exps(int(e) for e in r[2:])
        else:
            den[int(r[0])] = poly_from_exps(int(e) for e in r[2:])
    for b in (0, 1, 2):
        bits = series_bits(num[b], den[b], 400)
        L, _ = O.berlekamp_massey(bits)
        assert L == expect[b]
    # the text's bounds: C(6,1) = 6 and C(6,1)+C(6,2)+C(6,3) = 41 are attained
    assert expect[0] == math.comb(6, 1)
    assert expect[2] == sum(math.comb(6, i) for i in (1, 2, 3))


# ---------------------------------------------------------------- p(x)

def test_charpoly_weights_match_table():
    rows = read_golden("tab_par64.txt")
    probe = {"xoroshiro128": "xoroshiro128+", "xoroshiro128++": "xoroshiro128++",
             "xoshiro256": "xoshiro256+", "xoshiro512": "xoshiro512+",
             "xoroshiro1024": "xoroshiro1024+"}
    for eng, _a, _b, _c, wt in rows:
        g = O.GEN64[probe[eng]]
        p = O.charpoly(g)
        assert p.bit_length() - 1 == g.n
        assert bin(p).count("1") == int(wt), eng


@pytest.mark.parametrize("engine,old,new", [
    ("xoshiro256+", '{"I", "I", "Sa", "Rb"},', '{"I", "I", "I", "Rb"},'),
    ("xoshiro256+", '{"I", "0", "0",  "Rb"},', '{"0", "I", "0",  "Rb"},'),
    ("xoshiro512+", '{"0", "0", "0", "I", "0", "0", "I",  "Rb"},',
     '{"0", "0", "0", "I", "0", "0", "0",  "Rb"},'),
    ("xoroshiro128+", 'return "Sb+I";', 'return "Sb";'),
    ("xoroshiro1024+", 'return "Ra+Sb+I";', 'return "Ra+I";'),
    ("xoroshiro1024+", "j == i - 1) return", "j == i) return")])
def test_planted_block_mistakes_fail_the_table_pins(tmp_path, engine, old, new):
    # a block of the transition matrix mistyped in a copy of the oracle must
    # fail the pins of Table tab:par64: degree n, the printed weight of p(x),
    # irreducibility (a full-period engine)
    import ctypes
    import subprocess
    src = open(O._SRC).read()
    assert src.count(old) == 1
    path = tmp_path / "orc_planted.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "liborc_planted.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", str(lib), str(path),
                           "-lpthread"])
    L = ctypes.CDLL(str(lib))
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.orc_charpoly.argtypes = [ctypes.POINTER(O._Gen), u64p, u64p]
    L.orc_charpoly.restype = ctypes.c_long
    g = O.GEN64[engine]
    x0 = O.splitmix_fill(1, g.k)
    out = np.zeros(g.n // 64 + 1, dtype=np.uint64)
    cs = g.c_struct()
    deg = L.orc_charpoly(ctypes.byref(cs), x0.ctypes.data_as(u64p), out.ctypes.data_as(u64p))
    p = sum(int(w) << (64 * i) for i, w in enumerate(out.tolist()))
    weights = {r[0]: int(r[4]) for r in read_golden("tab_par64.txt")}
    row = {"xoshiro256+": "xoshiro256", "xoshiro512+": "xoshiro512", "xoroshiro128+": "xoroshiro128",
           "xoroshiro1024+": "xoroshiro1024"}[engine]
    passes = deg == g.n and bin(p).count("1") == weights[row] and rabin_irreducible_pow2(p)
    assert not passes


def test_charpoly_annihilates_the_matrix_sequence():
    # p(M) = 0: sum_i p_i (x M^i) = 0 for any x, on the state as a whole
    # (not only on the bit BM was run on)
    for name in ["xoroshiro128+", "xoshiro256+", "xoshiro512+", "xoroshiro1024+"]:
        g = O.GEN64[name]
        p = O.charpoly(g)
        x = O.splitmix_fill(77, g.k)
        acc = np.zeros(g.k, dtype=np.uint64)
        cur = x.copy()
        for i in range(g.n + 1):
            if (p >> i) & 1:
                acc ^= cur
            cur = O.advance(g, cur, 1)
        assert not acc.any(), name


def test_charpoly_independent_of_start_bit():
    g = O.GEN64["xoshiro256**"]
    p1 = O.charpoly(g)
    p2 = O.charpoly(g, O.splitmix_fill(999, 4))
    assert p1 == p2


@pytest.mark.parametrize("name", ["xoroshiro128+", "xoroshiro128++", "xoshiro256+", "xoshiro512+",
                                  "xoroshiro1024+"])
def test_charpoly_irreducible(name):
    assert rabin_irreducible_pow2(O.charpoly(O.GEN64[name]))


@pytest.mark.parametrize("name", ["xoroshiro128+", "xoroshiro128++"])
def test_charpoly_primitive_n128(name):
    assert is_primitive(O.charpoly(O.GEN64[name]))


def test_small_generators_full_period_by_brute_force():
    # Section "Equidistribution": the 5-bit xoroshiro with 10 bits of state and
    # a=1, b=3, c=1 has full period; so has the 4-bit one with 16 bits of
    # state and a=3, b=1, c=2.
    g = O.Gen(O.XOROSHIRO, 5, 2, 1, 3, 1)
    assert O.period(g, [1, 0], 1 << 11) == (1 << 10) - 1
    g = O.Gen(O.XOROSHIRO, 4, 4, 3, 1, 2)
    assert O.period(g, [1, 0, 0, 0], 1 << 17) == (1 << 16) - 1
    # and primitivity of their BM polynomials agrees with the brute force
    assert is_primitive(O.charpoly(O.Gen(O.XOROSHIRO, 5, 2, 1, 3, 1), [1, 0]))


def test_full_period_parameter_counts_w16_k4():
    rows = read_golden("full_period_counts.txt")
    expect = {r[0]: int(r[3]) for r in rows}
    w, k = 16, 4
    cnt_xor = 0
    for a in range(1, w):
        for b in range(1, w):
            for c in range(1, w):
                p = O.charpoly(O.Gen(O.XOROSHIRO, w, k, a, b, c), [1, 0, 0, 0])
                if p.bit_length() - 1 == 64 and is_primitive(p):
                    cnt_xor += 1
    assert cnt_xor == expect["xoroshiro"]
    cnt_xos = 0
    for a in range(1, w):
        for b in range(1, w):
            p = O.charpoly(O.Gen(O.XOSHIRO, w, k, a, b), [1, 0, 0, 0])
            if p.bit_length() - 1 == 64 and is_primitive(p):
                cnt_xos += 1
    assert cnt_xos == expect["xoshiro"]


# ---------------------------------------------------------------- LC of scrambled bits

def U(n, d):
    """Upper bound sum_{i=1..d} C(n, i) of Section "Filtered LFSRs"."""
    return sum(math.comb(n, i) for i in range(1, d + 1))


def output_bit_lc(g, bit, N, seed=3):
    x = O.splitmix_fill(seed, g.k)
    out, _ = O.generate(g, x, N)
    bits = ((out >> np.uint64(bit)) & np.uint64(1)).astype(np.uint8)
    return O.berlekamp_massey(bits)[0]


def test_plus_low_bits_linear_complexity_table():
    rows = read_golden("tab_plusdeg.txt")
    names = ["xoroshiro128+", "xoshiro256+", "xoshiro512+", "xoroshiro1024+"]
    for col, name in enumerate(names):
        g = O.GEN64[name]
        # bit 0 has the engine's linear complexity n
        assert output_bit_lc(g, 0, 2 * g.n + 64) == int(rows[0][col]) == g.n
    for col, name in enumerate(names[:3]):
        g = O.GEN64[name]
        expect = int(rows[1][col])
        assert expect == U(g.n, 2)
        assert output_bit_lc(g, 1, 2 * expect + 64) == expect


@pytest.mark.slow
def test_plus_bit1_xoroshiro1024_and_bit2_xoroshiro128():
    rows = read_golden("tab_plusdeg.txt")
    g = O.GEN64["xoroshiro1024+"]
    assert output_bit_lc(g, 1, 2 * int(rows[1][3]) + 64) == int(rows[1][3])
    g = O.GEN64["xoroshiro128+"]
    assert output_bit_lc(g, 2, 2 * int(rows[2][0]) + 64) == int(rows[2][0])


def test_star_low_bits_linear_complexity():
    # Section "Multiplication": with bit 1 of the multiplier set the lowest
    # bit is unmodified and the next is a xor of bits 0 and 1, so both have the
    # engine's linear complexity; bit 2 reaches U(n, 2) (Section on the *
    # scrambler's theory).
    g = O.GEN64["xoroshiro128*"]
    assert output_bit_lc(g, 0, 400) == 128
    assert output_bit_lc(g, 1, 400) == 128
    assert output_bit_lc(g, 2, 2 * U(128, 2) + 64) == U(128, 2)


def test_star_multiplier_is_golden_ratio_with_bit_one_set():
    # Section "Multiplication": a multiplier close to phi * 2^w, lower bits
    # adjusted so that bit 1 is set.  floor(2^64/phi) ends in ...c15 (binary
    # ...0101); setting bit 1 and clearing bit 2 gives ...c13, the value of
    # tab:scr64 (nearest such value with bit 1 set).
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    phi = (1 + Decimal(5).sqrt()) / 2
    f = int(Decimal(2 ** 64) / phi)
    S = O.STAR_S
    assert S & 1 and (S >> 1) & 1
    assert abs(S - f) < 4
    assert f >> 8 == S >> 8

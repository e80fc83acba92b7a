"""Pins of the oracle's 32-bit generators (Section "The 32-bit case"):
engine transcription against the block matrices, the parameters of
tab:par32 and tab:scr32 through the weights and primitivity of the
characteristic polynomials, the full-period counts of tab:xorpol/tab:xospol
and maximum weights of tab:xordeg/tab:xosdeg for w = 32, the linear
complexity of the low bits of the weak scramblers, jumps and floats."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import matrices as Mx
from conftest import read_golden
from test_oracle_poly import is_primitive, prime_factors, rabin_irreducible_pow2

ENGINES_32 = ["xoroshiro64*", "xoshiro128+"]


def U(n, d):
    return sum(math.comb(n, i) for i in range(1, d + 1))


def output_bit_lc(g, bit, N, seed=3):
    x = O.seed_state(g, seed)
    out, _ = O.generate(g, x, N)
    bits = ((out >> np.uint64(bit)) & np.uint64(1)).astype(np.uint8)
    return O.berlekamp_massey(bits)[0]


@pytest.mark.parametrize("name", ENGINES_32)
def test_step32_equals_block_matrix(name):
    g = O.GEN32[name]
    M = Mx.matrix_for(g)
    rng = np.random.default_rng(321)
    for _ in range(8):
        x = rng.integers(0, 2**32, size=g.k, dtype=np.uint64)
        assert O.advance(g, x, 1).tolist() == Mx.apply(M, x.tolist(), 32)
        assert O.advance(g, x, 5).tolist() == Mx.apply(Mx.mpow(M, 5), x.tolist(), 32)


def test_par32_parameters_and_weights():
    rows = {r[0]: r[1:] for r in read_golden("tab_par32.txt")}
    for eng, name in (("xoroshiro64", "xoroshiro64**"), ("xoshiro128", "xoshiro128**")):
        A, B, C, wt = rows[eng]
        g = O.GEN32[name]
        assert (g.a, g.b) == (int(A), int(B))
        if C != "-":
            assert g.c == int(C)
        p = O.charpoly(g)
        assert p.bit_length() - 1 == g.n == 32 * g.k
        assert bin(p).count("1") == int(wt)


def test_scr32_constants():
    rows = {r[0]: r[1:] for r in read_golden("tab_scr32.txt")}
    for name, (S, R, T) in rows.items():
        g = O.GEN32[name]
        if S != "-":
            assert g.ms == int(S, 16 if S.startswith("0x") else 10)
        if R != "-":
            assert g.r == int(R)
        if T != "-":
            assert g.mt == int(T)
    # the multiplier is the 32-bit analogue of the 64-bit one: close to
    # 2^32/phi, odd, with bit 1 set
    phi = (1 + 5 ** 0.5) / 2
    f = int(2**32 / phi)
    assert O.STAR32_S & 1 and (O.STAR32_S >> 1) & 1 and abs(O.STAR32_S - f) < 4


@pytest.mark.parametrize("name", ENGINES_32)
def test_32bit_engines_have_full_period(name):
    p = O.charpoly(O.GEN32[name])
    assert rabin_irreducible_pow2(p)
    assert is_primitive(p)


def _count_full_period(fam, w, k, fac):
    n = w * k
    order = (1 << n) - 1
    cnt, maxw = 0, 0
    x0 = [1] + [0] * (k - 1)
    rng = range(1, w)
    params = ([(a, b, c) for a in rng for b in rng for c in rng] if fam == O.XOROSHIRO
              else [(a, b, 0) for a in rng for b in rng])
    for a, b, c in params:
        p = O.charpoly(O.Gen(fam, w, k, a, b, c), x0)
        if p.bit_length() - 1 != n or O.xpow_mod(order, p) != 1:
            continue
        if all(O.xpow_mod(order // q, p) != 1 for q in fac):
            cnt += 1
            maxw = max(maxw, bin(p).count("1"))
    return cnt, maxw


def test_full_period_counts_w32():
    rows = {r[0]: r[1:] for r in read_golden("full_period_w32.txt")}
    w, k, cnt, mw = rows["xoshiro"]
    assert _count_full_period(O.XOSHIRO, 32, 4, prime_factors((1 << 128) - 1)) == (int(cnt), int(mw))
    w, k, cnt, mw = rows["xoroshiro"]
    assert _count_full_period(O.XOROSHIRO, 32, 2, prime_factors((1 << 64) - 1)) == (int(cnt), int(mw))


def test_weak_scramblers_low_bits_linear_complexity():
    # + on xoshiro128: bit 0 has the engine's complexity n = 128, bit 1 reaches
    # U(128, 2) = 8256 (the n = 128 column of tab:plusdeg)
    g = O.GEN32["xoshiro128+"]
    assert output_bit_lc(g, 0, 2 * 128 + 64) == 128
    assert output_bit_lc(g, 1, 2 * U(128, 2) + 64) == U(128, 2) == 8256
    # * on xoroshiro64 (multiplier with bit 1 set): bits 0 and 1 have
    # complexity n = 64, bit 2 reaches U(64, 2)
    g = O.GEN32["xoroshiro64*"]
    assert output_bit_lc(g, 0, 200) == 64
    assert output_bit_lc(g, 1, 200) == 64
    assert output_bit_lc(g, 2, 2 * U(64, 2) + 64) == U(64, 2)


def test_planted_wrong_parameters_fail_the_pins():
    # transposing the xoshiro128 shift and rotation gives an engine without
    # full period (tab:xospol: (9, 11) is the only one), and dropping the
    # scrambler's carry (xor instead of +) leaves bit 1 at complexity n
    bad = O.Gen(O.XOSHIRO, 32, 4, 11, 9, 0, O.PLUS)
    assert not is_primitive(O.charpoly(bad))
    g = O.GEN32["xoshiro128+"]
    x = O.seed_state(g, 3)
    eng = O.Gen(O.XOSHIRO, 32, 4, 9, 11, 0)
    st = O.advance(eng, x, 0)
    bits = []
    for _ in range(600):
        bits.append(((int(st[0]) ^ int(st[3])) >> 1) & 1)
        st = O.advance(eng, st, 1)
    assert O.berlekamp_massey(bits)[0] == 128 != U(128, 2)


@pytest.mark.parametrize("name", list(O.GEN32))
def test_jumps_32(name):
    g = O.GEN32[name]
    x = O.seed_state(g, 17)
    for J in (0, 1, 2, 63, 64, 1000):
        assert O.jump(g, x, J).tolist() == O.advance(g, x, J).tolist()
    a, b = 3 << 40, (1 << g.n // 2) + 12345
    assert O.jump(g, O.jump(g, x, a), b).tolist() == O.jump(g, x, a + b).tolist()
    assert O.jump(g, x, (1 << g.n) - 1).tolist() == x.tolist()


def test_seed_state_reading_and_floats():
    # the SplitMix64 output stream cut into 32-bit words, low half first
    for seed in (0, 1, 42, 2**64 - 1):
        o = O.splitmix_fill(seed, 2)
        x = O.seed_state(O.GEN32["xoshiro128**"], seed)
        assert x.tolist() == [int(o[0]) & 0xFFFFFFFF, int(o[0]) >> 32,
                              int(o[1]) & 0xFFFFFFFF, int(o[1]) >> 32]
        assert O.seed_state(O.GEN32["xoroshiro64*"], seed).tolist() == x.tolist()[:2]
    # floats: the upper 24 bits, exactly, in [0, 1)
    v = np.array([0, 1, 255, 256, 2**31, 2**32 - 1, 0x12345678], dtype=np.uint64)
    f = O.to_float32(v)
    assert f.dtype == np.float32
    assert ((f.astype(np.float64) * 2**24).astype(np.uint64) == (v >> np.uint64(8))).all()
    assert (f >= 0).all() and (f < 1).all()

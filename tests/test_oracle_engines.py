"""Pins of the oracle's linear engines against the block matrices of Section
"Linear engines" (X_2w, X_kw of equation eq:M, S_4w, S_8w), which are built
independently of the code figures the oracle transcribes."""
import numpy as np
import pytest

import oracle as O
from oracle import matrices as Mx
from conftest import read_golden

ENGINES_64 = ["xoroshiro128+", "xoroshiro128++", "xoshiro256+", "xoshiro512+", "xoroshiro1024+"]


@pytest.mark.parametrize("name", ENGINES_64)
def test_step_equals_block_matrix(name):
    g = O.GEN64[name]
    M = Mx.matrix_for(g)
    rng = np.random.default_rng(1234)
    for _ in range(8):
        x = rng.integers(0, 2**64, size=g.k, dtype=np.uint64)
        assert O.advance(g, x, 1).tolist() == Mx.apply(M, x.tolist(), 64)


@pytest.mark.parametrize("name", ENGINES_64)
def test_several_steps_equal_matrix_power(name):
    # exercises the cyclic index of xoroshiro1024 through more than one wrap
    g = O.GEN64[name]
    M = Mx.matrix_for(g)
    rng = np.random.default_rng(99)
    x = rng.integers(0, 2**64, size=g.k, dtype=np.uint64)
    for steps in (2, 15, 16, 17, 37):
        assert O.advance(g, x, steps).tolist() == Mx.apply(Mx.mpow(M, steps), x.tolist(), 64)


@pytest.mark.parametrize("fam,w,k,a,b,c", [
    (O.XOROSHIRO, 5, 2, 1, 3, 1),
    (O.XOROSHIRO, 4, 4, 3, 1, 2),
    (O.XOROSHIRO, 7, 16, 2, 3, 5),
    (O.XOSHIRO, 5, 4, 1, 3, 0),
    (O.XOSHIRO, 6, 8, 2, 3, 0),
])
def test_small_word_engines_match_matrix(fam, w, k, a, b, c):
    g = O.Gen(fam, w, k, a, b, c)
    M = Mx.matrix_for(g)
    rng = np.random.default_rng(7)
    for _ in range(10):
        x = rng.integers(0, 1 << w, size=k, dtype=np.uint64)
        assert O.advance(g, x, 1).tolist() == Mx.apply(M, x.tolist(), w)


def test_engine_parameters_match_table():
    # the oracle's parameter table against the fixture typed from tab:par64
    rows = {r[0]: r[1:] for r in read_golden("tab_par64.txt")}
    probe = {"xoroshiro128": "xoroshiro128+", "xoroshiro128++": "xoroshiro128++",
             "xoshiro256": "xoshiro256**", "xoshiro512": "xoshiro512**",
             "xoroshiro1024": "xoroshiro1024**"}
    for eng, name in probe.items():
        A, B, C, _wt = rows[eng]
        g = O.GEN64[name]
        assert (g.a, g.b) == (int(A), int(B))
        if C != "-":
            assert g.c == int(C)


def test_scrambler_constants_match_table():
    rows = {r[0]: r[1:] for r in read_golden("tab_scr64.txt")}
    assert O.GEN64["xoroshiro128*"].ms == int(rows["*"][0], 16)
    for name, g in O.GEN64.items():
        if g.scr == O.STARSTAR:
            assert (g.ms, g.r, g.mt) == tuple(int(v) for v in rows["**"])
        if g.scr == O.PLUSPLUS:
            assert g.r == int(rows[name][1])


def test_zero_state_is_fixed_and_nonzero_stays_nonzero():
    # M is invertible (det = 1, Section "Linear engines"), so the zero state
    # is a fixed point and no nonzero state ever reaches it.
    for name in ENGINES_64:
        g = O.GEN64[name]
        z = np.zeros(g.k, dtype=np.uint64)
        assert O.advance(g, z, 5).tolist() == [0] * g.k
        M = Mx.matrix_for(g)
        assert Mx.rank(M) == g.n
        x = np.zeros(g.k, dtype=np.uint64)
        x[g.k - 1] = 1
        for _ in range(50):
            x = O.advance(g, x, 1)
            assert any(int(v) for v in x)


def test_max_dimension_equidistribution_of_words():
    # Section "Equidistribution": juxtaposing the j-th block columns of
    # M^0..M^(k-1) gives an invertible matrix for every xoroshiro word and
    # every xoshiro512 word; for xoshiro256 the words other than the third.
    for name in ["xoroshiro128+", "xoroshiro128++", "xoshiro256+", "xoshiro512+"]:
        g = O.GEN64[name]
        M = Mx.matrix_for(g)
        pows = [np.eye(g.n, dtype=np.uint8)]
        for _ in range(g.k - 1):
            pows.append(Mx.mul(pows[-1], M))
        words = range(g.k)
        if g.k == 4 and g.family == O.XOSHIRO:
            words = [0, 1, 3]
        for j in words:
            blk = np.concatenate([P[:, j * 64:(j + 1) * 64] for P in pows], axis=1)
            assert Mx.rank(blk) == g.n, (name, j)

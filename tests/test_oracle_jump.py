"""Pins of the oracle's jump: x^J mod p(x) applied by accumulate-and-step must
equal J single steps, compose additively, agree with the matrix power M^J
computed by repeated squaring of the block matrix, and return to the start
after a full period."""
import numpy as np
import pytest

import oracle as O
from oracle import matrices as Mx

ALL = ["xoroshiro128+", "xoroshiro128++", "xoshiro256+", "xoshiro512+", "xoroshiro1024+"]


@pytest.mark.parametrize("name", ALL)
def test_jump_equals_single_steps(name):
    g = O.GEN64[name]
    x = O.splitmix_fill(11, g.k)
    rng = np.random.default_rng(3)
    Js = [0, 1, 2, 15, 16, 17, g.n - 1, g.n, g.n + 1] + rng.integers(0, 4096, 6).tolist()
    for J in Js:
        assert O.jump(g, x, J).tolist() == O.advance(g, x, J).tolist(), J


@pytest.mark.parametrize("name", ALL)
def test_jump_homomorphism(name):
    g = O.GEN64[name]
    x = O.splitmix_fill(12, g.k)
    a = O.jump_distance(g, "jump")
    b = O.jump_distance(g, "long")
    c = (1 << (g.n - 3)) + 123456789
    assert O.jump(g, O.jump(g, x, a), b).tolist() == O.jump(g, x, a + b).tolist()
    assert O.jump(g, O.jump(g, x, b), a).tolist() == O.jump(g, x, a + b).tolist()
    assert O.jump(g, O.jump(g, x, c), 77).tolist() == O.jump(g, x, c + 77).tolist()


@pytest.mark.parametrize("name", ALL)
def test_full_period_returns_to_start(name):
    g = O.GEN64[name]
    x = O.splitmix_fill(13, g.k)
    assert O.jump(g, x, (1 << g.n) - 1).tolist() == x.tolist()
    # and no smaller power of two minus one does (the order is exactly 2^n-1
    # only with primitivity; here: x M^(2^(n/2)) is not x)
    assert O.jump(g, x, 1 << (g.n // 2)).tolist() != x.tolist()


def _matrix_jump(g, x, log2J):
    M = Mx.matrix_for(g)
    for _ in range(log2J):
        M = Mx.mul(M, M)
    return Mx.apply(M, [int(v) for v in x], 64)


@pytest.mark.parametrize("name", ["xoroshiro128+", "xoroshiro128++", "xoshiro256+", "xoshiro512+"])
def test_jump_matches_matrix_squaring(name):
    g = O.GEN64[name]
    x = O.splitmix_fill(14, g.k)
    for log2J in (g.n // 2, 3 * g.n // 4):
        assert O.jump(g, x, 1 << log2J).tolist() == _matrix_jump(g, x, log2J)


@pytest.mark.slow
def test_jump_matches_matrix_squaring_xoroshiro1024():
    g = O.GEN64["xoroshiro1024+"]
    x = O.splitmix_fill(14, g.k)
    M = Mx.matrix_for(g)
    for _ in range(512):
        M = Mx.mul(M, M)
    assert O.jump(g, x, 1 << 512).tolist() == Mx.apply(M, [int(v) for v in x], 64)
    for _ in range(256):
        M = Mx.mul(M, M)
    assert O.jump(g, x, 1 << 768).tolist() == Mx.apply(M, [int(v) for v in x], 64)


@pytest.mark.parametrize("name", ["xoshiro256**", "xoroshiro1024**", "xoroshiro128++"])
def test_stream_chain_equals_direct_positioning(name):
    g = O.GEN64[name]
    S = 37
    chain = O.stream_chain(g, 42, S)
    for i in (0, 1, 2, 17, 36):
        assert chain[i].tolist() == O.stream_state(g, 42, i).tolist()
    assert chain[0].tolist() == O.splitmix_fill(42, g.k).tolist()


def test_jump_many_matches_single():
    g = O.GEN64["xoshiro512++"]
    st = np.stack([O.splitmix_fill(s, g.k) for s in range(9)])
    J = O.jump_distance(g, "long")
    many = O.jump_many(g, st, J, nthreads=3)
    for i in range(9):
        assert many[i].tolist() == O.jump(g, st[i], J).tolist()

"""GPU parity of the on-device equidistribution test
(slrng_equidistribution_rank) and of the Gaussian elimination behind it
(slrng_gf2_rank).

The expected ranks come from the oracle: the engine matrices built from the
block matrices of Section "Linear engines" (not from the code figures), the
j-th block columns of M^0 .. M^(dims-1) juxtaposed as in Section
"Equidistribution", and the oracle's own elimination.  Row and column order
differ between the two sides (the oracle reads words most significant bit
first); the rank does not depend on either.  The elimination is pinned on
random matrices of planted rank, where a kernel that always answered the
maximum would fail."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import matrices as Mx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_01407_amd as P
    P.lib()
    return P


def announce(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def oracle_equidist_rank(g, word, dims):
    """Rank of the juxtaposed j-th block columns of M^0 .. M^(dims-1)."""
    M = Mx.matrix_for(g).astype(np.int64)
    n, w = g.n, g.w
    col = np.eye(n, dtype=np.int64)[:, word * w:(word + 1) * w]
    blocks = [col]
    for _ in range(dims - 1):
        col = (M @ col) & 1  # M^t's block columns: M times M^(t-1)'s
        blocks.append(col)
    return Mx.rank(np.concatenate(blocks, axis=1).astype(np.uint8))


CASES = [("xoroshiro128+", w, d) for w in (0, 1) for d in (1, 2)] + \
        [("xoroshiro128++", w, 2) for w in (0, 1)] + \
        [("xoshiro256+", w, d) for w in range(4) for d in (1, 2, 4)] + \
        [("xoshiro512+", w, d) for w in (0, 2, 7) for d in (3, 8)] + \
        [("xoroshiro1024+", w, d) for w, d in ((0, 16), (15, 16), (7, 5))] + \
        [("xoroshiro64*", w, d) for w in (0, 1) for d in (1, 2)] + \
        [("xoshiro128+", w, d) for w in range(4) for d in (1, 3, 4)]


def third_word_of_four(g, word):
    """The one word Section "Equidistribution" leaves open: the third word
    of the four-word xoshiro engines, equidistributed or not depending on
    the shift and rotation parameters."""
    return g.family == O.XOSHIRO and g.k == 4 and word == 2


# The ranks of that word for the parameters of table tab:par64 (17/45) and
# tab:par32 (9/11), as computed by the oracle (and matched by the kernel):
# full for xoshiro256, one short of full for xoshiro128, whose scramblers
# read words 0, 1 and 3 only.
THIRD_WORD_RANK = {256: 256, 128: 127}


@pytest.mark.parametrize("name,word,dims", CASES)
def test_equidistribution_rank_matches_oracle(P, name, word, dims):
    g = O.GEN64.get(name) or O.GEN32[name]
    announce("equidistribution rank", name, word, dims)
    got = P.equidistribution_rank(name, word, dims)
    assert got == oracle_equidist_rank(g, word, dims)
    if third_word_of_four(g, word):
        if dims == g.k:
            assert got == THIRD_WORD_RANK[g.n]
    else:
        # Section "Equidistribution": every other word of these engines is
        # equidistributed in the maximum dimension, hence in every lower one
        assert got == min(g.n, dims * g.w)


def test_every_generator_word_in_the_maximum_dimension(P):
    # the check a user would run: every word of every generator's engine
    for name in P.VARIANTS + P.VARIANTS32:
        g = O.GEN64.get(name) or O.GEN32[name]
        announce("maximum dimension", name)
        for word in range(g.k):
            want = THIRD_WORD_RANK[g.n] if third_word_of_four(g, word) else g.n
            assert P.equidistribution_rank(name, word) == want, (name, word)


def planted(rng, nrows, ncols, r):
    """A random nrows x ncols matrix of rank at most r (a product B C)."""
    if r == 0:
        return np.zeros((nrows, ncols), dtype=np.uint8)
    B = rng.integers(0, 2, (nrows, r))
    C = rng.integers(0, 2, (r, ncols))
    return ((B @ C) & 1).astype(np.uint8)


@pytest.mark.parametrize("nrows,ncols,r", [
    (1, 1, 0), (1, 1, 1), (64, 64, 64), (64, 64, 17), (65, 63, 63), (63, 65, 5),
    (100, 1024, 99), (1024, 100, 100), (1024, 1024, 1024), (1024, 1024, 700),
    (37, 500, 3), (1000, 129, 128), (777, 777, 0)])
def test_gf2_rank_matches_oracle_elimination(P, nrows, ncols, r):
    rng = np.random.default_rng(nrows * 7919 + ncols * 31 + r)
    a = planted(rng, nrows, ncols, r)
    announce("gf2 rank", nrows, ncols, r)
    got = P.gf2_rank(a)
    assert got == Mx.rank(a)
    assert got <= r


def test_gf2_rank_special_matrices(P):
    announce("gf2 rank special")
    assert P.gf2_rank(np.eye(1024, dtype=np.uint8)) == 1024
    assert P.gf2_rank(np.ones((300, 400), dtype=np.uint8)) == 1
    # a row that is the sum of two others, and a repeated row
    rng = np.random.default_rng(5)
    a = rng.integers(0, 2, (10, 70)).astype(np.uint8)
    a[3] = a[1] ^ a[2]
    a[7] = a[0]
    assert P.gf2_rank(a) == Mx.rank(a) == 8
    # the same matrix with its rows and columns permuted keeps its rank
    b = a[rng.permutation(10)][:, rng.permutation(70)]
    assert P.gf2_rank(b) == 8

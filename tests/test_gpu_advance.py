"""GPU parity of per-stream arbitrary jumps (slrng_streams_advance_each): every
stream advances by its own 128-bit distance, on the device, through the
radix-1024 digit tables.  Expected states come from the oracle's own jump
(x^J mod p by square-and-multiply, then accumulate-and-step) and, for small
distances, from plain stepping."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

ALL = list(O.GEN64)


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


def distances(S: int, seed: int, distinct: int | None = None) -> list[int]:
    """A mix of zero, small, 64-bit, word-boundary and full 128-bit distances;
    with `distinct`, only that many different values (cycled)."""
    rng = np.random.default_rng(seed)
    m = distinct or S
    base = []
    for i in range(m):
        c = i % 7
        if c == 0:
            J = 0
        elif c == 1:
            J = int(rng.integers(1, 5000))
        elif c == 2:
            J = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        elif c == 3:
            J = (1 << 64) - 1 + int(rng.integers(0, 3))  # carries into the high word
        elif c == 4:
            J = (1 << 128) - 1 - int(rng.integers(0, 1000))
        elif c == 5:
            J = 1023 << (10 * int(rng.integers(0, 12)))  # one full digit
        else:
            J = int.from_bytes(rng.bytes(16), "little")
        base.append(J)
    return [base[i % m] for i in range(S)]


def oracle_jumped(g, states: np.ndarray, Js: list[int]) -> np.ndarray:
    """x_i * M^(J_i) for every row, polynomials computed in parallel."""
    p = O.charpoly(g)
    uniq = sorted(set(Js))
    with ThreadPoolExecutor(16) as ex:
        polys = dict(zip(uniq, ex.map(lambda J: O.xpow_mod(J, p), uniq)))
    return np.stack([O.jump_poly(g, states[i], polys[J]) for i, J in enumerate(Js)])


@pytest.mark.parametrize("name", ALL)
def test_advance_each_matches_oracle(P, name):
    g = O.GEN64[name]
    S = 131  # two full waves and a ragged one
    announce("advance_each", name, S)
    chain = O.stream_chain(g, 7, S)
    Js = distances(S, seed=11, distinct=28 if g.k == 16 else None)
    exp = oracle_jumped(g, chain, Js)
    with P.Streams(name, 7, S) as h:
        h.advance_each(Js)
        got = h.get_state()
    assert np.array_equal(got, exp)


def test_advance_each_small_distances_equal_steps(P):
    name = "xoshiro256**"
    g = O.GEN64[name]
    S = 200
    announce("advance_each small", name)
    chain = O.stream_chain(g, 3, S)
    rng = np.random.default_rng(5)
    Js = [int(v) for v in rng.integers(0, 3000, size=S)]
    Js[:4] = [0, 1, 1023, 1024]
    exp = np.stack([O.advance(g, chain[i], Js[i]) for i in range(S)])
    with P.Streams(name, 3, S) as h:
        h.advance_each(Js)
        got = h.get_state()
        out = h.generate(37).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, exp)
    for i in range(0, S, 17):
        assert np.array_equal(out[i], O.generate(g, exp[i], 37)[0])


def test_advance_each_composes_and_period(P):
    import torch
    announce("advance_each compose")
    for name in ("xoroshiro128++", "xoshiro512**"):
        g = O.GEN64[name]
        S = 96
        rng = np.random.default_rng(9)
        a = [int.from_bytes(rng.bytes(15), "little") for _ in range(S)]
        b = [int.from_bytes(rng.bytes(15), "little") for _ in range(S)]
        with P.Streams(name, 1, S) as h1, P.Streams(name, 1, S) as h2:
            h1.advance_each(a)
            h1.advance_each(b)
            # the same sum given as a device tensor of (low, high) words
            w = np.zeros((S, 2), dtype=np.uint64)
            for i in range(S):
                J = a[i] + b[i]
                w[i] = (J & (2**64 - 1), J >> 64)
            h2.advance_each(torch.from_numpy(w.view(np.int64)).cuda())
            torch.cuda.synchronize()
            assert np.array_equal(h1.get_state(), h2.get_state())
    # xoroshiro128 has period 2^128 - 1: that distance is the identity
    for name in ("xoroshiro128+", "xoroshiro128++", "xoroshiro128*"):
        with P.Streams(name, 2, 70) as h:
            before = h.get_state()
            h.advance_each([(1 << 128) - 1] * 70)
            assert np.array_equal(h.get_state(), before)


def test_advance_each_full_size_sampled(P):
    """2^20 xoshiro256++ streams (seed 42), each advanced by its own random
    128-bit distance; sampled streams against the oracle, then 256 outputs of
    each sampled stream."""
    import torch
    name, seed, S, N = "xoshiro256++", 42, 1 << 20, 256
    g = O.GEN64[name]
    announce("advance_each full size", name, S)
    rng = np.random.default_rng(2024)
    words = rng.integers(0, 2**63, size=(S, 2), dtype=np.int64) * 2 + rng.integers(0, 2, size=(S, 2))
    words = words.astype(np.int64)
    steps = torch.from_numpy(words).cuda()
    rows = np.unique(np.concatenate([np.arange(64), rng.integers(0, S, 1500), S - 1 - np.arange(64)]))
    chain = O.stream_chain(g, seed, S)
    uw = words.view(np.uint64)
    Js = [int(uw[i, 0]) | (int(uw[i, 1]) << 64) for i in rows]
    exp = oracle_jumped(g, chain[rows], Js)
    buf = torch.empty((S, N), dtype=torch.int64, device="cuda")
    with P.Streams(name, seed, S) as h:
        h.advance_each(steps)
        P.slrng_generate(h.h, P.SLRNG_U64, N, buf.data_ptr(), N, 0)
        torch.cuda.synchronize()
        got = h.get_state()
    out = buf[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint64)
    del buf
    torch.cuda.empty_cache()
    for j, i in enumerate(rows):
        o, fin = O.generate(g, exp[j], N)
        assert np.array_equal(out[j], o), i
        assert np.array_equal(got[i], fin), i

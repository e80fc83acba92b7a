"""GPU parity of jump polynomials computed on the device
(slrng_jump_poly_device): x^J mod p for 128-bit distances J, from tables of
x^(d 2^(10 l)) mod p that the device builds from p alone.  Expected values
come from the oracle's own square-and-multiply (x^J mod p over its own
characteristic polynomial); states jumped with the device polynomials are
checked against plain stepping for small J."""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

ALL = list(O.GEN64) + list(O.GEN32)


def gen(name):
    return O.GEN64[name] if name in O.GEN64 else O.GEN32[name]


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


def distances(m: int, seed: int) -> list[int]:
    """Zero, one, small, single digits at every radix-1024 level (the table
    entries themselves), 64-bit boundaries, the maximum and random 128-bit
    values."""
    rng = np.random.default_rng(seed)
    out = [0, 1, 2, 1023, 1024, (1 << 64) - 1, 1 << 64, (1 << 128) - 1]
    # level 12 holds bits 120..127 only: digits below 256 there
    out += [int(rng.integers(1, 1024 if l < 12 else 256)) << (10 * l) for l in range(13)]
    out += [255 << 120, 1 << 127, (1 << 70) + 5]
    while len(out) < m:
        out.append(int.from_bytes(rng.bytes(16), "little"))
    return out[:m]


def rows_to_ints(t) -> list[int]:
    a = t.cpu().numpy().view(np.uint64)
    return [sum(int(v) << (64 * w) for w, v in enumerate(row)) for row in a]


@pytest.mark.parametrize("name", ALL)
def test_jump_poly_device_matches_oracle(P, name):
    g = gen(name)
    m = 40 if g.k == 16 else 67  # a ragged second wave
    announce("jump_poly_device", name, m)
    Js = distances(m, seed=len(name))
    p = O.charpoly(g)
    got = rows_to_ints(P.slrng_jump_poly_device(name, Js))
    exp = [O.xpow_mod(J, p) for J in Js]
    bad = [i for i in range(m) if got[i] != exp[i]]
    assert not bad, f"{name}: {len(bad)} of {m} differ, first J = {Js[bad[0]]:#x}"


@pytest.mark.parametrize("name", ["xoroshiro128+", "xoshiro256**", "xoshiro512++", "xoroshiro1024*",
                                  "xoshiro128+"])
def test_jump_poly_device_small_distances_step(P, name):
    """For J < 3000, the state jumped with the device polynomial equals the
    state stepped J times (the oracle's plain step)."""
    g = gen(name)
    announce("jump_poly_device steps", name)
    Js = [0, 1, 2, 3, 63, 64, 65, 1000, 1023, 1024, 2999]
    polys = rows_to_ints(P.slrng_jump_poly_device(name, Js))
    x0 = O.seed_state(g, 99)
    for J, r in zip(Js, polys):
        assert np.array_equal(O.jump_poly(g, x0, r), O.advance(g, x0, J)), (name, J)


def test_jump_poly_device_tensor_input_and_empty(P):
    import torch
    announce("jump_poly_device tensor")
    Js = distances(300, seed=5)
    w = np.array([[J & ((1 << 64) - 1), J >> 64] for J in Js], dtype=np.uint64)
    t = torch.from_numpy(w.view(np.int64)).cuda()
    a = rows_to_ints(P.slrng_jump_poly_device("xoshiro256++", t))
    b = rows_to_ints(P.slrng_jump_poly_device("xoshiro256++", Js))
    assert a == b
    assert P.slrng_jump_poly_device("xoshiro256++", []).shape == (0, 4)

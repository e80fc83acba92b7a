"""The batch entry point that allocates no device memory
(slrng_batch_run_static) against slrng_batch_run on the same requests, bit for
bit, on two calls in a row (the second smaller, so that stale contents of the
library's fixed device array would show), with a sample of requests also
checked against the oracle; and its size limit."""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

NAMES = ["xoroshiro128+", "xoroshiro128++", "xoroshiro128**", "xoshiro256+", "xoshiro256++",
         "xoshiro256**", "xoshiro512+", "xoshiro512++", "xoshiro512**", "xoroshiro1024+",
         "xoroshiro1024++", "xoroshiro1024**", "xoroshiro128*", "xoroshiro1024*"]


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


def requests(rng, count):
    variant = rng.integers(0, 14, count)
    kind = rng.integers(0, 2, count)
    seed = rng.integers(0, 2**63, count, dtype=np.uint64)
    lens = np.array([0, 1, 17, 33, 1000, 4095, 9000, 70000, 300000], dtype=np.uint64)
    n = lens[rng.integers(0, len(lens), count)]
    start = np.array([0, 0, 5, 1 << 33], dtype=np.uint64)[rng.integers(0, 4, count)]
    off = np.zeros(count, dtype=np.int64)
    pos = 0
    for i, m in enumerate(n.tolist()):
        pos = (pos + 31) // 32 * 32 + (i % 5 == 3)  # some requests only 8-byte aligned
        off[i] = pos
        pos += int(m)
    return variant, kind, seed, start, n, off, pos + 1


def oracle_request(variant, kind, seed, start, n):
    g = O.GEN64[NAMES[int(variant)]]
    x = O.splitmix_fill(int(seed), g.k)
    if int(start):
        x = O.jump(g, x, int(start))
    out, _ = O.generate(g, x, int(n))
    if int(kind) == 1:
        out = ((out >> np.uint64(11)).astype(np.float64) * 2.0**-53).view(np.uint64)
    return out


@pytest.mark.parametrize("tile", [32, 16])
def test_static_batch_equals_batch_run_twice(P, tile):
    import torch
    rng = np.random.default_rng(77 + tile)
    for call, count in enumerate((240, 37)):
        variant, kind, seed, start, n, off, elems = requests(rng, count)
        announce(f"batch_run_static tile={tile} call={call} requests={count} outputs={int(n.sum())}")
        ref = torch.full((elems,), -1, dtype=torch.int64, device="cuda")
        got = torch.full((elems,), -2, dtype=torch.int64, device="cuda")
        opts = P.slrng_batch_default_opts(mode=P.SLRNG_BATCH_PERSISTENT, tile=tile)
        P.slrng_batch_run(P.make_requests(variant, kind, seed, start, n, ref.data_ptr() + 8 * off), opts, 0)
        P.slrng_batch_run_static(P.make_requests(variant, kind, seed, start, n, got.data_ptr() + 8 * off),
                                 opts, 0)
        torch.cuda.synchronize()
        a = ref.cpu().numpy().view(np.uint64)
        b = got.cpu().numpy().view(np.uint64)
        for r in range(count):
            lo, hi = int(off[r]), int(off[r] + n[r])
            assert (a[lo:hi] == b[lo:hi]).all(), (call, r)
        for r in rng.choice(count, 12, replace=False):
            lo, hi = int(off[r]), int(off[r] + n[r])
            exp = oracle_request(variant[r], kind[r], seed[r], start[r], n[r])
            assert (b[lo:hi] == exp).all(), (call, r)


def test_static_batch_graph_mode_and_empty(P):
    import torch
    rng = np.random.default_rng(5)
    variant, kind, seed, start, n, off, elems = requests(rng, 20)
    announce("batch_run_static graph mode, empty batch")
    ref = torch.zeros((elems,), dtype=torch.int64, device="cuda")
    got = torch.zeros((elems,), dtype=torch.int64, device="cuda")
    P.slrng_batch_run(P.make_requests(variant, kind, seed, start, n, ref.data_ptr() + 8 * off), None, 0)
    P.slrng_batch_run_static(P.make_requests(variant, kind, seed, start, n, got.data_ptr() + 8 * off), None, 0)
    torch.cuda.synchronize()
    assert torch.equal(ref, got)
    P.slrng_batch_run_static(P.make_requests([], [], [], [], [], 0), None, 0)


def test_static_batch_limits(P):
    import torch
    # the plain form needs per-request tables: refused
    buf = torch.zeros(64, dtype=torch.int64, device="cuda")
    with pytest.raises(P.SlrngError):
        P.slrng_batch_run_static(P.make_requests([0], [0], [1], [0], [10], buf.data_ptr()),
                                 P.slrng_batch_default_opts(mode=P.SLRNG_BATCH_PLAIN), 0)
    # more lane descriptors than the fixed array holds (32 bytes each): refused
    # before anything is launched (the outputs are valid memory all the same)
    count = (P.SLRNG_BATCH_STATIC_SCRATCH_BYTES // 32) + 4096
    announce(f"batch_run_static over the limit: {count} one-output requests")
    out = torch.zeros(count, dtype=torch.int64, device="cuda")
    z = np.zeros(count, dtype=np.uint64)
    reqs = P.make_requests(np.zeros(count, np.int64), np.zeros(count, np.int64), np.arange(count, dtype=np.uint64),
                           z, np.ones(count, dtype=np.uint64), out.data_ptr() + 8 * np.arange(count))
    with pytest.raises(P.SlrngError) as ei:
        P.slrng_batch_run_static(reqs, None, 0)
    assert ei.value.name == "ERANGE"
    torch.cuda.synchronize()
    assert not out.any()

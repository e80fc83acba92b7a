"""GPU parity of batched generation (persistent kernel, hipGraph replay, and the
plain one-launch-per-request form) against the oracle, bit for bit; every
request must give the same values alone and in any mix."""
import concurrent.futures as cf
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

NAMES = list(O.GEN64)  # the library's variant ids follow this order
ID = {name: i for i, name in enumerate(["xoroshiro128+", "xoroshiro128++", "xoroshiro128**",
                                        "xoshiro256+", "xoshiro256++", "xoshiro256**",
                                        "xoshiro512+", "xoshiro512++", "xoshiro512**",
                                        "xoroshiro1024+", "xoroshiro1024++", "xoroshiro1024**",
                                        "xoroshiro128*", "xoroshiro1024*"])}
NAME_OF = {v: k for k, v in ID.items()}


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


def oracle_request(variant, kind, seed, start, n):
    g = O.GEN64[NAME_OF[int(variant)]]
    x = O.splitmix_fill(int(seed), g.k)
    if int(start):
        x = O.jump(g, x, int(start))
    out, _ = O.generate(g, x, int(n))
    if int(kind) == 1:
        out = ((out >> np.uint64(11)).astype(np.float64) * 2.0**-53).view(np.uint64)
    return out


def mixed_requests(rng, count, big_start_ok=True):
    variant = rng.integers(0, 14, count)
    kind = rng.integers(0, 2, count)
    seed = rng.integers(0, 2**63, count, dtype=np.uint64)
    lens = np.array([0, 1, 2, 15, 16, 17, 31, 33, 100, 1000, 1007, 3000, 5000, 12000], dtype=np.uint64)
    n = lens[rng.integers(0, len(lens), count)]
    starts = np.array([0, 0, 0, 1, 7, 1000, (1 << 40) + 3], dtype=np.uint64)
    start = starts[rng.integers(0, len(starts), count)]
    if not big_start_ok:
        start[variant >= 9] = np.minimum(start[variant >= 9], 1000)
    return variant, kind, seed, start, n


def layout(n, misalign_every=0):
    """Element offsets in an arena, each request 256-byte aligned, some shifted
    by one element (8-byte aligned only)."""
    off = np.zeros(len(n), dtype=np.int64)
    pos = 0
    for i, m in enumerate(n.tolist()):
        pos = (pos + 31) // 32 * 32
        if misalign_every and i % misalign_every == 1:
            pos += 1
        off[i] = pos
        pos += int(m)
    return off, pos + 1


def run_batch(P, reqs_np, mode, chunk=None, tile=None):
    import torch
    opts = P.slrng_batch_default_opts(mode=mode, chunk=chunk, tile=tile)
    P.slrng_batch_run(reqs_np, opts, 0)
    torch.cuda.synchronize()


def check_all(arena_host, variant, kind, seed, start, n, off):
    def one(i):
        exp = oracle_request(variant[i], kind[i], seed[i], start[i], n[i])
        got = arena_host[off[i]:off[i] + int(n[i])]
        return i, np.array_equal(got, exp)
    with cf.ThreadPoolExecutor(8) as ex:
        for i, ok in ex.map(one, range(len(n))):
            assert ok, (i, NAME_OF[int(variant[i])], int(kind[i]), int(start[i]), int(n[i]))


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_mixed_batch_matches_oracle(P, mode):
    import torch
    rng = np.random.default_rng(100 + mode)
    variant, kind, seed, start, n = mixed_requests(rng, 160, big_start_ok=(mode == 0))
    off, total = layout(n, misalign_every=5)
    arena = torch.full((total,), -1, dtype=torch.int64, device="cuda")
    base = arena.data_ptr()
    reqs = P.make_requests(variant, kind, seed, start, n, base + 8 * off.astype(np.uint64))
    announce("mixed batch mode", mode)
    # small chunks so that short requests still span several lanes
    run_batch(P, reqs, mode, chunk={v: 1000 for v in range(14)})
    host = arena.cpu().numpy().view(np.uint64)
    check_all(host, variant, kind, seed, start, n, off)
    # nothing outside the requests was written
    mask = np.ones(total, dtype=bool)
    for o, m in zip(off.tolist(), n.tolist()):
        mask[o:o + m] = False
    assert (host[mask] == np.uint64(0xFFFFFFFFFFFFFFFF)).all()


def test_alone_equals_in_mix_and_modes_agree(P):
    import torch
    rng = np.random.default_rng(7)
    variant, kind, seed, start, n = mixed_requests(rng, 120, big_start_ok=False)
    n[:5] = [40000, 70000, 5, 16384, 16385]
    off, total = layout(n)
    results = []
    for mode in (0, 1, 2):
        arena = torch.full((total,), -1, dtype=torch.int64, device="cuda")
        reqs = P.make_requests(variant, kind, seed, start, n,
                               arena.data_ptr() + 8 * off.astype(np.uint64))
        run_batch(P, reqs, mode)
        results.append(arena.cpu().numpy().view(np.uint64).copy())
    assert np.array_equal(results[0], results[1]) and np.array_equal(results[0], results[2])
    for i in range(8):
        out = torch.full((int(n[i]) + 1,), -1, dtype=torch.int64, device="cuda")
        one = P.make_requests(variant[i], kind[i], seed[i], start[i], n[i], out.data_ptr())
        run_batch(P, one, 0)
        alone = out.cpu().numpy().view(np.uint64)
        assert np.array_equal(alone[:int(n[i])], results[0][off[i]:off[i] + int(n[i])])
        assert alone[int(n[i])] == np.uint64(0xFFFFFFFFFFFFFFFF)


def test_graph_replays_are_identical(P):
    """Replay a captured batch several times with eager work in between."""
    import torch
    rng = np.random.default_rng(9)
    variant, kind, seed, start, n = mixed_requests(rng, 60, big_start_ok=False)
    off, total = layout(n)
    arena = torch.full((total,), -1, dtype=torch.int64, device="cuda")
    reqs = P.make_requests(variant, kind, seed, start, n, arena.data_ptr() + 8 * off.astype(np.uint64))
    opts = P.slrng_batch_default_opts(mode=P.SLRNG_BATCH_GRAPH, chunk={v: 2000 for v in range(14)})
    b = P.slrng_batch_plan(reqs, opts)
    try:
        first = None
        for rep in range(4):
            arena.fill_(-1)
            torch.cuda.synchronize()
            P.slrng_batch_launch(b, 0)
            torch.cuda.synchronize()
            host = arena.cpu().numpy().view(np.uint64).copy()
            if first is None:
                first = host
                check_all(host, variant, kind, seed, start, n, off)
            else:
                assert np.array_equal(host, first), rep
    finally:
        P.slrng_batch_destroy(b)


def test_batched_workload_full_size(P):
    """The batched workload at full size: 10,000 requests, generator uniform
    over the eight swept variants, lengths log-uniform in [1, 2^24), 30%
    doubles (about 78 GB of outputs), one persistent launch captured in a
    hipGraph; every request compared in full with the oracle."""
    import torch
    from paper_1805_01407_amd import workloads as W
    w = W.batch_requests()
    announce("batched workload", int(w["n"].sum()), "outputs")
    arena = torch.empty((w["arena_elems"],), dtype=torch.int64, device="cuda")
    base = arena.data_ptr()
    reqs = P.make_requests(w["variant"], w["kind"], w["seed"], w["start"], w["n"],
                           base + 8 * w["offset"])
    run_batch(P, reqs, P.SLRNG_BATCH_GRAPH)

    order = np.argsort(-w["n"].astype(np.int64))

    def one(i):
        n_i, o_i = int(w["n"][i]), int(w["offset"][i])
        got = arena[o_i:o_i + n_i].cpu().numpy().view(np.uint64)
        exp = oracle_request(w["variant"][i], w["kind"][i], w["seed"][i], 0, n_i)
        return i, np.array_equal(got, exp)

    with cf.ThreadPoolExecutor(16) as ex:
        for i, ok in ex.map(one, order.tolist()):
            assert ok, ("request", i)
    del arena
    torch.cuda.empty_cache()

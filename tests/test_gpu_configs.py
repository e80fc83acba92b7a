"""GPU parity at the full sizes of the benchmark configurations, in the launch
configuration bench.py times (default tuning), bit for bit against the oracle.

* sweep: 65,536 streams x 65,536 outputs (32 GiB per kind, written into
  memory from slrng_output_alloc as bench.py does) — xoshiro256** (seed 3)
  compared in full (uint64 and doubles); each of the eight swept generators
  on its own seed (generator i on seed i + 1, as the sweep's steps use them)
  in its tuned launch shape, on rows covering every stagger class and slot
  boundary, plus every final state;
* jump-ahead: 1,048,576 xoshiro256++ streams positioned by the jump chain,
  then long-jumped once: all states compared, then 1,024 outputs per stream
  (8 GiB) compared in full.
"""
import sys

import numpy as np
import pytest

import oracle as O

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


def compare_blocks(buf, st0, g, N, kind, block=2048):
    """Compare a device [S, N] buffer with the oracle, block of rows at a time."""
    S = st0.shape[0]
    for r0 in range(0, S, block):
        r1 = min(S, r0 + block)
        got = buf[r0:r1].cpu().numpy().view(np.uint64)
        exp, _ = O.generate_many(g, st0[r0:r1], N, kind="u64", nthreads=16)
        if kind == 1:
            exp = ((exp >> np.uint64(11)).astype(np.float64) * 2.0**-53).view(np.uint64)
        if not np.array_equal(got, exp):
            bad = np.argwhere(got != exp)[0]
            raise AssertionError(f"rows {r0}..{r1}: first mismatch at {bad}")


def test_sweep_full_size_xoshiro256ss_complete(P):
    import torch
    name, seed, S, N = "xoshiro256**", 3, 65536, 65536
    g = O.GEN64[name]
    announce("sweep full", name, S, N)
    st0 = O.stream_chain(g, seed, S)
    buf = P.output_empty((S, N), torch.int64)  # the memory bench.py writes into
    with P.Streams(name, seed, S) as h:
        assert np.array_equal(h.get_state(), st0)
        P.slrng_generate(h.h, P.SLRNG_U64, N, buf.data_ptr(), N, 0)
        torch.cuda.synchronize()
        fin = h.get_state()
        compare_blocks(buf, st0, g, N, 0)
        h.seed(seed)
        P.slrng_generate(h.h, P.SLRNG_F64, N, buf.data_ptr(), N, 0)
        torch.cuda.synchronize()
        compare_blocks(buf, st0, g, N, 1)
    exp_fin = O.jump_many(g, st0, N, nthreads=16)
    assert np.array_equal(fin, exp_fin)
    del buf
    torch.cuda.empty_cache()


SWEEP = ["xoroshiro128+", "xoroshiro128++", "xoroshiro128**", "xoshiro256+", "xoshiro256++",
         "xoshiro256**", "xoshiro512**", "xoroshiro1024**"]


def sweep_rows(S, seed):
    """Rows that cover every stagger class of the slot boundaries (the class
    of a row is its group of 64 streams modulo the skew, at most 16), with the
    first, a middle and the last lane of each chosen group; plus the first and
    last rows of the launch.  Every row spans every slot boundary."""
    rng = np.random.default_rng(seed)
    groups = S // 64
    rows = {0, 1, S - 2, S - 1}
    for d in range(16):
        g = d + 16 * int(rng.integers(0, groups // 16))
        rows |= {g * 64, g * 64 + 31, g * 64 + 63}
    rows |= {(groups - 1) * 64, (groups - 1) * 64 + 63}
    return sorted(rows)


@pytest.mark.parametrize("gi", range(len(SWEEP)))
def test_sweep_full_size_every_generator(P, gi):
    """Generator i of the sweep on seed i + 1 at 65,536 x 65,536, uint64 and
    doubles, in the launch shape the autotuner chose for it (the one bench.py
    times): sampled rows covering every stagger class and slot boundary, and
    every stream's final state after each kind."""
    import torch
    name, seed, S, N = SWEEP[gi], gi + 1, 65536, 65536
    g = O.GEN64[name]
    announce("sweep full size", name, "seed", seed, S, N)
    st0 = O.stream_chain(g, seed, S)
    exp_fin = O.jump_many(g, st0, N, nthreads=16)
    rows = sweep_rows(S, seed)
    idx = None
    buf = P.output_empty((S, N), torch.int64)
    exp_u, _ = O.generate_many(g, st0[rows], N, kind="u64", nthreads=16)
    with P.Streams(name, seed, S) as h:
        assert np.array_equal(h.get_state(), st0)
        for kind in (P.SLRNG_U64, P.SLRNG_F64):
            h.seed(seed)
            P.slrng_generate(h.h, kind, N, buf.data_ptr(), N, 0)
            torch.cuda.synchronize()
            if idx is None:
                idx = torch.tensor(rows, device="cuda")
            got = buf.index_select(0, idx).cpu().numpy().view(np.uint64)
            exp = exp_u
            if kind == P.SLRNG_F64:
                exp = ((exp_u >> np.uint64(11)).astype(np.float64) * 2.0**-53).view(np.uint64)
            if not np.array_equal(got, exp):
                bad = np.argwhere(got != exp)[0]
                raise AssertionError(f"{name} kind {kind}: row {rows[bad[0]]} output {bad[1]} differs")
            assert np.array_equal(h.get_state(), exp_fin), (name, kind)
    del buf
    torch.cuda.empty_cache()


def test_jump_ahead_at_scale_1m_xoshiro256pp(P):
    import torch
    name, seed, S, N = "xoshiro256++", 42, 1 << 20, 1024
    g = O.GEN64[name]
    announce("jump ahead", name, S)
    chain = O.stream_chain(g, seed, S)
    exp = O.jump_many(g, chain, O.jump_distance(g, "long"), nthreads=16)
    buf = torch.empty((S, N), dtype=torch.int64, device="cuda")
    with P.Streams(name, seed, S) as h:
        assert np.array_equal(h.get_state(), chain)
        h.jump(P.SLRNG_LONG_JUMP)
        assert np.array_equal(h.get_state(), exp)
        P.slrng_generate(h.h, P.SLRNG_U64, N, buf.data_ptr(), N, 0)
        torch.cuda.synchronize()
        compare_blocks(buf, exp, g, N, 0, block=1 << 17)
        fin = h.get_state()
    assert np.array_equal(fin, O.jump_many(g, exp, N, nthreads=16))
    del buf
    torch.cuda.empty_cache()

"""GPU tests of the serving loop: every served request equals the oracle and the
same request run alone (a fresh handle advanced to the request's position),
at positions up to and past 2^64 (start states computed on the device from
the digits of the position); admission never exceeds the budget; requests
submitted while others are in flight run in iterations that overlap on the
device (shown by the iterations' device intervals)."""
import ctypes
import sys
import threading

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

NAME = "xoshiro256**"


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


def d2h(ptr, n):
    """Copy n uint64 from a device address (HIP runtime, the one torch loaded)."""
    import torch  # noqa: F401
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    out = np.zeros(n, dtype=np.uint64)
    rc = hip.hipMemcpy(out.ctypes.data, ptr, n * 8, 2)  # hipMemcpyDeviceToHost
    assert rc == 0
    return out


def expected(chain, stream, pos, n, kind=0):
    g = O.GEN64[NAME]
    x = O.jump(g, chain[stream], pos) if pos else chain[stream]
    out, _ = O.generate(g, x, n)
    if kind == 1:
        out = ((out >> np.uint64(11)).astype(np.float64) * 2.0**-53).view(np.uint64)
    return out


def test_served_requests_match_oracle_and_alone(P):
    S = 64
    chain = O.stream_chain(O.GEN64[NAME], 42, S)
    opts = P.slrng_server_default_opts(n_streams=S, budget_bytes=256 << 20, seed=42, variant=NAME,
                                       inflight=3)
    sv = P.slrng_server_create(opts)
    results = {}
    lock = threading.Lock()
    try:
        def client(cid):
            rng = np.random.default_rng(cid)
            for k in range(60):
                stream = int(rng.integers(0, 8))  # few streams: many requests per stream
                n = int(rng.choice([1, 7, 33, 1000, 5000, 20000, 70000]))
                kind = int(rng.integers(0, 2))
                t = P.slrng_server_submit(sv, stream, n, kind)
                with lock:
                    results[t] = (stream, n, kind)
        ths = [threading.Thread(target=client, args=(c,)) for c in range(4)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        announce("served", len(results))
        got = {}
        for t, (stream, n, kind) in results.items():
            ptr, pos = P.slrng_server_wait(sv, t)
            got[t] = (pos, d2h(ptr, n))
            P.slrng_server_release(sv, t)
        st = P.slrng_server_get_stats(sv)
    finally:
        P.slrng_server_destroy(sv)
    # positions on each stream are consecutive in admission (ticket) order
    heads = {}
    for t in sorted(results):
        stream, n, kind = results[t]
        pos, out = got[t]
        assert pos == heads.get(stream, 0)
        heads[stream] = pos + n
        assert np.array_equal(out, expected(chain, stream, pos, n, kind)), (t, stream, pos, n)
    assert st["completed"] == len(results) and st["failed"] == 0
    # the same requests alone: a fresh handle at the stream state, advanced to pos
    for t in sorted(results)[::17]:
        stream, n, kind = results[t]
        pos, out = got[t]
        with P.Streams(NAME, states=chain[stream]) as h:
            h.advance(pos)
            alone = h.generate(n, kind).cpu().numpy().view(np.uint64)[0]
        assert np.array_equal(alone, out)


@pytest.mark.parametrize("store,inflight", [(1, 8), (2, 1), (0, 8)])
def test_served_store_policies_and_slots(P, store, inflight):
    """Every store policy of the served kernel (the completion signal then
    follows a write-back fence or a counter wait) and one to eight slots:
    bursts of requests of many sizes, compared in full with the oracle."""
    S = 16
    chain = O.stream_chain(O.GEN64[NAME], 9, S)
    # room for every request of the burst at once: they are released only
    # after all are submitted
    opts = P.slrng_server_default_opts(n_streams=S, budget_bytes=2 << 30, seed=9, variant=NAME,
                                       inflight=inflight, store=store)
    sv = P.slrng_server_create(opts)
    rng = np.random.default_rng(store * 10 + inflight)
    sizes = [int(x) for x in rng.choice([1, 3, 64, 500, 8192, 8193, 100000, 1 << 20], 120)]
    announce("store/slots", store, inflight, len(sizes))
    try:
        tickets = [(P.slrng_server_submit(sv, k % S, n, k % 2), k % S, n, k % 2) for k, n in enumerate(sizes)]
        got = []
        for t, stream, n, kind in tickets:
            ptr, pos = P.slrng_server_wait(sv, t)
            got.append((stream, pos, n, kind, d2h(ptr, n)))
            P.slrng_server_release(sv, t)
        st = P.slrng_server_get_stats(sv)
    finally:
        P.slrng_server_destroy(sv)
    for stream, pos, n, kind, out in got:
        assert np.array_equal(out, expected(chain, stream, pos, n, kind)), (store, inflight, stream, pos, n)
    assert st["completed"] == len(sizes) and st["failed"] == 0
    # each iteration's busy interval contains its kernel interval
    assert 0 < st["kernel_s"] <= st["busy_s"]


def test_budget_admission_and_overlap(P):
    import time
    S = 16
    budget = 1 << 20  # 1 MiB arena
    # no batching window: every iteration launches as soon as a slot is free,
    # so a burst keeps several iterations in flight
    opts = P.slrng_server_default_opts(n_streams=S, budget_bytes=budget, seed=7, variant=NAME,
                                       inflight=3, window_us=0)
    sv = P.slrng_server_create(opts)
    try:
        # fill the arena with unreleased requests, then a non-blocking submit
        # that does not fit is rejected
        held = [P.slrng_server_submit(sv, i % S, 16384) for i in range(8)]  # 8 x 128 KiB
        for t in held:
            P.slrng_server_wait(sv, t)
        with pytest.raises(P.SlrngError) as e:
            P.slrng_server_submit(sv, 0, 1, flags=P.SLRNG_SUBMIT_NONBLOCK)
        assert e.value.name == "EAGAIN"
        # a blocking submit waits until a release makes room
        done = []

        def blocked():
            done.append(P.slrng_server_submit(sv, 1, 16384))
        th = threading.Thread(target=blocked)
        th.start()
        time.sleep(0.2)
        assert not done
        P.slrng_server_release(sv, held[0])
        th.join(timeout=30)
        assert done
        P.slrng_server_wait(sv, done[0])
        P.slrng_server_release(sv, done[0])
        for t in held[1:]:
            P.slrng_server_release(sv, t)
        # a burst of auto-released requests, batched into fewer iterations
        P.slrng_server_reset_stats(sv)
        for i in range(3000):
            P.slrng_server_submit(sv, i % S, 8000, flags=P.SLRNG_SUBMIT_AUTORELEASE)
        P.slrng_server_drain(sv)
        st = P.slrng_server_get_stats(sv)
    finally:
        P.slrng_server_destroy(sv)
    assert st["completed"] == 3000 and st["failed"] == 0
    assert st["peak_reserved_bytes"] <= budget
    assert st["iterations"] < 3000  # requests were batched


def test_iterations_overlap_on_the_device(P):
    """A long iteration (one request of two lane-chunks of 2^20 outputs, tens
    of ms on two lanes) and short requests submitted while it runs: the short
    ones complete in iterations on other HIP streams whose device intervals
    lie inside the long one's, and every value is right."""
    import time
    S = 8
    g = O.GEN64[NAME]
    chain = O.stream_chain(g, 9, S)
    opts = P.slrng_server_default_opts(n_streams=S, budget_bytes=64 << 20, seed=9, variant=NAME,
                                       inflight=3, window_us=0, chunk=1 << 20, min_chunk=1 << 20)
    sv = P.slrng_server_create(opts)
    try:
        long_t = P.slrng_server_submit(sv, 0, 1 << 21)
        time.sleep(0.003)
        short = []
        for k in range(4):
            short.append((P.slrng_server_submit(sv, 1 + k, 1000 + k), 1 + k, 1000 + k))
            time.sleep(0.002)
        outs = []
        for t, st, n in short:
            ptr, pos = P.slrng_server_wait(sv, t)
            outs.append((st, pos, n, d2h(ptr, n)))
        ptr, pos = P.slrng_server_wait(sv, long_t)
        head, tail = d2h(ptr, 4096), d2h(ptr + 8 * ((1 << 21) - 4096), 4096)
        iv = P.slrng_server_intervals(sv)
        stats = P.slrng_server_get_stats(sv)
    finally:
        P.slrng_server_destroy(sv)
    announce("overlap intervals (ms)", iv.round(3).tolist())
    assert stats["failed"] == 0 and stats["iterations"] >= 2
    # the long iteration completes last; some other iteration ran entirely
    # inside its interval on the device
    lo, hi = iv[-1]
    assert hi - lo > 1.0
    inside = [(a, b) for a, b in iv[:-1] if lo < a and b < hi]
    assert inside, iv.tolist()
    for st, pos, n, out in outs:
        assert np.array_equal(out, expected(chain, st, pos, n)), (st, pos, n)
    assert np.array_equal(head, O.generate(g, chain[0], 4096)[0])
    assert np.array_equal(tail, O.generate(g, O.jump(g, chain[0], (1 << 21) - 4096), 4096)[0])


@pytest.mark.parametrize("name", [NAME, "xoroshiro1024**", "xoroshiro128++"])
def test_served_positions_past_2_64(P, name):
    """Heads moved with slrng_server_advance to positions around and far past
    2^64 (one request straddles 2^64, one starts near 2^128 and wraps): the
    served values equal the oracle's jump to the same position and a fresh
    handle advanced there."""
    S = 6
    g = O.GEN64[name]
    chain = O.stream_chain(g, 21, S)
    skips = [(1 << 64) - 3, (1 << 64) + 12345, (1 << 100) + (1 << 70) + 99, (1 << 128) - 5,
             0x0123456789ABCDEF_FEDCBA9876543210, 5]
    opts = P.slrng_server_default_opts(n_streams=S, budget_bytes=64 << 20, seed=21, variant=name)
    sv = P.slrng_server_create(opts)
    got = []
    try:
        for st, k in enumerate(skips):
            P.slrng_server_advance(sv, st, k)
        tickets = []
        for st in range(S):
            for n in (10, 70000, 3):
                tickets.append((P.slrng_server_submit(sv, st, n, st % 2), st, n, st % 2))
        for t, st, n, kind in tickets:
            ptr, pos = P.slrng_server_wait(sv, t)
            got.append((st, pos, n, kind, d2h(ptr, n)))
            P.slrng_server_release(sv, t)
    finally:
        P.slrng_server_destroy(sv)
    announce("served past 2^64", name, len(got))
    heads = list(skips)
    for st, pos, n, kind, out in got:
        full = heads[st] % (1 << 128)
        assert pos == full % (1 << 64)
        heads[st] = full + n
        e, _ = O.generate(g, O.jump(g, chain[st], full), n)
        if kind == 1:
            e = ((e >> np.uint64(11)).astype(np.float64) * 2.0**-53).view(np.uint64)
        assert np.array_equal(out, e), (name, st, full, n)
    # the same request alone: a fresh handle advanced by the full position
    st, pos, n, kind, out = got[4]  # stream 1, 70,000 outputs past 2^64 + 12,355
    with P.Streams(name, states=chain[st]) as h:
        h.advance((1 << 64) + 12345 + 10)
        alone = h.generate(n, kind).cpu().numpy().view(np.uint64)[0]
    assert np.array_equal(alone, out)


def test_replay_small_trace(P):
    from paper_1805_01407_amd import workloads as W
    tr = W.serve_trace(rate=20000, seconds=0.5, streams=256, max_bytes=1 << 16, seed=11)
    opts = P.slrng_server_default_opts(n_streams=256, budget_bytes=1 << 30, seed=42, variant=NAME)
    sv = P.slrng_server_create(opts)
    try:
        P.slrng_server_replay(sv, tr["t"], tr["stream"], tr["n"], tr["kind"])
        st = P.slrng_server_get_stats(sv)
    finally:
        P.slrng_server_destroy(sv)
    assert st["completed"] == tr["t"].size and st["failed"] == 0
    assert st["outputs"] == int(tr["n"].sum())
    assert 0 < st["p50_us"] <= st["p99_us"] <= st["max_us"]


@pytest.mark.parametrize("name", ["xoroshiro128+", "xoshiro512**", "xoroshiro1024++"])
def test_served_requests_other_generators(P, name):
    """Request start states computed on the device from the digits of the
    position: two-word, eight-word and the cyclic sixteen-word engines,
    positions from 0 to past several digit levels."""
    S = 8
    g = O.GEN64[name]
    chain = O.stream_chain(g, 3, S)
    opts = P.slrng_server_default_opts(n_streams=S, budget_bytes=64 << 20, seed=3, variant=name)
    sv = P.slrng_server_create(opts)
    sizes = [1, 5, 64, 1000, 3, 40000, 777, 2]
    try:
        tickets = [(P.slrng_server_submit(sv, (k * 3) % S, n, k % 2), (k * 3) % S, n, k % 2)
                   for k, n in enumerate(sizes * 3)]
        got = []
        for t, st, n, kind in tickets:
            ptr, pos = P.slrng_server_wait(sv, t)
            got.append((st, pos, n, kind, d2h(ptr, n)))
            P.slrng_server_release(sv, t)
    finally:
        P.slrng_server_destroy(sv)
    announce("served", name, len(got))
    for st, pos, n, kind, out in got:
        x = O.jump(g, chain[st], pos) if pos else chain[st]
        e, _ = O.generate(g, x, n)
        if kind == 1:
            e = ((e >> np.uint64(11)).astype(np.float64) * 2.0**-53).view(np.uint64)
        assert np.array_equal(out, e), (name, st, pos, n)


def test_served_trace_values_at_workload_shape(P):
    """The first 0.2 s of the serving trace (the bench's recipe: Poisson
    arrivals at 20,000 requests/s, 4,096 resident xoshiro256** streams,
    64 B .. 256 MiB) through the default server (16 GiB budget), submitted as
    one burst so that admission blocks on the budget: every request of at
    most 1 MiB compared in full with the oracle, larger ones on their first
    and last 4,096 outputs and on eight interior blocks of 512 outputs, each
    straddling a multiple of 8,192 (a lane-chunk boundary for every chunk
    length the server can fit), all at the positions the server assigned."""
    import queue
    from concurrent.futures import ThreadPoolExecutor
    from paper_1805_01407_amd import workloads as W
    tr = W.serve_trace(seconds=0.2)
    g = O.GEN64[NAME]
    opts = P.slrng_server_default_opts()
    chain = O.stream_chain(g, opts.seed, opts.n_streams)
    announce("trace values", tr["t"].size)
    sv = P.slrng_server_create(opts)
    results = []
    work = queue.Queue()

    def consumer():
        while True:
            item = work.get()
            if item is None:
                return
            t, st, n = item
            ptr, pos = P.slrng_server_wait(sv, t)
            if n <= 131072:
                results.append((st, pos, n, d2h(ptr, n), None, []))
            else:
                rng = np.random.default_rng(t)
                offs = sorted({int(m) * 8192 - 256 for m in rng.integers(1, n // 8192, 8)})
                blocks = [(o, d2h(ptr + 8 * o, 512)) for o in offs]
                results.append((st, pos, n, d2h(ptr, 4096), d2h(ptr + 8 * (n - 4096), 4096), blocks))
            P.slrng_server_release(sv, t)

    th = threading.Thread(target=consumer)
    th.start()
    try:
        for i in range(tr["t"].size):
            st, n = int(tr["stream"][i]), int(tr["n"][i])
            work.put((P.slrng_server_submit(sv, st, n, 0), st, n))
        work.put(None)
        th.join()
        stats = P.slrng_server_get_stats(sv)
    finally:
        P.slrng_server_destroy(sv)
    assert len(results) == tr["t"].size and stats["failed"] == 0
    assert stats["peak_reserved_bytes"] <= opts.budget_bytes
    p = O.charpoly(g)

    def check(res):
        st, pos, n, head, tail, blocks = res
        x = O.jump_poly(g, chain[st], O.xpow_mod(pos, p)) if pos else chain[st]
        if tail is None:
            return np.array_equal(head, O.generate(g, x, n)[0])
        y = O.jump_poly(g, x, O.xpow_mod(n - 4096, p))
        ok = (np.array_equal(head, O.generate(g, x, 4096)[0]) and
              np.array_equal(tail, O.generate(g, y, 4096)[0]))
        for o, blk in blocks:
            z = O.jump_poly(g, x, O.xpow_mod(o, p))
            ok = ok and np.array_equal(blk, O.generate(g, z, 512)[0])
        return ok

    with ThreadPoolExecutor(16) as ex:
        ok = list(ex.map(check, results))
    assert all(ok), [results[i][:3] for i, v in enumerate(ok) if not v][:5]

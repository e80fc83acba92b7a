"""Throughput benchmark: the full-family sweep of 64-bit generation on one GPU.

Workload (one step): for each of the eight generators xoroshiro128+/++/**,
xoshiro256+/++/**, xoshiro512** and xoroshiro1024**, position 65,536 streams
from a seed (SplitMix64 fill, stream i jumped i times by 2^(n/2)), generate
65,536 uint64 outputs per stream (32 GiB, stream-major), re-position the same
streams and generate the same outputs as [0,1) doubles (another 32 GiB).
Step k uses seed (k mod 8) + 1, so 8 steps cover seeds 1..8.  Inputs are the
seeds alone; all outputs stay in HBM, in memory from the library's output
allocator (slrng_output_alloc: physical pages spread over the HBM; the
`placement` entry measures the same writes into compact memory beside it).

Prints one JSON line (rank 0).  `value` = outputs (uint64 + double) per
second over the timed steps; `roofline` describes the generation kernel
(HIP events around each launch; `traffic` from the committed HBM counters).
The same line carries the other workloads, each run once after the sweep:
the small case (1,024 streams), jump-ahead at scale (2^20 streams), the
32-bit generators, the on-device linearity check, the batched-requests
workload (one graph launch against one launch per request), the serving
trace (continuous batching against the plain form) and the CPU oracle on a
bounded sample (`cpu_baseline`; its `per_config` entry times the oracle on
samples of the other workloads, on one thread and on all).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SWEEP = ["xoroshiro128+", "xoroshiro128++", "xoroshiro128**", "xoshiro256+", "xoshiro256++",
         "xoshiro256**", "xoshiro512**", "xoroshiro1024**"]
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources of the generation kernel: a change to any of them invalidates the
# committed counter summary.
KERNEL_SOURCES = ["kernels.hip", "gen_device.hpp", "engines.hpp", "kernels.hpp"]


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1805_01407_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# Sources of the batched kernel: a change to any of them invalidates its
# committed counter summary.
BATCH_SOURCES = ["batch.hip", "batch.hpp", "gen_device.hpp", "engines.hpp", "kernels.hpp"]


def batch_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in BATCH_SOURCES:
        with open(os.path.join(ROOT, "paper_1805_01407_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_batch_traffic() -> int | None:
    """HBM bytes per launch of the batched workload's persistent kernel from
    the committed counter summary (FETCH_SIZE and WRITE_SIZE scaled by a copy
    kernel), or None when its sources have changed since."""
    path = os.path.join(ROOT, "profiles", "k_batch_batched_requests_pmc.md")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                      if line.startswith(("traffic_bytes_per_launch: ", "source_sha256: ")))
        sha = batch_source_sha()
    except (OSError, ValueError):
        return None
    if fields.get("source_sha256") != sha:
        return None
    return int(fields["traffic_bytes_per_launch"])


def profiled_valu() -> dict | None:
    """VALU instructions per dispatch of the positioning kernels (k_position,
    k_jump, k_advance_each for xoshiro256++ at 2^20 streams) from the
    committed counter summary (SQ_INSTS_VALU), or None when the kernel
    sources have changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", "jump_kernels_valu_pmc.md")
    try:
        lines = open(path).read().splitlines()
        sha = kernel_source_sha()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in lines if line.startswith(("valu_", "source_sha256: ")))
    if fields.get("source_sha256") != sha:
        return None
    return {k[len("valu_insts_per_dispatch_"):]: int(v) for k, v in fields.items()
            if k.startswith("valu_insts_per_dispatch_")}


def profiled_traffic() -> int | None:
    """HBM bytes per generation launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a copy kernel), or None when the
    kernel sources have changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_generate_full_family_sweep_pmc.md")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                      if line.startswith(("traffic_bytes_per_launch: ", "source_sha256: ")))
        sha = kernel_source_sha()
    except (OSError, ValueError):
        return None
    if fields.get("source_sha256") != sha:
        return None
    return int(fields["traffic_bytes_per_launch"])


# Worker threads for the CPU oracle: the host threads this process may use,
# at most 16 (the host share that goes with one GPU on a shared multi-GPU
# host, whatever nproc shows).
CPU_THREAD_CAP = 16


def host_cpu() -> dict:
    """nproc, the usable host threads, the cap applied and the CPU model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"nproc": os.cpu_count(), "usable_threads": usable, "thread_cap": CPU_THREAD_CAP,
            "threads": max(1, min(usable, CPU_THREAD_CAP)), "cpu_model": model}


def cpu_baseline(batch: int, N: int, seconds: float = 15.0) -> dict:
    """The oracle (plain serial C, threaded over streams only) on a bounded
    sample of the same workload: for each of the eight generators in turn,
    batches of `batch` streams of the seed-1 chain, N outputs each, as uint64
    and as doubles, until `seconds` of host time are spent, on all the host
    threads available up to CPU_THREAD_CAP; then the same on one thread for a
    third of the time."""
    import oracle as O
    host = host_cpu()
    nth = host["threads"]
    chains = {name: O.stream_chain(O.GEN64[name], 1, batch) for name in SWEEP}

    def run(threads: int, budget: float):
        outs = rounds = 0
        t0 = time.perf_counter()
        while True:
            for name in SWEEP:
                g = O.GEN64[name]
                O.generate_many(g, chains[name], N, kind="u64", nthreads=threads)
                O.generate_many(g, chains[name], N, kind="f64", nthreads=threads)
                outs += 2 * batch * N
            rounds += 1
            if time.perf_counter() - t0 >= budget:
                break
        return outs, rounds, time.perf_counter() - t0

    outs, rounds, dt = run(nth, seconds)
    outs1, rounds1, dt1 = run(1, seconds / 3)
    return {"value": outs / dt, "unit": "outputs/s", "cores": nth, "kind": "oracle", "host": host,
            "sample": f"{rounds} round(s) of 8 generators x {batch} streams x {N} outputs x "
                      f"(u64 + f64) from the seed-1 chains; {outs:.3g} outputs in {dt:.1f} s",
            "value_1thread": outs1 / dt1,
            "sample_1thread": f"{rounds1} round(s) of the same on one thread; {outs1:.3g} outputs "
                              f"in {dt1:.1f} s"}


def cpu_per_config(budget: float = 3.0) -> dict:
    """The oracle on the other configurations, each on a bounded sample, on
    one host thread and on all of them (at most 16): the small case in full;
    jump-ahead at scale on the first 2^14 of its 2^20 streams (the stream
    chain is serial by definition; the long jumps and the outputs are
    threaded over streams); the batched requests in list order until
    `budget` seconds of host time, threaded over requests."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O
    from paper_1805_01407_amd import workloads as W
    from paper_1805_01407_amd.binding import VARIANT_IDS
    nth = host_cpu()["threads"]
    out = {"cores": nth}

    g = O.GEN64["xoshiro256**"]
    t0 = time.perf_counter()
    st = O.stream_chain(g, 42, 1024)
    t_chain = time.perf_counter() - t0
    small = {"streams": 1024, "outputs_per_stream": 4096, "position_ms": round(t_chain * 1e3, 2)}
    for label, th in (("1thread", 1), ("all", nth)):
        t0 = time.perf_counter()
        O.generate_many(g, st, 4096, kind="u64", nthreads=th)
        small[f"generate_ms_{label}"] = round((time.perf_counter() - t0) * 1e3, 2)
    out["small_case"] = small

    g = O.GEN64["xoshiro256++"]
    S = 1 << 14
    t0 = time.perf_counter()
    chain = O.stream_chain(g, 42, S)
    t_chain = time.perf_counter() - t0
    jump = {"streams_sampled": S, "chain_streams_per_s": S / t_chain}
    J = O.jump_distance(g, "long")
    for label, th in (("1thread", 1), ("all", nth)):
        t0 = time.perf_counter()
        lj = O.jump_many(g, chain, J, nthreads=th)
        jump[f"long_jumps_per_s_{label}"] = S / (time.perf_counter() - t0)
        t0 = time.perf_counter()
        O.generate_many(g, lj, 1024, kind="u64", nthreads=th)
        jump[f"outputs_per_s_{label}"] = S * 1024 / (time.perf_counter() - t0)
    out["jump_ahead_at_scale"] = jump

    w = W.batch_requests()
    gens = {v: O.GEN64[name] for name, v in VARIANT_IDS.items() if name in O.GEN64}

    def one(r):
        gr = gens[int(w["variant"][r])]
        x = O.seed_state(gr, int(w["seed"][r]))
        O.generate_many(gr, x.reshape(1, -1), int(w["n"][r]), kind="f64" if w["kind"][r] else "u64",
                        nthreads=1)
        return int(w["n"][r])

    batched = {}
    for label, th in (("1thread", 1), ("all", nth)):
        done = r = 0
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=th) as ex:
            while time.perf_counter() - t0 < budget and r < len(w["n"]):
                step = th * 4
                done += sum(ex.map(one, range(r, min(r + step, len(w["n"])))))
                r += step
        dt = time.perf_counter() - t0
        batched[f"outputs_per_s_{label}"] = done / dt
        batched[f"requests_{label}"] = min(r, len(w["n"]))
    out["batched_requests"] = batched
    return out


def batched_section(P, torch, stream, launches: int = 3, forms=("graph", "plain")) -> dict:
    """The batched-requests workload (10,000 requests, generator uniform over
    the eight swept variants, lengths log-uniform in [1, 2^24), 30% doubles):
    one persistent launch replayed from a hipGraph, against the plain form (one
    launch of the same kernel per request).  Per-request latency is the time
    from the start of the launch until that request's outputs are complete."""
    import numpy as np
    from paper_1805_01407_amd import workloads as W
    w = W.batch_requests()
    arena = P.output_empty((w["arena_elems"],), torch.int64)
    reqs = P.make_requests(w["variant"], w["kind"], w["seed"], w["start"], w["n"],
                           arena.data_ptr() + 8 * w["offset"])
    total = int(w["n"].sum())
    out = {"requests": len(w["n"]), "outputs": total}
    chosen = [(label, mode, reps) for form, label, mode, reps in
              (("graph", "batched_graph", P.SLRNG_BATCH_GRAPH, launches),
               ("plain", "plain_per_request", P.SLRNG_BATCH_PLAIN, 1)) if form in forms]
    for label, mode, reps in chosen:
        t0 = time.perf_counter()
        b = P.slrng_batch_plan(reqs, P.slrng_batch_default_opts(mode=mode))
        plan_ms = (time.perf_counter() - t0) * 1e3
        try:
            P.slrng_batch_launch(b, stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                P.slrng_batch_launch(b, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            lat = P.slrng_batch_latencies(b, len(w["n"]), stream)
        finally:
            P.slrng_batch_destroy(b)
        gbs = 8 * total / (ms * 1e-3) / 1e9
        out[label] = {"ms_per_launch": round(ms, 3), "outputs_per_s": total / (ms * 1e-3),
                      "bytes_per_launch": 8 * total,
                      "GBs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                      "latency_p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "latency_p99_ms": round(float(np.percentile(lat, 99)), 3),
                      "plan_ms": round(plan_ms, 1)}
    if "batched_graph" in out:
        out["batched_graph"]["traffic"] = profiled_batch_traffic()
    # a plain copy of known size inside the arena, for scaling the hardware
    # memory counters of a profiled run of this section
    P.slrng_calib_copy(arena.data_ptr() + (4 << 30), arena.data_ptr(), 4 << 30, stream)
    torch.cuda.synchronize()
    del arena
    torch.cuda.empty_cache()
    return out


def placement_section(P, torch, stream, S: int, N: int, reps: int = 3) -> dict:
    """Store bandwidth against the physical placement of the output: the same
    fill kernel and one generator (xoshiro256**, uint64) writing S x N words
    into (a) the process's first large device allocation (torch.empty: one
    compact physical range) and (b) memory from slrng_output_alloc (the same
    virtual layout, physical pieces spread over the HBM).  Runs first, before
    any other large allocation, so that (a) is compact."""
    nbytes = 8 * S * N
    out = {"bytes": nbytes}

    def rate(ptr, fn):
        fn(ptr)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn(ptr)
        e1.record(stream)
        torch.cuda.synchronize()
        return round(nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)

    with P.Streams("xoshiro256**", 1, S) as h:
        for label, alloc in (("compact_first_allocation", lambda: torch.empty((S, N), dtype=torch.int64,
                                                                               device="cuda")),
                             ("output_alloc_spread", lambda: P.output_empty((S, N), torch.int64))):
            buf = alloc()
            out[label] = {
                "fill_GBs": rate(buf.data_ptr(), lambda p: P.slrng_calib_write(p, nbytes, stream)),
                "generate_GBs": rate(buf.data_ptr(),
                                     lambda p: P.slrng_generate(h.h, P.SLRNG_U64, N, p, N, stream))}
            del buf
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    return out


def small_case_section(P, torch, stream, reps: int = 20) -> dict:
    """The small case: xoshiro256**, 1,024 streams from seed 42 (stream i
    jumped i times by 2^128), 4,096 uint64 outputs each (32 MiB).  Too small
    to approach the HBM roof (about 4 us of writes at 8 TB/s): reported as
    times, positioning included."""
    name, seed, S, N = "xoshiro256**", 42, 1024, 4096
    buf = torch.empty((S, N), dtype=torch.int64, device="cuda")
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    pos_ms = gen_ms = 0.0
    with P.Streams(name, seed, S) as h:
        for rep in range(reps + 1):
            e = [ev() for _ in range(3)]
            e[0].record(stream)
            P.slrng_streams_seed(h.h, seed, stream)
            e[1].record(stream)
            P.slrng_generate(h.h, P.SLRNG_U64, N, buf.data_ptr(), N, stream)
            e[2].record(stream)
            torch.cuda.synchronize()
            if rep:
                pos_ms += e[0].elapsed_time(e[1]) / reps
                gen_ms += e[1].elapsed_time(e[2]) / reps
    del buf
    torch.cuda.empty_cache()
    return {"generator": name, "streams": S, "outputs_per_stream": N,
            "position_us": round(pos_ms * 1e3, 2), "generate_us": round(gen_ms * 1e3, 2),
            "generate_GBs": round(8 * S * N / (gen_ms * 1e-3) / 1e9, 1)}


def positioning_section(P, torch, stream, reps: int = 5) -> dict:
    """Jump-ahead at scale: 2^20 xoshiro256++ streams from seed 42 (stream i is
    the SplitMix64 base state jumped i times by 2^128), every stream then
    long-jumped once (2^192), then 1,024 outputs per stream (8 GiB).

    Positioning and the long jump are bound by integer VALU issue, not by
    HBM.  Their instruction counts come from the hardware counters
    (SQ_INSTS_VALU per dispatch, committed under profiles/ with the hash of
    the kernel sources): lane-operations = instructions x 64 lanes, divided
    by the launch time measured here.  gfx950 issues one VALU instruction per
    SIMD every four clocks, and a second one from another wave in the same
    slot (dual issue, counted by SQ_ACTIVE_INST_VALU2): 256 CUs x 4 SIMDs x
    16 lanes x 2.4 GHz = 39.3 T lane-operations/s single issue, 78.6 T with
    dual issue in every slot; both fractions are reported.  The section also
    times the advance of every stream by its own random 128-bit distance."""
    name, seed, S, N = "xoshiro256++", 42, 1 << 20, 1024
    buf = P.output_empty((S, N), torch.int64)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    acc = {"position": 0.0, "long_jump": 0.0, "generate": 0.0, "advance_each": 0.0}
    # one random 128-bit distance per stream, for the per-stream advance
    g = torch.Generator().manual_seed(7)
    dist = torch.randint(-2**63, 2**63 - 1, (S, 2), generator=g, dtype=torch.int64).cuda()
    with P.Streams(name, seed, S) as h:
        for rep in range(reps + 1):
            e = [ev() for _ in range(4)]
            e[0].record(stream)
            P.slrng_streams_seed(h.h, seed, stream)
            e[1].record(stream)
            P.slrng_streams_jump(h.h, P.SLRNG_LONG_JUMP, stream)
            e[2].record(stream)
            P.slrng_generate(h.h, P.SLRNG_U64, N, buf.data_ptr(), N, stream)
            e[3].record(stream)
            P.slrng_streams_advance_each(h.h, dist.data_ptr(), stream)
            e4 = ev()
            e4.record(stream)
            torch.cuda.synchronize()
            if rep:  # the first round is a warm-up
                acc["position"] += e[0].elapsed_time(e[1]) / reps
                acc["long_jump"] += e[1].elapsed_time(e[2]) / reps
                acc["generate"] += e[2].elapsed_time(e[3]) / reps
                acc["advance_each"] += e[3].elapsed_time(e4) / reps
    del buf, dist
    torch.cuda.empty_cache()
    jump_s = acc["long_jump"] * 1e-3
    gbs = 8 * S * N / (acc["generate"] * 1e-3) / 1e9
    out = {"generator": name, "streams": S, "outputs_per_stream": N,
           "position_ms": round(acc["position"], 4),
           "positioned_streams_per_s": S / (acc["position"] * 1e-3),
           "long_jump_ms": round(acc["long_jump"], 4),
           "jumps_per_s": S / jump_s,
           "ns_per_jump_aggregate": round(jump_s / S * 1e9, 4),
           "advance_each_ms": round(acc["advance_each"], 4),
           "advance_each_per_s": S / (acc["advance_each"] * 1e-3),
           "generate_ms": round(acc["generate"], 4), "generate_GBs": round(gbs, 1),
           "generate_frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
    valu = profiled_valu()
    if valu:
        single, dual = 256 * 4 * 16 * 2.4e9, 256 * 4 * 32 * 2.4e9
        for label, key, ms in (("position", "k_position", acc["position"]),
                               ("long_jump", "k_jump", acc["long_jump"]),
                               ("advance_each", "k_advance_each", acc["advance_each"])):
            if key in valu:
                rate = valu[key] * 64 / (ms * 1e-3)
                out[f"{label}_valu"] = {"insts_per_launch": valu[key], "lane_ops_per_s": rate,
                                        "frac_single_issue": round(rate / single, 4),
                                        "frac_dual_issue": round(rate / dual, 4)}
    return out


SWEEP32 = ["xoroshiro64*", "xoroshiro64**", "xoshiro128+", "xoshiro128++", "xoshiro128**"]


def gen32_section(P, torch, stream, rounds: int = 2) -> dict:
    """The 32-bit generators (Section "The 32-bit case"): for each of the five,
    65,536 streams (seed 1) x 131,072 outputs as uint32 and as floats from the
    upper 24 bits: 32 GiB per launch, the same bytes as a 64-bit sweep launch.
    HIP events around every launch; average write bandwidth per generator."""
    S, N = 65536, 131072
    buf = P.output_empty((S, N), torch.int32)
    hs = {name: P.Streams(name, 1, S) for name in SWEEP32}
    per = {name: [] for name in SWEEP32}
    for r in range(rounds + 1):
        for name in SWEEP32:
            h = hs[name]
            for kind in (P.SLRNG_U32, P.SLRNG_F32):
                h.seed(1, stream)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                P.slrng_generate(h.h, kind, N, buf.data_ptr(), N, stream)
                e1.record(stream)
                torch.cuda.synchronize()
                if r:  # the first pass is a warm-up
                    per[name].append(e0.elapsed_time(e1))
    for h in hs.values():
        h.close()
    del buf
    torch.cuda.empty_cache()
    nbytes = 4 * S * N
    gbs = {name: round(nbytes / (sum(v) / len(v) * 1e-3) / 1e9, 1) for name, v in per.items()}
    allv = [t for v in per.values() for t in v]
    avg = nbytes / (sum(allv) / len(allv) * 1e-3) / 1e9
    return {"streams": S, "outputs_per_stream": N, "bytes_per_launch": nbytes,
            "outputs_per_s": avg * 1e9 / 4, "GBs": round(avg, 1),
            "frac_of_hbm_peak": round(avg / HBM_PEAK_GBS, 4), "GBs_per_generator": gbs}


def lincomp_section(P, torch, stream, reps: int = 3) -> dict:
    """On-device linearity checks: Berlekamp-Massey on bit 0 of 2n outputs of
    each of 65,536 xoshiro256+ streams (complexity n = 256 expected, table
    tab:plusdeg), with the time per check and the streams checked per second;
    then the maximum-dimension equidistribution test of Section
    "Equidistribution" (the rank of an n x n matrix over Z/2Z, one
    workgroup) for every word of xoroshiro1024 (n = 1,024) and of
    xoshiro256, with the time per word."""
    name, S, nbits = "xoshiro256+", 65536, 512
    with P.Streams(name, 1, S) as h:
        h.linear_complexity(0, nbits, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            lc = h.linear_complexity(0, nbits, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        ok = bool((lc == 256).all().item())
    out = {"generator": name, "streams": S, "bit": 0, "nbits": nbits, "ms": round(ms, 3),
           "streams_per_s": S / (ms * 1e-3), "all_equal_n": ok}
    ed = {}
    for gen, k, n in (("xoroshiro1024+", 16, 1024), ("xoshiro256+", 4, 256)):
        ranks = torch.zeros(k, dtype=torch.int32, device="cuda")
        P.slrng_equidistribution_rank(gen, 0, k, ranks.data_ptr(), stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for word in range(k):
            P.slrng_equidistribution_rank(gen, word, k, ranks.data_ptr() + 4 * word, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ed[gen] = {"n": n, "ms_per_word": round(e0.elapsed_time(e1) / k, 3),
                   "all_words_full_rank": bool((ranks == n).all().item())}
    out["equidistribution_rank"] = ed
    return out


def serving_section(P, seconds: float) -> dict:
    """The serving workload: Poisson arrivals at 20,000 requests/s on 4,096
    device-resident xoshiro256** streams (seed 42), sizes log-uniform in
    64 B .. 256 MiB, admission under a 16 GB output budget, replayed in real
    time; latency runs from each request's scheduled arrival to the
    completion of its iteration.  Three operating points on the same trace:
    continuous batching with the default options (an iteration starts as soon
    as a slot is free), the plain form (one request per iteration), and the
    throughput operating points of continuous batching (iterations gather up
    to 8 ms or 2 GiB, and 16 ms or 4 GiB, of requests), whose kernel-active
    time is compared with the HBM roof: kernel_active_frac_of_hbm_peak = bytes
    written / union of the generation kernels' device intervals / 8 TB/s."""
    from paper_1805_01407_amd import workloads as W
    tr = W.serve_trace(seconds=seconds)
    out = {"seconds": seconds, "requests": int(tr["t"].size), "outputs": int(tr["n"].sum()),
           "offered_GBs": round(8 * float(tr["n"].sum()) / seconds / 1e9, 1)}
    for label, kw in (("continuous_batching", {}), ("plain_per_request", {"max_batch": 1}),
                      ("continuous_batching_window_8ms", {"window_us": 8000,
                                                          "window_bytes": 2 << 30}),
                      ("continuous_batching_window_16ms", {"window_us": 16000,
                                                           "window_bytes": 4 << 30})):
        sv = P.slrng_server_create(P.slrng_server_default_opts(**kw))
        try:
            t0 = time.perf_counter()
            P.slrng_server_replay(sv, tr["t"], tr["stream"], tr["n"], tr["kind"])
            wall = time.perf_counter() - t0
            st = P.slrng_server_get_stats(sv)
        finally:
            P.slrng_server_destroy(sv)
        log(f"bench: serving replay ({label}) done in {wall:.1f} s")
        kgbs = 8 * st["outputs"] / max(st["kernel_s"], 1e-12) / 1e9
        out[label] = {"options": kw, "latency_p50_us": round(st["p50_us"], 1),
                      "latency_p99_us": round(st["p99_us"], 1),
                      "latency_max_us": round(st["max_us"], 1), "outputs_per_s": st["outputs"] / wall,
                      "wall_s": round(wall, 3), "iterations": st["iterations"],
                      "mean_batch": round(st["mean_batch"], 2), "max_inflight": st["max_inflight"],
                      "peak_reserved_GB": round(st["peak_reserved_bytes"] / 1e9, 2),
                      "kernel_active_s": round(st["kernel_s"], 4),
                      "kernel_active_GBs": round(kgbs, 1),
                      "kernel_active_frac_of_hbm_peak": round(kgbs / HBM_PEAK_GBS, 4),
                      "completed": st["completed"], "failed": st["failed"]}
    return out


SECTIONS = ["sweep", "small", "jump", "gen32", "lincomp", "batch", "serve", "cpu"]


def sweep_section(P, torch, stream, S: int, N: int, steps: int, warmup: int) -> dict:
    """The headline: `steps` timed steps of the full family sweep (after
    `warmup` untimed ones), HIP events around every generation launch, then
    the fill kernel's rate into each of the two sweep buffers and a copy of
    known size (for scaling the hardware memory counters)."""
    placement = placement_section(P, torch, stream, S, N)
    # output memory from the library's allocator: virtually contiguous, its
    # physical pages spread over the HBM (compact placement caps stores lower)
    buf_u = P.output_empty((S, N), torch.int64)
    buf_f = P.output_empty((S, N), torch.float64)
    hs = {name: P.Streams(name, 1, S) for name in SWEEP}
    torch.cuda.synchronize()

    gen_events = []  # (start, end) around every generation launch

    def step(k: int, record: bool):
        seed = (k % 8) + 1
        for name in SWEEP:
            h = hs[name]
            for kind, buf in ((P.SLRNG_U64, buf_u), (P.SLRNG_F64, buf_f)):
                h.seed(seed)
                if record:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                P.slrng_generate(h.h, kind, N, buf.data_ptr(), N, stream)
                if record:
                    e1.record(stream)
                    gen_events.append((e0, e1))

    for k in range(warmup):
        step(k, False)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for k in range(steps):
        step(k, True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    outputs_per_step = len(SWEEP) * 2 * S * N
    durs = [a.elapsed_time(b) for a, b in gen_events]  # ms
    avg_ms = sum(durs) / len(durs)
    bytes_per_launch = 8 * S * N

    # write ceiling of each sweep buffer: the fill kernel (16-byte stores,
    # grid-stride), same bytes, into the same memory
    def fill_rate(buf, reps: int = 5) -> float:
        for _ in range(2):
            P.slrng_calib_write(buf.data_ptr(), bytes_per_launch, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            P.slrng_calib_write(buf.data_ptr(), bytes_per_launch, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return round(bytes_per_launch * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)

    ceilings = {"u64_buffer": fill_rate(buf_u), "f64_buffer": fill_rate(buf_f)}

    # launch j of the timed steps: generator (j // 2) % 8, kind j % 2
    per_variant, per_kind = {}, {}
    for i, name in enumerate(SWEEP):
        ds = [durs[j] for j in range(len(durs)) if (j // 2) % len(SWEEP) == i]
        per_variant[name] = round(bytes_per_launch / (sum(ds) / len(ds) * 1e-3) / 1e9, 1)
        per_kind[name] = {}
        for kk, label in ((0, "u64"), (1, "f64")):
            dk = [durs[j] for j in range(len(durs)) if (j // 2) % len(SWEEP) == i and j % 2 == kk]
            per_kind[name][label] = round(bytes_per_launch / (sum(dk) / len(dk) * 1e-3) / 1e9, 1)
    per_buffer = {}
    for kk, label in ((0, "u64_buffer"), (1, "f64_buffer")):
        dk = [durs[j] for j in range(len(durs)) if j % 2 == kk]
        per_buffer[label] = round(bytes_per_launch / (sum(dk) / len(dk) * 1e-3) / 1e9, 1)

    # a plain copy of known size, for scaling the hardware memory counters
    copy_bytes = 4 << 30
    P.slrng_calib_copy(buf_f.data_ptr(), buf_u.data_ptr(), copy_bytes, stream)
    torch.cuda.synchronize()

    for h in hs.values():
        h.close()
    del buf_u, buf_f
    torch.cuda.empty_cache()
    return {"dt": dt, "outputs": outputs_per_step * steps, "avg_ms": avg_ms,
            "achieved": bytes_per_launch / (avg_ms * 1e-3) / 1e9, "ceilings": ceilings,
            "per_buffer": per_buffer, "placement": placement, "per_variant": per_variant,
            "per_kind": per_kind}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--streams", type=int, default=65536)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-requests section")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving trace (0 skips the serving section)")
    ap.add_argument("--cpu-streams", type=int, default=512, help="streams per oracle batch")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma-separated sections to run (default: all): " + ",".join(SECTIONS))
    ap.add_argument("--batch-forms", default="graph,plain",
                    help="forms of the batched section: graph (one persistent launch) and/or plain")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (the streams are independent and "
              "would shard by stream range with no exchange); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    sections = set(args.sections.split(","))
    unknown = sections - set(SECTIONS)
    if unknown:
        print(f"bench.py: unknown sections {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)
    if args.no_cpu:
        sections.discard("cpu")
    if args.no_batch:
        sections.discard("batch")
    if args.serve_seconds <= 0:
        sections.discard("serve")

    import torch

    import paper_1805_01407_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    S, N = args.streams, args.n
    stream = torch.cuda.current_stream()
    sw = sweep_section(P, torch, stream, S, N, args.steps, args.warmup) if "sweep" in sections else None
    small = small_case_section(P, torch, stream) if "small" in sections else None
    positioned = positioning_section(P, torch, stream) if "jump" in sections else None
    gen32 = gen32_section(P, torch, stream) if "gen32" in sections else None
    lincomp = lincomp_section(P, torch, stream) if "lincomp" in sections else None
    batched = batched_section(P, torch, stream, forms=args.batch_forms.split(",")) \
        if "batch" in sections else None
    served = serving_section(P, args.serve_seconds) if "serve" in sections else None

    cpu = cpu_baseline(args.cpu_streams, N, args.cpu_seconds) if "cpu" in sections else None
    if cpu is not None:
        cpu["per_config"] = cpu_per_config()

    out = {
        "metric": "64-bit outputs/s (uint64 + [0,1) doubles), full family sweep",
        "value": sw["outputs"] / sw["dt"] if sw else None,
        "unit": "outputs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sw["dt"] / args.steps * 1e3 if sw else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "full family sweep: 8 generators x 65,536 streams x 65,536 "
                               "outputs, uint64 + doubles, seeds 1..8",
                   "streams": S, "outputs_per_stream": N, "generators": SWEEP},
        "roofline": {"bound": "hbm", "achieved": sw["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": sw["achieved"] / HBM_PEAK_GBS,
                     "traffic": profiled_traffic()} if sw else None,
        "write_ceiling_GBs": sw["ceilings"] if sw else None,
        "gen_GBs_per_buffer": sw["per_buffer"] if sw else None,
        "placement": sw["placement"] if sw else None,
        "gen_GBs_per_generator": sw["per_variant"] if sw else None,
        "gen_GBs_per_generator_kind": sw["per_kind"] if sw else None,
        "small_case": small,
        "jump_ahead_at_scale": positioned,
        "generators_32bit": gen32,
        "linearity_check": lincomp,
        "batched_requests": batched,
        "serving": served,
        "cpu_baseline": cpu,
    }
    if sorted(sections) != sorted(SECTIONS):
        out["sections"] = sorted(sections)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

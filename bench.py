"""Throughput benchmark: the full-family sweep of 64-bit generation on one GPU.

Workload (one step): for each of the eight generators xoroshiro128+/++/**,
xoshiro256+/++/**, xoshiro512** and xoroshiro1024**, position 65,536 streams
from a seed (SplitMix64 fill, stream i jumped i times by 2^(n/2)), generate
65,536 uint64 outputs per stream (32 GiB, stream-major), re-position the same
streams and generate the same outputs as [0,1) doubles (another 32 GiB).
Step k uses seed (k mod 8) + 1, so 8 steps cover seeds 1..8.  Inputs are the
seeds alone; all outputs stay in HBM.

Prints one JSON line (rank 0).  `value` = outputs (uint64 + double) per
second over the timed steps; `roofline` describes the generation kernel.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SWEEP = ["xoroshiro128+", "xoroshiro128++", "xoroshiro128**", "xoshiro256+", "xoshiro256++",
         "xoshiro256**", "xoshiro512**", "xoroshiro1024**"]
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(S_sample: int, N: int, seconds_cap: float = 30.0) -> dict:
    """The oracle (plain serial C, threaded over streams) on a bounded sample of
    the same workload: for each of the eight generators, S_sample streams of
    the seed-1 chain, N outputs each, as uint64 and as doubles."""
    import oracle as O
    nth = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nth = min(nth, 16)
    outs = 0
    t0 = time.perf_counter()
    for name in SWEEP:
        g = O.GEN64[name]
        st = O.stream_chain(g, 1, S_sample)
        O.generate_many(g, st, N, kind="u64", nthreads=nth)
        O.generate_many(g, st, N, kind="f64", nthreads=nth)
        outs += 2 * S_sample * N
        if time.perf_counter() - t0 > seconds_cap:
            break
    dt = time.perf_counter() - t0
    return {"value": outs / dt, "unit": "outputs/s", "cores": nth, "kind": "oracle",
            "sample": f"8 generators x {S_sample} streams x {N} outputs x (u64 + f64), "
                      f"seed 1, stream chain included; {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--streams", type=int, default=65536)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-streams", type=int, default=256)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (the streams are independent and "
              "would shard by stream range with no exchange); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1805_01407_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    S, N = args.streams, args.n
    buf_u = torch.empty((S, N), dtype=torch.int64, device=dev)
    buf_f = torch.empty((S, N), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
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

    for k in range(args.warmup):
        step(k, False)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    outputs_per_step = len(SWEEP) * 2 * S * N
    value = outputs_per_step * args.steps / dt
    durs = [a.elapsed_time(b) for a, b in gen_events]  # ms
    avg_ms = sum(durs) / len(durs)
    bytes_per_launch = 8 * S * N
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9

    # write ceiling of the same store path, same size
    for _ in range(2):
        P.slrng_calib_write(buf_u.data_ptr(), bytes_per_launch, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    reps = 5
    for _ in range(reps):
        P.slrng_calib_write(buf_u.data_ptr(), bytes_per_launch, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ceiling = bytes_per_launch * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9

    per_variant = {}
    for i, name in enumerate(SWEEP):
        ds = [durs[j] for j in range(len(durs)) if (j // 2) % len(SWEEP) == i]
        per_variant[name] = round(bytes_per_launch / (sum(ds) / len(ds) * 1e-3) / 1e9, 1)

    cpu = None if args.no_cpu else cpu_baseline(args.cpu_streams, N)
    for h in hs.values():
        h.close()

    out = {
        "metric": "64-bit outputs/s (uint64 + [0,1) doubles), full family sweep",
        "value": value,
        "unit": "outputs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "full family sweep: 8 generators x 65,536 streams x 65,536 "
                               "outputs, uint64 + doubles, seeds 1..8",
                   "streams": S, "outputs_per_stream": N, "generators": SWEEP},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "write_ceiling_GBs": ceiling,
        "gen_GBs_per_generator": per_variant,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

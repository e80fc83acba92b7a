"""Seeded synthetic workloads (inputs only: request lists and arrival traces).

This module holds none of the generators' arithmetic; it only draws request
parameters with numpy's PCG64 so that the library and the oracle can be fed
the same inputs.

batch_requests: the batched-requests workload — `count` requests, generator
uniform over the eight swept variants, length floor(2^(24 U)) with U uniform
in [0, 1) (log-uniform in [1, 2^24)), doubles with probability 0.3, origin
seed r + 1, start position 0.  Outputs are laid out in one arena, each request
aligned to 256 bytes.

serve_trace: the serving workload — Poisson arrivals at `rate` requests per
second for `seconds`, each on a stream uniform in [0, streams), asking for
floor(bytes / 8) uint64 outputs with bytes log-uniform in [64 B, 256 MiB].
"""
from __future__ import annotations

import numpy as np

SWEEP = ["xoroshiro128+", "xoroshiro128++", "xoroshiro128**", "xoshiro256+", "xoshiro256++",
         "xoshiro256**", "xoshiro512**", "xoroshiro1024**"]
VARIANT_IDS = {"xoroshiro128+": 0, "xoroshiro128++": 1, "xoroshiro128**": 2, "xoshiro256+": 3,
               "xoshiro256++": 4, "xoshiro256**": 5, "xoshiro512**": 8, "xoroshiro1024**": 11}


def batch_requests(count: int = 10000, seed: int = 4, max_log2: int = 24, p_double: float = 0.3):
    """Returns dict of arrays: variant ids, kind (0 u64 / 1 f64), origin seed,
    start, n, and the element offset of each request in the output arena,
    plus the arena size in elements."""
    rng = np.random.default_rng(seed)
    vi = rng.integers(0, len(SWEEP), count)
    variant = np.array([VARIANT_IDS[SWEEP[i]] for i in vi], dtype=np.int32)
    n = np.floor(2.0 ** (max_log2 * rng.random(count))).astype(np.uint64)
    n = np.maximum(n, 1)
    kind = (rng.random(count) < p_double).astype(np.int32)
    seeds = np.arange(1, count + 1, dtype=np.uint64)
    start = np.zeros(count, dtype=np.uint64)
    # 256-byte aligned offsets (32 elements of 8 bytes)
    padded = (n + np.uint64(31)) // np.uint64(32) * np.uint64(32)
    offset = np.zeros(count, dtype=np.uint64)
    offset[1:] = np.cumsum(padded)[:-1]
    arena = int(padded.sum())
    return {"variant": variant, "kind": kind, "seed": seeds, "start": start, "n": n,
            "offset": offset, "arena_elems": arena}


def serve_trace(rate: float = 20000.0, seconds: float = 60.0, streams: int = 4096,
                min_bytes: int = 64, max_bytes: int = 1 << 28, seed: int = 5,
                p_double: float = 0.0):
    """Returns dict of arrays: arrival time (s), stream id, n, kind."""
    rng = np.random.default_rng(seed)
    count = int(rate * seconds * 1.2) + 16
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    m = t.size
    sid = rng.integers(0, streams, m).astype(np.uint32)
    lo, hi = np.log(min_bytes), np.log(max_bytes)
    nbytes = np.exp(lo + (hi - lo) * rng.random(m))
    n = np.maximum(np.floor(nbytes / 8.0), 1).astype(np.uint64)
    kind = (rng.random(m) < p_double).astype(np.int32)
    return {"t": t, "stream": sid, "n": n, "kind": kind}

"""Autotuner for the launch shapes of slrng on the current GPU.

It times the library's own kernels through the C ABI (HIP events on the
current torch stream) and keeps the fastest shape:

* ``slrng_generate``, per variant and kind: LDS tile (16 or 32 outputs per lane
  per round), wave target (how finely short, wide requests are split into
  jumped slots) and the number of staggered slot-boundary classes, timed on
  the 65,536 x 65,536 sweep in memory from slrng_output_alloc, with plain or
  nontemporal output stores; then the shortest slot (min_chunk), which only
  matters when there are few streams, by the latency of a 1,024-stream
  launch of 4,096 outputs per stream;
* batched generation: LDS tile, persistent grid (waves per CU) and lane-chunk
  length per variant, on a seeded batched workload.

The result is a JSON file keyed by GPU architecture; the binding applies it
when it loads the library (``apply``).  The launch shape never changes any
output value, only speed.

    python -m paper_1805_01407_amd.autotune [--out FILE] [--quick] [--only generate|batch|min_chunk]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "tuning.json")


def _arch() -> str | None:
    import torch
    if not torch.cuda.is_available():
        return None
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _time_ms(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune_generate(variants, S=65536, N=65536, reps=5, quick=False, log=print) -> dict:
    """64-bit generators: S x N outputs; 32-bit ones: S x 2N (the same bytes)."""
    import torch
    from . import binding as B
    buf = B.output_empty((S, N), torch.int64)  # the memory large outputs live in
    out = {}
    waves = (4096, 8192) if quick else (2048, 4096, 8192, 16384)
    skews = (1, 4) if quick else (1, 4, 16)
    for name in variants:
        w32 = name in B.VARIANTS32
        tiles = (64,) if w32 else (16, 32)
        n_out = 2 * N if w32 else N
        kinds = (B.SLRNG_U32, B.SLRNG_F32) if w32 else (B.SLRNG_U64, B.SLRNG_F64)
        for kind in kinds:
            best = None
            with B.Streams(name, 1, S) as h:
                for tile in tiles:
                    for tw in waves:
                        for sk in skews:
                            for store in (0, 1):
                                B.slrng_set_tuning(name, kind, tile, tw, 1024, sk, store)
                                ms = _time_ms(lambda: B.slrng_generate(h.h, kind, n_out, buf.data_ptr(),
                                                                       n_out), reps)
                                if best is None or ms < best[0]:
                                    best = (ms, {"tile": tile, "target_waves": tw, "skew": sk,
                                                 "min_chunk": 1024, "store": store})
            gbs = 8 * S * N / (best[0] * 1e-3) / 1e9
            cfg = best[1]
            cfg["min_chunk"], lat_us = _best_min_chunk(name, kind, cfg, reps)
            log(f"generate {name} kind {kind}: {cfg} {gbs:.0f} GB/s; 1,024 streams: {lat_us:.1f} us")
            out[f"{name}/{kind}"] = dict(cfg, GBs=round(gbs, 1))
            B.slrng_set_tuning(name, kind, **{k: cfg[k] for k in
                                              ("tile", "target_waves", "min_chunk", "skew", "store")})
    del buf
    torch.cuda.empty_cache()
    return out


def _best_min_chunk(name, kind, cfg, reps=9):
    """Shortest slot for a launch shape: the latency of 1,024 streams x 4,096
    outputs (8,192 for 32-bit generators) in ordinary device memory, where
    outputs of that size live (the sweep's slots are far longer than any
    candidate, so its timing does not change).  Returns (min_chunk, us)."""
    import torch
    from . import binding as B
    small_n = 2 * 4096 if name in B.VARIANTS32 else 4096
    buf = torch.empty((1024, small_n), dtype=torch.int64, device="cuda")
    lat = []
    with B.Streams(name, 1, 1024) as h:
        for mc in (256, 512, 1024):
            B.slrng_set_tuning(name, kind, cfg["tile"], cfg["target_waves"], mc, cfg["skew"],
                               cfg.get("store", 0))
            lat.append((_time_ms(lambda: B.slrng_generate(h.h, kind, small_n, buf.data_ptr(), small_n),
                                 reps), mc))
    ms, mc = min(lat)
    return mc, ms * 1e3


def tune_min_chunk(data: dict, log=print) -> dict:
    """Re-tune min_chunk alone for every saved (generator, kind) entry."""
    from . import binding as B
    for key, cfg in data.items():
        name, kind = key.rsplit("/", 1)
        cfg["min_chunk"], lat_us = _best_min_chunk(name, int(kind), cfg)
        B.slrng_set_tuning(name, int(kind), cfg["tile"], cfg["target_waves"], cfg["min_chunk"],
                           cfg["skew"], cfg.get("store", 0))
        log(f"min_chunk {key}: {cfg['min_chunk']} ({lat_us:.1f} us)")
    return data


def tune_batch(reps=5, quick=False, log=print) -> dict:
    import torch
    from . import binding as B
    from . import workloads as W
    w = W.batch_requests()
    arena = B.output_empty((w["arena_elems"],), torch.int64)
    reqs = B.make_requests(w["variant"], w["kind"], w["seed"], w["start"], w["n"],
                           arena.data_ptr() + 8 * w["offset"])
    total = int(w["n"].sum())
    heavy = {9, 10, 11, 13}  # 16-word engine: longer chunks amortise its jump
    best = None
    for tile in (16, 32):
        for wpc in ((8, 12) if quick else (8, 12, 16)):
            for light in ((8192, 16384) if quick else (4096, 8192, 16384)):
                for hv in ((32768, 65536) if quick else (16384, 32768, 65536)):
                    chunk = {v: (hv if v in heavy else light) for v in range(B.NUM_VARIANTS)}
                    opts = B.slrng_batch_default_opts(mode=B.SLRNG_BATCH_GRAPH, tile=tile,
                                                      waves_per_cu=wpc, chunk=chunk)
                    b = B.slrng_batch_plan(reqs, opts)
                    try:
                        ms = _time_ms(lambda: B.slrng_batch_launch(b), reps)
                    finally:
                        B.slrng_batch_destroy(b)
                    if best is None or ms < best[0]:
                        best = (ms, {"tile": tile, "waves_per_cu": wpc, "chunk_light": light,
                                     "chunk_heavy": hv})
    gbs = 8 * total / (best[0] * 1e-3) / 1e9
    log(f"batch: {best[1]} {gbs:.0f} GB/s")
    del arena
    torch.cuda.empty_cache()
    return dict(best[1], GBs=round(gbs, 1))


def load(path: str = DEFAULT_PATH) -> dict | None:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def apply(path: str = DEFAULT_PATH) -> bool:
    """Apply saved tuning for this GPU's architecture (no-op without a GPU or a
    matching entry).  Returns True if something was applied."""
    data = load(path)
    arch = _arch() if data else None
    if not data or not arch or arch not in data:
        return False
    from . import binding as B
    t = data[arch]
    for key, cfg in t.get("generate", {}).items():
        name, kind = key.rsplit("/", 1)
        B.slrng_set_tuning(name, int(kind), cfg["tile"], cfg["target_waves"], cfg["min_chunk"],
                           cfg["skew"], cfg.get("store", 0))
    if "batch" in t:
        B.set_batch_defaults(t["batch"])
    return True


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--only", choices=["generate", "batch", "min_chunk"], default=None)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    from . import binding as B
    B.lib()
    arch = _arch()
    if arch is None:
        print("autotune: no GPU", file=sys.stderr)
        return 2
    data = load(args.out) or {}
    entry = data.get(arch, {})
    if args.only in (None, "generate"):
        entry["generate"] = tune_generate(B.VARIANTS + B.VARIANTS32, quick=args.quick)
    if args.only == "min_chunk":
        entry["generate"] = tune_min_chunk(entry.get("generate", {}))
    if args.only in (None, "batch"):
        entry["batch"] = tune_batch(quick=args.quick)
    data[arch] = entry
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(f"autotune: wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())

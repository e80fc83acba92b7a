"""ctypes binding of libslrng.so (include/slrng.h).  Argument marshalling only:
every computation happens in the library.

Functions named ``slrng_*`` mirror the C ABI one to one and raise
``SlrngError`` on a negative return code.  ``Streams`` is a small object
wrapper over a stream handle that allocates output tensors with torch.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libslrng.so")

SLRNG_U64, SLRNG_F64, SLRNG_U32, SLRNG_F32 = 0, 1, 2, 3
SLRNG_JUMP, SLRNG_LONG_JUMP = 0, 1

VARIANTS = [
    "xoroshiro128+", "xoroshiro128++", "xoroshiro128**",
    "xoshiro256+", "xoshiro256++", "xoshiro256**",
    "xoshiro512+", "xoshiro512++", "xoshiro512**",
    "xoroshiro1024+", "xoroshiro1024++", "xoroshiro1024**",
    "xoroshiro128*", "xoroshiro1024*",
]
# 32-bit generators (ids 14 .. 18; uint32 / float outputs)
VARIANTS32 = ["xoroshiro64*", "xoroshiro64**", "xoshiro128+", "xoshiro128++", "xoshiro128**"]
VARIANT_IDS = {name: i for i, name in enumerate(VARIANTS + VARIANTS32)}
_ERRNAMES = {-1: "EINVAL", -2: "ERANGE", -3: "ENOMEM", -4: "EZEROSTATE", -5: "EAGAIN",
             -6: "EHIP", -7: "ENOTIMPL"}


class SlrngError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        self.name = _ERRNAMES.get(code, str(code))
        msg = f"{where}: {self.name}"
        if code == -6:
            msg += f" (HIP error {_lib.slrng_last_hip_error()})" if _lib is not None else ""
        super().__init__(msg)


class _Tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("target_waves", ctypes.c_int32),
                ("skew", ctypes.c_int32), ("store", ctypes.c_int32),
                ("min_chunk", ctypes.c_uint64)]


NUM_VARIANTS = 14
SLRNG_BATCH_GRAPH, SLRNG_BATCH_PERSISTENT, SLRNG_BATCH_PLAIN = 0, 1, 2
SLRNG_BATCH_STATIC_SCRATCH_BYTES = 32 << 20  # the fixed device array of slrng_batch_run_static

# slrng_request as a numpy record (40 bytes, the C layout)
REQUEST_DTYPE = np.dtype([("variant", "<i4"), ("kind", "<i4"), ("seed", "<u8"), ("start", "<u8"),
                          ("n", "<u8"), ("dev_out", "<u8")])


class _BatchOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("chunk", ctypes.c_uint64 * NUM_VARIANTS)]


SLRNG_SUBMIT_NONBLOCK, SLRNG_SUBMIT_AUTORELEASE = 1, 2


class _ServerOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("chunk", ctypes.c_uint64), ("n_streams", ctypes.c_uint32),
                ("variant", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("inflight", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("window_us", ctypes.c_int32),
                ("min_chunk", ctypes.c_int32), ("window_bytes", ctypes.c_uint64),
                ("arena_plain", ctypes.c_int32), ("store", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in
                ("submitted", "completed", "failed", "rejected", "outputs", "iterations",
                 "max_inflight", "max_batch", "peak_reserved_bytes", "reserved_bytes")] + \
               [(f, ctypes.c_double) for f in
                ("wall_s", "busy_s", "mean_batch", "p50_us", "p99_us", "max_us", "kernel_s")]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libslrng.so (torch first, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_1805_01407_amd.build`")
    L = ctypes.CDLL(_LIB_PATH)
    vp, u64, u64p = ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)
    i32 = ctypes.c_int
    sig = {
        "slrng_version": ([], i32),
        "slrng_strerror": ([i32], ctypes.c_char_p),
        "slrng_last_hip_error": ([], i32),
        "slrng_state_words": ([i32], i32),
        "slrng_charpoly": ([i32, u64p, i32], i32),
        "slrng_jump_poly": ([i32, u64p, i32, u64p, i32], i32),
        "slrng_jump_poly_device": ([i32, vp, u64, vp, vp], i32),
        "slrng_streams_create": ([i32, u64, u64, vp, ctypes.POINTER(vp)], i32),
        "slrng_streams_create_from_states": ([i32, u64p, u64, vp, ctypes.POINTER(vp)], i32),
        "slrng_streams_seed": ([vp, u64, vp], i32),
        "slrng_streams_count": ([vp, u64p], i32),
        "slrng_streams_variant": ([vp, ctypes.POINTER(i32)], i32),
        "slrng_streams_jump": ([vp, i32, vp], i32),
        "slrng_streams_advance": ([vp, u64, u64, vp], i32),
        "slrng_streams_advance_each": ([vp, vp, vp], i32),
        "slrng_linear_complexity": ([vp, i32, ctypes.c_uint32, vp, vp], i32),
        "slrng_equidistribution_rank": ([i32, i32, i32, vp, vp], i32),
        "slrng_gf2_rank": ([vp, ctypes.c_uint32, ctypes.c_uint32, vp, vp], i32),
        "slrng_generate": ([vp, i32, u64, vp, u64, vp], i32),
        "slrng_get_state": ([vp, u64p, vp], i32),
        "slrng_set_state": ([vp, u64p, vp], i32),
        "slrng_streams_destroy": ([vp], i32),
        "slrng_get_tuning": ([i32, i32, ctypes.POINTER(_Tuning)], i32),
        "slrng_set_tuning": ([i32, i32, ctypes.POINTER(_Tuning)], i32),
        "slrng_batch_default_opts": ([ctypes.POINTER(_BatchOpts)], i32),
        "slrng_batch_plan": ([vp, ctypes.c_size_t, ctypes.POINTER(_BatchOpts), ctypes.POINTER(vp)], i32),
        "slrng_batch_launch": ([vp, vp], i32),
        "slrng_batch_info": ([vp, u64p, u64p, u64p], i32),
        "slrng_batch_latencies": ([vp, vp, ctypes.POINTER(ctypes.c_double)], i32),
        "slrng_batch_destroy": ([vp], i32),
        "slrng_batch_run": ([vp, ctypes.c_size_t, ctypes.POINTER(_BatchOpts), vp], i32),
        "slrng_batch_run_static": ([vp, ctypes.c_size_t, ctypes.POINTER(_BatchOpts), vp], i32),
        "slrng_server_default_opts": ([ctypes.POINTER(_ServerOpts)], i32),
        "slrng_server_create": ([ctypes.POINTER(_ServerOpts), ctypes.POINTER(vp)], i32),
        "slrng_server_submit": ([vp, ctypes.c_uint32, u64, i32, i32, u64p], i32),
        "slrng_server_poll": ([vp, u64, ctypes.POINTER(vp), u64p], i32),
        "slrng_server_wait": ([vp, u64, ctypes.POINTER(vp), u64p], i32),
        "slrng_server_release": ([vp, u64], i32),
        "slrng_server_drain": ([vp], i32),
        "slrng_server_get_stats": ([vp, ctypes.POINTER(_ServerStats)], i32),
        "slrng_server_reset_stats": ([vp], i32),
        "slrng_server_replay": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint32),
                                 u64p, ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t], i32),
        "slrng_server_destroy": ([vp], i32),
        "slrng_server_advance": ([vp, ctypes.c_uint32, u64, u64], i32),
        "slrng_server_intervals": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    u64, u64p], i32),
        "slrng_calib_write": ([vp, u64, vp], i32),
        "slrng_calib_copy": ([vp, vp, u64, vp], i32),
        "slrng_output_alloc": ([u64, ctypes.POINTER(vp)], i32),
        "slrng_output_free": ([vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    # launch shapes chosen by the autotuner for this GPU, if any were saved
    from . import autotune
    autotune.apply()
    return L


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise SlrngError(rc, where)
    return rc


def _stream(stream) -> int | None:
    """hipStream_t of a torch stream, an int, or the current torch stream."""
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _u64p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _variant(v) -> int:
    return VARIANT_IDS[v] if isinstance(v, str) else int(v)


# ---------------------------------------------------------------- C ABI mirror

def slrng_version() -> int:
    return lib().slrng_version()


def slrng_strerror(err: int) -> str:
    return lib().slrng_strerror(err).decode()


def slrng_last_hip_error() -> int:
    return lib().slrng_last_hip_error()


def slrng_state_words(variant) -> int:
    return _check(lib().slrng_state_words(_variant(variant)), "slrng_state_words")


def _words_to_int(a: np.ndarray) -> int:
    v = 0
    for i, w in enumerate(a.tolist()):
        v |= int(w) << (64 * i)
    return v


def slrng_charpoly(variant) -> int:
    """Characteristic polynomial as a Python int (bit i = coefficient of x^i)."""
    n = 64 * slrng_state_words(variant)
    out = np.zeros(n // 64 + 1, dtype=np.uint64)
    _check(lib().slrng_charpoly(_variant(variant), _u64p(out), out.size), "slrng_charpoly")
    return _words_to_int(out)


def slrng_jump_poly(variant, J: int) -> int:
    """x^J mod p(x) as a Python int."""
    n = 64 * slrng_state_words(variant)
    nj = max(0, (J.bit_length() + 63) // 64)
    jw = np.array([(J >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(max(nj, 1))],
                  dtype=np.uint64)
    out = np.zeros(n // 64, dtype=np.uint64)
    _check(lib().slrng_jump_poly(_variant(variant), _u64p(jw), nj, _u64p(out), out.size),
           "slrng_jump_poly")
    return _words_to_int(out)


def slrng_jump_poly_device(variant, J, stream=None):
    """x^J mod p(x) for each 128-bit distance in J (Python ints, or a CUDA
    int64 tensor of shape (m, 2) holding (low, high) words), computed on the
    device: a CUDA int64 tensor of shape (m, n/64), row j the words of
    x^(J_j) mod p."""
    import torch
    if isinstance(J, torch.Tensor):
        assert J.is_cuda and J.dtype == torch.int64 and J.dim() == 2 and J.shape[1] == 2
        buf = J.contiguous()
    else:
        words = np.zeros((len(J), 2), dtype=np.uint64)
        for i, x in enumerate(J):
            x = int(x)
            words[i, 0] = x & 0xFFFFFFFFFFFFFFFF
            words[i, 1] = (x >> 64) & 0xFFFFFFFFFFFFFFFF
        buf = torch.from_numpy(words.view(np.int64)).cuda()
    m = buf.shape[0]
    nw = (slrng_charpoly(variant).bit_length() - 1) // 64
    out = torch.empty((m, nw), dtype=torch.int64, device=buf.device)
    _check(lib().slrng_jump_poly_device(_variant(variant), buf.data_ptr(), m, out.data_ptr(),
                                        _stream(stream)), "slrng_jump_poly_device")
    if buf is not J:
        # the staging tensor must outlive the queued kernel
        torch.cuda.synchronize()
    return out


def slrng_streams_create(variant, seed: int, n_streams: int, stream=None) -> int:
    h = ctypes.c_void_p()
    _check(lib().slrng_streams_create(_variant(variant), seed & 0xFFFFFFFFFFFFFFFF, n_streams,
                                      _stream(stream), ctypes.byref(h)), "slrng_streams_create")
    return h.value


def slrng_streams_create_from_states(variant, states: np.ndarray, stream=None) -> int:
    st = np.ascontiguousarray(np.asarray(states, dtype=np.uint64))
    k = slrng_state_words(variant)
    S = st.size // k
    h = ctypes.c_void_p()
    _check(lib().slrng_streams_create_from_states(_variant(variant), _u64p(st), S,
                                                  _stream(stream), ctypes.byref(h)),
           "slrng_streams_create_from_states")
    return h.value


def slrng_streams_seed(h: int, seed: int, stream=None) -> None:
    _check(lib().slrng_streams_seed(h, seed & 0xFFFFFFFFFFFFFFFF, _stream(stream)),
           "slrng_streams_seed")


def slrng_streams_count(h: int) -> int:
    n = ctypes.c_uint64()
    _check(lib().slrng_streams_count(h, ctypes.byref(n)), "slrng_streams_count")
    return n.value


def slrng_streams_variant(h: int) -> int:
    v = ctypes.c_int()
    _check(lib().slrng_streams_variant(h, ctypes.byref(v)), "slrng_streams_variant")
    return v.value


def slrng_streams_jump(h: int, jump_kind: int = SLRNG_JUMP, stream=None) -> None:
    _check(lib().slrng_streams_jump(h, jump_kind, _stream(stream)), "slrng_streams_jump")


def slrng_streams_advance(h: int, steps: int, stream=None) -> None:
    _check(lib().slrng_streams_advance(h, (steps >> 64) & 0xFFFFFFFFFFFFFFFF,
                                       steps & 0xFFFFFFFFFFFFFFFF, _stream(stream)),
           "slrng_streams_advance")


def slrng_streams_advance_each(h: int, dev_steps: int, stream=None) -> None:
    """dev_steps: device address of 2 S uint64 words (low, high) per stream."""
    _check(lib().slrng_streams_advance_each(h, dev_steps, _stream(stream)),
           "slrng_streams_advance_each")


def slrng_linear_complexity(h: int, bit: int, nbits: int, dev_lc: int, stream=None) -> None:
    """dev_lc: device address of S uint32 results."""
    _check(lib().slrng_linear_complexity(h, bit, nbits, dev_lc, _stream(stream)),
           "slrng_linear_complexity")


def slrng_equidistribution_rank(variant, word: int, dims: int, dev_rank: int, stream=None) -> None:
    """dev_rank: device address of one uint32 result."""
    _check(lib().slrng_equidistribution_rank(_variant(variant), word, dims, dev_rank, _stream(stream)),
           "slrng_equidistribution_rank")


def slrng_gf2_rank(dev_rows: int, nrows: int, ncols: int, dev_rank: int, stream=None) -> None:
    _check(lib().slrng_gf2_rank(dev_rows, nrows, ncols, dev_rank, _stream(stream)), "slrng_gf2_rank")


def equidistribution_rank(variant, word: int, dims: int | None = None) -> int:
    """The rank of slrng_equidistribution_rank as a Python int (dims defaults
    to k, the maximum dimension); synchronises the current stream."""
    import torch
    if dims is None:
        dims = slrng_state_words(variant)
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    slrng_equidistribution_rank(variant, word, dims, out.data_ptr())
    return int(out.item())


def gf2_rank(bits) -> int:
    """Rank over Z/2Z of a 0/1 matrix (nrows x ncols, both <= 1024), packed
    into the row layout of slrng_gf2_rank; synchronises the current stream."""
    import torch
    a = np.asarray(bits, dtype=np.uint8) & 1
    nrows, ncols = a.shape
    nw = (ncols + 63) // 64
    padded = np.zeros((nrows, nw * 64), dtype=np.uint8)
    padded[:, :ncols] = a
    words = np.packbits(padded, axis=1, bitorder="little").view("<u8").reshape(nrows, nw)
    dev = torch.from_numpy(np.ascontiguousarray(words).view(np.int64)).cuda()
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    slrng_gf2_rank(dev.data_ptr(), nrows, ncols, out.data_ptr())
    return int(out.item())


def slrng_generate(h: int, kind: int, n: int, dev_out: int, ld: int, stream=None) -> None:
    _check(lib().slrng_generate(h, kind, n, dev_out, ld, _stream(stream)), "slrng_generate")


def slrng_get_state(h: int, stream=None) -> np.ndarray:
    """States as an S x k uint64 array (logical order)."""
    S = slrng_streams_count(h)
    k = slrng_state_words(slrng_streams_variant(h))
    out = np.zeros(S * k, dtype=np.uint64)
    _check(lib().slrng_get_state(h, _u64p(out), _stream(stream)), "slrng_get_state")
    return out.reshape(S, k)


def slrng_set_state(h: int, states: np.ndarray, stream=None) -> None:
    st = np.ascontiguousarray(np.asarray(states, dtype=np.uint64))
    _check(lib().slrng_set_state(h, _u64p(st), _stream(stream)), "slrng_set_state")


def slrng_streams_destroy(h: int) -> None:
    _check(lib().slrng_streams_destroy(h), "slrng_streams_destroy")


def slrng_get_tuning(variant, kind: int = SLRNG_U64) -> dict:
    t = _Tuning()
    _check(lib().slrng_get_tuning(_variant(variant), kind, ctypes.byref(t)), "slrng_get_tuning")
    return {"tile": t.tile, "target_waves": t.target_waves, "skew": t.skew,
            "min_chunk": t.min_chunk, "store": t.store}


def slrng_set_tuning(variant, kind: int, tile: int, target_waves: int, min_chunk: int,
                     skew: int = 1, store: int = 0) -> None:
    t = _Tuning(tile, target_waves, skew, store, min_chunk)
    _check(lib().slrng_set_tuning(_variant(variant), kind, ctypes.byref(t)), "slrng_set_tuning")


def slrng_calib_write(dev_out: int, nbytes: int, stream=None) -> None:
    _check(lib().slrng_calib_write(dev_out, nbytes, _stream(stream)), "slrng_calib_write")


def slrng_calib_copy(dev_dst: int, dev_src: int, nbytes: int, stream=None) -> None:
    _check(lib().slrng_calib_copy(dev_dst, dev_src, nbytes, _stream(stream)), "slrng_calib_copy")


def slrng_output_alloc(nbytes: int) -> int:
    """Device memory for large outputs (physical pages spread over the HBM
    from 1 GiB up); returns the device address."""
    p = ctypes.c_void_p()
    _check(lib().slrng_output_alloc(nbytes, ctypes.byref(p)), "slrng_output_alloc")
    return p.value


def slrng_output_free(dev_ptr: int) -> None:
    _check(lib().slrng_output_free(dev_ptr), "slrng_output_free")


class _OutputMemory:
    """One slrng_output_alloc block, exposed through the CUDA array interface
    so that torch wraps it without a copy; freed when the last tensor on it
    is gone."""

    _TYPESTR = {"int64": "<i8", "float64": "<f8", "int32": "<i4", "float32": "<f4", "uint8": "|u1"}

    def __init__(self, shape, dtype_name: str, itemsize: int):
        n = 1
        for s in shape:
            n *= s
        self.ptr = 0
        self.ptr = slrng_output_alloc(max(n, 1) * itemsize)
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": self._TYPESTR[dtype_name],
                                         "data": (self.ptr, False), "version": 2, "strides": None}

    def __del__(self):
        if self.ptr and _lib is not None:
            try:
                _lib.slrng_output_free(self.ptr)
            except Exception:  # interpreter shutdown
                pass
            self.ptr = 0


def output_empty(shape, dtype=None):
    """An uninitialised CUDA tensor on memory from slrng_output_alloc: the
    layout of torch.empty(shape, dtype) (contiguous), with its physical pages
    spread over the HBM for the store bandwidth of large outputs."""
    import torch
    dtype = torch.int64 if dtype is None else dtype
    shape = tuple(int(s) for s in (shape if isinstance(shape, (tuple, list)) else (shape,)))
    name = str(dtype).replace("torch.", "")
    if name not in _OutputMemory._TYPESTR:
        raise ValueError(f"output_empty: unsupported dtype {dtype} "
                         f"(one of {', '.join(sorted(_OutputMemory._TYPESTR))})")
    mem = _OutputMemory(shape, name, torch.empty((), dtype=dtype).element_size())
    return torch.as_tensor(mem, device="cuda")


_batch_defaults: dict = {}
_HEAVY = (9, 10, 11, 13)  # variants of the 16-word engine


def set_batch_defaults(cfg: dict) -> None:
    """Tuned batch defaults: tile, waves_per_cu, chunk_light, chunk_heavy."""
    _batch_defaults.clear()
    _batch_defaults.update(cfg)


def slrng_batch_default_opts(mode: int = SLRNG_BATCH_GRAPH, tile: int | None = None,
                             waves_per_cu: int | None = None, chunk: dict | None = None):
    """Default batch options (the library's, then tuned values if the
    autotuner saved any), with optional overrides (chunk: {variant: length})."""
    o = _BatchOpts()
    _check(lib().slrng_batch_default_opts(ctypes.byref(o)), "slrng_batch_default_opts")
    if _batch_defaults:
        o.tile = _batch_defaults.get("tile", o.tile)
        o.waves_per_cu = _batch_defaults.get("waves_per_cu", o.waves_per_cu)
        for v in range(NUM_VARIANTS):
            key = "chunk_heavy" if v in _HEAVY else "chunk_light"
            if key in _batch_defaults:
                o.chunk[v] = _batch_defaults[key]
    o.mode = mode
    if tile is not None:
        o.tile = tile
    if waves_per_cu is not None:
        o.waves_per_cu = waves_per_cu
    for v, c in (chunk or {}).items():
        o.chunk[_variant(v)] = c
    return o


def make_requests(variant, kind, seed, start, n, dev_out) -> np.ndarray:
    """Pack request fields (scalars or arrays) into slrng_request records."""
    cols = np.broadcast_arrays(np.asarray(variant), np.asarray(kind), np.asarray(seed, dtype=np.uint64),
                               np.asarray(start, dtype=np.uint64), np.asarray(n, dtype=np.uint64),
                               np.asarray(dev_out, dtype=np.uint64))
    r = np.zeros(cols[0].shape, dtype=REQUEST_DTYPE).reshape(-1)
    for name, c in zip(REQUEST_DTYPE.names, cols):
        r[name] = c.reshape(-1)
    return r


def _reqs(reqs: np.ndarray):
    reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
    return reqs, reqs.ctypes.data_as(ctypes.c_void_p), reqs.size


def slrng_batch_plan(reqs: np.ndarray, opts=None) -> int:
    reqs, ptr, n = _reqs(reqs)
    b = ctypes.c_void_p()
    _check(lib().slrng_batch_plan(ptr, n, ctypes.byref(opts) if opts is not None else None,
                                  ctypes.byref(b)), "slrng_batch_plan")
    return b.value


def slrng_batch_launch(b: int, stream=None) -> None:
    _check(lib().slrng_batch_launch(b, _stream(stream)), "slrng_batch_launch")


def slrng_batch_info(b: int) -> dict:
    t, l, o = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().slrng_batch_info(b, ctypes.byref(t), ctypes.byref(l), ctypes.byref(o)),
           "slrng_batch_info")
    return {"tiles": t.value, "lanes": l.value, "outputs": o.value}


def slrng_batch_latencies(b: int, n_requests: int, stream=None) -> np.ndarray:
    """Per-request completion times (ms from launch start) of one timed launch."""
    out = np.zeros(max(n_requests, 1), dtype=np.float64)
    _check(lib().slrng_batch_latencies(b, _stream(stream),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "slrng_batch_latencies")
    return out[:n_requests]


def slrng_batch_destroy(b: int) -> None:
    _check(lib().slrng_batch_destroy(b), "slrng_batch_destroy")


def slrng_batch_run(reqs: np.ndarray, opts=None, stream=None) -> None:
    reqs, ptr, n = _reqs(reqs)
    _check(lib().slrng_batch_run(ptr, n, ctypes.byref(opts) if opts is not None else None,
                                 _stream(stream)), "slrng_batch_run")


def slrng_batch_run_static(reqs: np.ndarray, opts=None, stream=None) -> None:
    reqs, ptr, n = _reqs(reqs)
    _check(lib().slrng_batch_run_static(ptr, n, ctypes.byref(opts) if opts is not None else None,
                                        _stream(stream)), "slrng_batch_run_static")


def slrng_server_default_opts(**overrides):
    o = _ServerOpts()
    _check(lib().slrng_server_default_opts(ctypes.byref(o)), "slrng_server_default_opts")
    for k, v in overrides.items():
        setattr(o, k, _variant(v) if k == "variant" else v)
    return o


def slrng_server_create(opts=None) -> int:
    sv = ctypes.c_void_p()
    _check(lib().slrng_server_create(ctypes.byref(opts) if opts is not None else None,
                                     ctypes.byref(sv)), "slrng_server_create")
    return sv.value


def slrng_server_submit(sv: int, stream_id: int, n: int, kind: int = SLRNG_U64,
                        flags: int = 0) -> int:
    t = ctypes.c_uint64()
    _check(lib().slrng_server_submit(sv, stream_id, n, kind, flags, ctypes.byref(t)),
           "slrng_server_submit")
    return t.value


def slrng_server_poll(sv: int, ticket: int):
    """(status, device pointer, stream position); status 1 done, 0 pending."""
    p, pos = ctypes.c_void_p(), ctypes.c_uint64()
    rc = _check(lib().slrng_server_poll(sv, ticket, ctypes.byref(p), ctypes.byref(pos)),
                "slrng_server_poll")
    return rc, p.value, pos.value


def slrng_server_wait(sv: int, ticket: int):
    """Blocks until done; returns (device pointer, stream position)."""
    p, pos = ctypes.c_void_p(), ctypes.c_uint64()
    _check(lib().slrng_server_wait(sv, ticket, ctypes.byref(p), ctypes.byref(pos)),
           "slrng_server_wait")
    return p.value, pos.value


def slrng_server_release(sv: int, ticket: int) -> None:
    _check(lib().slrng_server_release(sv, ticket), "slrng_server_release")


def slrng_server_drain(sv: int) -> None:
    _check(lib().slrng_server_drain(sv), "slrng_server_drain")


def slrng_server_get_stats(sv: int) -> dict:
    st = _ServerStats()
    _check(lib().slrng_server_get_stats(sv, ctypes.byref(st)), "slrng_server_get_stats")
    return {f: getattr(st, f) for f, _ in _ServerStats._fields_}


def slrng_server_reset_stats(sv: int) -> None:
    _check(lib().slrng_server_reset_stats(sv), "slrng_server_reset_stats")


def slrng_server_replay(sv: int, t_arrival_s, stream_ids, n, kinds) -> None:
    t = np.ascontiguousarray(t_arrival_s, dtype=np.float64)
    sid = np.ascontiguousarray(stream_ids, dtype=np.uint32)
    nn = np.ascontiguousarray(n, dtype=np.uint64)
    kk = np.ascontiguousarray(kinds, dtype=np.int32)
    _check(lib().slrng_server_replay(sv, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     sid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), _u64p(nn),
                                     kk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), t.size),
           "slrng_server_replay")


def slrng_server_destroy(sv: int) -> None:
    _check(lib().slrng_server_destroy(sv), "slrng_server_destroy")


def slrng_server_advance(sv: int, stream_id: int, steps: int) -> None:
    """Move a resident stream's head by `steps` (any value below 2^128)."""
    steps %= 1 << 128
    _check(lib().slrng_server_advance(sv, stream_id, steps >> 64, steps & ((1 << 64) - 1)),
           "slrng_server_advance")


def slrng_server_intervals(sv: int) -> np.ndarray:
    """The generation kernels' device intervals, shape (iterations, 2), in ms."""
    cnt = ctypes.c_uint64()
    _check(lib().slrng_server_intervals(sv, None, None, 0, ctypes.byref(cnt)), "slrng_server_intervals")
    n = cnt.value + 64  # room for iterations completing meanwhile
    a = np.zeros(n, dtype=np.float64)
    b = np.zeros(n, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().slrng_server_intervals(sv, a.ctypes.data_as(dp), b.ctypes.data_as(dp), n, ctypes.byref(cnt)),
           "slrng_server_intervals")
    m = min(n, cnt.value)
    return np.stack([a[:m], b[:m]], axis=1)


# ---------------------------------------------------------------- object wrapper

class Streams:
    """S device-resident streams of one variant (see slrng_streams_create)."""

    def __init__(self, variant, seed: int = 0, n_streams: int = 1, states=None, stream=None):
        self.variant = _variant(variant)
        self.k = slrng_state_words(self.variant)
        if states is not None:
            self.h = slrng_streams_create_from_states(self.variant, states, stream)
        else:
            self.h = slrng_streams_create(self.variant, seed, n_streams, stream)
        self.S = slrng_streams_count(self.h)

    def close(self):
        if getattr(self, "h", None):
            slrng_streams_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def generate(self, n: int, kind: int | None = None, out=None, ld: int | None = None,
                 stream=None):
        """Outputs as a torch tensor [S, ld]: int64 / int32 bit patterns, or
        float64 / float32.  kind defaults to the generator's integers."""
        import torch
        if kind is None:
            kind = SLRNG_U32 if self.variant >= len(VARIANTS) else SLRNG_U64
        if ld is None:
            ld = n
        if out is None:
            dt = {SLRNG_U64: torch.int64, SLRNG_F64: torch.float64,
                  SLRNG_U32: torch.int32, SLRNG_F32: torch.float32}[kind]
            out = torch.empty((self.S, max(ld, 1)), dtype=dt, device="cuda")
        slrng_generate(self.h, kind, n, out.data_ptr(), ld, stream)
        return out

    def seed(self, seed: int, stream=None):
        slrng_streams_seed(self.h, seed, stream)

    def jump(self, jump_kind: int = SLRNG_JUMP, stream=None):
        slrng_streams_jump(self.h, jump_kind, stream)

    def advance(self, steps: int, stream=None):
        slrng_streams_advance(self.h, steps, stream)

    def advance_each(self, steps, stream=None):
        """Advance stream i by steps[i] (Python ints or uint64 pairs; any
        128-bit value).  `steps` may also be a CUDA int64 tensor of shape
        (S, 2) holding (low, high) words, used in place."""
        import torch
        if isinstance(steps, torch.Tensor):
            assert steps.is_cuda and steps.dtype == torch.int64 and steps.shape == (self.S, 2)
            buf = steps.contiguous()
        else:
            words = np.zeros((self.S, 2), dtype=np.uint64)
            for i, J in enumerate(steps):
                J = int(J)
                words[i, 0] = J & 0xFFFFFFFFFFFFFFFF
                words[i, 1] = (J >> 64) & 0xFFFFFFFFFFFFFFFF
            buf = torch.from_numpy(words.view(np.int64)).cuda()
        slrng_streams_advance_each(self.h, buf.data_ptr(), stream)
        if buf is not steps:
            # the staging tensor must outlive the queued kernel
            torch.cuda.synchronize()

    def get_state(self, stream=None) -> np.ndarray:
        return slrng_get_state(self.h, stream)

    def linear_complexity(self, bit: int, nbits: int, stream=None):
        """Per-stream linear complexity of output bit `bit` over the next
        nbits outputs (a CUDA int32 tensor of S values); streams unchanged."""
        import torch
        out = torch.empty((self.S,), dtype=torch.int32, device="cuda")
        slrng_linear_complexity(self.h, bit, nbits, out.data_ptr(), stream)
        return out

    def set_state(self, states, stream=None):
        slrng_set_state(self.h, np.asarray(states, dtype=np.uint64).reshape(-1), stream)

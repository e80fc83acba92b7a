"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and
its host-side polynomial planner agrees with the oracle's independent
Berlekamp-Massey and square-and-multiply routes.  No kernel is launched."""
import ctypes
import glob
import os
import random
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_1805_01407_amd as P
    if not os.path.exists(P.library_path()):
        from paper_1805_01407_amd import build
        build.build()
    P.lib()
    return P


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w \*]*?\b(slrng_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported(P):
    names = declared_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(P.library_path())
    for n in names:
        assert hasattr(L, n), n


def test_binding_mirrors_every_declared_symbol(P):
    for n in declared_functions():
        assert hasattr(P, n), n


def test_version_and_errors(P):
    assert P.slrng_version() == 1
    for code in range(0, -8, -1):
        assert P.slrng_strerror(code).startswith("SLRNG")
    assert "unknown" in P.slrng_strerror(-99)
    with pytest.raises(P.SlrngError):
        P.slrng_state_words(19)
    assert [P.slrng_state_words(v) for v in range(19)] == \
        [2, 2, 2, 4, 4, 4, 8, 8, 8, 16, 16, 16, 2, 16, 2, 2, 4, 4, 4]


def test_rank_argument_errors(P):
    # host-side checks only: every call below is rejected before any launch
    L = P.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced
    bad = [(99, 0, 1), (-1, 0, 1), (0, -1, 1), (0, 2, 1), (0, 0, 0), (0, 0, 3),  # xoroshiro128: k = 2
           (9, 16, 1), (9, 0, 17), (14, 2, 1), (16, 0, 5)]                     # k = 16, 2, 4
    for v, word, dims in bad:
        assert L.slrng_equidistribution_rank(v, word, dims, fake, None) == -1, (v, word, dims)
    assert L.slrng_equidistribution_rank(0, 0, 1, None, None) == -1
    assert L.slrng_equidistribution_rank(0, 0, 1, ctypes.c_void_p(0x1002), None) == -1  # misaligned
    for nrows, ncols in ((0, 1), (1, 0), (1025, 1), (1, 1025)):
        assert L.slrng_gf2_rank(fake, nrows, ncols, fake, None) == -1
    assert L.slrng_gf2_rank(None, 1, 1, fake, None) == -1
    assert L.slrng_gf2_rank(ctypes.c_void_p(0x1004), 1, 1, fake, None) == -1  # rows misaligned


def test_output_memory_argument_errors(P):
    # host-side checks only: no device memory is touched
    import torch
    with pytest.raises(ValueError, match="unsupported dtype"):
        P.output_empty((4, 4), torch.bfloat16)
    L = P.lib()
    p = ctypes.c_void_p(1234)
    assert L.slrng_output_alloc(0, ctypes.byref(p)) == -1 and p.value is None  # EINVAL, *out cleared
    assert L.slrng_output_alloc(1 << 20, None) == -1
    assert L.slrng_output_free(None) == 0
    assert L.slrng_output_free(ctypes.c_void_p(0x1000)) == -1  # not from slrng_output_alloc


@pytest.mark.parametrize("name", list(O.GEN64))
def test_charpoly_matches_oracle(P, name):
    assert P.slrng_charpoly(name) == O.charpoly(O.GEN64[name])


@pytest.mark.parametrize("name", ["xoroshiro128+", "xoroshiro128++", "xoshiro256++",
                                  "xoshiro512**", "xoroshiro1024**"])
def test_jump_poly_matches_oracle(P, name):
    g = O.GEN64[name]
    p = O.charpoly(g)
    rnd = random.Random(name)
    Js = [0, 1, 2, 63, 64, g.n - 1, g.n, 1 << (g.n // 2), 1 << (3 * g.n // 4),
          (1 << 128) - 1, rnd.getrandbits(64), rnd.getrandbits(100)]
    for J in Js:
        assert P.slrng_jump_poly(name, J) == O.xpow_mod(J, p), J


def test_jump_poly_homomorphism_in_the_library(P):
    # r_a * r_b = r_{a+b} mod p, the products taken with the oracle's multiplier
    name = "xoshiro256**"
    p = O.charpoly(O.GEN64[name])
    a, b = 1 << 128, 1 << 192
    ra, rb = P.slrng_jump_poly(name, a), P.slrng_jump_poly(name, b)
    assert O.poly_mulmod(ra, rb, p) == P.slrng_jump_poly(name, a + b)


def test_zero_state_rejected_before_any_device_call(P):
    st = np.zeros((3, 4), dtype=np.uint64)
    st[0, 1] = 5
    with pytest.raises(P.SlrngError) as e:
        P.slrng_streams_create_from_states("xoshiro256**", st.reshape(-1), stream=0)
    assert e.value.name == "EZEROSTATE"


def test_tuning_validation(P):
    t = P.slrng_get_tuning("xoshiro256**")
    assert t["tile"] in (16, 32)
    with pytest.raises(P.SlrngError):
        P.slrng_set_tuning("xoshiro256**", 0, 24, 1024, 1024)
    with pytest.raises(P.SlrngError):
        P.slrng_set_tuning("xoshiro256**", 2, 16, 1024, 1024)
    with pytest.raises(P.SlrngError):
        P.slrng_set_tuning("xoshiro256**", 0, 16, 1024, 1024, skew=3)
    with pytest.raises(P.SlrngError):
        P.slrng_set_tuning("xoshiro256**", 0, 16, 1024, 1024, store=2)
    P.slrng_set_tuning("xoshiro256**", 0, t["tile"], t["target_waves"], t["min_chunk"], t["skew"], 1)
    assert P.slrng_get_tuning("xoshiro256**")["store"] == 1
    P.slrng_set_tuning("xoshiro256**", 0, t["tile"], t["target_waves"], t["min_chunk"], t["skew"],
                       t["store"])


def test_invalid_arguments_return_einval(P):
    L = P.lib()
    assert L.slrng_streams_jump(None, 0, None) == -1
    assert L.slrng_generate(None, 0, 10, None, 10, None) == -1
    assert L.slrng_streams_destroy(None) == -1
    h = ctypes.c_void_p()
    assert L.slrng_streams_create(99, 1, 1, None, ctypes.byref(h)) == -1
    assert L.slrng_streams_create(0, 1, 0, None, ctypes.byref(h)) == -2
    assert L.slrng_streams_create(0, 1, (1 << 31) + 1, None, ctypes.byref(h)) == -2
    assert L.slrng_calib_write(None, 16, None) == -1


def test_jump_poly_device_argument_errors_before_any_device_call(P):
    """slrng_jump_poly_device rejects a bad variant, null or unaligned
    pointers and m > 2^32 before touching the device; m = 0 does nothing."""
    L = P.lib()
    fake = 1 << 20  # aligned, never dereferenced: the checks come first
    assert L.slrng_jump_poly_device(99, fake, 1, fake, None) == -1
    assert L.slrng_jump_poly_device(-1, fake, 1, fake, None) == -1
    assert L.slrng_jump_poly_device(3, None, 1, fake, None) == -1
    assert L.slrng_jump_poly_device(3, fake, 1, None, None) == -1
    assert L.slrng_jump_poly_device(3, fake + 4, 1, fake, None) == -1
    assert L.slrng_jump_poly_device(3, fake, 1, fake + 4, None) == -1
    assert L.slrng_jump_poly_device(3, fake, (1 << 32) + 1, fake, None) == -2
    assert L.slrng_jump_poly_device(3, None, 0, None, None) == 0


def test_batch_argument_errors_before_any_device_call(P):
    bad_variant = P.make_requests(14, 0, 1, 0, 10, 4096)
    misaligned = P.make_requests(0, 0, 1, 0, 10, 4100)
    bad_kind = P.make_requests(0, 2, 1, 0, 10, 4096)
    null_out = P.make_requests(0, 0, 1, 0, 10, 0)
    for reqs in (bad_variant, misaligned, bad_kind, null_out):
        with pytest.raises(P.SlrngError) as e:
            P.slrng_batch_run(reqs, None, 0)
        assert e.value.name == "EINVAL"
    o = P.slrng_batch_default_opts()
    o.mode = 7
    with pytest.raises(P.SlrngError):
        P.slrng_batch_run(P.make_requests(0, 0, 1, 0, 10, 4096), o, 0)
    o = P.slrng_batch_default_opts(tile=24)
    with pytest.raises(P.SlrngError):
        P.slrng_batch_run(P.make_requests(0, 0, 1, 0, 10, 4096), o, 0)


def test_request_record_layout(P):
    assert P.REQUEST_DTYPE.itemsize == 40
    r = P.make_requests([1, 2], 1, [5, 6], 0, 7, [8, 16])
    assert r["variant"].tolist() == [1, 2] and r["seed"].tolist() == [5, 6]
    assert r["dev_out"].tolist() == [8, 16]


def test_server_argument_errors_before_any_device_call(P):
    for kw in ({"n_streams": 0}, {"variant": 14}, {"budget_bytes": 16}, {"inflight": 9}):
        o = P.slrng_server_default_opts(**kw)
        with pytest.raises(P.SlrngError) as e:
            P.slrng_server_create(o)
        assert e.value.name == "EINVAL"
    L = P.lib()
    t = ctypes.c_uint64()
    assert L.slrng_server_submit(None, 0, 1, 0, 0, ctypes.byref(t)) == -1
    assert L.slrng_server_drain(None) == -1
    assert L.slrng_server_destroy(None) == -1


def test_serve_trace_shape():
    from paper_1805_01407_amd import workloads as W
    tr = W.serve_trace(rate=20000, seconds=1.0)
    m = tr["t"].size
    assert 19000 < m < 21000
    assert np.all(np.diff(tr["t"]) >= 0) and tr["t"][-1] < 1.0
    assert tr["n"].min() >= 8 and tr["n"].max() <= (1 << 28) // 8
    assert tr["stream"].max() < 4096
    mean_bytes = float((tr["n"] * 8).mean())
    assert 8e6 < mean_bytes < 3e7  # log-uniform 64 B .. 256 MiB: mean about 17.6 MB


# ---------------------------------------------------------------- 32-bit generators

@pytest.mark.parametrize("name", list(O.GEN32))
def test_charpoly_and_jump_poly_32_match_oracle(P, name):
    g = O.GEN32[name]
    p = O.charpoly(g)
    assert P.slrng_charpoly(name) == p
    assert P.slrng_state_words(name) == g.k
    rnd = random.Random(name)
    for J in (0, 1, 63, g.n, 1 << (g.n // 2), 1 << (3 * g.n // 4), (1 << 128) - 1,
              rnd.getrandbits(100)):
        assert P.slrng_jump_poly(name, J) == O.xpow_mod(J, p), J


def test_32bit_argument_errors_before_any_device_call(P):
    # a 32-bit state word must fit in 32 bits; all-zero states are rejected
    st = np.ones((3, 4), dtype=np.uint64)
    st[1, 2] = 1 << 32
    with pytest.raises(P.SlrngError) as e:
        P.slrng_streams_create_from_states("xoshiro128**", st.reshape(-1), stream=0)
    assert e.value.name == "EINVAL"
    st = np.ones((2, 2), dtype=np.uint64)
    st[1] = 0
    with pytest.raises(P.SlrngError) as e:
        P.slrng_streams_create_from_states("xoroshiro64*", st.reshape(-1), stream=0)
    assert e.value.name == "EZEROSTATE"
    # 32-bit kinds and a 64-output tile for the 32-bit generators only
    t = P.slrng_get_tuning("xoshiro128+", P.SLRNG_U32)
    assert t["tile"] == 64
    for bad in ((P.SLRNG_U64, 64), (P.SLRNG_U32, 32)):
        with pytest.raises(P.SlrngError):
            P.slrng_set_tuning("xoshiro128+", bad[0], bad[1], 1024, 1024)
    with pytest.raises(P.SlrngError):
        P.slrng_get_tuning("xoshiro256+", P.SLRNG_U32)
    P.slrng_set_tuning("xoshiro128+", P.SLRNG_U32, t["tile"], t["target_waves"], t["min_chunk"],
                       t["skew"], t["store"])


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_oracle_baselines_per_config():
    # the host-only part of bench.py: the oracle timed on samples of the
    # small case, jump-ahead and batched workloads
    import sys
    sys.path.insert(0, ROOT)
    import bench
    r = bench.cpu_per_config(budget=0.2)
    assert r["cores"] >= 1
    assert r["small_case"]["generate_ms_1thread"] > 0 and r["small_case"]["generate_ms_all"] > 0
    j = r["jump_ahead_at_scale"]
    assert j["chain_streams_per_s"] > 0 and j["long_jumps_per_s_all"] > 0 and j["outputs_per_s_all"] > 0
    b = r["batched_requests"]
    assert b["requests_1thread"] >= 1 and b["outputs_per_s_all"] > 0


def test_plain_c_program_uses_the_abi(tmp_path):
    """A C program compiled against include/slrng.h and linked with
    libslrng.so (no Python in between) gets the same polynomials as the
    oracle."""
    import shutil
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lib_dir = os.path.join(root, "paper_1805_01407_amd")
    if not os.path.exists(os.path.join(lib_dir, "libslrng.so")) or not shutil.which("gcc"):
        pytest.skip("library not built or no C compiler")
    exe = str(tmp_path / "abi_host_calls")
    subprocess.run(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"),
                    "-I", "/opt/rocm/include", os.path.join(root, "tests", "c", "abi_host_calls.c"),
                    "-L", lib_dir, "-Wl,-rpath," + lib_dir, "-lslrng", "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    lines = dict(line.split(" ", 1) for line in out.stdout.strip().splitlines() if " " in line)
    g = O.GEN64["xoshiro256**"]
    p = O.charpoly(g)
    words = lambda v, k: " ".join(f"{(v >> (64 * i)) & (2**64 - 1):016x}" for i in range(k))  # noqa: E731
    assert lines["charpoly"] == words(p, 5)
    assert lines["jump"] == words(O.xpow_mod(1 << 128, p), 4)
    assert lines["longjump"] == words(O.xpow_mod(1 << 192, p), 4)
    assert "ZEROSTATE" in out.stdout

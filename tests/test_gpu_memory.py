"""GPU checks of the output allocator (slrng_output_alloc / slrng_output_free):
plain and spread blocks hold what the generators write into them, bit for bit
the same as ordinary device memory, including across piece boundaries and at
the last element; torch tensors on them behave like torch.empty; argument and
double-free errors."""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
GiB = 1 << 30


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


def test_output_alloc_errors(P):
    import torch
    announce("output alloc errors")
    with pytest.raises(P.SlrngError, match="EINVAL"):
        P.slrng_output_alloc(0)
    p = P.slrng_output_alloc(4096)  # plain block
    P.slrng_output_free(p)
    with pytest.raises(P.SlrngError, match="EINVAL"):
        P.slrng_output_free(p)  # already freed
    x = torch.empty(16, dtype=torch.int64, device="cuda")
    with pytest.raises(P.SlrngError, match="EINVAL"):
        P.slrng_output_free(x.data_ptr())  # not from the allocator
    P.slrng_output_free(0)  # NULL: no-op


@pytest.mark.parametrize("nbytes", [1 << 20, (5 * GiB) // 2 + 8 * 1000])
def test_generate_into_output_memory_matches_plain_memory(P, nbytes):
    # 1 MiB: a plain block; just under 2.5 GiB: ten spread pieces of 256 MiB,
    # the last one not quite full.  Rows of 8 * N bytes straddle the piece
    # boundaries.
    import torch
    name, seed = "xoshiro512**", 11
    N = 3001
    S = nbytes // (8 * N)
    announce("output memory generate", nbytes, S, N)
    p = P.slrng_output_alloc(8 * S * N)
    try:
        ref = torch.empty((S, N), dtype=torch.int64, device="cuda")
        got = torch.empty((S, N), dtype=torch.int64, device="cuda")
        with P.Streams(name, seed, S) as h:
            P.slrng_generate(h.h, P.SLRNG_U64, N, p, N, 0)
            h.seed(seed)
            P.slrng_generate(h.h, P.SLRNG_U64, N, ref.data_ptr(), N, 0)
        # read the allocator's block back with the library's own copy kernel
        P.slrng_calib_copy(got.data_ptr(), p, 8 * S * N // 16 * 16, 0)
        torch.cuda.synchronize()
        flat_g, flat_r = got.view(-1), ref.view(-1)
        m = 8 * S * N // 16 * 2  # elements covered by the 16-byte copy
        assert torch.equal(flat_g[:m], flat_r[:m])
        # the first and last rows against the oracle as well
        g = O.GEN64[name]
        st0 = O.stream_chain(g, seed, S)
        exp, _ = O.generate_many(g, st0[[0, S - 1]], N)
        assert np.array_equal(ref[[0, S - 1]].cpu().numpy().view(np.uint64), exp)
    finally:
        P.slrng_output_free(p)


@pytest.mark.parametrize("dtype_name", ["int64", "float64", "int32", "float32"])
def test_output_empty_tensor(P, dtype_name):
    import torch
    dtype = getattr(torch, dtype_name)
    announce("output_empty", dtype_name)
    name = "xoshiro128**" if dtype in (torch.int32, torch.float32) else "xoshiro256++"
    kind = {torch.int64: P.SLRNG_U64, torch.float64: P.SLRNG_F64,
            torch.int32: P.SLRNG_U32, torch.float32: P.SLRNG_F32}[dtype]
    S, N = 257, 5000
    t = P.output_empty((S, N), dtype)
    assert t.is_cuda and t.dtype == dtype and t.shape == (S, N) and t.is_contiguous()
    with P.Streams(name, 9, S) as h:
        h.generate(N, kind, out=t)
        h.seed(9)
        ref = h.generate(N, kind)
    torch.cuda.synchronize()
    assert torch.equal(t.view(torch.int64 if t.element_size() == 8 else torch.int32),
                       ref.view(torch.int64 if ref.element_size() == 8 else torch.int32))
    del t
    torch.cuda.synchronize()


def test_output_empty_spread_tensor_views_keep_memory(P):
    # a spread block (1.5 GiB) wrapped by torch; a view keeps it alive after
    # the tensor itself is dropped
    import torch
    announce("output_empty spread views")
    S, N = 3, (3 * GiB // 2) // 24
    t = P.output_empty((S, N), torch.float64)
    with P.Streams("xoroshiro1024++", 2, S) as h:
        h.generate(N, P.SLRNG_F64, out=t)
        h.seed(2)
        ref = h.generate(N, P.SLRNG_F64)
    v = t[2, -7:]
    del t
    torch.cuda.synchronize()
    assert torch.equal(v.view(torch.int64), ref[2, -7:].view(torch.int64))
    del v, ref
    torch.cuda.synchronize()

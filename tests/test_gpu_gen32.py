"""GPU parity of the 32-bit generators (xoroshiro64*, xoroshiro64**,
xoshiro128+, xoshiro128++, xoshiro128**) against the oracle: positioning,
uint32 and float outputs, ragged shapes, misaligned buffers and row strides,
stream splitting with and without staggered boundaries, jumps, advances,
per-stream advances, checkpoint and restore, argument errors."""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

NAMES = list(O.GEN32)


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


def oracle_outputs(g, states, n):
    out, fin = O.generate_many(g, states, n, kind="u64")
    return out.astype(np.uint32), fin


def as_u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("kind", ["u32", "f32"])
def test_generate32_matches_oracle(P, name, kind):
    g = O.GEN32[name]
    S, N = 200, 1000  # ragged: not multiples of 64 streams or of the 64-output tile
    announce("gen32", name, kind, S, N)
    chain = O.stream_chain(g, 42, S)
    exp, fin = oracle_outputs(g, chain, N)
    k = P.SLRNG_U32 if kind == "u32" else P.SLRNG_F32
    with P.Streams(name, 42, S) as h:
        assert np.array_equal(h.get_state(), chain)
        out = h.generate(N, k)
        got_fin = h.get_state()
    if kind == "u32":
        assert np.array_equal(as_u32(out), exp)
    else:
        f = out.cpu().numpy()
        assert f.dtype == np.float32
        assert np.array_equal(f.view(np.uint32), O.to_float32(exp).view(np.uint32))
    assert np.array_equal(got_fin, fin)


@pytest.mark.parametrize("name", ["xoroshiro64**", "xoshiro128++"])
def test_generate32_edge_cases(P, name):
    import torch
    g = O.GEN32[name]
    announce("gen32 edges", name)
    # misaligned buffer (4-byte aligned only), odd row stride, single stream,
    # zero length, repeated calls equal one long call
    S, N, ld = 67, 333, 339
    chain = O.stream_chain(g, 9, S)
    exp, fin = oracle_outputs(g, chain, N)
    buf = torch.full((S * ld + 8,), -1, dtype=torch.int32, device="cuda")
    with P.Streams(name, 9, S) as h:
        P.slrng_generate(h.h, P.SLRNG_U32, N, buf.data_ptr() + 4, ld, 0)
        torch.cuda.synchronize()
        host = buf.cpu().numpy().view(np.uint32)[1:1 + S * ld].reshape(S, ld)
        assert np.array_equal(host[:, :N], exp)
        assert (host[:, N:] == 0xFFFFFFFF).all()
        assert np.array_equal(h.get_state(), fin)
        P.slrng_generate(h.h, P.SLRNG_U32, 0, buf.data_ptr(), 1, 0)  # no-op
        assert np.array_equal(h.get_state(), fin)
    with P.Streams(name, 5, 1) as h:
        a = as_u32(h.generate(100))
        b = as_u32(h.generate(157))
    e, _ = oracle_outputs(g, O.stream_chain(g, 5, 1), 257)
    assert np.array_equal(np.concatenate([a[0], b[0]]), e[0])


@pytest.mark.parametrize("name", NAMES)
def test_generate32_split_streams(P, name):
    """Few streams, long rows: the streams are split into jumped slots, with
    and without staggered boundaries."""
    g = O.GEN32[name]
    S, N = 70, 40000
    chain = O.stream_chain(g, 3, S)
    exp, fin = oracle_outputs(g, chain, N)
    for skew, store in ((1, 0), (4, 1), (1, 1)):
        announce("gen32 split", name, skew, store)
        old = P.slrng_get_tuning(name, P.SLRNG_U32)
        P.slrng_set_tuning(name, P.SLRNG_U32, 64, 4096, 1024, skew, store)
        try:
            with P.Streams(name, 3, S) as h:
                out = as_u32(h.generate(N))
                assert np.array_equal(h.get_state(), fin)
        finally:
            P.slrng_set_tuning(name, P.SLRNG_U32, old["tile"], old["target_waves"],
                               old["min_chunk"], old["skew"], old["store"])
        assert np.array_equal(out, exp)


@pytest.mark.parametrize("name", NAMES)
def test_jumps32(P, name):
    g = O.GEN32[name]
    S = 130
    announce("jumps32", name)
    chain = O.stream_chain(g, 77, S)
    p = O.charpoly(g)
    with P.Streams(name, 77, S) as h:
        h.jump(P.SLRNG_JUMP)
        exp = O.jump_many(g, chain, O.jump_distance(g, "jump"))
        assert np.array_equal(h.get_state(), exp)
        h.jump(P.SLRNG_LONG_JUMP)
        exp = O.jump_many(g, exp, O.jump_distance(g, "long"))
        assert np.array_equal(h.get_state(), exp)
        J = (1 << 70) + 12345
        h.advance(J)
        exp = O.jump_many(g, exp, J)
        assert np.array_equal(h.get_state(), exp)
        rng = np.random.default_rng(4)
        Js = [int.from_bytes(rng.bytes(16), "little") for _ in range(S)]
        Js[:3] = [0, 1, (1 << g.n) - 1]
        h.advance_each(Js)
        exp = np.stack([O.jump_poly(g, exp[i], O.xpow_mod(Js[i], p)) for i in range(S)])
        assert np.array_equal(h.get_state(), exp)
        out = as_u32(h.generate(129))
    e, _ = oracle_outputs(g, exp, 129)
    assert np.array_equal(out, e)


def test_state32_checkpoint_and_errors(P):
    name = "xoshiro128**"
    g = O.GEN32[name]
    announce("state32")
    with P.Streams(name, 1, 100) as h:
        h.generate(77)
        st = h.get_state()
        a = as_u32(h.generate(500))
        h.set_state(st)
        b = as_u32(h.generate(500))
        assert np.array_equal(a, b)
        bad = st.copy()
        bad[3, 1] = 1 << 32  # does not fit a 32-bit word
        with pytest.raises(P.SlrngError) as e:
            h.set_state(bad)
        assert e.value.name == "EINVAL"
        zero = st.copy()
        zero[5] = 0
        with pytest.raises(P.SlrngError) as e:
            h.set_state(zero)
        assert e.value.name == "EZEROSTATE"
        # a 32-bit generator takes 32-bit kinds only
        with pytest.raises(P.SlrngError):
            h.generate(10, P.SLRNG_U64)
    with P.Streams("xoshiro256**", 1, 4) as h:
        with pytest.raises(P.SlrngError):
            h.generate(10, P.SLRNG_U32)
    st = O.stream_chain(g, 8, 3)
    with P.Streams(name, states=st) as h:
        e, _ = oracle_outputs(g, st, 64)
        assert np.array_equal(as_u32(h.generate(64)), e)


def test_generate32_full_size_sampled(P):
    """65,536 xoshiro128** streams x 131,072 outputs (32 GiB of uint32), as the
    bench runs it; sampled rows against the oracle."""
    import torch
    name = "xoshiro128**"
    g = O.GEN32[name]
    S, N = 65536, 131072
    announce("gen32 full size", name, S, N)
    buf = torch.empty((S, N), dtype=torch.int32, device="cuda")
    rows = np.array([0, 1, 63, 64, 4095, 32768, 65471, S - 1])
    with P.Streams(name, 1, S) as h:
        P.slrng_generate(h.h, P.SLRNG_U32, N, buf.data_ptr(), N, 0)
        torch.cuda.synchronize()
        fin = h.get_state()
    got = buf[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32)
    del buf
    torch.cuda.empty_cache()
    for j, i in enumerate(rows):
        x = O.stream_state(g, 1, int(i))
        e, f = O.generate(g, x, N)
        assert np.array_equal(got[j], e.astype(np.uint32)), i
        assert np.array_equal(fin[i], f), i


def test_zero_base_state_rejected(P):
    """SplitMix64's finalizer maps 0 to 0, so the seed -gamma (mod 2^64) makes
    the first SplitMix64 output zero: the whole xoroshiro64 state.  Creating
    or re-seeding such streams is refused; xoshiro128 (two outputs) is fine."""
    seed = (-O.splitmix_gamma()) % 2**64
    assert O.seed_state(O.GEN32["xoroshiro64*"], seed).tolist() == [0, 0]
    announce("zero base", hex(seed))
    with pytest.raises(P.SlrngError) as e:
        P.Streams("xoroshiro64*", seed, 4)
    assert e.value.name == "EZEROSTATE"
    with P.Streams("xoroshiro64**", 1, 4) as h:
        with pytest.raises(P.SlrngError) as e:
            h.seed(seed)
        assert e.value.name == "EZEROSTATE"
    with P.Streams("xoshiro128+", seed, 3) as h:
        g = O.GEN32["xoshiro128+"]
        assert np.array_equal(h.get_state(), O.stream_chain(g, seed, 3))

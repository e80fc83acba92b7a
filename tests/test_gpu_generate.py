"""GPU parity of the generation, positioning and jump kernels against the oracle,
bit for bit (tolerance 0 for integers and for doubles).  Every call goes
through the C ABI."""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

ALL14 = list(O.GEN64)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_01407_amd as P
    P.lib()
    return P


def announce(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def to_u64(t):
    return t.cpu().numpy().view(np.uint64)


def oracle_streams(name, seed, S):
    return O.stream_chain(O.GEN64[name], seed, S)


def check_generate(P, name, seed, S, n, kind=0, ld=None, offset=0):
    """Create S streams on the GPU, generate n outputs, compare with the oracle."""
    import torch
    announce("generate", name, "seed", seed, "S", S, "n", n, "kind", kind, "ld", ld, "off", offset)
    g = O.GEN64[name]
    ld = n if ld is None else ld
    st0 = oracle_streams(name, seed, S)
    with P.Streams(name, seed, S) as s:
        assert (s.get_state() == st0).all(), "positioning"
        total = S * ld + offset + 1
        buf = torch.full((total,), -1, dtype=torch.int64, device="cuda")
        view = buf[offset:offset + S * ld]
        P.slrng_generate(s.h, kind, n, view.data_ptr(), ld, 0)
        torch.cuda.synchronize()
        got = buf.cpu().numpy().view(np.uint64)
        fin = s.get_state()
    exp, exp_fin = O.generate_many(g, st0, n, kind="u64")
    rows = got[offset:offset + S * ld].reshape(S, ld)
    if kind == 0:
        assert (rows[:, :n] == exp).all()
    else:
        d = rows[:, :n].view(np.float64)
        ed = (exp >> np.uint64(11)).astype(np.float64) * 2.0**-53
        assert (d.view(np.uint64) == ed.view(np.uint64)).all()
    # untouched gaps and guards
    assert (rows[:, n:] == np.uint64(0xFFFFFFFFFFFFFFFF)).all()
    assert (got[:offset] == np.uint64(0xFFFFFFFFFFFFFFFF)).all()
    assert got[-1] == np.uint64(0xFFFFFFFFFFFFFFFF)
    assert (fin == exp_fin).all(), "final state"


@pytest.mark.parametrize("name", ALL14)
def test_all_variants_ragged(P, name):
    check_generate(P, name, 7, 200, 1000)


@pytest.mark.parametrize("name", ["xoshiro256**", "xoroshiro1024++", "xoroshiro128+"])
def test_doubles_bit_exact(P, name):
    check_generate(P, name, 3, 130, 517, kind=1)


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 31, 32, 33, 16 * 5 + 7, 4096 + 3])
def test_tail_lengths_xoroshiro1024(P, n):
    check_generate(P, "xoroshiro1024**", 11, 65, n)


@pytest.mark.parametrize("n", [1, 15, 16, 17, 100])
def test_tail_lengths_xoshiro512(P, n):
    check_generate(P, "xoshiro512++", 12, 70, n)


def test_row_stride_and_misaligned_output(P):
    check_generate(P, "xoshiro256++", 5, 100, 333, ld=341)       # odd ld: 8-byte store path
    check_generate(P, "xoshiro256++", 5, 100, 334, ld=340, offset=1)  # 8-byte aligned only
    check_generate(P, "xoroshiro1024+", 6, 64, 160, ld=170, offset=3)


def test_single_stream(P):
    check_generate(P, "xoroshiro128**", 99, 1, 4097)


def test_zero_length_is_noop(P):
    import torch
    with P.Streams("xoshiro256**", 1, 10) as s:
        st = s.get_state()
        buf = torch.zeros(4, dtype=torch.int64, device="cuda")
        P.slrng_generate(s.h, 0, 0, buf.data_ptr(), 0, 0)
        assert (s.get_state() == st).all()


@pytest.mark.parametrize("name", ["xoshiro256**", "xoroshiro1024**", "xoroshiro128++", "xoshiro512+"])
def test_chunk_split_matches_unsplit(P, name):
    """Force the stream-splitting path (slots jumped ahead, with and without
    staggered boundaries) with plain and nontemporal stores: the values never
    depend on the launch shape."""
    t = P.slrng_get_tuning(name)
    try:
        for tile, skew, store in ((16, 1, 0), (32, 1, 1), (16, 4, 1), (32, 16, 0), (32, 16, 1)):
            P.slrng_set_tuning(name, 0, tile, 1 << 16, 64, skew, store)
            check_generate(P, name, 21, 300, 3001)
            check_generate(P, name, 22, 3, 100)
            check_generate(P, name, 23, 64, 1)
    finally:
        P.slrng_set_tuning(name, 0, t["tile"], t["target_waves"], t["min_chunk"], t["skew"],
                           t["store"])


def test_split_calls_equal_one_call(P):
    import torch
    name = "xoshiro512**"
    with P.Streams(name, 4, 150) as a, P.Streams(name, 4, 150) as b:
        x = a.generate(777)
        y1 = b.generate(300)
        y2 = b.generate(477)
        torch.cuda.synchronize()
        assert torch.equal(x[:, :300], y1) and torch.equal(x[:, 300:], y2)
        assert (a.get_state() == b.get_state()).all()


@pytest.mark.parametrize("name", ["xoshiro256**", "xoroshiro1024*", "xoroshiro128++", "xoshiro512++"])
def test_jump_long_jump_and_advance(P, name):
    g = O.GEN64[name]
    S = 77
    st0 = oracle_streams(name, 8, S)
    with P.Streams(name, 8, S) as s:
        announce("jump", name)
        s.jump(P.SLRNG_JUMP)
        exp = O.jump_many(g, st0, O.jump_distance(g, "jump"))
        assert (s.get_state() == exp).all()
        s.jump(P.SLRNG_LONG_JUMP)
        exp = O.jump_many(g, exp, O.jump_distance(g, "long"))
        assert (s.get_state() == exp).all()
        for steps in (1, 17, 12345, (1 << 64) + 99, (1 << 127) + 5):
            s.advance(steps)
            exp = O.jump_many(g, exp, steps)
            assert (s.get_state() == exp).all(), steps


def test_set_get_state_roundtrip(P):
    name = "xoroshiro1024++"
    g = O.GEN64[name]
    rng = np.random.default_rng(1)
    st = rng.integers(0, 2**64, size=(90, 16), dtype=np.uint64)
    with P.Streams(name, states=st.reshape(-1)) as s:
        assert (s.get_state() == st).all()
        out = to_u64(s.generate(50))
        exp, fin = O.generate_many(g, st, 50)
        assert (out == exp).all() and (s.get_state() == fin).all()
        bad = st.copy()
        bad[5] = 0
        with pytest.raises(P.SlrngError):
            s.set_state(bad)
        assert (s.get_state() == fin).all()


# outputs at the edges of the float conversions: the low bits that are
# dropped, the 2^11 (2^8) threshold, each word of the upper part, all ones
EDGE64 = [0, 1, 0x7FF, 0x800, 0xFFF, 0xFFFFF7FF, 0xFFFFF800, 0xFFFFFFFF, 1 << 32, (1 << 32) | 0x7FF,
          (1 << 32) + 0x800, 0x7FFFFFFFFFFFFFFF, 1 << 63, (1 << 63) | 0x7FF, (1 << 64) - 0x800,
          (1 << 64) - 0x801, (1 << 64) - 1, 0x0123456789ABCDEF, 0xFEDCBA9876543210, 0x00000000FFFFF800]
EDGE32 = [0, 1, 0x7F, 0x80, 0xFF, 0x100, 0x1FF, 0xFFFFFF, 0x1000000, 0x7FFFFFFF, 0x80000000,
          0xFFFFFF00, 0xFFFFFFFE, 0xFFFFFFFF, 0x12345678]


def test_float_conversion_at_edge_values(P):
    """Streams whose first output is a chosen value: xoroshiro128+ emits
    s0 + s1 and xoshiro128+ emits s0 + s3, so the states (x, 0) and
    (x, 0, 0, 0) give x (and (1, 2^64 - 1), (1, 0, 0, 2^32 - 1) give 0, the
    zero state being excluded).  The doubles must be (x >> 11) 2^-53 and the
    floats (x >> 8) 2^-24, bit for bit."""
    import torch
    announce("float conversion edges")
    st = np.array([[x, 0] if x else [1, (1 << 64) - 1] for x in EDGE64], dtype=np.uint64)
    with P.Streams("xoroshiro128+", states=st.reshape(-1)) as s:
        u = to_u64(s.generate(1, P.SLRNG_U64))[:, 0]
        s.set_state(st)
        d = s.generate(1, P.SLRNG_F64).cpu().numpy()[:, 0]
    x = np.array(EDGE64, dtype=np.uint64)
    assert (u == x).all()
    exp = (x >> np.uint64(11)).astype(np.float64) * 2.0**-53
    assert (d.view(np.uint64) == exp.view(np.uint64)).all()
    assert (d < 1.0).all() and d[EDGE64.index((1 << 64) - 1)] == 1.0 - 2.0**-53
    st32 = np.array([[x, 0, 0, 0] if x else [1, 0, 0, (1 << 32) - 1] for x in EDGE32], dtype=np.uint64)
    with P.Streams("xoshiro128+", states=st32.reshape(-1)) as s:
        w = s.generate(1, P.SLRNG_U32).cpu().numpy().view(np.uint32)[:, 0]
        s.set_state(st32)
        f = s.generate(1, P.SLRNG_F32).cpu().numpy()[:, 0]
    x32 = np.array(EDGE32, dtype=np.uint64)
    assert (w == x32.astype(np.uint32)).all()
    assert (f.view(np.uint32) == O.to_float32(x32).view(np.uint32)).all()
    torch.cuda.synchronize()


def test_positioning_levels_beyond_1024(P):
    """Streams past 1024 use the second (wave-uniform) positioning level."""
    name = "xoshiro256++"
    g = O.GEN64[name]
    S = 3000
    chain = oracle_streams(name, 42, S)
    with P.Streams(name, 42, S) as s:
        assert (s.get_state() == chain).all()


def test_config1_xoshiro256ss_1024x4096(P):
    """xoshiro256**, 1,024 streams from seed 42, stream i = base jumped i times
    by 2^128, 4,096 outputs per stream, stream-major; compared in full."""
    check_generate(P, "xoshiro256**", 42, 1024, 4096)

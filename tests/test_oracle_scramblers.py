"""Pins of the oracle's scramblers, seeding and double conversion.

The equidistribution facts of Section "Equidistribution" are checked by
exhaustive enumeration of small-word instances that run through the same
oracle code as the 64-bit generators:
  * Prop. xoroshirop / xoroshiropp: (k-1)-dimensional equidistribution when ++
    scrambles "the last and first word" (adds the last word), and the 4-bit,
    16-bit-state instance (a, b, c) = (3, 1, 2) fails 3 dimensions when ++ adds
    the first word instead;
  * the 5-bit, 10-bit-state xoroshiro+ (1, 3, 1) is not 2-dimensionally
    equidistributed (but is 1-dimensionally);
  * Prop. xoshiro256p / xoshiro256pp: 3 dimensions for + on the first and last
    word and ++ adding the first; the 2-bit, 8-bit-state xoshiro+ is not
    4-dimensionally equidistributed;
  * Prop. xoshiro512p / xoshiro512pp: 7 dimensions for + on the first and third
    word and ++ adding the third.
A mistaken word choice or order in the +/++ code fails one of these (the
mutation checks below plant such mistakes in a Python copy and show that the
same criterion rejects them)."""
import collections

import numpy as np
import pytest

import oracle as O


def equidistributed(counts):
    return len(set(counts.tolist())) == 1


def test_xoroshiro_plus_small_counterexample():
    g = O.Gen(O.XOROSHIRO, 5, 2, 1, 3, 1, O.PLUS)
    assert equidistributed(O.tuple_counts(g, 1))
    assert not equidistributed(O.tuple_counts(g, 2))


@pytest.mark.parametrize("r", [1, 2, 3])
def test_xoroshiro_plusplus_last_and_first_is_k_minus_1_dim(r):
    g = O.Gen(O.XOROSHIRO, 4, 4, 3, 1, 2, O.PLUSPLUS, r)
    assert equidistributed(O.tuple_counts(g, 3))


def test_xoroshiro_plus_k4_is_3_dim():
    g = O.Gen(O.XOROSHIRO, 4, 4, 3, 1, 2, O.PLUS)
    assert equidistributed(O.tuple_counts(g, 3))


def test_xoroshiro128_plusplus_and_plus_1_dim():
    for scr in (O.PLUS, O.PLUSPLUS):
        g = O.Gen(O.XOROSHIRO, 5, 2, 1, 3, 1, scr, 2)
        assert equidistributed(O.tuple_counts(g, 1))


def test_xoshiro256_plus_3_dim_not_4():
    g = O.Gen(O.XOSHIRO, 2, 4, 1, 1, 0, O.PLUS)
    assert equidistributed(O.tuple_counts(g, 3))
    assert not equidistributed(O.tuple_counts(g, 4))


@pytest.mark.parametrize("w,a,b", [(4, 1, 1), (5, 1, 3), (5, 2, 2)])
def test_xoshiro256_plusplus_3_dim(w, a, b):
    for r in range(1, w):
        g = O.Gen(O.XOSHIRO, w, 4, a, b, 0, O.PLUSPLUS, r)
        assert equidistributed(O.tuple_counts(g, 3))


def test_xoshiro512_plus_and_plusplus_7_dim():
    g = O.Gen(O.XOSHIRO, 2, 8, 1, 1, 0, O.PLUS)
    assert equidistributed(O.tuple_counts(g, 7))
    assert not equidistributed(O.tuple_counts(g, 8))
    g = O.Gen(O.XOSHIRO, 2, 8, 1, 1, 0, O.PLUSPLUS, 1)
    assert equidistributed(O.tuple_counts(g, 7))


def test_star_and_starstar_keep_max_dimension():
    # Section "Equidistribution": * and ** remap outputs bijectively, so a
    # k-dimensionally equidistributed word stays so.
    g = O.Gen(O.XOROSHIRO, 5, 2, 1, 3, 1, O.STARSTAR, 2, 5, 9)
    assert equidistributed(O.tuple_counts(g, 2))
    g = O.Gen(O.XOROSHIRO, 5, 2, 1, 3, 1, O.STAR, 0, 0b10011)
    assert equidistributed(O.tuple_counts(g, 2))
    g = O.Gen(O.XOSHIRO, 4, 4, 1, 1, 0, O.STARSTAR, 3, 5, 9)
    assert equidistributed(O.tuple_counts(g, 4))


# ------------------------------------------------------------ mutation checks

def _counts(w, k, fam, abc, d, fn):
    e = O.Gen(fam, w, k, *abc)
    m = (1 << w) - 1
    cnt = collections.Counter()
    for v in range(1 << (k * w)):
        x = [(v >> (w * j)) & m for j in range(k)]
        idx = 0
        for t in range(d):
            idx |= fn(x, m, w) << (w * t)
            x = [int(y) for y in O.advance(e, x, 1)]
        cnt[idx] += 1
    return len(cnt) == 1 << (d * w) and len(set(cnt.values())) == 1


def _rotl(x, r, w, m):
    return ((x << r) | (x >> (w - r))) & m


def test_planted_word_mistakes_fail_the_criteria():
    # ++ adding the first word on xoroshiro with k = 4 (text after Prop.
    # xoroshiropp): not 3-dimensionally equidistributed
    assert not _counts(4, 4, O.XOROSHIRO, (3, 1, 2), 3,
                       lambda x, m, w: (_rotl((x[0] + x[3]) & m, 1, w, m) + x[0]) & m)
    # xoshiro256++ adding the last word instead of the first
    assert not _counts(4, 4, O.XOSHIRO, (1, 1, 0), 3,
                       lambda x, m, w: (_rotl((x[0] + x[3]) & m, 1, w, m) + x[3]) & m)
    # xoshiro256+ on words 0 and 1
    assert not _counts(4, 4, O.XOSHIRO, (1, 1, 0), 3, lambda x, m, w: (x[0] + x[1]) & m)


# ------------------------------------------------------------ bijectivity

def test_starstar_and_star_are_bijections_64():
    # odd multipliers and a rotation are invertible: undo them
    rng = np.random.default_rng(8)
    M64 = (1 << 64) - 1
    inv5, inv9 = pow(5, -1, 1 << 64), pow(9, -1, 1 << 64)
    invS = pow(O.STAR_S, -1, 1 << 64)
    g = O.GEN64["xoshiro256**"]
    gs = O.GEN64["xoroshiro128*"]
    for _ in range(50):
        x = rng.integers(0, 2**64, size=4, dtype=np.uint64)
        y = O.output(g, x)
        z = (y * inv9) & M64
        z = ((z >> 7) | (z << 57)) & M64
        assert (z * inv5) & M64 == int(x[1])
        y = O.output(gs, x[:2])
        assert (y * invS) & M64 == int(x[0])


def test_plusplus_rotation_parameter_changes_output():
    # a dropped rotation would make ++ equal to 2*x + y
    g = O.GEN64["xoshiro256++"]
    x = O.splitmix_fill(5, 4)
    y = O.output(g, x)
    assert y != (2 * int(x[0]) + int(x[3])) & ((1 << 64) - 1)


# ------------------------------------------------------------ seeding

def test_splitmix_gamma_is_odd_integer_nearest_2_64_over_phi():
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    phi = (1 + Decimal(5).sqrt()) / 2
    v = Decimal(2 ** 64) / phi
    lo = int(v)
    cands = [c for c in (lo - 1, lo, lo + 1, lo + 2) if c % 2 == 1]
    nearest = min(cands, key=lambda c: abs(Decimal(c) - v))
    assert O.splitmix_gamma() == nearest


# The SplitMix64 finalizer as the SplitMix publication states it (Steele, Lea
# and Flood, OOPSLA 2014: xor-shift 30, multiply, xor-shift 27, multiply,
# xor-shift 31).  The inverse below is derived here, independently of the
# oracle's code: each xor-shift is undone by iterating it, each multiplication
# by the multiplicative inverse modulo 2^64.
MIX_SHIFTS = (30, 27, 31)
MIX_MULTS = (0xBF58476D1CE4E5B9, 0x94D049BB133111EB)
M64 = (1 << 64) - 1


def _unxorshift(y, s):
    # y = z ^ (z >> s)  =>  z = y ^ (y >> s) ^ (y >> 2s) ^ ...
    z, t = y, y >> s
    while t:
        z ^= t
        t >>= s
    return z


def _unmix(y):
    s1, s2, s3 = MIX_SHIFTS
    m1, m2 = MIX_MULTS
    z = _unxorshift(y, s3)
    z = (z * pow(m2, -1, 1 << 64)) & M64
    z = _unxorshift(z, s2)
    z = (z * pow(m1, -1, 1 << 64)) & M64
    return _unxorshift(z, s1)


def _round_trip_fails(mix, samples):
    return [z for z in samples if _unmix(mix(z)) != z]


def _samples(n=2000):
    rng = np.random.default_rng(20140)
    return [0, 1, M64, 1 << 63] + [int(v) for v in rng.integers(0, 2**64, n, dtype=np.uint64)]


def test_splitmix_finalizer_inverts_on_random_inputs():
    # Seeding, Section "Choosing a generator": the finalizer is a bijection of
    # 64-bit words (so distinct counters give distinct outputs); its inverse,
    # built from the publication's shifts and multipliers, undoes the oracle's
    # finalizer on every sample.
    assert _round_trip_fails(O.splitmix_mix, _samples()) == []
    # and the inverse is a true inverse of the publication's finalizer
    def mix_here(z):
        z = ((z ^ (z >> 30)) * MIX_MULTS[0]) & M64
        z = ((z ^ (z >> 27)) * MIX_MULTS[1]) & M64
        return z ^ (z >> 31)
    assert all(mix_here(_unmix(z)) == z for z in _samples(200))


@pytest.mark.parametrize("old,new", [
    ("z >> 30", "z >> 29"), ("z >> 27", "z >> 28"), ("z >> 31", "z >> 32"),
    ("0xbf58476d1ce4e5b9ULL", "0xbf58476d1ce4e5bbULL"),
    ("0x94d049bb133111ebULL", "0x94d049bb133111e9ULL")])
def test_one_constant_edit_of_the_finalizer_fails_the_inversion(tmp_path, old, new):
    # a planted mistake in a copy of the oracle: one shift or multiplier of
    # the finalizer changed (the multiplier stays odd, the map stays a
    # bijection) must make the inversion above fail
    import ctypes
    import subprocess
    src = open(O._SRC).read()
    assert src.count(old) == 1
    path = tmp_path / "orc_planted.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "liborc_planted.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", str(lib), str(path),
                           "-lpthread"])
    L = ctypes.CDLL(str(lib))
    L.orc_splitmix_mix.argtypes = [ctypes.c_uint64]
    L.orc_splitmix_mix.restype = ctypes.c_uint64
    assert len(_round_trip_fails(L.orc_splitmix_mix, _samples(200))) > 150


def test_seeded_states_are_never_all_zero():
    for k in (2, 4, 8, 16):
        for seed in list(range(200)) + [2**64 - 1, 2**63]:
            assert O.splitmix_fill(seed, k).any()


def test_fill_uses_consecutive_outputs():
    x = O.splitmix_fill(42, 16)
    y = O.splitmix_fill(42, 4)
    assert x[:4].tolist() == y.tolist()
    gam = O.splitmix_gamma()
    assert int(x[0]) == O.splitmix_mix((42 + gam) & ((1 << 64) - 1))
    assert int(x[3]) == O.splitmix_mix((42 + 4 * gam) & ((1 << 64) - 1))


# ------------------------------------------------------------ doubles

def test_double_is_exact_upper_53_bits():
    rng = np.random.default_rng(9)
    vals = [0, 1, (1 << 11) - 1, 1 << 11, (1 << 64) - 1, 1 << 63] + \
        rng.integers(0, 2**64, 200, dtype=np.uint64).tolist()
    for v in vals:
        d = O.to_double(int(v))
        assert 0.0 <= d < 1.0
        assert int(d * 2.0**53) == int(v) >> 11
        assert d * 2.0**53 == float(int(v) >> 11)
    assert O.to_double((1 << 64) - 1) == 1.0 - 2.0**-53


def test_generate_many_both_kinds_agree():
    g = O.GEN64["xoroshiro1024**"]
    st = np.stack([O.splitmix_fill(s, 16) for s in range(5)])
    (u, d), fin = O.generate_many(g, st, 100, kind="both", nthreads=2)
    assert (d * 2.0**53 == (u >> np.uint64(11)).astype(np.float64)).all()
    d2, fin2 = O.generate_many(g, st, 100, kind="f64", nthreads=1)
    assert (d2 == d).all() and (fin2 == fin).all()
    for i in range(5):
        o, f = O.generate(g, st[i], 100)
        assert (o == u[i]).all() and (f == fin[i]).all()

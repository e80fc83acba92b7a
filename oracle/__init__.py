"""CPU oracle for the scrambled linear generators of Blackman & Vigna,
"Scrambled Linear Pseudorandom Number Generators".

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only code allowed to import this package.  It is
a plain, slow, serial restatement of the paper (``orc.c`` for the engines,
scramblers, seeding, Berlekamp-Massey and polynomial arithmetic;
``matrices.py`` for the block matrices of Section "Linear engines").  It shares
no code with the GPU library and never imports it.

Polynomials over Z/2Z are Python integers: bit i is the coefficient of x^i.
States are numpy uint64 arrays in the logical order of the block matrices
(word j of the row vector the transition matrix multiplies from the right).

The engine step is the product of the state with the block matrix the paper
prints (X_2w, X_kw of equation eq:M, S_4w, S_8w), expanded block by block; the
code figures are not transcribed.

Parity unpinned (no fact of the paper fixes these; they follow the code
figures or the cited publication, and no external test vector exists here):
  * the SplitMix64 finalizer constants (shifts 30, 27, 31 and its two
    multipliers), checked only by inverting the finalizer with the test's own
    statement of them;
  * the word that ``**`` scrambles (the first logical word of xoroshiro, word
    1 of xoshiro);
  * the word ``++`` adds back for the two-word xoroshiro (the first);
  * the split of SplitMix64 outputs into the 32-bit generators' words (low
    half first).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

XOROSHIRO, XOSHIRO = 0, 1
NONE, PLUS, PLUSPLUS, STAR, STARSTAR = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile orc.c into liborc.so with plain gcc (-O2, no vector flags)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _Gen(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("w", ctypes.c_int32), ("k", ctypes.c_int32),
                ("a", ctypes.c_int32), ("b", ctypes.c_int32), ("c", ctypes.c_int32),
                ("scr", ctypes.c_int32), ("r", ctypes.c_int32),
                ("ms", ctypes.c_uint64), ("mt", ctypes.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        u64p, u8p = P(ctypes.c_uint64), P(ctypes.c_uint8)
        g = P(_Gen)
        L.orc_valid.argtypes = [g]
        L.orc_advance.argtypes = [g, u64p, ctypes.c_uint64]
        L.orc_output.argtypes = [g, u64p]
        L.orc_output.restype = ctypes.c_uint64
        L.orc_generate1.argtypes = [g, u64p, ctypes.c_uint64, u64p]
        L.orc_generate_window.argtypes = [g, u64p, ctypes.c_uint64, ctypes.c_uint64, u64p]
        L.orc_generate_many.argtypes = [g, u64p, ctypes.c_uint64, ctypes.c_uint64, u64p,
                                        P(ctypes.c_double), ctypes.c_uint64, ctypes.c_int]
        L.orc_to_double.argtypes = [ctypes.c_uint64]
        L.orc_to_double.restype = ctypes.c_double
        L.orc_splitmix_gamma.restype = ctypes.c_uint64
        L.orc_splitmix_mix.argtypes = [ctypes.c_uint64]
        L.orc_splitmix_mix.restype = ctypes.c_uint64
        L.orc_splitmix_fill.argtypes = [ctypes.c_uint64, u64p, ctypes.c_int]
        L.orc_berlekamp_massey.argtypes = [u8p, ctypes.c_long, u8p]
        L.orc_berlekamp_massey.restype = ctypes.c_long
        L.orc_poly_mulmod.argtypes = [u64p, u64p, u64p, ctypes.c_int, u64p]
        L.orc_poly_xpow.argtypes = [u64p, ctypes.c_int, u64p, ctypes.c_int, u64p]
        L.orc_charpoly.argtypes = [g, u64p, u64p]
        L.orc_charpoly.restype = ctypes.c_long
        L.orc_jump_poly.argtypes = [g, u64p, u64p]
        L.orc_stream_chain.argtypes = [g, ctypes.c_uint64, u64p, ctypes.c_uint64, u64p]
        L.orc_seed_state.argtypes = [g, ctypes.c_uint64, u64p]
        L.orc_jump_many.argtypes = [g, u64p, ctypes.c_uint64, u64p, ctypes.c_int]
        L.orc_period.argtypes = [g, u64p, ctypes.c_uint64]
        L.orc_period.restype = ctypes.c_uint64
        L.orc_tuple_counts.argtypes = [g, ctypes.c_int, P(ctypes.c_uint32)]
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# Generators
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Gen:
    family: int
    w: int
    k: int
    a: int
    b: int
    c: int = 0
    scr: int = NONE
    r: int = 0
    ms: int = 0
    mt: int = 0

    @property
    def n(self) -> int:
        return self.k * self.w

    def c_struct(self) -> _Gen:
        return _Gen(self.family, self.w, self.k, self.a, self.b, self.c, self.scr, self.r,
                    self.ms, self.mt)

    def engine(self) -> "Gen":
        return replace(self, scr=NONE, r=0, ms=0, mt=0)


# Table tab:scr64: the * multiplier, and ** with S = 5, R = 7, T = 9.
STAR_S = 0x9E3779B97F4A7C13
SS = dict(scr=STARSTAR, r=7, ms=5, mt=9)

# Table tab:par64 (engine parameters) and tab:scr64 (++ rotations).  The
# xoroshiro128 row applies to +, * and **; xoroshiro128++ has its own row.
GEN64 = {
    "xoroshiro128+": Gen(XOROSHIRO, 64, 2, 24, 16, 37, PLUS),
    "xoroshiro128++": Gen(XOROSHIRO, 64, 2, 49, 21, 28, PLUSPLUS, 17),
    "xoroshiro128**": Gen(XOROSHIRO, 64, 2, 24, 16, 37, **SS),
    "xoroshiro128*": Gen(XOROSHIRO, 64, 2, 24, 16, 37, STAR, ms=STAR_S),
    "xoshiro256+": Gen(XOSHIRO, 64, 4, 17, 45, 0, PLUS),
    "xoshiro256++": Gen(XOSHIRO, 64, 4, 17, 45, 0, PLUSPLUS, 23),
    "xoshiro256**": Gen(XOSHIRO, 64, 4, 17, 45, 0, **SS),
    "xoshiro512+": Gen(XOSHIRO, 64, 8, 11, 21, 0, PLUS),
    "xoshiro512++": Gen(XOSHIRO, 64, 8, 11, 21, 0, PLUSPLUS, 17),
    "xoshiro512**": Gen(XOSHIRO, 64, 8, 11, 21, 0, **SS),
    "xoroshiro1024+": Gen(XOROSHIRO, 64, 16, 25, 27, 36, PLUS),
    "xoroshiro1024++": Gen(XOROSHIRO, 64, 16, 25, 27, 36, PLUSPLUS, 23),
    "xoroshiro1024**": Gen(XOROSHIRO, 64, 16, 25, 27, 36, **SS),
    "xoroshiro1024*": Gen(XOROSHIRO, 64, 16, 25, 27, 36, STAR, ms=STAR_S),
}


# Section "The 32-bit case": tables tab:par32 (engines xoroshiro64 26/9/13,
# xoshiro128 9/11) and tab:scr32 (scramblers).  The * and ** of xoroshiro64
# multiply by 0x9E3779BB (** with R = 5, T = 5); ** of xoshiro128 has S = 5,
# R = 7, T = 9, and its ++ rotates by 7.
STAR32_S = 0x9E3779BB
GEN32 = {
    "xoroshiro64*": Gen(XOROSHIRO, 32, 2, 26, 9, 13, STAR, ms=STAR32_S),
    "xoroshiro64**": Gen(XOROSHIRO, 32, 2, 26, 9, 13, STARSTAR, r=5, ms=STAR32_S, mt=5),
    "xoshiro128+": Gen(XOSHIRO, 32, 4, 9, 11, 0, PLUS),
    "xoshiro128++": Gen(XOSHIRO, 32, 4, 9, 11, 0, PLUSPLUS, 7),
    "xoshiro128**": Gen(XOSHIRO, 32, 4, 9, 11, 0, STARSTAR, r=7, ms=5, mt=9),
}


def to_float32(v) -> np.ndarray:
    """Upper 24 bits of 32-bit outputs as floats in [0, 1): (v >> 8) * 2^-24,
    exact (the 32-bit analogue of the 53-bit doubles)."""
    v = np.asarray(v, dtype=np.uint64)
    return ((v >> np.uint64(8)).astype(np.float64) * 2.0**-24).astype(np.float32)


def _u64p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _words(x: int, nwords: int) -> np.ndarray:
    out = np.zeros(nwords, dtype=np.uint64)
    for i in range(nwords):
        out[i] = (x >> (64 * i)) & 0xFFFFFFFFFFFFFFFF
    return out


def _int(words: np.ndarray) -> int:
    v = 0
    for i, wd in enumerate(words.tolist()):
        v |= int(wd) << (64 * i)
    return v


def _state(x, k) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.uint64).reshape(-1).copy())
    assert a.size == k
    return a


# --------------------------------------------------------------------------
# Engine, scrambler, generation
# --------------------------------------------------------------------------

def advance(g: Gen, x, nsteps: int) -> np.ndarray:
    s = _state(x, g.k)
    lib().orc_advance(ctypes.byref(g.c_struct()), _u64p(s), nsteps)
    return s


def output(g: Gen, x) -> int:
    s = _state(x, g.k)
    return int(lib().orc_output(ctypes.byref(g.c_struct()), _u64p(s)))


def generate(g: Gen, x, n: int):
    """One stream: returns (outputs[n], state after n steps)."""
    s = _state(x, g.k)
    out = np.zeros(max(n, 1), dtype=np.uint64)
    lib().orc_generate1(ctypes.byref(g.c_struct()), _u64p(s), n, _u64p(out))
    return out[:n], s


def generate_window(g: Gen, x, t_lo: int, t_hi: int):
    s = _state(x, g.k)
    out = np.zeros(max(t_hi - t_lo, 1), dtype=np.uint64)
    lib().orc_generate_window(ctypes.byref(g.c_struct()), _u64p(s), t_lo, t_hi, _u64p(out))
    return out[:t_hi - t_lo], s


def generate_many(g: Gen, states: np.ndarray, n: int, kind: str = "u64", nthreads: int = 0):
    """Stream-major outputs for S streams: returns (out[S, n], final states[S, k]).

    kind: "u64" for integers, "f64" for doubles, "both" for (u64, f64)."""
    st = np.ascontiguousarray(np.asarray(states, dtype=np.uint64).reshape(-1, g.k).copy())
    S = st.shape[0]
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    u = np.zeros((S, n), dtype=np.uint64) if kind in ("u64", "both") else None
    d = np.zeros((S, n), dtype=np.float64) if kind in ("f64", "both") else None
    if S and n:
        rc = lib().orc_generate_many(
            ctypes.byref(g.c_struct()), _u64p(st), S, n,
            _u64p(u) if u is not None else None,
            d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if d is not None else None,
            n, nthreads)
        assert rc == 0
    elif S and n == 0:
        pass
    if kind == "u64":
        return u, st
    if kind == "f64":
        return d, st
    return (u, d), st


def to_double(v: int) -> float:
    return float(lib().orc_to_double(v))


# --------------------------------------------------------------------------
# Seeding
# --------------------------------------------------------------------------

def splitmix_gamma() -> int:
    return int(lib().orc_splitmix_gamma())


def splitmix_mix(z: int) -> int:
    return int(lib().orc_splitmix_mix(z))


def splitmix_fill(seed: int, k: int) -> np.ndarray:
    x = np.zeros(k, dtype=np.uint64)
    lib().orc_splitmix_fill(seed & 0xFFFFFFFFFFFFFFFF, _u64p(x), k)
    return x


# --------------------------------------------------------------------------
# F2 tools: Berlekamp-Massey and polynomial arithmetic
# --------------------------------------------------------------------------

def berlekamp_massey(bits) -> tuple[int, list[int]]:
    """Linear complexity L and connection polynomial coefficients c_0..c_L."""
    s = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8) & 1)
    N = s.size
    conn = np.zeros(N + 1, dtype=np.uint8)
    L = lib().orc_berlekamp_massey(s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), N,
                                   conn.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    assert L >= 0
    return int(L), conn[:L + 1].tolist()


def poly_mulmod(a: int, b: int, p: int) -> int:
    n = p.bit_length() - 1
    W = n // 64 + 1
    out = np.zeros(W, dtype=np.uint64)
    A, B, Pw = _words(a, W), _words(b, W), _words(p, W)
    lib().orc_poly_mulmod(_u64p(A), _u64p(B), _u64p(Pw), n, _u64p(out))
    return _int(out)


def xpow_mod(J: int, p: int) -> int:
    """x^J mod p."""
    n = p.bit_length() - 1
    W = n // 64 + 1
    nj = max(1, (J.bit_length() + 63) // 64)
    jw = _words(J, nj)
    out = np.zeros(W, dtype=np.uint64)
    Pw = _words(p, W)
    lib().orc_poly_xpow(_u64p(jw), nj, _u64p(Pw), n, _u64p(out))
    return _int(out)


_charpoly_cache: dict = {}


def charpoly(g: Gen, x0=None) -> int:
    """Characteristic polynomial of g's engine by Berlekamp-Massey on bit 0 of
    word 0 over 2n steps from x0 (default: a SplitMix-filled state)."""
    e = g.engine()
    key = (e, None if x0 is None else tuple(int(v) for v in x0))
    if key in _charpoly_cache:
        return _charpoly_cache[key]
    if x0 is None:
        x0 = splitmix_fill(1, g.k) & np.uint64((1 << g.w) - 1 if g.w < 64 else 0xFFFFFFFFFFFFFFFF)
    s = _state(x0, g.k)
    W = g.n // 64 + 1
    out = np.zeros(W, dtype=np.uint64)
    L = lib().orc_charpoly(ctypes.byref(e.c_struct()), _u64p(s), _u64p(out))
    p = _int(out)
    assert p.bit_length() - 1 == L
    _charpoly_cache[key] = p
    return p


def jump_poly(g: Gen, x, r: int) -> np.ndarray:
    """x * M^J given r = x^J mod p."""
    s = _state(x, g.k)
    R = _words(r, g.n // 64 + 1)
    lib().orc_jump_poly(ctypes.byref(g.c_struct()), _u64p(s), _u64p(R))
    return s


def jump(g: Gen, x, J: int) -> np.ndarray:
    """x * M^J for an arbitrary nonnegative J (x^J mod p, then accumulate)."""
    return jump_poly(g, x, xpow_mod(J, charpoly(g)))


def jump_many(g: Gen, states: np.ndarray, J: int, nthreads: int = 0) -> np.ndarray:
    st = np.ascontiguousarray(np.asarray(states, dtype=np.uint64).reshape(-1, g.k).copy())
    R = _words(xpow_mod(J, charpoly(g)), g.n // 64 + 1)
    lib().orc_jump_many(ctypes.byref(g.c_struct()), _u64p(st), st.shape[0], _u64p(R),
                        nthreads or (os.cpu_count() or 1))
    return st


def jump_distance(g: Gen, kind: str = "jump") -> int:
    """The jump distances: 2^(n/2) for "jump", 2^(3n/4) for "long"."""
    return 1 << (g.n // 2) if kind == "jump" else 1 << (3 * g.n // 4)


def stream_chain(g: Gen, seed: int, S: int, J: int | None = None) -> np.ndarray:
    """Streams i = 0..S-1: SplitMix-filled base state jumped i times by J
    (default: the 2^(n/2) jump).  Returns S x k."""
    if J is None:
        J = jump_distance(g, "jump")
    r = xpow_mod(J, charpoly(g))
    R = _words(r, g.n // 64 + 1)
    out = np.zeros((S, g.k), dtype=np.uint64)
    lib().orc_stream_chain(ctypes.byref(g.c_struct()), seed & 0xFFFFFFFFFFFFFFFF, _u64p(R), S,
                           _u64p(out))
    return out


def seed_state(g: Gen, seed: int) -> np.ndarray:
    """The seeded base state: SplitMix64 outputs as the words (64-bit words),
    or the SplitMix64 output stream cut into 32-bit words, low half first."""
    x = np.zeros(g.k, dtype=np.uint64)
    lib().orc_seed_state(ctypes.byref(g.c_struct()), seed & 0xFFFFFFFFFFFFFFFF, _u64p(x))
    return x


def stream_state(g: Gen, seed: int, i: int, extra_steps: int = 0) -> np.ndarray:
    """Stream i of the chain, advanced by extra_steps, computed directly by one
    jump of distance i*2^(n/2) + extra_steps."""
    base = seed_state(g, seed)
    return jump(g, base, i * jump_distance(g, "jump") + extra_steps)


# --------------------------------------------------------------------------
# Small-instance tools
# --------------------------------------------------------------------------

def period(g: Gen, x0, limit: int) -> int:
    s = _state(x0, g.k)
    return int(lib().orc_period(ctypes.byref(g.c_struct()), _u64p(s), limit))


def tuple_counts(g: Gen, d: int) -> np.ndarray:
    counts = np.zeros(1 << (d * g.w), dtype=np.uint32)
    rc = lib().orc_tuple_counts(ctypes.byref(g.c_struct()), d,
                                counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    assert rc == 0
    return counts

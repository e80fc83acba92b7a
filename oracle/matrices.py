"""Transition matrices of the linear engines, built from the block matrices of
Section "Linear engines" (X_kw of equation eq:M, S_4w and S_8w), independently
of the code figures.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions taken from the text of Section "Linear engines":
  * a state is a row vector and the next state is the vector times M;
  * S is the w x w matrix with ones on the principal subdiagonal (a left shift
    of one position of a binary row vector) and R adds a one in the upper right
    corner (a left rotation).  With the row vector read most significant bit
    first, x S^b is the C expression x << b and x R^a is rotl(x, a);
  * a kw-bit state is the concatenation of its k words in the order of the
    matrix blocks.

Matrices are numpy uint8 arrays over Z/2Z.
"""
from __future__ import annotations

import numpy as np


def I(w: int) -> np.ndarray:
    return np.eye(w, dtype=np.uint8)


def Z(w: int) -> np.ndarray:
    return np.zeros((w, w), dtype=np.uint8)


def S(w: int) -> np.ndarray:
    """Ones on the principal subdiagonal: entry (i, j) = 1 iff i = j + 1."""
    m = np.zeros((w, w), dtype=np.uint8)
    for j in range(w - 1):
        m[j + 1, j] = 1
    return m


def R(w: int) -> np.ndarray:
    """S plus a one in the upper right corner."""
    m = S(w)
    m[0, w - 1] = 1
    return m


def mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Product over Z/2Z (exact: float32 sums stay below 2^24 for n <= 4096)."""
    return (a.astype(np.float32) @ b.astype(np.float32)).astype(np.int64).astype(np.uint8) & 1


def mpow(m: np.ndarray, e: int) -> np.ndarray:
    out = np.eye(m.shape[0], dtype=np.uint8)
    base = m.copy()
    while e:
        if e & 1:
            out = mul(out, base)
        e >>= 1
        if e:
            base = mul(base, base)
    return out


def _blocks(rows, w: int) -> np.ndarray:
    return np.block([[blk if not isinstance(blk, int) else (I(w) if blk == 1 else Z(w))
                      for blk in row] for row in rows]).astype(np.uint8) & 1


def xoroshiro(w: int, k: int, a: int, b: int, c: int) -> np.ndarray:
    """X_kw of equation eq:M (for k = 2, the matrix X_2w)."""
    Ra, Sb, Rc = mpow(R(w), a), mpow(S(w), b), mpow(R(w), c)
    top = (Ra + Sb + I(w)) & 1
    bot = (Sb + I(w)) & 1
    if k == 2:
        return _blocks([[top, Rc], [bot, Rc]], w)
    rows = []
    rows.append([0] * (k - 2) + [top, Rc])
    for i in range(1, k - 1):
        rows.append([1 if j == i - 1 else 0 for j in range(k)])
    rows.append([0] * (k - 2) + [bot, Rc])
    return _blocks(rows, w)


def xoshiro(w: int, k: int, a: int, b: int) -> np.ndarray:
    """S_4w and S_8w of Section "Linear engines"."""
    Sa, Rb = mpow(S(w), a), mpow(R(w), b)
    if k == 4:
        rows = [[1, 1, 1, 0],
                [1, 1, Sa, Rb],
                [0, 1, 1, 0],
                [1, 0, 0, Rb]]
    elif k == 8:
        rows = [[1, 1, 1, 0, 0, 0, 0, 0],
                [0, 1, 0, 0, 1, 1, Sa, 0],
                [0, 1, 1, 0, 0, 0, 0, 0],
                [0, 0, 0, 1, 0, 0, 1, Rb],
                [0, 0, 0, 1, 1, 0, 0, 0],
                [0, 0, 0, 0, 1, 1, 0, 0],
                [1, 0, 0, 0, 0, 0, 1, 0],
                [0, 0, 0, 0, 0, 0, 1, Rb]]
    else:
        raise ValueError("xoshiro is defined for 4 and 8 words")
    return _blocks(rows, w)


def matrix_for(gen) -> np.ndarray:
    """Transition matrix of an ``oracle.Gen``'s engine."""
    if gen.family == 0:
        return xoroshiro(gen.w, gen.k, gen.a, gen.b, gen.c)
    return xoshiro(gen.w, gen.k, gen.a, gen.b)


def to_bits(words, w: int) -> np.ndarray:
    """Row vector of a state: each word most significant bit first."""
    out = []
    for x in words:
        x = int(x)
        out.extend((x >> (w - 1 - i)) & 1 for i in range(w))
    return np.array(out, dtype=np.uint8)


def from_bits(bits: np.ndarray, w: int) -> list[int]:
    words = []
    for j in range(0, bits.size, w):
        v = 0
        for i in range(w):
            v = (v << 1) | int(bits[j + i])
        words.append(v)
    return words


def apply(m: np.ndarray, words, w: int) -> list[int]:
    """Next state x * M of a state given as words."""
    v = to_bits(words, w)
    return from_bits(mul(v[None, :], m)[0], w)


def rank(m: np.ndarray) -> int:
    """Rank over Z/2Z by Gaussian elimination."""
    a = m.copy() & 1
    rows, cols = a.shape
    r = 0
    for c in range(cols):
        piv = None
        for i in range(r, rows):
            if a[i, c]:
                piv = i
                break
        if piv is None:
            continue
        if piv != r:
            a[[r, piv]] = a[[piv, r]]
        nz = np.nonzero(a[:, c])[0]
        for i in nz:
            if i != r:
                a[i] ^= a[r]
        r += 1
        if r == rows:
            break
    return r

"""The paper's horizontal Z_17 layout and its relation to the vertical one.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4.5 stores one codeword of R_17 per 16-bit word: bit r of the word
is the coefficient of x^r, and multiplying by g is
``y = (x + x) XOR (all ones if x is negative as an int16)``.  The library
slices bits vertically instead: a strip is 16 rows of W bytes and the
codeword of lane (byte j, bit b) has its x^r coefficient in bit b of byte j
of row r.  Codeword c of a horizontal strip of 8W words is taken to be lane
(c // 8, c % 8) of the vertical strip; both layouts then hold the same ring
elements, so a stripe has the same parity in either.
"""

from __future__ import annotations

import numpy as np

ROWS = 16


def to_vertical(words: np.ndarray) -> np.ndarray:
    """(..., n) uint16 codewords, n a multiple of 8 -> (..., 16, n // 8) bytes."""
    words = np.asarray(words, dtype=np.uint16)
    n = words.shape[-1]
    if n % 8:
        raise ValueError("the number of codewords must be a multiple of 8")
    out = np.zeros(words.shape[:-1] + (ROWS, n // 8), dtype=np.uint8)
    for r in range(ROWS):
        bits = ((words >> r) & 1).astype(np.uint8).reshape(words.shape[:-1] + (n // 8, 8))
        for b in range(8):
            out[..., r, :] |= bits[..., b] << b
    return out


def to_horizontal(strip: np.ndarray) -> np.ndarray:
    """(..., 16, W) bytes -> (..., 8W) uint16 codewords (inverse of to_vertical)."""
    strip = np.asarray(strip, dtype=np.uint8)
    if strip.shape[-2] != ROWS:
        raise ValueError("a Z_17 strip has 16 rows")
    w = strip.shape[-1]
    out = np.zeros(strip.shape[:-2] + (8 * w,), dtype=np.uint16)
    for r in range(ROWS):
        for b in range(8):
            bit = ((strip[..., r, :] >> b) & 1).astype(np.uint16)       # (..., W): codewords 8j + b
            out[..., b::8] |= bit << r
    return out


def mul_g_packed(x: np.ndarray) -> np.ndarray:
    """g . x on 16-bit words by the Section 4.5 formula."""
    x = np.asarray(x, dtype=np.uint16)
    neg = (x & 0x8000) != 0
    return ((x.astype(np.uint32) << 1) & 0xFFFF).astype(np.uint16) ^ np.where(neg, 0xFFFF, 0).astype(np.uint16)


def encode_packed(data: np.ndarray):
    """(P, Q) of k horizontal data strips ``(..., k, n)`` uint16, by the loop of
    Section 4.5: for i = k-1 down to 0, q = g q + d[i], p = p + d[i]."""
    data = np.asarray(data, dtype=np.uint16)
    k = data.shape[-2]
    p = np.zeros(data.shape[:-2] + data.shape[-1:], dtype=np.uint16)
    q = np.zeros_like(p)
    for i in range(k - 1, -1, -1):
        q = mul_g_packed(q) ^ data[..., i, :]
        p ^= data[..., i, :]
    return p, q

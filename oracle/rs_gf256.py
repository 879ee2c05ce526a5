"""Reed-Solomon RAID-6 over GF(256), the conventional comparison code.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4.1: GF(256) = GF(2)[x]/(x^8+x^4+x^3+x^2+1) (0x11D), generator
``g = {02}``, and for data bytes ``D_0 .. D_{N-1}``::

    P = D_0 + D_1 + ... + D_{N-1}
    Q = D_0 + g D_1 + ... + g^{N-1} D_{N-1}

Every byte position is independent, so a strip is any byte array; the data
array has shape ``(..., N, *strip_shape)`` with axis ``-1 - len(strip_shape)``
indexing the disk.  Here strips are given as ``(..., N, n)`` byte vectors.
"""

from __future__ import annotations

import numpy as np

POLY = 0x11D


def mul2(b: np.ndarray) -> np.ndarray:
    """Multiply bytes by ``{02}``: shift left one place, and when the bit
    shifted out was set, XOR in 0x1D (the low byte of 0x11D) -- Section 4.2."""
    b = np.asarray(b, dtype=np.uint8)
    hi = (b & 0x80) != 0
    return (((b.astype(np.uint16) << 1) & 0xFF) ^ np.where(hi, 0x1D, 0)).astype(np.uint8)


def gf_mul_const(b: np.ndarray, c: int) -> np.ndarray:
    """``c . b`` for a constant byte ``c``: the sum of ``{02}^i . b`` over the
    set bits ``i`` of ``c`` (polynomial multiplication, reduced step by step)."""
    acc = np.zeros_like(np.asarray(b, dtype=np.uint8))
    term = np.asarray(b, dtype=np.uint8).copy()
    for i in range(8):
        if (c >> i) & 1:
            acc ^= term
        term = mul2(term)
    return acc


def gf_mul(a: int, c: int) -> int:
    return int(gf_mul_const(np.array([a], dtype=np.uint8), c)[0])


def gf_pow2(e: int) -> int:
    """``{02}^e`` for ``e >= 0``."""
    v = np.array([1], dtype=np.uint8)
    for _ in range(e % 255):
        v = mul2(v)
    return int(v[0])


def gf_inv(a: int) -> int:
    """Multiplicative inverse by search (the field has 255 nonzero elements)."""
    if a == 0:
        raise ZeroDivisionError("0 has no inverse in GF(256)")
    for c in range(1, 256):
        if gf_mul(a, c) == 1:
            return c
    raise AssertionError("no inverse found: polynomial is not irreducible")


def encode(data: np.ndarray):
    """``(P, Q)`` for data of shape ``(..., N, n)``; Q by Horner's rule
    ``Q = D_0 + g(D_1 + g(... + g D_{N-1}))`` of Section 4.2."""
    n_disks = data.shape[-2]
    P = np.zeros(data.shape[:-2] + data.shape[-1:], dtype=np.uint8)
    for t in range(n_disks):
        P ^= data[..., t, :]
    Q = data[..., n_disks - 1, :].copy()
    for t in range(n_disks - 2, -1, -1):
        Q = mul2(Q) ^ data[..., t, :]
    return P, Q


def recover_two_data(stripe: np.ndarray, x: int, y: int) -> np.ndarray:
    """Rebuild data disks ``x < y`` of an RS stripe ``(..., N+2, n)``
    (disks 0..N-1, then P, then Q), Sections 4.3 and 4.4::

        dP = P + P_xy,  dQ = Q + Q_xy,
        A = (1 + g^{y-x})^{-1},  B = (g^x + g^y)^{-1},
        D_y = A dP + B dQ,  D_x = D_y + dP.
    """
    n_disks = stripe.shape[-2] - 2
    if not 0 <= x < y < n_disks:
        raise ValueError("need two data disks x < y")
    out = stripe.copy()
    data = out[..., :n_disks, :].copy()
    data[..., x, :] = 0
    data[..., y, :] = 0
    pxy, qxy = encode(data)
    dP = out[..., n_disks, :] ^ pxy
    dQ = out[..., n_disks + 1, :] ^ qxy
    A = gf_inv(1 ^ gf_pow2(y - x))
    B = gf_inv(gf_pow2(x) ^ gf_pow2(y))
    dy = gf_mul_const(dP, A) ^ gf_mul_const(dQ, B)
    out[..., y, :] = dy
    out[..., x, :] = dy ^ dP
    return out


def recover(stripe: np.ndarray, erased) -> np.ndarray:
    """Rebuild one or two erased disks (indices ``0 .. N+1``; ``N`` = P,
    ``N+1`` = Q) of an RS stripe ``(..., N+2, n)``, by the cases of the proof
    of Lemma 3.1.2 with the cone ``{g^t}`` of Section 4.1:

    * P and Q, P alone, Q alone: recompute from the data.
    * one data disk ``x``: ``D_x = P + P_x`` (RAID-5 parity).
    * data ``x`` and P: ``D_x = g^{-x} (Q + Q_x)``, then ``P``.
    * data ``x`` and Q: ``D_x = P + P_x``, then ``Q``.
    * data ``x < y``: Sections 4.3 and 4.4 (``recover_two_data``).

    ``P_x``, ``Q_x`` are the syndromes with the erased disks taken as zero.
    ``g^{-x}`` is the inverse of ``g^x``, found by search.
    """
    n_disks = stripe.shape[-2] - 2
    er = sorted(set(int(e) for e in erased))
    if len(er) != len(tuple(erased)) or not 1 <= len(er) <= 2:
        raise ValueError("need one or two distinct erased disks")
    if any(e < 0 or e > n_disks + 1 for e in er):
        raise ValueError("erased index out of range")
    iP, iQ = n_disks, n_disks + 1
    out = stripe.copy()
    data = out[..., :n_disks, :].copy()
    for e in er:
        if e < n_disks:
            data[..., e, :] = 0
    px, qx = encode(data)                 # syndromes without the erased data disks
    if len(er) == 1:
        e = er[0]
        if e < n_disks:
            out[..., e, :] = out[..., iP, :] ^ px
        elif e == iP:
            out[..., iP, :] = px
        else:
            out[..., iQ, :] = qx
        return out
    x, y = er
    if (x, y) == (iP, iQ):
        out[..., iP, :] = px
        out[..., iQ, :] = qx
    elif y == iP:
        dx = gf_mul_const(out[..., iQ, :] ^ qx, gf_inv(gf_pow2(x)))
        out[..., x, :] = dx
        out[..., iP, :] = px ^ dx
    elif y == iQ:
        dx = out[..., iP, :] ^ px
        out[..., x, :] = dx
        out[..., iQ, :] = qx ^ gf_mul_const(dx, gf_pow2(x))
    else:
        out = recover_two_data(out, x, y)
    return out


"""The ring R_p = F2[x]/(1+x+...+x^(p-1)) as the action of the Sylvester matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring).

An element is an array whose axis ``-2`` has ``p-1`` rows; row ``r`` is the
coefficient of ``x^r``.  The trailing axis (bytes) and any leading axes are
independent lanes: every operation below is a whole-row XOR.

Multiplication by the generator ``g = S_p`` follows the Sylvester (companion)
matrix of Lemma 3.4.1, whose p = 17 instance is written out in Section 4.5:
the new row 0 is the old top row ``a_{p-2}``, and the new row ``r >= 1`` is
``a_{r-1} XOR a_{p-2}``.  Powers ``g^i`` are taken as ``i`` such single steps,
never by a closed form: the oracle follows the matrix definition only.
"""

from __future__ import annotations

import numpy as np


def is_odd_prime(p: int) -> bool:
    """True when ``p`` is an odd prime (the condition under which Lemma 3.4.1
    and Corollary 3.2.4 give a two-erasure code with g = S_p)."""
    if p < 3 or p % 2 == 0:
        return False
    d = 3
    while d * d <= p:
        if p % d == 0:
            return False
        d += 2
    return True


def check_prime(p: int) -> None:
    if not is_odd_prime(p):
        raise ValueError(f"p = {p} is not an odd prime")


def zero(p: int, width: int, lead=()) -> np.ndarray:
    return np.zeros(tuple(lead) + (p - 1, width), dtype=np.uint8)


def sylvester_step(a: np.ndarray, p: int) -> np.ndarray:
    """Return ``S_p . a`` (multiplication by ``g``; Lemma 3.4.1, Section 4.5)."""
    if a.shape[-2] != p - 1:
        raise ValueError("element must have p-1 rows")
    top = a[..., p - 2:p - 1, :]          # a_{p-2}, kept as a 1-row slice
    y = np.empty_like(a)
    y[..., 0:1, :] = top
    y[..., 1:, :] = a[..., :p - 2, :] ^ top
    return y


def mul_g_power(a: np.ndarray, i: int, p: int) -> np.ndarray:
    """Return ``g^i . a`` as ``i mod p`` single Sylvester steps (``g^p = Id``,
    Lemma 3.4.1 (i); negative exponents use ``g^{-k} = g^{p-k}``, Section 4.6)."""
    y = a.copy()
    for _ in range(i % p):
        y = sylvester_step(y, p)
    return y


def add(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Ring addition: XOR (characteristic 2)."""
    return a ^ b


def inv_one_plus_g_power(v: np.ndarray, z: int, p: int) -> np.ndarray:
    """Return ``(1 + g^z)^{-1} . v`` for ``z`` not divisible by ``p``.

    Section 4.6 writes, for p = 17, ``(1 + g^z)^{-1} = 1 + g^{2z} + ... + g^{16z}``
    and evaluates it by Horner's rule with the step ``g^{2z}``.  For any odd
    prime the sum has ``(p+1)/2`` terms ``g^{2jz}``, ``j = 0 .. (p-1)/2``:
    multiplying it by ``1 + g^z`` gives ``sum_{m=0}^{p} g^{mz} = Phi(g^z) + g^{pz}
    = 0 + 1`` by Lemma 3.2.2 applied to ``g^z`` (which also has order p).

    Horner: ``acc = v``; then ``(p-1)/2`` times ``acc = v + g^{2z} acc``.
    """
    if z % p == 0:
        raise ValueError("1 + g^z is singular for z = 0 mod p")
    acc = v.copy()
    for _ in range((p - 1) // 2):
        acc = v ^ mul_g_power(acc, 2 * z, p)
    return acc


def element_from_bits(bits, p: int) -> np.ndarray:
    """One-lane element from a sequence of ``p-1`` bits (row r = bits[r])."""
    arr = np.asarray(bits, dtype=np.uint8).reshape(p - 1, 1)
    if arr.shape[0] != p - 1:
        raise ValueError("need p-1 bits")
    return arr & 1


def matrix_of(fn, p: int) -> np.ndarray:
    """The (p-1)x(p-1) GF(2) matrix of a linear map given as a function on
    one-lane elements: column c is the image of the c-th unit vector."""
    n = p - 1
    m = np.zeros((n, n), dtype=np.uint8)
    for c in range(n):
        e = np.zeros((n, 1), dtype=np.uint8)
        e[c, 0] = 1
        m[:, c] = fn(e)[:, 0] & 1
    return m

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


def poly_mod(a: int, m: int) -> int:
    """Remainder of ``a`` modulo ``m`` in F2[X]; a polynomial is an int whose
    bit i is the coefficient of X^i."""
    if m == 0:
        raise ZeroDivisionError("polynomial modulus is zero")
    dm = m.bit_length()
    while a.bit_length() >= dm:
        a ^= m << (a.bit_length() - dm)
    return a


def poly_gcd(a: int, b: int) -> int:
    """Greatest common divisor in F2[X] (Euclid's algorithm)."""
    while b:
        a, b = b, poly_mod(a, b)
    return a


def extension_ok(p: int) -> bool:
    """Condition (3) of Theorem 3.3.3: for every 0 < m < p the polynomials
    X^p + 1 and X^m + X + 1 are relatively prime over F2.  Exactly then the
    2p-1 matrices g^i and Id + g^j form a cone, so the extended Q parity of
    Section 3.3 protects up to 2p-1 data strips."""
    check_prime(p)
    xp1 = (1 << p) | 1
    return all(poly_gcd(xp1, (1 << m) ^ 0b10 ^ 1) == 1 for m in range(1, p))


def gf2_inverse(m: np.ndarray) -> np.ndarray:
    """Inverse of a square GF(2) matrix by Gauss-Jordan elimination; raises
    ValueError when it is singular."""
    n = m.shape[0]
    a = np.concatenate([m & 1, np.eye(n, dtype=np.uint8)], axis=1).astype(np.uint8)
    for c in range(n):
        rows = [r for r in range(c, n) if a[r, c]]
        if not rows:
            raise ValueError("singular matrix")
        if rows[0] != c:
            a[[c, rows[0]]] = a[[rows[0], c]]
        for r in range(n):
            if r != c and a[r, c]:
                a[r] ^= a[c]
    return a[:, n:]


def apply_matrix(m: np.ndarray, v: np.ndarray) -> np.ndarray:
    """``m . v`` for a GF(2) matrix acting on the rows of ``v`` (row r of the
    result is the XOR of the rows c of ``v`` with m[r, c] = 1)."""
    out = np.zeros_like(v)
    for r in range(m.shape[0]):
        for c in range(m.shape[1]):
            if m[r, c]:
                out[..., r, :] ^= v[..., c, :]
    return out


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

"""Z_p-RAID: P/Q encode and recovery of one or two erased strips.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A stripe is an array of shape ``(..., k+2, p-1, W)``: data strips
``D_0 .. D_{k-1}``, then ``P`` (index ``k``) and ``Q`` (index ``k+1``).  Leading
axes are independent stripes that share the same erasure pattern.

Parity (Corollary 3.2.4, with ``g_t = g^t`` for the 0-based data index t, as in
the Reed-Solomon parity of Section 4.1)::

    P = D_0 + D_1 + ... + D_{k-1}
    Q = D_0 + g D_1 + ... + g^{k-1} D_{k-1}

with ``g = S_p`` (Lemma 3.4.1) and ``1 <= k <= p``.  Recovery follows the four
cases of the proof of Lemma 3.1.2; the two-data case uses the formulas of
Sections 4.3 and 4.6.  The input contents of erased strips are never read.

Extended Q parity (Section 3.3, eq. *qext*): for primes that satisfy
Theorem 3.3.3, up to ``2p - 1`` data strips are allowed, and strip
``t >= p`` enters Q with the coefficient ``Id + g^{t-p+1}``::

    Q = sum_{t < p} g^t D_t + sum_{t >= p} (Id + g^{t-p+1}) D_t

For ``k <= p`` this is the code above.  A recovery that involves a strip
``t >= p`` uses the general formulas of the proof of Lemma 3.1.2, with the
inverse of the coefficient (or of the sum of two coefficients) taken by
GF(2) elimination of its matrix: the paper gives no closed form for these.
"""

from __future__ import annotations

import numpy as np

from .ring import (apply_matrix, check_prime, extension_ok, gf2_inverse, inv_one_plus_g_power, matrix_of,
                   mul_g_power, sylvester_step)


def max_data_strips(p: int) -> int:
    """``2p - 1`` when the extended cone of Theorem 3.3.3 exists for ``p``,
    else ``p`` (Corollary 3.2.4)."""
    check_prime(p)
    return 2 * p - 1 if extension_ok(p) else p


def _check(p: int, k: int, rows: int) -> None:
    check_prime(p)
    if not 1 <= k <= p and not (p < k <= max_data_strips(p)):
        raise ValueError(f"k = {k} must satisfy 1 <= k <= p = {p} "
                         f"(or <= 2p-1 where Theorem 3.3.3 holds)")
    if rows != p - 1:
        raise ValueError("strips must have p-1 rows")


def coefficient(v: np.ndarray, t: int, p: int) -> np.ndarray:
    """``g_t . v``: ``g^t v`` for ``t < p``, ``v + g^{t-p+1} v`` for ``t >= p``
    (eq. *qext*)."""
    if t < p:
        return mul_g_power(v, t, p)
    return v ^ mul_g_power(v, t - p + 1, p)


def _solve(fn, v: np.ndarray, p: int) -> np.ndarray:
    """``M^{-1} v`` where ``M`` is the matrix of the linear map ``fn``."""
    return apply_matrix(gf2_inverse(matrix_of(fn, p)), v)


def p_parity(data: np.ndarray, skip=()) -> np.ndarray:
    """``sum_t D_t`` over the data strips not in ``skip`` (axis -3 indexes t)."""
    acc = np.zeros(data.shape[:-3] + data.shape[-2:], dtype=np.uint8)
    for t in range(data.shape[-3]):
        if t not in skip:
            acc ^= data[..., t, :, :]
    return acc


def q_parity(data: np.ndarray, p: int, skip=()) -> np.ndarray:
    """``sum_t g_t D_t`` over the data strips not in ``skip``.

    Horner's rule of Section 4.2, ``Q = D_0 + g(D_1 + g(... + g D_{k-1}))``,
    over the strips ``t < p``, with the strips in ``skip`` taken as zero; with
    the two failed strips skipped this is the syndrome ``Q_xy`` of Section
    4.3.  Strips ``t >= p`` (extended parity) add ``(Id + g^{t-p+1}) D_t``.
    """
    k = data.shape[-3]
    acc = np.zeros(data.shape[:-3] + data.shape[-2:], dtype=np.uint8)
    for t in range(min(k, p) - 1, -1, -1):
        acc = sylvester_step(acc, p)
        if t not in skip:
            acc ^= data[..., t, :, :]
    for t in range(p, k):
        if t not in skip:
            acc ^= coefficient(data[..., t, :, :], t, p)
    return acc


def encode(data: np.ndarray, p: int):
    """Return ``(P, Q)`` for data strips of shape ``(..., k, p-1, W)``."""
    _check(p, data.shape[-3], data.shape[-2])
    return p_parity(data), q_parity(data, p)


def encode_stripe(data: np.ndarray, p: int) -> np.ndarray:
    """Full stripe ``(..., k+2, p-1, W)`` from its data strips."""
    P, Q = encode(data, p)
    return np.concatenate([data, P[..., None, :, :], Q[..., None, :, :]], axis=-3)


def check_stripe(stripe: np.ndarray, p: int):
    """The two parity-check sums of Corollary 3.2.4; both are zero for a
    consistent stripe.  Returns ``(P + sum D, Q + sum g^t D_t)``."""
    k = stripe.shape[-3] - 2
    _check(p, k, stripe.shape[-2])
    data = stripe[..., :k, :, :]
    return stripe[..., k, :, :] ^ p_parity(data), stripe[..., k + 1, :, :] ^ q_parity(data, p)


def recover(stripe: np.ndarray, p: int, erased) -> np.ndarray:
    """Return a copy of ``stripe`` with the strips in ``erased`` (one or two
    distinct indices in ``0 .. k+1``) rebuilt from the others.

    Cases (proof of Lemma 3.1.2):

    * P and Q: recompute both from the data.
    * data ``j`` and P: ``D_j = g^{-j}(Q + sum_{t != j} g^t D_t)`` with
      ``g^{-j} = g^{p-j}`` (Section 4.6), then ``P`` from the first equation.
    * data ``j`` and Q: ``D_j = P + sum_{t != j} D_t``, then ``Q``.
    * data ``x < y``: Sections 4.3 and 4.6 -- ``z = y - x``,
      ``dP = P + P_xy``, ``dQ = Q + Q_xy``,
      ``D_y = (1+g^z)^{-1} dP + g^{p-x} (1+g^z)^{-1} dQ``, ``D_x = D_y + dP``.
    * one data strip ``e``: ``D_e = P + sum_{t != e} D_t`` (RAID-5, Section 1).
    * P alone or Q alone: recompute it from the data.
    """
    k = stripe.shape[-3] - 2
    _check(p, k, stripe.shape[-2])
    er = sorted(set(int(e) for e in erased))
    if len(er) != len(tuple(erased)) or not 1 <= len(er) <= 2:
        raise ValueError("need one or two distinct erased strips")
    if any(e < 0 or e > k + 1 for e in er):
        raise ValueError("erased index out of range")

    out = stripe.copy()
    data = out[..., :k, :, :]
    iP, iQ = k, k + 1
    P = out[..., iP, :, :]
    Q = out[..., iQ, :, :]
    skip = tuple(e for e in er if e < k)

    if len(er) == 1:
        e = er[0]
        if e == iP:
            out[..., iP, :, :] = p_parity(data)
        elif e == iQ:
            out[..., iQ, :, :] = q_parity(data, p)
        else:
            out[..., e, :, :] = P ^ p_parity(data, skip)
        return out

    x, y = er
    if (x, y) == (iP, iQ):
        out[..., iP, :, :] = p_parity(data)
        out[..., iQ, :, :] = q_parity(data, p)
    elif y == iP:                      # data x and P
        t = Q ^ q_parity(data, p, skip)
        if x < p:
            out[..., x, :, :] = mul_g_power(t, p - x, p)
        else:                          # D_x = g_x^{-1} (Q + sum_{t != x} g_t D_t)
            out[..., x, :, :] = _solve(lambda v: coefficient(v, x, p), t, p)
        out[..., iP, :, :] = p_parity(out[..., :k, :, :])
    elif y == iQ:                      # data x and Q
        out[..., x, :, :] = P ^ p_parity(data, skip)
        out[..., iQ, :, :] = q_parity(out[..., :k, :, :], p)
    elif y < p:                        # two data strips x < y < p
        z = y - x
        dP = P ^ p_parity(data, skip)
        dQ = Q ^ q_parity(data, p, skip)
        dy = inv_one_plus_g_power(dP, z, p) ^ mul_g_power(inv_one_plus_g_power(dQ, z, p), p - x, p)
        out[..., y, :, :] = dy
        out[..., x, :, :] = dy ^ dP
    else:                              # two data strips, y >= p (extended parity)
        # Lemma 3.1.2: D_y = (g_x + g_y)^{-1} (g_x dP + dQ), then D_x = D_y + dP.
        dP = P ^ p_parity(data, skip)
        dQ = Q ^ q_parity(data, p, skip)
        dy = _solve(lambda v: coefficient(v, x, p) ^ coefficient(v, y, p), coefficient(dP, x, p) ^ dQ, p)
        out[..., y, :, :] = dy
        out[..., x, :, :] = dy ^ dP
    return out


def update(stripe: np.ndarray, p: int, t: int, new_strip: np.ndarray) -> np.ndarray:
    """Stripe after data strip ``t`` is overwritten with ``new_strip``.

    The parity equations of Corollary 3.2.4 are linear, so a small write
    updates the parity from the change alone (the Q-parity update that the
    end of Section 3.4 prices at shifts, XOR and AND per power of S_N)::

        dD = D_t + D_t',   P' = P + dD,   Q' = Q + g_t dD

    with ``g_t = g^t`` (``Id + g^{t-p+1}`` for an extended strip ``t >= p``).
    Only strips ``t``, P and Q change.
    """
    k = stripe.shape[-3] - 2
    _check(p, k, stripe.shape[-2])
    if not 0 <= t < k:
        raise ValueError("t must index a data strip")
    out = stripe.copy()
    delta = out[..., t, :, :] ^ new_strip
    out[..., t, :, :] = new_strip
    out[..., k, :, :] ^= delta
    out[..., k + 1, :, :] ^= coefficient(delta, t, p)
    return out

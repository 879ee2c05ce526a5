"""GF(2) linear algebra for the tests (independent of the oracle).

Matrices are uint8 NumPy arrays of 0/1.  Used to check the oracle's decode
against plain Gaussian elimination on the parity-check matrix.
"""

import numpy as np


def matmul(a, b):
    return (a.astype(np.int64) @ b.astype(np.int64) % 2).astype(np.uint8)


def identity(n):
    return np.eye(n, dtype=np.uint8)


def power(m, e):
    r = identity(m.shape[0])
    for _ in range(e):
        r = matmul(r, m)
    return r


def rank(m):
    a = (m.copy() & 1).astype(np.uint8)
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
        mask = a[:, c].astype(bool)
        mask[r] = False
        a[mask] ^= a[r]
        r += 1
        if r == rows:
            break
    return r


def solve(a, b):
    """Solve ``a x = b`` over GF(2) for square nonsingular ``a`` and any number
    of right-hand-side columns ``b``; raises ValueError when ``a`` is singular."""
    n = a.shape[0]
    aug = np.concatenate([a & 1, b & 1], axis=1).astype(np.uint8)
    for c in range(n):
        piv = None
        for i in range(c, n):
            if aug[i, c]:
                piv = i
                break
        if piv is None:
            raise ValueError("singular matrix")
        if piv != c:
            aug[[c, piv]] = aug[[piv, c]]
        mask = aug[:, c].astype(bool)
        mask[c] = False
        aug[mask] ^= aug[c]
    return aug[:, n:]


def sylvester_matrix(n):
    """The (n-1)x(n-1) Sylvester matrix S_n as displayed in Lemma 3.4.1:
    ones on the subdiagonal and in the whole last column."""
    s = np.zeros((n - 1, n - 1), dtype=np.uint8)
    for r in range(1, n - 1):
        s[r, r - 1] = 1
    s[:, n - 2] = 1
    return s


_H_CACHE = {}


def parity_check_matrix(p, k):
    key = (p, k)
    if key not in _H_CACHE:
        _H_CACHE[key] = _parity_check_matrix(p, k)
    return _H_CACHE[key]


def _parity_check_matrix(p, k):
    """The parity-check matrix of Corollary 3.2.4 with g = S_p, for k data
    strips: block rows [I .. I I 0] and [I g .. g^{k-1} 0 I], block columns in
    strip order D_0 .. D_{k-1}, P, Q.  For k > p the blocks of strips t >= p
    are I + g^{t-p+1} (extended Q parity, eq. qext of Section 3.3)."""
    n = p - 1
    g = sylvester_matrix(p)
    h = np.zeros((2 * n, (k + 2) * n), dtype=np.uint8)
    for t in range(k):
        h[:n, t * n:(t + 1) * n] = identity(n)
        h[n:, t * n:(t + 1) * n] = power(g, t) if t < p else identity(n) ^ power(g, t - p + 1)
    h[:n, k * n:(k + 1) * n] = identity(n)
    h[n:, (k + 1) * n:(k + 2) * n] = identity(n)
    return h

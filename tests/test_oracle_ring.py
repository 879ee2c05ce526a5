"""Pins of the ring arithmetic of the oracle (multiplication by g = S_p and its
powers) against what the paper prints and what the mathematics fixes."""

import itertools

import numpy as np
import pytest

import gf2
import golden_io
from oracle import ring


PRIMES = [3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53]


def _rand(p, w, seed=0, lead=()):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=tuple(lead) + (p - 1, w), dtype=np.uint8)


def test_is_odd_prime():
    assert [n for n in range(60) if ring.is_odd_prime(n)] == [
        3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59]


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 9, 13, 17, 29, 53])
def test_step_is_the_displayed_sylvester_matrix(n):
    # Lemma 3.4.1 displays S_N: ones on the subdiagonal and in the last column.
    m = ring.matrix_of(lambda e: ring.sylvester_step(e, n), n)
    assert (m == gf2.sylvester_matrix(n)).all()


def test_step_matches_printed_z17_matrix():
    # Section 4.5 prints the full 16x16 matrix for p = 17.
    printed = golden_io.matrix(golden_io.sections("sylvester_s17.txt")[""])
    assert printed.shape == (16, 16)
    m = ring.matrix_of(lambda e: ring.sylvester_step(e, 17), 17)
    assert (m == printed).all()


def test_step_matches_printed_z3_generator():
    # Sections 2.1 / 3.2: for N = 3 the generator is G = [[0,1],[1,1]].
    g = golden_io.matrix(golden_io.sections("z3_matrices.txt")["G"])
    m = ring.matrix_of(lambda e: ring.sylvester_step(e, 3), 3)
    assert (m == g).all()
    idg = golden_io.matrix(golden_io.sections("z3_matrices.txt")["Id+G"])
    assert ((gf2.identity(2) ^ m) == idg).all()
    assert gf2.rank(idg) == 2


@pytest.mark.parametrize("n", [3, 5, 7, 9, 11, 15, 17, 29])
def test_order_is_exactly_n(n):
    # Lemma 3.4.1 (i): S_N has order N.
    m = ring.matrix_of(lambda e: ring.sylvester_step(e, n), n)
    acc = gf2.identity(n - 1)
    for i in range(1, n + 1):
        acc = gf2.matmul(m, acc)
        assert (acc == gf2.identity(n - 1)).all() == (i == n), i


@pytest.mark.parametrize("n", list(range(3, 24)))
def test_id_plus_s_invertible_iff_odd(n):
    # Lemma 3.4.1 (ii): Id + S_N is non-degenerate for odd N, degenerate for even N.
    m = ring.matrix_of(lambda e: ring.sylvester_step(e, n), n)
    r = gf2.rank(gf2.identity(n - 1) ^ m)
    assert (r == n - 1) == (n % 2 == 1)


def _powers_closed_form(a_col, n, k):
    """S_N^k applied to a vector, transcribed from the display in the proof of
    Lemma 3.4.1: the vector is listed top-down as (x_{N-1}, ..., x_1); the image
    is x_k in every position plus the list (x_{k-1}, ..., x_1, 0, x_{N-1}, ..., x_{k+1}),
    with x_j = 0 unless 1 <= j <= N-1."""
    # position i from the top holds x_{N-1-i}
    x = {j: int(a_col[n - 1 - j]) for j in range(1, n)}
    xj = lambda j: x.get(j, 0)  # noqa: E731
    listed = [xj(j) for j in range(k - 1, 0, -1)]
    listed += [0] if k >= 1 else []
    listed += [xj(j) for j in range(n - 1, k, -1)]
    listed = listed[:n - 1]
    return np.array([xj(k) ^ v for v in listed], dtype=np.uint8)


@pytest.mark.parametrize("n", [3, 5, 7, 13, 17])
def test_powers_match_closed_form_display(n):
    rng = np.random.default_rng(n)
    for _ in range(20):
        a = rng.integers(0, 2, size=n - 1).astype(np.uint8)
        for k in range(1, n + 1):
            got = ring.mul_g_power(a.reshape(n - 1, 1), k, n)[:, 0]
            assert (got == _powers_closed_form(a, n, k)).all(), (n, k)


def _pack16(col):
    return int(sum(int(b) << r for r, b in enumerate(col)))


def _unpack16(v):
    return np.array([(v >> r) & 1 for r in range(16)], dtype=np.uint8)


def test_z17_packed_int16_step():
    # Section 4.5: on a 16-bit word whose bit r is the row-r coefficient,
    # g.x = (x + x) XOR (all ones if x is negative as a signed int16).
    for v in range(0, 1 << 16, 7):
        s = v - (1 << 16) if v >= 1 << 15 else v
        y = ((s + s) ^ (-1 if s < 0 else 0)) & 0xFFFF
        got = ring.sylvester_step(_unpack16(v).reshape(16, 1), 17)[:, 0]
        assert (got == _unpack16(y)).all(), v


def test_z17_packed_int16_power():
    # Section 4.6: g^k x = (x << k) ^ (x >> (17-k)) ^ (all ones if (x << (k-1)) is
    # negative as an int16), 1 <= k <= 16.  The right shift is the logical one (the
    # SSE2 sequence there uses psrlw).
    rng = np.random.default_rng(17)
    for v in rng.integers(0, 1 << 16, size=300):
        v = int(v)
        for k in range(1, 17):
            sh = (v << (k - 1)) & 0xFFFF
            neg = sh >= 1 << 15
            y = ((v << k) & 0xFFFF) ^ (v >> (17 - k)) ^ (0xFFFF if neg else 0)
            got = ring.mul_g_power(_unpack16(v).reshape(16, 1), k, 17)[:, 0]
            assert (got == _unpack16(y)).all(), (v, k)


@pytest.mark.parametrize("p", PRIMES)
def test_sum_of_all_powers_is_zero(p):
    # Lemma 3.2.2: sum_{k<N} g^k = 0.
    a = _rand(p, 8, p)
    acc = np.zeros_like(a)
    for i in range(p):
        acc ^= ring.mul_g_power(a, i, p)
    assert not acc.any()


@pytest.mark.parametrize("p", [3, 5, 7, 11, 13, 17, 19])
def test_differences_of_powers_invertible(p):
    # Lemma 3.2.3: g^l + g^k is non-degenerate for 0 <= k < l < p.
    mats = [ring.matrix_of(lambda e, i=i: ring.mul_g_power(e, i, p), p) for i in range(p)]
    for k, l in itertools.combinations(range(p), 2):
        assert gf2.rank(mats[k] ^ mats[l]) == p - 1, (k, l)


@pytest.mark.parametrize("p", PRIMES)
def test_horner_inverse_inverts(p):
    # Section 4.6: (1 + g^z)^{-1} by Horner with step g^{2z}; check (1 + g^z) A v = v.
    v = _rand(p, 4, 100 + p)
    for z in range(1, p):
        a = ring.inv_one_plus_g_power(v, z, p)
        back = a ^ ring.mul_g_power(a, z, p)
        assert (back == v).all(), z


def test_z3_gf4_field():
    # Section 2.2: {0, 1, G, G^2} is closed under + and x, and non-zero elements
    # are invertible (the field GF(4)).
    g = ring.matrix_of(lambda e: ring.sylvester_step(e, 3), 3)
    elems = [np.zeros((2, 2), np.uint8), gf2.identity(2), g, gf2.matmul(g, g)]
    key = lambda m: m.tobytes()  # noqa: E731
    keys = {key(m) for m in elems}
    assert len(keys) == 4
    for a in elems:
        for b in elems:
            assert key(a ^ b) in keys
            assert key(gf2.matmul(a, b)) in keys
    for a in elems[1:]:
        assert gf2.rank(a) == 2


def test_composite_n_is_rejected_by_check_prime():
    for n in (1, 2, 4, 9, 15, 21, 25, 49):
        with pytest.raises(ValueError):
            ring.check_prime(n)


def test_composite_odd_n_breaks_the_cone():
    # Theorem 3.2.1 needs Id + g^m non-degenerate for proper divisors m of N;
    # for N = 9, m = 3 fails (1 + x^3 shares a factor with 1 + x + ... + x^8).
    n = 9
    m3 = ring.matrix_of(lambda e: ring.mul_g_power(e, 3, n), n)
    assert gf2.rank(gf2.identity(n - 1) ^ m3) < n - 1

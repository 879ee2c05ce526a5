"""Pins of the oracle's Z_p-RAID encode and recovery against the paper's
printed example, EVENODD, brute force and GF(2) Gaussian elimination."""

import itertools

import numpy as np
import pytest

import gf2
import golden_io
from oracle import zp_raid as zp

CONFIG_PRIMES = [5, 11, 13, 19, 29, 37, 53]


def _rand_data(p, k, w, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=(k, p - 1, w), dtype=np.uint8)


def _bits_to_lanes(values):
    """Pack a list of 0/1 values (one per lane) into bytes, lane 8*j+b = bit b of byte j."""
    v = np.asarray(values, dtype=np.uint8)
    w = (len(v) + 7) // 8
    out = np.zeros(w, dtype=np.uint8)
    for i, b in enumerate(v):
        out[i // 8] |= (int(b) & 1) << (i % 8)
    return out


def _lane_bits(row, n):
    return np.array([(int(row[i // 8]) >> (i % 8)) & 1 for i in range(n)], dtype=np.uint8)


def _eval(terms, env):
    acc = np.zeros_like(next(iter(env.values())))
    for t in terms:
        acc ^= env[t]
    return acc


def test_four_disk_example_bits():
    # Section 2.1 with p = 3, k = 2: all 16 data patterns at once, one per lane.
    fx = golden_io.sections("z3_four_disk.txt")
    pats = list(itertools.product([0, 1], repeat=4))          # (d11, d12, d21, d22)
    d = {name: np.array([pt[i] for pt in pats], dtype=np.uint8)
         for i, name in enumerate(["d11", "d12", "d21", "d22"])}
    data = np.zeros((2, 2, 2), dtype=np.uint8)
    data[0, 0], data[0, 1] = _bits_to_lanes(d["d11"]), _bits_to_lanes(d["d12"])
    data[1, 0], data[1, 1] = _bits_to_lanes(d["d21"]), _bits_to_lanes(d["d22"])
    P, Q = zp.encode(data, 3)
    pi = {"pi11": _lane_bits(P[0], 16), "pi12": _lane_bits(P[1], 16),
          "pi21": _lane_bits(Q[0], 16), "pi22": _lane_bits(Q[1], 16)}
    for name, terms in golden_io.equations(fx["parity"]).items():
        assert (pi[name] == _eval(terms, d)).all(), name

    # RAID-DP naming of the same bits: disk 1 = (A, C), disk 2 = (B, D).
    dp_env = {"A": d["d11"], "C": d["d12"], "B": d["d21"], "D": d["d22"]}
    dp_names = {"HP": "pi11", "HP2": "pi12", "DP1": "pi21", "DP2": "pi22"}
    for name, terms in golden_io.equations(fx["raid_dp"]).items():
        assert (pi[dp_names[name]] == _eval(terms, dp_env)).all(), name

    # Recovery of both data disks: compare with the printed expressions.
    stripe = zp.encode_stripe(data, 3)
    stripe[0:2] = 0x5A
    rec = zp.recover(stripe, 3, (0, 1))
    got = {"d11": _lane_bits(rec[0, 0], 16), "d12": _lane_bits(rec[0, 1], 16),
           "d21": _lane_bits(rec[1, 0], 16), "d22": _lane_bits(rec[1, 1], 16)}
    for name, terms in golden_io.equations(fx["recovery"]).items():
        assert (got[name] == _eval(terms, pi)).all(), name
        assert (got[name] == d[name]).all(), name


def test_five_disk_code_with_printed_g():
    # Section 2.2: Q = d1 + G d2 + G^2 d3 with the printed G (three data disks, p = 3).
    g = golden_io.matrix(golden_io.sections("z3_matrices.txt")["G"])
    data = _rand_data(3, 3, 16, 1)
    _, Q = zp.encode(data, 3)
    for byte in range(16):
        for bit in range(8):
            cols = [((data[t, :, byte] >> bit) & 1).reshape(2, 1) for t in range(3)]
            want = cols[0] ^ gf2.matmul(g, cols[1]) ^ gf2.matmul(gf2.matmul(g, g), cols[2])
            assert (((Q[:, byte] >> bit) & 1).reshape(2, 1) == want).all()


@pytest.mark.parametrize("p", [3, 5, 7, 13, 17, 29])
def test_identical_strips_give_zero_q(p):
    # Lemma 3.2.2: with k = p copies of the same strip, Q = (sum_k g^k) D = 0.
    one = _rand_data(p, 1, 8, p)[0]
    data = np.broadcast_to(one, (p, p - 1, 8)).copy()
    P, Q = zp.encode(data, p)
    assert not Q.any()
    assert (P == one).all()


@pytest.mark.parametrize("p", [3, 5, 7, 11, 13])
def test_p_check_sum_is_zero(p):
    data = _rand_data(p, p - 1, 8, 7 * p)
    c1, c2 = zp.check_stripe(zp.encode_stripe(data, p), p)
    assert not c1.any() and not c2.any()


def _evenodd(data, p):
    """EVENODD parities (Blaum, Brady, Bruck, Menon) from their array definition:
    a (p-1) x p information array (column j = disk j, absent disks zero), an
    imaginary all-zero row p-1, horizontal parity = XOR of each row, and diagonal
    parity ``S + XOR_t a[(l - t) mod p][t]`` with the adjuster
    ``S = XOR_{t=1}^{p-1} a[p-1-t][t]``."""
    k, rows, w = data.shape
    a = np.zeros((p, p, w), dtype=np.uint8)      # a[row][column], row p-1 imaginary
    a[:rows, :k] = np.transpose(data, (1, 0, 2))
    horiz = np.zeros((p - 1, w), dtype=np.uint8)
    for r in range(p - 1):
        for t in range(p):
            horiz[r] ^= a[r, t]
    s = np.zeros(w, dtype=np.uint8)
    for t in range(1, p):
        s ^= a[p - 1 - t, t]
    diag = np.zeros((p - 1, w), dtype=np.uint8)
    for l in range(p - 1):
        diag[l] = s
        for t in range(p):
            diag[l] ^= a[(l - t) % p, t]
    return horiz, diag


@pytest.mark.parametrize("p", [3, 5, 7, 11, 13, 17])
def test_construction_is_evenodd(p):
    # Section 3.4: the non-extended code with the Sylvester matrix is EVENODD.
    for k in sorted({1, 2, p - 1, p}):
        data = _rand_data(p, k, 8, 1000 * p + k)
        P, Q = zp.encode(data, p)
        h, dg = _evenodd(data, p)
        assert (P == h).all(), k
        assert (Q == dg).all(), k


def _roundtrip(p, k, w, seed):
    data = _rand_data(p, k, w, seed)
    stripe = zp.encode_stripe(data, p)
    rng = np.random.default_rng(seed + 1)
    for e in itertools.chain(itertools.combinations(range(k + 2), 2),
                             ((i,) for i in range(k + 2))):
        bad = stripe.copy()
        bad[list(e)] = rng.integers(0, 256, size=(len(e), p - 1, w), dtype=np.uint8)
        rec = zp.recover(bad, p, e)
        assert (rec == stripe).all(), (p, k, e)


@pytest.mark.parametrize("p", [3, 5, 7])
def test_roundtrip_every_pair_tiny_p(p):
    for k in range(1, p + 1):
        _roundtrip(p, k, 5, 31 * p + k)


@pytest.mark.parametrize("p", [11, 13])
def test_roundtrip_every_pair_mid_p(p):
    _roundtrip(p, p - 1, 3, p)


@pytest.mark.parametrize("p", [3, 5])
def test_bruteforce_unique_solution(p):
    # Lemma 3.1.2: for every erased pair exactly one candidate satisfies both
    # parity equations, and it is the oracle's answer.  One lane, all candidates.
    n = p - 1
    for k in range(1, p + 1):
        h = gf2.parity_check_matrix(p, k)
        rng = np.random.default_rng(p * 10 + k)
        data = rng.integers(0, 2, size=(k, n, 1), dtype=np.uint8)
        stripe = zp.encode_stripe(data, p) & 1
        full = stripe[:, :, 0].reshape(-1)
        assert not gf2.matmul(h, full.reshape(-1, 1)).any()
        cands = np.array(list(itertools.product([0, 1], repeat=2 * n)), dtype=np.uint8)
        for i, j in itertools.combinations(range(k + 2), 2):
            hits = []
            for c in cands:
                v = full.copy()
                v[i * n:(i + 1) * n] = c[:n]
                v[j * n:(j + 1) * n] = c[n:]
                if not gf2.matmul(h, v.reshape(-1, 1)).any():
                    hits.append(c)
            assert len(hits) == 1, (k, i, j, len(hits))
            bad = stripe.copy()
            bad[[i, j]] = 1 - bad[[i, j]]
            rec = zp.recover(bad, p, (i, j)) & 1
            assert (rec[i, :, 0] == hits[0][:n]).all() and (rec[j, :, 0] == hits[0][n:]).all()


def _gauss_recover(stripe_bits, p, k, erased):
    """Solve H_E x_E = H_S x_S over GF(2) lane-wise (Corollary 3.2.4's matrix)."""
    n = p - 1
    h = gf2.parity_check_matrix(p, k)
    cols_e = [c for e in erased for c in range(e * n, (e + 1) * n)]
    cols_s = [c for c in range(h.shape[1]) if c not in set(cols_e)]
    x = stripe_bits.reshape((k + 2) * n, -1)
    rhs = gf2.matmul(h[:, cols_s], x[cols_s])
    return gf2.solve(h[:, cols_e], rhs)


def _bits(stripe):
    """(k+2, n, W) bytes -> ((k+2)*n, 8W) bits."""
    return np.unpackbits(stripe, axis=-1, bitorder="little").reshape(stripe.shape[0] * stripe.shape[1], -1)


@pytest.mark.parametrize("p", CONFIG_PRIMES)
def test_decode_matches_gauss(p):
    k = p - 1
    n = p - 1
    data = _rand_data(p, k, 2, 5 * p)
    stripe = zp.encode_stripe(data, p)
    bits = _bits(stripe).reshape(k + 2, n, -1)
    pairs = list(itertools.combinations(range(k + 2), 2))
    if len(pairs) > 120:
        rng = np.random.default_rng(p)
        special = [pr for pr in pairs if pr[1] >= k]          # every DP, DQ, PQ
        dd = [pr for pr in pairs if pr[1] < k]
        pick = rng.choice(len(dd), size=80, replace=False)
        pairs = special[:: max(1, len(special) // 40)] + [dd[i] for i in pick]
    for e in pairs:
        sol = _gauss_recover(bits, p, k, e)
        bad = stripe.copy()
        bad[list(e)] = 0xC3
        rec = zp.recover(bad, p, e)
        want = _bits(rec[list(e)])
        assert (sol == want).all(), e
        assert (rec == stripe).all(), e


def test_recover_ignores_erased_contents():
    p, k, w = 7, 5, 16
    stripe = zp.encode_stripe(_rand_data(p, k, w, 3), p)
    for e in [(0, 1), (2, k), (3, k + 1), (k, k + 1), (4,)]:
        a = stripe.copy()
        b = stripe.copy()
        a[list(e)] = 0
        b[list(e)] = 0xFF
        assert (zp.recover(a, p, e) == zp.recover(b, p, e)).all()


def test_single_bit_flip_is_detected():
    p, k = 13, 12
    stripe = zp.encode_stripe(_rand_data(p, k, 8, 4), p)
    stripe[3, 5, 2] ^= 0x10
    c1, c2 = zp.check_stripe(stripe, p)
    assert c1.any() and c2.any()


def test_update_matches_reencode():
    # The small-write update (by linearity) against a full re-encode of the
    # changed data: every data strip, plain and extended parity.
    for p, k in ((11, 9), (7, 7), (5, 9), (13, 25)):
        w = 8
        data = _rand_data(p, k, w, 9 + k)
        stripe = zp.encode_stripe(data, p)
        for t in range(k):
            new = _rand_data(p, 1, w, 100 + t)[0]
            upd = zp.update(stripe, p, t, new)
            changed = data.copy()
            changed[t] = new
            assert (upd == zp.encode_stripe(changed, p)).all(), (p, k, t)
    with pytest.raises(ValueError):
        zp.update(stripe, 13, 25, new)


def test_argument_checks():
    with pytest.raises(ValueError):
        zp.encode(np.zeros((2, 8, 4), np.uint8), 9)         # 9 is not prime
    with pytest.raises(ValueError):
        zp.encode(np.zeros((10, 4, 4), np.uint8), 5)        # k > 2p-1
    with pytest.raises(ValueError):
        zp.encode(np.zeros((8, 6, 4), np.uint8), 7)         # k > p, and p = 7 has no extended cone
    with pytest.raises(ValueError):
        zp.encode(np.zeros((2, 3, 4), np.uint8), 5)         # wrong row count
    st = zp.encode_stripe(np.zeros((3, 4, 4), np.uint8), 5)
    for bad in [(1, 1), (0, 5), (-1,), (0, 1, 2), ()]:
        with pytest.raises(ValueError):
            zp.recover(st, 5, bad)


def test_leading_axes_are_independent_stripes():
    p, k, w = 5, 4, 8
    rng = np.random.default_rng(12)
    data = rng.integers(0, 256, size=(3, k, p - 1, w), dtype=np.uint8)
    st = zp.encode_stripe(data, p)
    for s in range(3):
        assert (st[s] == zp.encode_stripe(data[s], p)).all()
    rec = zp.recover(st, p, (0, 2))
    assert (rec == st).all()

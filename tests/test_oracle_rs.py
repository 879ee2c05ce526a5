"""Pins of the GF(256) Reed-Solomon comparison oracle."""

import itertools

import numpy as np

import gf2
import golden_io
from oracle import rs_gf256 as rs


def _bits(b):
    return np.array([(b >> i) & 1 for i in range(8)], dtype=np.uint8).reshape(8, 1)


def test_mul2_matches_printed_matrix():
    # Section 4.1 prints multiplication by {02} as an 8x8 matrix on (x_0..x_7).
    m = golden_io.matrix(golden_io.sections("gf256_mul02.txt")[""])
    allb = np.arange(256, dtype=np.uint8)
    y = rs.mul2(allb)
    for b in range(256):
        assert (gf2.matmul(m, _bits(b)) == _bits(int(y[b]))).all(), b


def test_signed_form_of_mul2():
    # Section 4.2: the signed-byte form (x + x) ^ (((x < 0) ? 0xff : 0) & 0x1d).
    for b in range(256):
        s = b - 256 if b >= 128 else b
        y = ((s + s) ^ ((-1 if s < 0 else 0) & 0x1D)) & 0xFF
        assert int(rs.mul2(np.array([b], np.uint8))[0]) == y


def test_generator_has_order_255():
    # 0x11D is primitive: {02} generates the 255 non-zero elements, which is what
    # allows up to 255 data disks (Section 1).
    seen = set()
    v = 1
    for i in range(1, 256):
        v = int(rs.mul2(np.array([v], np.uint8))[0])
        if i < 255:
            assert v != 1
        seen.add(v)
    assert v == 1 and len(seen) == 255


def _clmul_mod(a, b, poly=0x11D):
    """Carry-less product of two bytes reduced modulo ``poly`` (long division)."""
    r = 0
    for i in range(8):
        if (b >> i) & 1:
            r ^= a << i
    for bit in range(14, 7, -1):
        if (r >> bit) & 1:
            r ^= poly << (bit - 8)
    return r


def test_field_multiplication_matches_clmul():
    rng = np.random.default_rng(0)
    for a, c in rng.integers(0, 256, size=(400, 2)):
        assert rs.gf_mul(int(a), int(c)) == _clmul_mod(int(a), int(c))


def test_q_is_sum_of_powers():
    # Q = sum_i g^i D_i (Section 4.1) against Horner (Section 4.2).
    rng = np.random.default_rng(1)
    for n_disks in (1, 2, 5, 12, 30):
        data = rng.integers(0, 256, size=(n_disks, 64), dtype=np.uint8)
        P, Q = rs.encode(data)
        want_q = np.zeros(64, dtype=np.int64)
        want_p = np.zeros(64, dtype=np.int64)
        for j in range(64):
            q = 0
            pp = 0
            for i in range(n_disks):
                gi = 1
                for _ in range(i):
                    gi = _clmul_mod(gi, 2)
                q ^= _clmul_mod(int(data[i, j]), gi)
                pp ^= int(data[i, j])
            want_q[j] = q
            want_p[j] = pp
        assert (Q == want_q).all() and (P == want_p).all()


def test_inverse():
    for a in range(1, 256):
        assert rs.gf_mul(a, rs.gf_inv(a)) == 1


def test_two_data_recovery_roundtrip():
    rng = np.random.default_rng(2)
    n_disks = 8
    data = rng.integers(0, 256, size=(n_disks, 32), dtype=np.uint8)
    P, Q = rs.encode(data)
    stripe = np.concatenate([data, P[None], Q[None]])
    for x, y in itertools.combinations(range(n_disks), 2):
        bad = stripe.copy()
        bad[[x, y]] = 0x77
        assert (rs.recover_two_data(bad, x, y) == stripe).all(), (x, y)


def _rs_stripe(n_disks, width, seed):
    data = np.random.default_rng(seed).integers(0, 256, size=(n_disks, width), dtype=np.uint8)
    P, Q = rs.encode(data)
    return np.concatenate([data, P[None], Q[None]], axis=0)


def test_recover_every_erasure_roundtrip():
    for n_disks in (1, 2, 3, 5, 12):
        st = _rs_stripe(n_disks, 33, n_disks)
        rng = np.random.default_rng(n_disks + 100)
        for e in itertools.chain(itertools.combinations(range(n_disks + 2), 2), ((i,) for i in range(n_disks + 2))):
            bad = st.copy()
            bad[list(e)] = rng.integers(0, 256, size=(len(e), 33), dtype=np.uint8)
            assert (rs.recover(bad, e) == st).all(), (n_disks, e)


def test_recover_bruteforce_unique():
    # Lemma 3.1.2 for the cone {g^t}: for every erased pair of a 4-data-disk
    # stripe exactly one of the 65536 byte pairs satisfies both parity
    # equations (checked with the encoder only), and it is the oracle's answer.
    n_disks = 4
    st = _rs_stripe(n_disks, 1, 9)
    cand = np.array(list(itertools.product(range(256), repeat=2)), dtype=np.uint8)      # (65536, 2)
    for i, j in itertools.combinations(range(n_disks + 2), 2):
        trial = np.repeat(st[None, :, 0], len(cand), axis=0)                              # (65536, N+2)
        trial[:, i] = cand[:, 0]
        trial[:, j] = cand[:, 1]
        P, Q = rs.encode(trial[:, :n_disks, None])
        ok = (P[:, 0] == trial[:, n_disks]) & (Q[:, 0] == trial[:, n_disks + 1])
        assert ok.sum() == 1, (i, j)
        hit = cand[np.argmax(ok)]
        bad = st.copy()
        bad[[i, j]] ^= 0xFF
        rec = rs.recover(bad, (i, j))
        assert rec[i, 0] == hit[0] and rec[j, 0] == hit[1]


def test_recover_matches_gauss_with_printed_matrix():
    # Bit-level parity-check matrix from the printed {02} matrix M of Section
    # 4.1: rows [I .. I I 0] and [M^0 .. M^{N-1} 0 I]; GF(2) elimination on the
    # erased columns, for every pair at N = 20 (sampled) and N = 254.
    m = golden_io.matrix(golden_io.sections("gf256_mul02.txt")[""])
    for n_disks, count in ((20, 60), (254, 40)):
        h = np.zeros((16, (n_disks + 2) * 8), dtype=np.uint8)
        mt = gf2.identity(8)
        for t in range(n_disks):
            h[:8, t * 8:(t + 1) * 8] = gf2.identity(8)
            h[8:, t * 8:(t + 1) * 8] = mt
            mt = gf2.matmul(m, mt)
        h[:8, n_disks * 8:(n_disks + 1) * 8] = gf2.identity(8)
        h[8:, (n_disks + 1) * 8:] = gf2.identity(8)
        st = _rs_stripe(n_disks, 4, n_disks)
        bits = np.unpackbits(st[:, :, None], axis=-1, bitorder="little")          # (N+2, 4, 8)
        x = bits.transpose(0, 2, 1).reshape((n_disks + 2) * 8, 4)                 # bit b of disk t = row 8t+b
        pairs = list(itertools.combinations(range(n_disks + 2), 2))
        rng = np.random.default_rng(n_disks)
        special = [pr for pr in pairs if pr[1] >= n_disks]
        pick = [pairs[i] for i in rng.choice(len(pairs), size=count, replace=False)]
        for e in special[:: max(1, len(special) // 20)] + pick:
            cols_e = [c for d in e for c in range(d * 8, d * 8 + 8)]
            cols_s = [c for c in range(h.shape[1]) if c not in set(cols_e)]
            sol = gf2.solve(h[:, cols_e], gf2.matmul(h[:, cols_s], x[cols_s]))
            bad = st.copy()
            bad[list(e)] = 0
            rec = rs.recover(bad, e)
            want = np.unpackbits(rec[list(e)][:, :, None], axis=-1, bitorder="little").transpose(0, 2, 1).reshape(16, 4)
            assert (sol == want).all(), (n_disks, e)

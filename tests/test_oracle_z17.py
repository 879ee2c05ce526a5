"""Pins of the horizontal Z_17 layout of Section 4.5 (one codeword per
int16) against the vertical oracle."""

import numpy as np

from oracle import ring
from oracle import z17_layout as z
from oracle import zp_raid as zp


def test_single_bit_goes_to_its_lane_and_row():
    # codeword c, coefficient of x^r  <->  row r, byte c // 8, bit c % 8
    for c in (0, 1, 7, 8, 13, 127):
        for r in (0, 5, 15):
            words = np.zeros(128, dtype=np.uint16)
            words[c] = 1 << r
            v = z.to_vertical(words)
            want = np.zeros((16, 16), dtype=np.uint8)
            want[r, c // 8] = 1 << (c % 8)
            assert (v == want).all()
            assert (z.to_horizontal(v) == words).all()


def test_round_trip():
    rng = np.random.default_rng(1)
    words = rng.integers(0, 1 << 16, size=(3, 4, 256), dtype=np.uint16)
    assert (z.to_horizontal(z.to_vertical(words)) == words).all()
    strip = rng.integers(0, 256, size=(2, 16, 48), dtype=np.uint8)
    assert (z.to_vertical(z.to_horizontal(strip)) == strip).all()


def test_packed_step_is_the_sylvester_step():
    rng = np.random.default_rng(2)
    words = rng.integers(0, 1 << 16, size=512, dtype=np.uint16)
    assert (z.to_vertical(z.mul_g_packed(words)) == ring.sylvester_step(z.to_vertical(words), 17)).all()


def test_packed_encode_equals_vertical_encode():
    # The paper's int16 routine, on horizontal strips, and the vertical oracle
    # give the same P and Q once transposed (k = 1, 2, 16, 17; and the
    # extended code is out of reach of the packed routine, so k <= 17).
    rng = np.random.default_rng(3)
    for k in (1, 2, 16, 17):
        data = rng.integers(0, 1 << 16, size=(2, k, 128), dtype=np.uint16)
        P, Q = z.encode_packed(data)
        vp, vq = zp.encode(z.to_vertical(data), 17)
        assert (z.to_vertical(P) == vp).all() and (z.to_vertical(Q) == vq).all(), k

"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in the oracle (on the CPU, through
monkeypatch) and runs a set of the pins; at least one must fail.  This shows
that the pins constrain the oracle, not just that the oracle agrees with
itself."""

import numpy as np
import pytest

import test_oracle_ext as T_ext
import test_oracle_rs as T_rs
import test_oracle_ring as T_ring
import test_oracle_z17 as T_z17
import test_oracle_zp as T_zp
from oracle import ring, rs_gf256, z17_layout, zp_raid


def _zp_pins():
    yield lambda: T_zp.test_four_disk_example_bits()
    yield lambda: T_zp.test_construction_is_evenodd(5)
    yield lambda: T_zp.test_construction_is_evenodd(7)
    yield lambda: T_zp.test_roundtrip_every_pair_tiny_p(5)
    yield lambda: T_zp.test_decode_matches_gauss(5)
    yield lambda: T_zp.test_decode_matches_gauss(13)
    yield lambda: T_zp.test_update_matches_reencode()
    yield lambda: T_ring.test_step_matches_printed_z17_matrix()
    yield lambda: T_ring.test_horner_inverse_inverts(7)


def _ext_pins():
    yield lambda: T_ext.test_first_primes_that_fail_are_mersenne_and_73()
    yield lambda: T_ext.test_parity_check_matrix_annihilates_extended_stripes(5, 9)
    yield lambda: T_ext.test_extended_decode_matches_gauss(5)
    yield lambda: T_ext.test_extended_roundtrip_every_pair_p5(9)


def _rs_pins():
    yield lambda: T_rs.test_mul2_matches_printed_matrix()
    yield lambda: T_rs.test_recover_bruteforce_unique()
    yield lambda: T_rs.test_recover_matches_gauss_with_printed_matrix()


def _z17_pins():
    yield lambda: T_z17.test_single_bit_goes_to_its_lane_and_row()
    yield lambda: T_z17.test_packed_encode_equals_vertical_encode()


def _some_pin_fails(pins):
    for pin in pins:
        try:
            pin()
        except (AssertionError, ValueError, IndexError):
            return True
    return False


def _step_wrong_broadcast(a, p):
    top = a[..., p - 3:p - 2, :]          # the row below the top one
    y = np.empty_like(a)
    y[..., 0:1, :] = a[..., p - 2:p - 1, :]
    y[..., 1:, :] = a[..., :p - 2, :] ^ top
    return y


def _step_wrong_direction(a, p):
    top = a[..., 0:1, :]
    y = np.empty_like(a)
    y[..., p - 2:p - 1, :] = top
    y[..., :p - 2, :] = a[..., 1:, :] ^ top
    return y


def _q_reversed_horner(data, p, skip=()):
    k = data.shape[-3]
    acc = np.zeros(data.shape[:-3] + data.shape[-2:], dtype=np.uint8)
    for t in range(min(k, p)):
        acc = ring.sylvester_step(acc, p)
        if t not in skip:
            acc ^= data[..., t, :, :]
    for t in range(p, k):
        if t not in skip:
            acc ^= zp_raid.coefficient(data[..., t, :, :], t, p)
    return acc


def _inverse_one_term_short(v, z, p):
    acc = v.copy()
    for _ in range((p - 1) // 2 - 1):
        acc = v ^ ring.mul_g_power(acc, 2 * z, p)
    return acc


def _mul_g_power_off_by_one(a, i, p):
    y = a.copy()
    for _ in range((i + 1) % p):
        y = ring.sylvester_step(y, p)
    return y


def _coefficient_wrong_exponent(v, t, p):
    if t < p:
        return ring.mul_g_power(v, t, p)
    return v ^ ring.mul_g_power(v, t - p, p)


def _extension_no_plus_one(p):
    return all(ring.poly_gcd((1 << p) | 1, (1 << m) ^ 0b10) == 1 for m in range(1, p))


def _mul2_aes(b):
    b = np.asarray(b, dtype=np.uint8)
    hi = (b & 0x80) != 0
    return (((b.astype(np.uint16) << 1) & 0xFF) ^ np.where(hi, 0x1B, 0)).astype(np.uint8)


def _update_wrong_power(stripe, p, t, new):
    k = stripe.shape[-3] - 2
    out = stripe.copy()
    delta = out[..., t, :, :] ^ new
    out[..., t, :, :] = new
    out[..., k, :, :] ^= delta
    out[..., k + 1, :, :] ^= ring.mul_g_power(delta, t + 1, p)
    return out


def _to_vertical_msb_first(words):
    words = np.asarray(words, dtype=np.uint16)
    n = words.shape[-1]
    out = np.zeros(words.shape[:-1] + (16, n // 8), dtype=np.uint8)
    for r in range(16):
        bits = ((words >> r) & 1).astype(np.uint8).reshape(words.shape[:-1] + (n // 8, 8))
        for b in range(8):
            out[..., r, :] |= bits[..., b] << (7 - b)
    return out


MUTATIONS = {
    "step: broadcast of the wrong row": (
        [(ring, "sylvester_step", _step_wrong_broadcast), (zp_raid, "sylvester_step", _step_wrong_broadcast)],
        _zp_pins),
    "step: rotation the wrong way": (
        [(ring, "sylvester_step", _step_wrong_direction), (zp_raid, "sylvester_step", _step_wrong_direction)],
        _zp_pins),
    "Q: Horner over the strips in the wrong order": ([(zp_raid, "q_parity", _q_reversed_horner)], _zp_pins),
    "inverse of 1 + g^z: one Horner term dropped": (
        [(ring, "inv_one_plus_g_power", _inverse_one_term_short),
         (zp_raid, "inv_one_plus_g_power", _inverse_one_term_short)], _zp_pins),
    "g^i: exponent off by one": (
        [(ring, "mul_g_power", _mul_g_power_off_by_one), (zp_raid, "mul_g_power", _mul_g_power_off_by_one)],
        _zp_pins),
    "extended coefficient: exponent t-p instead of t-p+1": (
        [(zp_raid, "coefficient", _coefficient_wrong_exponent)], _ext_pins),
    "Theorem 3.3.3 test: X^m + X instead of X^m + X + 1": (
        [(ring, "extension_ok", _extension_no_plus_one), (zp_raid, "extension_ok", _extension_no_plus_one)],
        _ext_pins),
    "RS: multiply by {02} with 0x1B": ([(rs_gf256, "mul2", _mul2_aes)], _rs_pins),
    "small write: Q updated with g^(t+1)": ([(zp_raid, "update", _update_wrong_power)], _zp_pins),
    "Z17 layout: bit order within a byte reversed": (
        [(z17_layout, "to_vertical", _to_vertical_msb_first)], _z17_pins),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    patches, pins = MUTATIONS[name]
    for mod, attr, fn in patches:
        monkeypatch.setattr(mod, attr, fn)
    assert _some_pin_fails(pins()), f"no pin caught: {name}"


def test_pins_pass_without_mistakes():
    for pins in (_zp_pins, _ext_pins, _rs_pins, _z17_pins):
        assert not _some_pin_fails(pins())

"""GPU parity of the GF(256) Reed-Solomon kernels (encode and recovery of
every one- and two-disk erasure) against the CPU oracle, bit-exact.

Stripes are encoded by the oracle; erased disks are overwritten with random
bytes before each recovery and whole stripes are compared.
"""

import itertools

import numpy as np
import pytest

import datagen
import paper_cs_0611109_amd as r
from gpu_util import device, log, to_dev, to_host
from oracle import rs_gf256 as rs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _default_config():
    device()
    r.raid6c_rs_set_config(0, 0, 0)
    yield
    r.raid6c_rs_set_config(0, 0, 0)


def _stripes(k, nbytes, n, seed):
    data = datagen.fill_stripes(seed, 0, n, k, 2, nbytes)[:, :, 0, :]       # (n, k, nbytes)
    P, Q = rs.encode(data)
    return np.concatenate([data, P[:, None], Q[:, None]], axis=1)            # (n, k+2, nbytes)


def _recover(want, k, nbytes, er):
    import torch
    n = want.shape[0]
    dev = to_dev(want)
    for s in range(n):
        for e in er[s]:
            if e >= 0:
                dev[s, e] = to_dev(datagen.poison((nbytes,), index=s * 512 + int(e)))
    bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    r.raid6c_rs_recover_n(k, nbytes, dev, nbytes, (k + 2) * nbytes, n, to_dev(er.astype(np.int32)), bad)
    assert int(bad.item()) == 0
    return to_host(dev)


def _all_entries(k):
    return np.array(list(itertools.combinations(range(k + 2), 2)) + [(e, -1) for e in range(k + 2)], np.int32)


@pytest.mark.parametrize("k", [1, 2, 3, 12, 40])
def test_rs_recover_every_erasure(k):
    nbytes = 1040
    er = _all_entries(k)
    log(f"rs recover k={k} entries={len(er)}")
    want = _stripes(k, nbytes, len(er), seed=300 + k)
    assert np.array_equal(_recover(want, k, nbytes, er), want)


def test_rs_recover_largest_k():
    # k = 255 data disks (the order of {02}); pairs at the ends of the range.
    k, nbytes = 255, 64
    er = np.array([(0, 1), (0, 254), (253, 254), (100, 200), (254, k), (0, k), (17, k + 1), (254, k + 1),
                   (k, k + 1), (254, -1), (k + 1, -1)], np.int32)
    want = _stripes(k, nbytes, len(er), seed=255)
    assert np.array_equal(_recover(want, k, nbytes, er), want)


def test_rs_every_launch_configuration():
    import torch
    k, nbytes = 9, 2064
    er = _all_entries(k)
    want = _stripes(k, nbytes, len(er), seed=99)
    for v in (1, 2, 4):
        for u in (1, 4, 8):
            for t in (64, 128, 256):
                log(f"rs config vec={v} unroll={u} threads={t}")
                r.raid6c_rs_set_config(v, u, t)
                dev = to_dev(want.copy())
                dev[:, k:] = to_dev(datagen.poison((len(er), 2, nbytes), index=v * 100 + u * 10 + t))
                r.raid6c_rs_encode_n(k, nbytes, dev, nbytes, (k + 2) * nbytes, len(er))
                assert np.array_equal(to_host(dev), want), (v, u, t)
                assert np.array_equal(_recover(want, k, nbytes, er), want), (v, u, t)
    r.raid6c_rs_set_config(0, 0, 0)


def test_rs_invalid_entries_are_counted_and_skipped():
    import torch
    k, nbytes = 6, 256
    want = _stripes(k, nbytes, 5, seed=7)
    er = np.array([(0, 0), (-1, 3), (2, 9), (1, 4), (8, -1)], np.int32)    # only (1, 4) is valid
    dev = to_dev(want)
    dev[3, 1] = 0
    dev[3, 4] = 0
    bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    r.raid6c_rs_recover_n(k, nbytes, dev, nbytes, (k + 2) * nbytes, 5, to_dev(er), bad)
    assert int(bad.item()) == 4
    assert np.array_equal(to_host(dev), want)

"""GPU parity of the small-write update (P' = P + dD, Q' = Q + g_t dD)
against the CPU oracle, bit-exact, plain and extended Q parity."""

import numpy as np
import pytest

import datagen
import paper_cs_0611109_amd as r
from gpu_util import device, log, to_dev, to_host
from oracle import zp_raid as zp

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _dev():
    device()


def _stripes(p, k, w, n, seed):
    return zp.encode_stripe(datagen.fill_stripes(seed, 0, n, k, p, w), p)


CASES = [(3, 2, 48), (3, 3, 32), (5, 4, 272), (5, 9, 272), (7, 7, 80), (13, 12, 1040), (13, 25, 1040),
         (29, 28, 272), (29, 57, 48), (61, 60, 48), (61, 121, 32)]


@pytest.mark.parametrize("p,k,w,n", [(p, k, w, None) for p, k, w in CASES] + [(13, 12, 1040, 300), (5, 4, 272, 600)])
def test_update_n_matches_oracle(p, k, w, n):
    """Small writes against the oracle.  The last two cases (rows off
    128-byte lines, grids of 600 work-groups) go through the renumbered
    work-group order, which leaves grids under 128 work-groups as they are."""
    import torch
    n = n or max(k, 8)
    log(f"update p={p} k={k} W={w} stripes={n}")
    before = _stripes(p, k, w, n, seed=p * 7 + k)
    targets = np.array([s % k for s in range(n)], dtype=np.int32)
    new = datagen.fill_stripes(p * 7 + k + 1, 0, n, 1, p, w)[:, 0]          # (n, p-1, w)
    want = np.stack([zp.update(before[s], p, int(targets[s]), new[s]) for s in range(n)])
    dev = to_dev(before)
    src = to_dev(new)
    bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    r.raid6c_update_n(p, k, w, dev, (p - 1) * w, (k + 2) * (p - 1) * w, n, to_dev(targets), src, (p - 1) * w, bad)
    assert int(bad.item()) == 0
    assert np.array_equal(to_host(dev), want)
    assert np.array_equal(to_host(src), new)             # the source is only read


def test_update_single_stripe_scattered_strips():
    import torch
    p, k, w = 13, 12, 4096 + 48
    stripe = _stripes(p, k, w, 1, seed=5)[0]
    bufs = [to_dev(np.concatenate([datagen.poison((64,), index=j), stripe[j].reshape(-1),
                                   datagen.poison((80,), index=100 + j)])) for j in range(k + 2)]
    views = [b[64:64 + (p - 1) * w] for b in bufs]
    guard = [to_host(b[:64]).copy() for b in bufs] + [to_host(b[-80:]).copy() for b in bufs]
    cur = stripe
    for i, t in enumerate((0, 5, k - 1, 5)):
        new = datagen.fill_stripes(50 + i, 0, 1, 1, p, w)[0, 0]
        r.raid6c_update(p, k, w, views, t, to_dev(new))
        cur = zp.update(cur, p, t, new)
        torch.cuda.synchronize()
        for j in range(k + 2):
            assert np.array_equal(to_host(views[j]).reshape(p - 1, w), cur[j]), (t, j)
    after = [to_host(b[:64]) for b in bufs] + [to_host(b[-80:]) for b in bufs]
    assert all(np.array_equal(a, b) for a, b in zip(guard, after))


def test_update_invalid_targets_are_counted_and_skipped():
    import torch
    p, k, w = 5, 4, 64
    before = _stripes(p, k, w, 5, seed=3)
    targets = np.array([-1, 4, 2, 7, 0], dtype=np.int32)      # 2 and 0 are valid
    new = datagen.fill_stripes(4, 0, 5, 1, p, w)[:, 0]
    want = before.copy()
    for s in (2, 4):
        want[s] = zp.update(before[s], p, int(targets[s]), new[s])
    dev = to_dev(before)
    bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    r.raid6c_update_n(p, k, w, dev, (p - 1) * w, (k + 2) * (p - 1) * w, 5, to_dev(targets), to_dev(new),
                      (p - 1) * w, bad)
    assert int(bad.item()) == 3
    assert np.array_equal(to_host(dev), want)


def test_updated_stripes_recover():
    # After small writes the stripes are consistent: every erasure pair of the
    # updated stripes is rebuilt to the updated contents.
    import torch
    p, k, w = 13, 12, 512
    n = 91
    before = _stripes(p, k, w, n, seed=11)
    targets = np.array([s % k for s in range(n)], dtype=np.int32)
    new = datagen.fill_stripes(12, 0, n, 1, p, w)[:, 0]
    dev = to_dev(before)
    r.raid6c_update_n(p, k, w, dev, (p - 1) * w, (k + 2) * (p - 1) * w, n, to_dev(targets), to_dev(new),
                      (p - 1) * w)
    updated = to_host(dev).copy()
    pairs = np.array([(i, j) for i in range(k + 2) for j in range(i + 1, k + 2)], dtype=np.int32)
    for s in range(n):
        for e in pairs[s]:
            dev[s, e] = to_dev(datagen.poison((p - 1, w), index=s * 16 + int(e)))
    bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    r.raid6c_recover_n(p, k, w, dev, (p - 1) * w, (k + 2) * (p - 1) * w, n, to_dev(pairs), bad)
    assert int(bad.item()) == 0
    assert np.array_equal(to_host(dev), updated)

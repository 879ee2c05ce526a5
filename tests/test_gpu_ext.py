"""GPU parity of the extended Q parity (Section 3.3, eq. qext: up to 2p-1
data strips) against the CPU oracle, bit-exact.

Stripes are encoded by the oracle; the GPU encodes them again over poisoned
parity strips, and rebuilds poisoned erased strips for every class of pair
(two plain data strips, plain + extended, two extended, data + P, data + Q,
P + Q and single strips).  Whole stripes are compared.
"""

import itertools

import numpy as np
import pytest

import datagen
import paper_cs_0611109_amd as r
from gpu_util import device, log, to_dev, to_host
from oracle import zp_raid as zp

pytestmark = pytest.mark.gpu

EXT_PRIMES = [5, 11, 13, 17, 19, 23, 29, 37, 41, 43, 47, 53, 59, 61]


@pytest.fixture(autouse=True)
def _clean_tuning():
    device()
    r.raid6c_tune_clear()
    yield
    r.raid6c_tune_clear()


def _stripes(p, k, w, n, seed):
    return zp.encode_stripe(datagen.fill_stripes(seed, 0, n, k, p, w), p)


def _encode(want, p, k, w):
    n = want.shape[0]
    dev = to_dev(want.copy())
    dev[:, k:] = to_dev(datagen.poison((n, 2, p - 1, w), index=p * 1000 + k))
    r.raid6c_encode_n(p, k, w, dev, (p - 1) * w, (k + 2) * (p - 1) * w, n)
    return to_host(dev)


def _recover(want, p, k, w, er):
    import torch
    n = want.shape[0]
    dev = to_dev(want)
    for s in range(n):
        for e in er[s]:
            if e >= 0:
                dev[s, e] = to_dev(datagen.poison((p - 1, w), index=s * 256 + int(e)))
    bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    r.raid6c_recover_n(p, k, w, dev, (p - 1) * w, (k + 2) * (p - 1) * w, n, to_dev(er.astype(np.int32)), bad)
    assert int(bad.item()) == 0
    return to_host(dev)


def _classes(p, k):
    """Every erasure entry of a stripe with k data strips, grouped by class."""
    out = {}
    for x, y in itertools.combinations(range(k + 2), 2):
        if y == k + 1:
            key = "pq" if x == k else ("dq_ext" if x >= p else "dq")
        elif y == k:
            key = "dp_ext" if x >= p else "dp"
        elif y < p:
            key = "dd"
        elif x < p:
            key = "dd_mixed"
        else:
            key = "dd_ext"
        out.setdefault(key, []).append((x, y))
    out["single"] = [(e, -1) for e in range(k + 2)]
    return out


def _pick(p, k, per_class, seed):
    rng = np.random.default_rng(seed)
    rows = []
    for key, lst in sorted(_classes(p, k).items()):
        idx = rng.choice(len(lst), size=min(per_class, len(lst)), replace=False)
        rows += [lst[i] for i in idx]
    return np.array(rows, dtype=np.int32)


@pytest.mark.parametrize("p", EXT_PRIMES)
def test_extended_encode_matches_oracle(p):
    w = 48 if p > 40 else 272
    for k in sorted({p + 1, (3 * p) // 2, 2 * p - 1}):
        log(f"extended encode p={p} k={k} W={w}")
        want = _stripes(p, k, w, 2, seed=p * 100 + k)
        assert np.array_equal(_encode(want, p, k, w), want), (p, k)


@pytest.mark.parametrize("p", EXT_PRIMES)
def test_extended_recover_every_class(p):
    k = 2 * p - 1
    w = 48 if p > 40 else 144
    er = _pick(p, k, 6 if p > 30 else 10, seed=p)
    log(f"extended recover p={p} k={k} W={w} entries={len(er)}")
    want = _stripes(p, k, w, len(er), seed=7 * p)
    assert np.array_equal(_recover(want, p, k, w, er), want)


@pytest.mark.parametrize("p", [5, 11, 13])
def test_extended_recover_every_pair(p):
    k = 2 * p - 1
    w = 80
    er = np.array(list(itertools.combinations(range(k + 2), 2)) + [(e, -1) for e in range(k + 2)], np.int32)
    log(f"extended recover every pair p={p} k={k} entries={len(er)}")
    want = _stripes(p, k, w, len(er), seed=11 * p)
    assert np.array_equal(_recover(want, p, k, w, er), want)


@pytest.mark.parametrize("p", [5, 13, 29, 61])
def test_extended_every_launch_configuration(p):
    k = p + 3 if p > 5 else 9
    w = 1040 if p <= 13 else 272
    er = _pick(p, k, 3, seed=3 * p)
    want = _stripes(p, k, w, len(er), seed=13 * p)
    for v in (1, 2, 4):
        for u in (1, 2, 4):
            if not r.raid6c_unroll_mask(p, v) & u:
                continue
            # split-K entries run the split-K extended kernels
            cfgs = [(t, 1) for t in (64, 128, 256)] + [(64 * sp, sp) for sp in (2, 4) if r.raid6c_split_mask(p, v) & sp]
            for t, sp in cfgs:
                order = (v + u + t // 64 + sp) % 3
                log(f"extended config p={p} k={k} vec={v} unroll={u} threads={t} split={sp} order={order}")
                _set_ext(p, w, v, u, t, sp, order)
                assert np.array_equal(_encode(want[:2], p, k, w), want[:2]), (v, u, t, sp)
                assert np.array_equal(_recover(want, p, k, w, er), want), (v, u, t, sp)
    r.raid6c_tune_clear()


def _set_ext(p, w, v, u, t, sp, order=0):
    """Launch configuration of stripes with k > p (table slots 2: encode, 3:
    recovery), checked to be the one the next launches will use."""
    for op in (2, 3):
        r.raid6c_tune_set(p, op, w, v, u, t, sp, order)
        assert r.raid6c_tune_get(p, op, w) == (v, u, t, sp, order), (p, op, w)


@pytest.mark.parametrize("p", [5, 13, 29])
def test_extended_split_every_class(p):
    # k = 2p-1: the waves' strip ranges fall below p, straddle it, and lie
    # wholly above it; every erasure class, every built split configuration.
    k = 2 * p - 1
    w = 1040 if p <= 13 else 272
    er = _pick(p, k, 4, seed=5 * p)
    want = _stripes(p, k, w, len(er), seed=17 * p)
    n = 0
    for v in (1, 2, 4):
        for u in (1, 2, 4):
            if not r.raid6c_unroll_mask(p, v) & u:
                continue
            for sp in (2, 4):
                if not r.raid6c_split_mask(p, v) & sp:
                    continue
                log(f"extended split p={p} k={k} vec={v} unroll={u} split={sp} entries={len(er)}")
                _set_ext(p, w, v, u, 64 * sp, sp)
                assert np.array_equal(_encode(want, p, k, w), want), (v, u, sp)
                assert np.array_equal(_recover(want, p, k, w, er), want), (v, u, sp)
                n += 1
    r.raid6c_tune_clear()
    assert n > 0


def test_extended_default_rule_large_prime_whole_tiles():
    """p = 53, k = 2p-1, rows of whole 512-byte tiles: the built-in rule's
    choice for extended stripes (no table entry), every erasure class."""
    p, k, w = 53, 105, 1024
    er = _pick(p, k, 4, seed=53)
    want = _stripes(p, k, w, len(er), seed=19 * p)
    log(f"extended default rule p={p} k={k} W={w}: encode {r.raid6c_tune_get(p, 2, w)}, "
        f"recovery {r.raid6c_tune_get(p, 3, w)}")
    assert np.array_equal(_encode(want, p, k, w), want)
    assert np.array_equal(_recover(want, p, k, w, er), want)


def test_extended_cached_entries():
    """Each extended-parity entry of the shipped tuning cache, at its own
    geometry (fewer stripes), every erasure class."""
    import json
    import os
    path = os.path.join(os.path.dirname(r.__file__), "tuned_mi355x.json")
    with open(path) as f:
        entries = [e for e in json.load(f)["entries"] if e["op"] in (2, 3)]
    assert entries
    for e in entries:
        p, w, k = e["p"], e["row_bytes"], e["k"]
        cfg = (e["vec"], e["unroll"], e["threads"], e["split"], e["order"])
        r.raid6c_tune_clear()
        r.raid6c_tune_set(p, e["op"], w, *cfg)
        assert r.raid6c_tune_get(p, e["op"], w) == cfg
        er = _pick(p, k, 3, seed=e["op"] * 100 + p)
        want = _stripes(p, k, w, len(er), seed=23 * p + e["op"])
        log(f"cached extended entry p={p} op={e['op']} W={w} k={k} config={cfg}")
        if e["op"] == 2:
            assert np.array_equal(_encode(want, p, k, w), want), cfg
        else:
            assert np.array_equal(_recover(want, p, k, w, er), want), cfg
    r.raid6c_tune_clear()


def test_extended_single_stripe_pointer_tables():
    # p = 61, k = 121: the largest strip table (123 strips), scattered strips.
    import torch
    p, k, w = 61, 121, 32
    want = _stripes(p, k, w, 1, seed=61)[0]
    bufs = [to_dev(np.ascontiguousarray(want[j])) for j in range(k + 2)]
    pads = [torch.empty(512, dtype=torch.uint8, device="cuda:0") for _ in range(k + 2)]   # keep strips apart
    for j in (k, k + 1):
        bufs[j].copy_(to_dev(datagen.poison((p - 1, w), index=j)))
    r.raid6c_encode(p, k, w, bufs[:k], bufs[k], bufs[k + 1])
    for j in range(k + 2):
        assert np.array_equal(to_host(bufs[j]), want[j]), j
    for e0, e1 in [(3, 70), (64, 100), (60, k), (90, k + 1), (0, 61), (5, 66), (k, k + 1)]:
        log(f"single-stripe recover p={p} k={k} ({e0}, {e1})")
        bufs[e0].copy_(to_dev(datagen.poison((p - 1, w), index=e0)))
        bufs[e1].copy_(to_dev(datagen.poison((p - 1, w), index=e1 + 1000)))
        r.raid6c_recover_2(p, k, w, bufs, e0, e1)
        for j in range(k + 2):
            assert np.array_equal(to_host(bufs[j]), want[j]), (e0, e1, j)
    del pads


def test_extended_write_and_degraded_read():
    import torch
    p, k, w = 13, 25, 64
    strip = (p - 1) * w
    want = _stripes(p, k, w, 1, seed=5)[0]
    src = to_dev(np.ascontiguousarray(want[:k]))
    store = torch.empty((k + 2, p - 1, w), dtype=torch.uint8, device="cuda:0")
    store.copy_(to_dev(datagen.poison((k + 2, p - 1, w), index=9)))
    strips = [store[j] for j in range(k + 2)]
    r.raid6c_write(p, k, w, src, strip, strips)
    assert np.array_equal(to_host(store), want)
    out = torch.empty((2, p - 1, w), dtype=torch.uint8, device="cuda:0")
    for e0, e1 in [(2, 20), (14, 24), (17, k), (19, k + 1), (4, -1)]:
        out.fill_(0x5A)
        r.raid6c_read_degraded(p, k, w, strips, e0, e1, out)
        got = to_host(out)
        assert np.array_equal(got[0], want[e0]), (e0, e1)
        if e1 >= 0:
            assert np.array_equal(got[1], want[e1]), (e0, e1)
    assert np.array_equal(to_host(store), want)      # a degraded read writes nothing in the stripe

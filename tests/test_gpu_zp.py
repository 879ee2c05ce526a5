"""GPU parity of the Z_p-RAID kernels against the CPU oracle, bit-exact.

Inputs come from the seeded generators; expected values come from the oracle
only.  Erased strips are overwritten with random bytes before each recovery,
and whole stripes (including strips and gaps a call must not write) are
compared.
"""

import itertools

import numpy as np
import pytest

import datagen
import paper_cs_0611109_amd as r
from gpu_util import device, log, to_dev, to_host
from oracle import zp_raid as zp

pytestmark = pytest.mark.gpu

PRIMES = [3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61]


def _stripes(p, k, w, n, seed):
    data = datagen.fill_stripes(seed, 0, n, k, p, w)
    return zp.encode_stripe(data, p)                       # (n, k+2, p-1, w), oracle


def _encode_on_gpu(want, p, k, w):
    import torch
    n = want.shape[0]
    dev = to_dev(want.copy())
    dev[:, k:] = to_dev(datagen.poison((n, 2, p - 1, w), index=p * 1000 + k))
    r.raid6c_encode_n(p, k, w, dev, (p - 1) * w, (k + 2) * (p - 1) * w, n)
    return to_host(dev)


def _recover_on_gpu(want, p, k, w, er):
    import torch
    n = want.shape[0]
    dev = to_dev(want)
    for s in range(n):
        for e in er[s]:
            if e >= 0:
                dev[s, e] = to_dev(datagen.poison((p - 1, w), index=s * 64 + int(e)))
    er_dev = to_dev(er.astype(np.int32))
    bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    r.raid6c_recover_n(p, k, w, dev, (p - 1) * w, (k + 2) * (p - 1) * w, n, er_dev, bad)
    assert int(bad.item()) == 0
    return to_host(dev)


def _configs(p):
    """Every built launch configuration (vec, unroll, threads, split)."""
    out = []
    for v in (1, 2, 4):
        for u in (1, 2, 4):
            if not r.raid6c_unroll_mask(p, v) & u:
                continue
            out += [(v, u, t, 1) for t in (64, 128, 256)]
            out += [(v, u, 64 * sp, sp) for sp in (2, 4) if r.raid6c_split_mask(p, v) & sp]
    return out


@pytest.fixture(autouse=True)
def _clean_tuning():
    device()
    r.raid6c_tune_clear()
    yield
    r.raid6c_tune_clear()


@pytest.mark.parametrize("p", PRIMES)
def test_encode_matches_oracle(p):
    for k in sorted({1, 2, p - 1, p}):
        for w in (16, 80, 1040):
            log(f"encode p={p} k={k} W={w}")
            want = _stripes(p, k, w, 3, seed=p * 100 + k)
            got = _encode_on_gpu(want, p, k, w)
            assert np.array_equal(got, want), (p, k, w)


@pytest.mark.parametrize("p", PRIMES)
def test_recover_every_case_matches_oracle(p):
    k = p - 1 if p > 3 else 2
    w = 272
    pairs = list(itertools.combinations(range(k + 2), 2)) + [(e, -1) for e in range(k + 2)]
    if len(pairs) > 96:
        rng = np.random.default_rng(p)
        keep = [pr for pr in pairs if pr[0] >= k or pr[1] >= k or pr[1] == -1]
        dd = [pr for pr in pairs if pr not in keep]
        pairs = keep + [dd[i] for i in rng.choice(len(dd), size=48, replace=False)]
    er = np.array(pairs, dtype=np.int32)
    log(f"recover p={p} k={k} W={w} cases={len(er)}")
    want = _stripes(p, k, w, len(er), seed=p)
    got = _recover_on_gpu(want, p, k, w, er)
    bad = [tuple(er[s]) for s in range(len(er)) if not np.array_equal(got[s], want[s])]
    assert not bad, bad[:8]


@pytest.mark.parametrize("p", [3, 5, 7, 11, 13, 17, 29, 31, 37, 61])
def test_every_launch_config(p):
    for k in sorted({min(p, 6), p}):
        for ci, (v, u, t, sp) in enumerate(_configs(p)):
            # 128: rows on cache lines (non-temporal loads, work-group order
            # as configured: each of the three in turn); the others not
            # (chunked order, or spread stripes when order 2 is configured).
            order = ci % 3
            for w in (16, 128, 64 * 4 * v + 16):
                log(f"config p={p} k={k} vec={v} unroll={u} threads={t} split={sp} order={order} W={w}")
                r.raid6c_tune_set(p, 0, w, v, u, t, sp, order)
                r.raid6c_tune_set(p, 1, w, v, u, t, sp, order)
                want = _stripes(p, k, w, 4, seed=7 * p + v + t + u)
                assert np.array_equal(_encode_on_gpu(want, p, k, w), want), (v, u, t, sp, w)
                er = datagen.erasures(v * 1000 + t + u, 4, k, "any")
                assert np.array_equal(_recover_on_gpu(want, p, k, w, er), want), (v, u, t, sp, w)
                _single_stripe_calls(want[0], p, k, w, (v, u, t, sp, w))


def _single_stripe_calls(stripe, p, k, w, tag):
    """recover_2, recover_1 and read_degraded on one stripe: the erasures come
    from the call's arguments, not from a device array."""
    import torch
    dev = to_dev(stripe)
    strips = [dev[j] for j in range(k + 2)]
    pairs = [(0, k), (k, k + 1)] + ([(0, 1)] if k > 1 else []) + [(k - 1, k + 1)]
    for e0, e1 in pairs:
        dev[e0] = to_dev(datagen.poison((p - 1, w), index=e0))
        dev[e1] = to_dev(datagen.poison((p - 1, w), index=e1 + 64))
        r.raid6c_recover_2(p, k, w, strips, e0, e1)
        assert np.array_equal(to_host(dev), stripe), ("recover_2", e0, e1, tag)
    for e in (0, k, k + 1):
        dev[e] = to_dev(datagen.poison((p - 1, w), index=e + 128))
        r.raid6c_recover_1(p, k, w, strips, e)
        assert np.array_equal(to_host(dev), stripe), ("recover_1", e, tag)
    out = torch.empty((2, p - 1, w), dtype=torch.uint8, device="cuda:0")
    e0, e1 = pairs[-1]
    out.fill_(0xEE)
    r.raid6c_read_degraded(p, k, w, strips, e0, e1, out)
    got = to_host(out)
    assert np.array_equal(got[0], stripe[e0]) and np.array_equal(got[1], stripe[e1]), ("read", tag)
    assert np.array_equal(to_host(dev), stripe), ("read wrote the stripe", tag)


def test_config1_all_pairs():
    # p = 5, k = 4, W = 64, 1024 stripes: encode, then each of the 15 pairs and
    # the 6 single erasures applied to all stripes.
    p, k, w, n = 5, 4, 64, 1024
    data = datagen.fill_stripes(1, 0, n, k, p, w)
    want = zp.encode_stripe(data, p)
    got = _encode_on_gpu(want, p, k, w)
    assert np.array_equal(got, want)
    cases = list(itertools.combinations(range(k + 2), 2)) + [(e, -1) for e in range(k + 2)]
    for e in cases:
        log(f"config1 erasure {e}")
        er = np.tile(np.array(e, dtype=np.int32), (n, 1))
        assert np.array_equal(_recover_on_gpu(want, p, k, w, er), want), e
    # The oracle's own recovery agrees on a sample (same expected values).
    for e in [(0, 1), (2, 4), (1, 5), (4, 5)]:
        bad = want[:8].copy()
        bad[:, list(e)] = 0
        assert np.array_equal(zp.recover(bad, p, e), want[:8])


def test_single_stripe_entry_points_scattered_strips():
    import torch
    p, k, w = 13, 12, 4096 + 48
    want = _stripes(p, k, w, 1, seed=99)[0]
    bufs = [to_dev(np.concatenate([datagen.poison((64,), index=j), want[j].reshape(-1),
                                   datagen.poison((80,), index=100 + j)])) for j in range(k + 2)]
    views = [b[64:64 + (p - 1) * w] for b in bufs]
    for j in (k, k + 1):
        views[j].copy_(to_dev(datagen.poison(((p - 1) * w,), index=200 + j)))
    r.raid6c_encode(p, k, w, views[:k], views[k], views[k + 1])
    torch.cuda.synchronize()
    for j in range(k + 2):
        assert np.array_equal(to_host(views[j]).reshape(p - 1, w), want[j]), j
    guard = [to_host(b[:64]).copy() for b in bufs] + [to_host(b[-80:]).copy() for b in bufs]
    for e in [(0, 1), (3, 9), (5, k), (7, k + 1), (k, k + 1)]:
        for j in e:
            views[j].copy_(to_dev(datagen.poison(((p - 1) * w,), index=300 + j)))
        r.raid6c_recover_2(p, k, w, views, e[1], e[0])
        for j in range(k + 2):
            assert np.array_equal(to_host(views[j]).reshape(p - 1, w), want[j]), (e, j)
    for e in [0, 6, k, k + 1]:
        views[e].copy_(to_dev(datagen.poison(((p - 1) * w,), index=400 + e)))
        r.raid6c_recover_1(p, k, w, views, e)
        assert np.array_equal(to_host(views[e]).reshape(p - 1, w), want[e]), e
    after = [to_host(b[:64]) for b in bufs] + [to_host(b[-80:]) for b in bufs]
    assert all(np.array_equal(a, b) for a, b in zip(guard, after))


def test_gaps_between_strips_untouched():
    import torch
    p, k, w, n = 11, 7, 160, 5
    strip = (p - 1) * w
    strip_stride = strip + 48
    stripe_stride = (k + 2) * strip_stride + 96
    want = _stripes(p, k, w, n, seed=5)
    raw = datagen.poison((n * stripe_stride,), index=77)
    for s in range(n):
        for j in range(k):
            off = s * stripe_stride + j * strip_stride
            raw[off:off + strip] = want[s, j].reshape(-1)
    dev = to_dev(raw)
    r.raid6c_encode_n(p, k, w, dev, strip_stride, stripe_stride, n)
    got = to_host(dev)
    mask = np.ones(raw.shape, dtype=bool)
    for s in range(n):
        for j in range(k + 2):
            off = s * stripe_stride + j * strip_stride
            assert np.array_equal(got[off:off + strip], want[s, j].reshape(-1)), (s, j)
            mask[off:off + strip] = False
    assert np.array_equal(got[mask], raw[mask])
    er = to_dev(datagen.erasures(3, n, k, "any"))
    r.raid6c_recover_n(p, k, w, dev, strip_stride, stripe_stride, n, er)
    got2 = to_host(dev)
    assert np.array_equal(got2, got)
    del torch


def test_invalid_erasure_entries_are_counted_and_skipped():
    import torch
    p, k, w = 7, 5, 64
    want = _stripes(p, k, w, 6, seed=8)
    dev = to_dev(want)
    er = np.array([[0, 1], [3, 3], [-1, -1], [9, 0], [2, 8], [1, -1]], dtype=np.int32)
    for s in (0, 5):
        for e in er[s]:
            if e >= 0:
                dev[s, e] = 0
    bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    r.raid6c_recover_n(p, k, w, dev, (p - 1) * w, (k + 2) * (p - 1) * w, 6, to_dev(er), bad)
    assert int(bad.item()) == 4
    assert np.array_equal(to_host(dev), want)


def test_empty_call_is_a_noop():
    r.raid6c_encode_n(5, 4, 64, 0, 256, 1536, 0)


def test_rs_encode_matches_oracle():
    from oracle import rs_gf256 as rs
    for k, nbytes, n in [(1, 16, 3), (4, 272, 5), (12, 48 * 1024, 3), (30, 4096 + 16, 2)]:
        log(f"rs k={k} bytes={nbytes}")
        rng = np.random.default_rng(k)
        data = rng.integers(0, 256, size=(n, k, nbytes), dtype=np.uint8)
        P, Q = rs.encode(data)
        dev = to_dev(np.concatenate([data, datagen.poison((n, 2, nbytes))], axis=1))
        r.raid6c_rs_encode_n(k, nbytes, dev, nbytes, (k + 2) * nbytes, n)
        got = to_host(dev)
        assert np.array_equal(got[:, k], P) and np.array_equal(got[:, k + 1], Q)
        assert np.array_equal(got[:, :k], data)


@pytest.mark.parametrize("p,w", [(5, 4096), (13, 4096), (29, 1024)])
def test_every_config_every_two_erasure_kind_many_stripes(p, w):
    # Many stripes per (configuration, case): a fault that hits a few lanes of
    # a few work-groups shows up here even when small tests pass.
    k = p - 1
    n = 192
    want = zp.encode_stripe(datagen.fill_stripes(p, 0, n, k, p, w), p)
    for ci, (v, u, t, sp) in enumerate(_configs(p)):
        order = ci % 3                  # every work-group order; grids of 10^3 work-groups
        r.raid6c_tune_set(p, 0, w, v, u, t, sp, order)
        r.raid6c_tune_set(p, 1, w, v, u, t, sp, order)
        log(f"many stripes p={p} W={w} vec={v} unroll={u} threads={t} split={sp} order={order}")
        assert np.array_equal(_encode_on_gpu(want, p, k, w), want), ("encode", v, u, t, sp)
        for kind in ("dd", "dp", "dq", "pq", "d"):
            er = datagen.erasures(p * 100 + v + u + t, n, k, kind)
            got = _recover_on_gpu(want, p, k, w, er)
            bad = [s for s in range(n) if not np.array_equal(got[s], want[s])]
            assert not bad, (kind, v, u, t, sp, bad[:5], [tuple(er[s]) for s in bad[:5]])


@pytest.mark.parametrize("p,k,w,n", [(13, 12, 4112, 250), (53, 6, 2064, 200)])
def test_rows_off_lines_many_work_groups(p, k, w, n):
    # Rows 16 bytes past a 128-byte multiple: every launch loads through the
    # caches and takes the XCD-chunked work-group order, which permutes full
    # super-blocks of 128 work-groups and leaves the tail in place.  These
    # grids hold several super-blocks and a tail in every configuration.
    want = zp.encode_stripe(datagen.fill_stripes(p + 1, 0, n, k, p, w), p)
    for (v, u, t, sp) in _configs(p):
        tile = (64 if sp > 1 else t) * v * 4
        grid = n * -(-w // tile)
        assert grid > 2 * 128 and grid % 128 != 0, (v, t, sp, grid)
        r.raid6c_tune_set(p, 0, w, v, u, t, sp)
        r.raid6c_tune_set(p, 1, w, v, u, t, sp)
        log(f"rows off lines p={p} k={k} W={w} vec={v} unroll={u} threads={t} split={sp} grid={grid}")
        assert np.array_equal(_encode_on_gpu(want, p, k, w), want), ("encode", v, u, t, sp)
        er = datagen.erasures(p * 7 + v + u + t, n, k, "any")
        got = _recover_on_gpu(want, p, k, w, er)
        bad = [s for s in range(n) if not np.array_equal(got[s], want[s])]
        assert not bad, (v, u, t, sp, bad[:5])


def _built(p, cfg):
    v, u, t, sp, order = cfg
    return (r.raid6c_unroll_mask(p, v) & u and order in (0, 1, 2) and
            (sp == 1 and t in (64, 128, 256) or r.raid6c_split_mask(p, v) & sp and t == 64 * sp))


def test_autotuner_records_per_slot_and_keeps_results():
    # The strided autotuner runs every configuration on the caller's stripes:
    # afterwards they must still be bit-exact, and the choice is recorded for
    # (p, op, row-size bucket) -- op + 2 for the extended Q parity -- without
    # touching the other slots.
    import torch
    r.raid6c_tune_clear()
    p, w, n = 13, 1040, 24
    strip = (p - 1) * w
    recorded = {}
    try:
        for k in (12, 20):
            want = _stripes(p, k, w, n, seed=50 + k)
            dev = to_dev(want.copy())
            stride = (k + 2) * strip
            log(f"autotune p={p} k={k} W={w} encode")
            assert r.raid6c_autotune_n(p, k, w, dev, strip, stride, n, 0, reps=1) > 0
            er = datagen.erasures(60 + k, n, k, "any")
            log(f"autotune p={p} k={k} W={w} recovery")
            assert r.raid6c_autotune_n(p, k, w, dev, strip, stride, n, 1, to_dev(er.astype(np.int32)), reps=1) > 0
            assert np.array_equal(to_host(dev), want), k
            base = 2 if k > p else 0
            for op in (0, 1):
                cfg = r.raid6c_tune_get(p, base + op, w)
                assert _built(p, cfg), (k, op, cfg)
                recorded[base + op] = cfg
        # the extended run left the plain entries alone
        assert r.raid6c_tune_get(p, 0, w) == recorded[0] and r.raid6c_tune_get(p, 1, w) == recorded[1]
        # and the recorded configurations still give the oracle's results
        for k in (12, 20):
            want = _stripes(p, k, w, 8, seed=70 + k)
            assert np.array_equal(_encode_on_gpu(want, p, k, w), want), k
            er = datagen.erasures(80 + k, 8, k, "any")
            assert np.array_equal(_recover_on_gpu(want, p, k, w, er), want), k
    finally:
        r.raid6c_tune_clear()


def test_more_stripes_than_one_launch_holds():
    # 2^31 threads is the most one launch takes: with 64-thread work-groups
    # and one column tile per stripe, 2^25 stripes.  2^25 + 4096 stripes of
    # p = 5, k = 2, 16-byte rows (8.6 GB) need a second launch; stripes on
    # both sides of the boundary are checked against the oracle.
    import torch
    device()
    p, k, w = 5, 2, 16
    per_launch = 1 << 25
    n = per_launch + 4096
    strip = (p - 1) * w
    stride = (k + 2) * strip
    free, _ = torch.cuda.mem_get_info()
    if free < n * stride + (8 << 30):
        pytest.skip("needs about 17 GB of free device memory")
    r.raid6c_tune_set(p, 0, w, 1, 1, 64)
    r.raid6c_tune_set(p, 1, w, 1, 1, 64)
    dev = None
    try:
        dev = torch.empty((n, k + 2, p - 1, w), dtype=torch.uint8, device="cuda:0")
        g = torch.Generator(device="cuda:0")
        g.manual_seed(91)
        dev.random_(0, 256, generator=g)
        sample = [0, 1, per_launch - 2, per_launch - 1, per_launch, per_launch + 1, n - 1, 12345, n - 777]
        log(f"encode {n} stripes (two launches)")
        r.raid6c_encode_n(p, k, w, dev, strip, stride, n)
        torch.cuda.synchronize()
        got = {s: to_host(dev[s]) for s in sample}
        for s in sample:
            want = zp.encode_stripe(got[s][None, :k], p)[0]
            assert np.array_equal(got[s], want), s
        # every stripe gets one of the six pairs of its 4 strips, in turn
        pairs = np.array(list(itertools.combinations(range(k + 2), 2)), dtype=np.int32)
        er = torch.from_numpy(pairs[np.arange(n) % len(pairs)]).to("cuda:0")
        for s in sample:
            for e in pairs[s % len(pairs)]:
                dev[s, e] = to_dev(datagen.poison((p - 1, w), index=s * 8 + int(e)))
        bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        log(f"recover {n} stripes (two launches)")
        r.raid6c_recover_n(p, k, w, dev, strip, stride, n, er, bad)
        torch.cuda.synchronize()
        assert int(bad.item()) == 0
        for s in sample:
            assert np.array_equal(to_host(dev[s]), got[s]), s
    finally:
        r.raid6c_tune_clear()
        del dev
        torch.cuda.empty_cache()

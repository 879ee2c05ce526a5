"""GPU parity of plans (mixed stripes in one persistent graph launch) against
the CPU oracle, bit-exact, for every schedule and after autotuning."""

import numpy as np
import pytest

import datagen
import paper_cs_0611109_amd as r
from gpu_util import device, log, to_dev, to_host
from oracle import zp_raid as zp

pytestmark = pytest.mark.gpu

PRIMES = [3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61]


def _mixed_jobs(seed, n, w_max=1200, ext=False):
    """Random geometries over every prime, all erasure cases, ragged rows;
    with `ext`, k up to 2p-1 (extended Q parity) where the prime allows it."""
    d = datagen.Draws(seed, datagen.TAG_GEOMETRY, 1)
    out = []
    for i in range(n):
        p = PRIMES[d.below(len(PRIMES))]
        k = d.between(1, r.raid6c_max_data_strips(p) if ext else p)
        w = 16 * d.between(1, w_max // 16)
        kind = d.below(3)
        if kind == 0:
            e = (-1, -1)
        elif kind == 1:
            e = (d.below(k + 2), -1)
        else:
            a = d.below(k + 2)
            b = d.below(k + 1)
            b += b >= a
            e = (a, b)
        out.append((p, k, w, e))
    return out


def _layout(specs, gap=48, align=16):
    """Byte offsets of each stripe in one buffer, with gaps between strips;
    strides and stripe offsets rounded up to `align` bytes."""
    up = lambda x: (x + align - 1) // align * align
    offs, pos = [], 0
    for (p, k, w, _) in specs:
        strip = (p - 1) * w
        stride = up(strip + gap)
        offs.append((pos, stride))
        pos = up(pos + (k + 2) * stride + 64)
    return offs, pos


def _run_plan(specs, seed, schedules=None, autotune=False, align=16):
    device()
    offs, total = _layout(specs, align=align)
    raw = datagen.poison((total,), index=seed)
    want = []
    for i, ((p, k, w, e), (off, stride)) in enumerate(zip(specs, offs)):
        st = zp.encode_stripe(datagen.stripe_data(seed, i, k, p, w), p)
        want.append(st)
        for j in range(k + 2):
            if e[0] == -1 and j >= k:
                continue                      # encode: P, Q stay poisoned
            if j in e:
                continue                      # erased: stays poisoned
            raw[off + j * stride: off + j * stride + (p - 1) * w] = st[j].reshape(-1)
    dev = to_dev(raw)
    base = dev.data_ptr()
    jobs = []
    for (p, k, w, e), (off, stride) in zip(specs, offs):
        op = r.RAID6C_JOB_ENCODE if e[0] == -1 else r.RAID6C_JOB_RECOVER
        jobs.append(r.raid6c_job(op, p, k, e[0], e[1], w, stride, base + off))
    plan = r.raid6c_plan_create(jobs)
    try:
        info = r.raid6c_plan_stats(plan)
        assert info.njobs == len(specs)
        results = []
        for sched in (schedules or [None]):
            if sched is not None:
                r.raid6c_plan_set_schedule(plan, *sched)
            if autotune:
                r.raid6c_plan_autotune(plan, reps=1)
            r.raid6c_plan_run(plan)
            results.append((sched, to_host(dev)))
    finally:
        r.raid6c_plan_destroy(plan)
    for sched, got in results:
        for i, ((p, k, w, e), (off, stride)) in enumerate(zip(specs, offs)):
            for j in range(k + 2):
                seg = got[off + j * stride: off + j * stride + (p - 1) * w].reshape(p - 1, w)
                assert np.array_equal(seg, want[i][j]), (sched, i, (p, k, w, e), j)
        # bytes outside the strips are untouched
        mask = np.ones(total, dtype=bool)
        for (p, k, w, e), (off, stride) in zip(specs, offs):
            for j in range(k + 2):
                mask[off + j * stride: off + j * stride + (p - 1) * w] = False
        assert np.array_equal(got[mask], raw[mask]), sched


def test_plan_mixed_geometries():
    specs = _mixed_jobs(1, 160)
    log(f"plan with {len(specs)} mixed jobs")
    _run_plan(specs, seed=21)


def test_plan_every_schedule():
    specs = _mixed_jobs(2, 60)
    scheds = [(w, c, o) for o in (0, 1, 2) for w in (1, 8) for c in (1, 5, 64)] + [(8, 4, 0, 1), (8, 4, 0, 2)]
    _run_plan(specs, seed=22, schedules=scheds)


def test_plan_after_autotune():
    specs = _mixed_jobs(3, 40)
    _run_plan(specs, seed=23, autotune=True)


def test_plan_rows_on_cache_lines():
    """Rows, strides and stripes on 128-byte lines (non-temporal loads) and,
    in the same plan's second half, rows 16 bytes past them (ordinary loads),
    through the chained job-list grids and through the persistent kernel."""
    specs = [(p, k, 128 * m, e) for (p, k, w, e), m in zip(_mixed_jobs(4, 40), [1, 2, 3, 5, 8] * 8)]
    specs = [s if i < 20 else (s[0], s[1], s[2] + 16, s[3]) for i, s in enumerate(specs)]
    _run_plan(specs, seed=25, align=128, schedules=[(8, 4, 0, 2), (8, 1, 0)])


def test_plan_every_case_large_prime():
    specs = []
    for p in (53, 61):
        k = p
        for e in [(-1, -1), (0, -1), (k, -1), (k + 1, -1), (0, 1), (3, k - 1), (5, k), (7, k + 1), (k, k + 1)]:
            specs.append((p, k, 272, e))
    _run_plan(specs, seed=24)


def test_empty_plan():
    device()
    plan = r.raid6c_plan_create([])
    r.raid6c_plan_run(plan)
    assert r.raid6c_plan_stats(plan).nitems == 0
    r.raid6c_plan_destroy(plan)


def test_plan_extended_q_parity_mixed_with_plain():
    """Jobs with k up to 2p-1 (extended Q parity, Section 3.3) beside plain
    ones, every case, both grouped schedules; the persistent kernel (plain
    code only) is refused for such a plan."""
    specs = _mixed_jobs(6, 120, w_max=640, ext=True)
    n_ext = sum(k > p for p, k, _, _ in specs)
    log(f"plan with {len(specs)} jobs, {n_ext} with k > p")
    assert n_ext >= 30
    _run_plan(specs, seed=26, schedules=[(8, 4, 0, 1), (8, 4, 0, 2)])
    _run_plan(specs[:40], seed=27, autotune=True)


def test_plan_extended_refuses_persistent_schedule():
    import torch
    device()
    p, k, w = 13, 20, 64
    buf = torch.zeros((k + 2) * (p - 1) * w, dtype=torch.uint8, device="cuda:0")
    plan = r.raid6c_plan_create([r.raid6c_job(r.RAID6C_JOB_ENCODE, p, k, -1, -1, w, (p - 1) * w, buf.data_ptr())])
    try:
        with pytest.raises(r.Raid6cError) as ex:
            r.raid6c_plan_set_schedule(plan, 8, 4, 0, 0)
        assert ex.value.code == r.RAID6C_E_UNSUPPORTED
        r.raid6c_plan_run(plan)
    finally:
        r.raid6c_plan_destroy(plan)

"""The seeded input generators: determinism and the ranges of their draws."""

import itertools

import numpy as np
import pytest

import datagen


def test_stripe_bytes_are_deterministic_and_chunk_independent():
    a = datagen.fill_stripes(3, 0, 10, 4, 5, 64)
    b = datagen.fill_stripes(3, 4, 3, 4, 5, 64, threads=1)
    assert (a[4:7] == b).all()
    assert (datagen.stripe_data(3, 9, 4, 5, 64) == a[9]).all()
    assert not (datagen.stripe_data(4, 9, 4, 5, 64) == a[9]).all()


def test_bytes_look_uniform():
    b = datagen.random_bytes(1, datagen.TAG_DATA, 0, 1 << 16)
    counts = np.bincount(b, minlength=256)
    assert counts.min() > 150 and counts.max() < 380


@pytest.mark.parametrize("kind", datagen.ERASURE_KINDS)
def test_erasure_kinds(kind):
    k = 6
    e = datagen.erasures(7, 2000, k, kind)
    assert e.shape == (2000, 2)
    for e0, e1 in e:
        if kind in ("d", "p", "q", "any1"):
            assert e1 == -1 and 0 <= e0 < k + 2
            if kind == "d":
                assert e0 < k
            if kind == "p":
                assert e0 == k
            if kind == "q":
                assert e0 == k + 1
        else:
            assert 0 <= e0 < e1 < k + 2
            if kind == "dd":
                assert e1 < k
            if kind == "dp":
                assert e1 == k and e0 < k
            if kind == "dq":
                assert e1 == k + 1 and e0 < k
            if kind == "pq":
                assert (e0, e1) == (k, k + 1)
    if kind == "any":
        seen = {tuple(x) for x in e}
        assert seen == set(itertools.combinations(range(k + 2), 2))


def test_below_is_uniform_enough():
    d = datagen.Draws(0, datagen.TAG_GEOMETRY, 9)
    c = np.bincount([d.below(7) for _ in range(14000)], minlength=7)
    assert c.min() > 1800 and c.max() < 2200


def test_batch_jobs_ranges():
    jobs = datagen.batch_jobs(4, 3000)
    assert {j.p for j in jobs} == set(datagen.BATCH_PRIMES)
    for j in jobs:
        assert 2 <= j.k <= j.p - 1
        assert 512 <= j.row_bytes <= 65536 and j.row_bytes % 16 == 0
        if j.op == "recover":
            assert 0 <= j.e0 < j.e1 < j.k + 2
    frac = sum(j.op == "encode" for j in jobs) / len(jobs)
    assert 0.56 < frac < 0.64


def test_serve_requests_ranges():
    reqs = datagen.serve_requests(5, 2000, qps=1000.0)
    t = [r.arrival_s for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    for r in reqs:
        assert r.k == r.p - 1 and r.row_bytes % 16 == 0
        assert r.row_bytes * r.k * (r.p - 1) >= r.payload
        if r.kind == "read":
            assert reqs[r.target].kind == "write" and r.target < r.index
            assert 0 <= r.e0 < r.k
            assert r.e1 == -1 or r.e0 < r.e1 < r.k + 2


@pytest.mark.parametrize("kind", datagen.EXTENDED_ERASURE_KINDS)
def test_extended_erasures_stay_in_their_class(kind):
    p, k = 13, 25
    e = datagen.erasures_extended(3, 3000, k, p, kind)
    assert e.shape == (3000, 2) and e.dtype == np.int32
    assert (e[:, 0] < e[:, 1]).all()
    x, y = e[:, 0], e[:, 1]
    if kind == "dd_mixed":
        assert (x < p).all() and (y >= p).all() and (y < k).all()
        assert len(set(map(tuple, e))) == p * (k - p)          # every mixed pair occurs
    elif kind == "dd_ext":
        assert (x >= p).all() and (y < k).all()
    elif kind == "dp_ext":
        assert (x >= p).all() and (x < k).all() and (y == k).all()
    else:
        assert (x >= p).all() and (x < k).all() and (y == k + 1).all()
    assert np.array_equal(e, datagen.erasures_extended(3, 3000, k, p, kind))

"""GPU tests of the request server: every write's stored stripe and every
degraded read's rebuilt strips equal the oracle's, and are identical whether
requests run alone (one plain launch each) or mixed in overlapping batches."""

import numpy as np
import pytest

import datagen
import paper_cs_0611109_amd as r
from gpu_util import device, log, to_host
from oracle import zp_raid as zp

pytestmark = pytest.mark.gpu


def _stage(reqs, seed):
    """Device payloads (writes) and output buffers (reads) for a request list."""
    import torch
    pay_off, out_off, pos_p, pos_o = {}, {}, 0, 0
    for q in reqs:
        strip = (q.p - 1) * q.row_bytes
        if q.kind == "write":
            pay_off[q.index] = pos_p
            pos_p += q.k * strip
        else:
            out_off[q.index] = pos_o
            pos_o += 2 * strip
    pay = torch.empty(max(16, pos_p), dtype=torch.uint8, device="cuda:0")
    out = torch.full((max(16, pos_o),), 0xEE, dtype=torch.uint8, device="cuda:0")
    data = {}
    for q in reqs:
        if q.kind == "write":
            d = datagen.stripe_data(seed, q.index, q.k, q.p, q.row_bytes)
            data[q.index] = d
            pay[pay_off[q.index]:pay_off[q.index] + d.size].copy_(torch.from_numpy(d.reshape(-1)))
    c = []
    for q in reqs:
        if q.kind == "write":
            c.append(r.raid6c_request(r.RAID6C_REQ_WRITE, q.p, q.k, -1, -1, q.row_bytes, q.index,
                                      pay.data_ptr() + pay_off[q.index], None, q.index))
        else:
            c.append(r.raid6c_request(r.RAID6C_REQ_READ, 0, 0, q.e0, q.e1, 0, q.target, None,
                                      out.data_ptr() + out_off[q.index], q.index))
    torch.cuda.synchronize()
    return c, pay, out, out_off, data


def _expected_stripes(reqs, data):
    return {q.index: zp.encode_stripe(data[q.index], q.p) for q in reqs if q.kind == "write"}


def _check(server, reqs, comps, out, out_off, stripes, allow_evicted=False):
    host_out = to_host(out)
    byidx = {q.index: q for q in reqs}
    for q, c in zip(reqs, comps):
        assert c.tag == q.index
        if q.kind == "read":
            if allow_evicted and c.status == r.RAID6C_ST_NOT_RESIDENT:
                continue
            assert c.status == r.RAID6C_ST_OK, (q, c.status)
            src = byidx[q.target]
            strip = (src.p - 1) * src.row_bytes
            want = stripes[q.target]
            es = sorted(e for e in (q.e0, q.e1) if e >= 0)
            for n, e in enumerate(es):
                got = host_out[out_off[q.index] + n * strip: out_off[q.index] + (n + 1) * strip]
                assert np.array_equal(got.reshape(src.p - 1, src.row_bytes), want[e]), (q, e)
        else:
            assert c.status == r.RAID6C_ST_OK, (q, c.status)
            assert c.arrival_ns <= c.launch_ns <= c.complete_ns
    # every resident stripe holds data + P + Q as the oracle computes them
    import torch
    for q in reqs:
        if q.kind != "write":
            continue
        try:
            base, stride = r.raid6c_server_stripe(server, q.index)
        except r.Raid6cError:
            assert allow_evicted
            continue
        want = stripes[q.index]
        n = want.shape[0] * stride
        t = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        got = _read_device(base, n, t)
        assert np.array_equal(got.reshape(want.shape), want), q


def _read_device(addr, n, tmp):
    """Copy n bytes from a raw device address (inside the server's store)."""
    import ctypes

    import torch
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    torch.cuda.synchronize()
    assert hip.hipMemcpy(ctypes.c_void_p(tmp.data_ptr()), ctypes.c_void_p(addr), n, 3) == 0  # device to device
    return to_host(tmp)


def _trace(seed, n, qps, pay_hi=256 << 10):
    return datagen.serve_requests(seed, n, qps, pay_hi=pay_hi)


@pytest.mark.parametrize("persistent", [False, True])
def test_served_results_match_oracle(persistent):
    device()
    reqs = _trace(31, 300, qps=20000.0)
    c, pay, out, out_off, data = _stage(reqs, 31)
    stripes = _expected_stripes(reqs, data)
    srv = r.raid6c_server_create(4 << 30, max_inflight=4, max_batch=64, persistent=persistent)
    try:
        comps = r.raid6c_server_replay(srv, c, [q.arrival_s for q in reqs])
        st = r.raid6c_server_get_stats(srv)
        log(f"served: {st.batches} batches for {st.completed} requests")
        _check(srv, reqs, comps, out, out_off, stripes)
        assert st.completed == len(reqs) and st.batches < len(reqs)
    finally:
        r.raid6c_server_destroy(srv)


def test_every_prime_up_to_31_in_shared_grids_matches_oracle():
    """Writes and degraded reads over every prime up to 31, small enough
    that each batch's groups of these primes run as one grid of the
    multi-prime kernel (every case of its switch), checked against the
    oracle (Lemma 3.1.2: the rebuilt strips are unique)."""
    device()
    primes = (3, 5, 7, 11, 13, 17, 19, 23, 29, 31)
    reqs = datagen.serve_requests(43, 500, qps=200000.0, primes=primes, pay_hi=64 << 10)
    assert {q.p for q in reqs} == set(primes)
    c, pay, out, out_off, data = _stage(reqs, 43)
    stripes = _expected_stripes(reqs, data)
    srv = r.raid6c_server_create(4 << 30, max_inflight=4, max_batch=128)
    try:
        comps = r.raid6c_server_replay(srv, c, [q.arrival_s for q in reqs])
        _check(srv, reqs, comps, out, out_off, stripes)
        st = r.raid6c_server_get_stats(srv)
        log(f"{st.batches} batches for {len(reqs)} requests")
        assert st.batches < len(reqs)
    finally:
        r.raid6c_server_destroy(srv)


def test_alone_and_in_the_mix_are_identical():
    import torch
    device()
    reqs = _trace(32, 240, qps=50000.0)
    results = []
    for plain, inflight, persistent in ((True, 8, False), (False, 4, False), (False, 1, False), (False, 4, True)):
        c, pay, out, out_off, data = _stage(reqs, 32)
        stripes = _expected_stripes(reqs, data)
        srv = r.raid6c_server_create(4 << 30, max_inflight=inflight, max_batch=32, plain=plain,
                                     persistent=persistent)
        try:
            comps = r.raid6c_server_replay(srv, c, [q.arrival_s for q in reqs])
            _check(srv, reqs, comps, out, out_off, stripes)
            stored = {}
            for q in reqs:
                if q.kind == "write":
                    base, stride = r.raid6c_server_stripe(srv, q.index)
                    n = (q.k + 2) * stride
                    stored[q.index] = _read_device(base, n, torch.empty(n, dtype=torch.uint8, device="cuda:0"))
            results.append((to_host(out), stored, max(x.batch_size for x in comps)))
        finally:
            r.raid6c_server_destroy(srv)
    (o0, s0, b0), (o1, s1, b1), (o2, s2, b2), (o3, s3, b3) = results
    assert b0 == 1 and b1 > 1 and b3 > 1
    assert np.array_equal(o0, o1) and np.array_equal(o0, o2) and np.array_equal(o0, o3)
    for k in s0:
        assert np.array_equal(s0[k], s1[k]) and np.array_equal(s0[k], s2[k]) and np.array_equal(s0[k], s3[k])


# The served workload's own payload range (4 KiB - 4 MiB, log-uniform): rows
# reach 41 KB at p = 11.  Slot tables start at max_batch x 64 column tiles of
# 256 bytes, so with two requests per batch any request with rows over 32 KiB
# (and many pairs over 16 KiB) makes its slot enlarge its tables, while the
# other slots' batches are in flight.
FULL_SEED, FULL_N = 41, 300


def _full_trace():
    reqs = datagen.serve_requests(FULL_SEED, FULL_N, qps=200000.0)   # default pay_hi = 4 MiB
    assert max(q.payload for q in reqs) > 3 << 20
    assert sum(q.kind == "write" and q.row_bytes > 32768 for q in reqs) >= 1
    return reqs


@pytest.mark.parametrize("mode", ["grouped", "persistent"])
def test_full_size_payloads_grow_tables_and_match_oracle(mode):
    device()
    reqs = _full_trace()
    c, pay, out, out_off, data = _stage(reqs, FULL_SEED)
    stripes = _expected_stripes(reqs, data)
    srv = r.raid6c_server_create(4 << 30, max_inflight=4, max_batch=2, persistent=mode == "persistent")
    try:
        comps = r.raid6c_server_replay(srv, c, [q.arrival_s for q in reqs])
        st = r.raid6c_server_get_stats(srv)
        log(f"{mode}: {st.batches} batches, {st.table_grows} table enlargements, "
            f"largest row {max(q.row_bytes for q in reqs)} B")
        assert st.table_grows >= 1
        _check(srv, reqs, comps, out, out_off, stripes)
    finally:
        r.raid6c_server_destroy(srv)


def test_full_size_payloads_alone_and_in_the_mix_are_identical():
    """Each request alone (one plain launch) and in batches of up to 16, in
    both launch modes: the same rebuilt strips and stored stripes, all equal
    to the oracle's."""
    import torch
    device()
    reqs = _full_trace()
    results = []
    for plain, inflight, batch, persistent in ((True, 8, 1, False), (False, 4, 16, False), (False, 4, 16, True)):
        c, pay, out, out_off, data = _stage(reqs, FULL_SEED)
        stripes = _expected_stripes(reqs, data)
        srv = r.raid6c_server_create(4 << 30, max_inflight=inflight, max_batch=batch, plain=plain,
                                     persistent=persistent)
        try:
            comps = r.raid6c_server_replay(srv, c, [q.arrival_s for q in reqs])
            _check(srv, reqs, comps, out, out_off, stripes)
            stored = {}
            for q in reqs:
                if q.kind == "write":
                    base, stride = r.raid6c_server_stripe(srv, q.index)
                    n = (q.k + 2) * stride
                    stored[q.index] = _read_device(base, n, torch.empty(n, dtype=torch.uint8, device="cuda:0"))
            results.append((to_host(out), stored, max(x.batch_size for x in comps)))
        finally:
            r.raid6c_server_destroy(srv)
        del pay, out
    (o0, s0, b0), (o1, s1, b1), (o2, s2, b2) = results
    log(f"largest batches: plain {b0}, grouped {b1}, persistent {b2}")
    assert b0 == 1 and b1 > 1 and b2 > 1
    assert np.array_equal(o0, o1) and np.array_equal(o0, o2)
    for k in s0:
        assert np.array_equal(s0[k], s1[k]) and np.array_equal(s0[k], s2[k])


def _ext_trace(seed, n):
    """Writes of stripes with the extended Q parity (p < k <= 2p-1, Section
    3.3) and degraded reads of them (one or two strips, at least one data
    strip, plain or extended)."""
    d = datagen.Draws(seed, datagen.TAG_ARRIVAL, 3)
    out, writes, t = [], [], 0.0
    for i in range(n):
        t += d.exponential(20000.0)
        if i < 8 or d.unit() < 0.5:
            p = (5, 11, 13, 29)[d.below(4)]
            k = d.between(p + 1, 2 * p - 1)
            w = 16 * d.between(1, 40)
            out.append(datagen.Request(i, t, "write", p, k, w, k * (p - 1) * w, -1, -1, -1))
            writes.append(i)
        else:
            tgt = writes[d.below(len(writes))]
            src = out[tgt]
            k = src.k
            e0 = d.below(k)
            e1 = -1
            if d.unit() < 0.5:
                e1 = d.below(k + 1)
                e1 += e1 >= e0
                e0, e1 = min(e0, e1), max(e0, e1)
            out.append(datagen.Request(i, t, "read", src.p, k, src.row_bytes, src.payload, e0, e1, tgt))
    return out


@pytest.mark.parametrize("mode", ["plain", "grouped", "persistent"])
def test_extended_q_parity_requests_match_oracle(mode):
    device()
    reqs = _ext_trace(36, 160)
    c, pay, out, out_off, data = _stage(reqs, 36)
    stripes = _expected_stripes(reqs, data)
    srv = r.raid6c_server_create(1 << 30, max_inflight=4, max_batch=16, plain=mode == "plain",
                                 persistent=mode == "persistent")
    try:
        comps = r.raid6c_server_replay(srv, c, [q.arrival_s for q in reqs])
        st = r.raid6c_server_get_stats(srv)
        log(f"extended, {mode}: {st.batches} batches for {st.completed} requests")
        _check(srv, reqs, comps, out, out_off, stripes)
    finally:
        r.raid6c_server_destroy(srv)


def test_small_budget_evicts_oldest_and_reports_not_resident():
    device()
    reqs = _trace(33, 200, qps=5000.0)
    c, pay, out, out_off, data = _stage(reqs, 33)
    stripes = _expected_stripes(reqs, data)
    srv = r.raid6c_server_create(8 << 20, max_inflight=2, max_batch=16)
    try:
        comps = r.raid6c_server_replay(srv, c, [q.arrival_s for q in reqs])
        st = r.raid6c_server_get_stats(srv)
        log(f"evictions {st.evictions}, resident {st.resident}, used {st.store_used}")
        assert st.evictions > 0 and st.store_used <= 8 << 20
        too_large = [q for q, x in zip(reqs, comps) if x.status == r.RAID6C_ST_TOO_LARGE]
        for q in too_large:
            assert (q.k + 2) * (q.p - 1) * q.row_bytes > 8 << 20
        ok_reqs = [(q, x) for q, x in zip(reqs, comps) if x.status != r.RAID6C_ST_TOO_LARGE]
        _check(srv, [q for q, _ in ok_reqs], [x for _, x in ok_reqs], out, out_off, stripes, allow_evicted=True)
    finally:
        r.raid6c_server_destroy(srv)


def test_bad_requests_complete_with_a_status():
    import torch
    device()
    srv = r.raid6c_server_create(1 << 24, max_inflight=2, max_batch=8)
    buf = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda:0")
    try:
        R = r.raid6c_request
        reqs = [
            R(r.RAID6C_REQ_READ, 0, 0, 0, 1, 0, 12345, None, buf.data_ptr(), 1),        # not resident
            R(r.RAID6C_REQ_WRITE, 9, 4, -1, -1, 64, 1, buf.data_ptr(), None, 2),        # not prime
            R(r.RAID6C_REQ_WRITE, 5, 4, -1, -1, 64, 7, buf.data_ptr(), None, 3),        # ok
            R(9, 5, 4, -1, -1, 64, 8, buf.data_ptr(), None, 4),                         # bad kind
        ]
        r.raid6c_server_submit(srv, reqs)
        r.raid6c_server_wait_idle(srv)
        r.raid6c_server_submit(srv, [R(r.RAID6C_REQ_WRITE, 5, 4, -1, -1, 64, 7, buf.data_ptr(), None, 5),
                                     R(r.RAID6C_REQ_READ, 0, 0, 2, 2, 0, 7, None, buf.data_ptr() + 4096, 6)])
        r.raid6c_server_wait_idle(srv)
        got = {c.tag: c.status for c in r.raid6c_server_poll(srv)}
        assert got == {1: r.RAID6C_ST_NOT_RESIDENT, 2: r.RAID6C_ST_INVALID, 3: r.RAID6C_ST_OK,
                       4: r.RAID6C_ST_INVALID, 5: r.RAID6C_ST_DUPLICATE, 6: r.RAID6C_ST_INVALID}
    finally:
        r.raid6c_server_destroy(srv)

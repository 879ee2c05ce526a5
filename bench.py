#!/usr/bin/env python3
"""Throughput of Z_p-RAID encode and two-erasure recovery on one MI355X.

Workload: p = 13, k = 12 data strips, rows of 4 KiB (48 KiB strips), 4096
stripes = 2.25 GiB of user data, uniform random bytes from the seeded
generators, resident in HBM before timing starts.  One step is the whole
hot path over that batch: one encode launch (P and Q of every stripe) and one
recovery launch in which every stripe rebuilds a pair of strips drawn
uniformly from its 91 pairs (two data strips, data + P, data + Q, or P + Q).
`value` is user bytes made whole per second: 2 x 2.25 GiB per step.

Also reported: per-kernel HIP-event timing and latency percentiles, the
roofline of the dominant kernel (HBM bound); recovery of each erasure class
at p = 29, k = 28, 1 KiB rows, 8192 stripes, each with its own roofline;
launch latency at p = 5, k = 4, 64-byte rows, 1024 stripes; the GF(256)
Reed-Solomon P+Q kernel on the same bytes, 20,000 mixed stripes in one plan
run against 20,000 plain launches, a served Poisson request stream against
per-request plain launches (a seeded sample of its results checked against
the oracle); and the CPU oracle timed on a bounded sample of the workload, on
every core and on one thread.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "encode & 2-erasure recovery GB/s user data; % HBM peak; p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
SEED = 2
P, K, W, NSTRIPES = 13, 12, 4096, 4096
# Cache-policy parameter of the kernels launched on this workload: its rows
# start on 128-byte lines, so the loads are non-temporal (policy 2).
LOAD_POLICY_STREAM = 2
KERNEL_SOURCES = ["paper_cs_0611109_amd/csrc/zp_core.hpp", "paper_cs_0611109_amd/csrc/zp_kernels.hip",
                  "paper_cs_0611109_amd/csrc/raid6c_internal.h"]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(vals, q):
    s = sorted(vals)
    if not s:
        return None
    i = min(len(s) - 1, max(0, int(round(q / 100.0 * (len(s) - 1)))))
    return s[i]


def source_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def lookup_traffic(kernel: str, cfg, bytes_per_launch: int, role: str = None):
    """Measured HBM bytes per launch of `kernel` (in `role`, where one kernel
    serves several) from the committed counter summaries, when they were
    taken on the current kernel source and launch configuration; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    e = table.get(kernel if role is None else f"{kernel} {role}")
    if not e or e.get("source_sha256") != source_digest() or tuple(e.get("config", ())) != tuple(cfg):
        return None
    if e.get("algorithmic_bytes") != bytes_per_launch:
        return None
    return e.get("hbm_bytes_per_launch")


def fill_batch(batch, seed, chunk=256):
    import numpy as np
    import torch

    import datagen
    p, k, w, n = batch.p, batch.k, batch.row_bytes, batch.nstripes
    host = torch.empty((chunk, k, p - 1, w), dtype=torch.uint8).pin_memory()
    for s0 in range(0, n, chunk):
        c = min(chunk, n - s0)
        datagen.fill_stripes(seed, s0, c, k, p, w, out=host.numpy()[:c])
        batch.tensor[s0:s0 + c, :k].copy_(host[:c], non_blocking=False)
    del np


def time_launches(fn, reps, stream):
    """HIP-event durations of `reps` calls of `fn` on `stream`, after one
    untimed call."""
    import torch
    fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def cpu_baseline(batch, er_host, seconds: float, parallel=None):
    """The CPU oracle (untuned, NumPy) on stripes of the same workload: one
    thread on successive stripes for about `seconds` (which also checks the
    GPU results on them), beside the parallel run over every core
    (`parallel`, from cpu_oracle_parallel, taken before the GPU was touched)."""
    import numpy as np

    import datagen
    from oracle import zp_raid as zp
    p, k, w = batch.p, batch.k, batch.row_bytes
    user = k * (p - 1) * w
    done, spent, verified = 0, 0.0, True
    while spent < seconds and done < batch.nstripes:
        data = datagen.stripe_data(SEED, done, k, p, w)
        e = tuple(int(v) for v in er_host[done])
        t0 = time.perf_counter()
        stripe = zp.encode_stripe(data, p)
        bad = stripe.copy()
        bad[list(e)] = 0
        rec = zp.recover(bad, p, e)
        spent += time.perf_counter() - t0
        got = batch.tensor[done].cpu().numpy()
        verified &= bool(np.array_equal(rec, stripe) and np.array_equal(got, stripe))
        done += 1
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    one = round(2 * user * done / spent / 1e9, 6)
    out = {
        "value": one,
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {done} stripes of the workload, encode + recovery of each stripe's pair, "
                  f"NumPy oracle on one thread, {spent:.1f} s",
        "one_thread_GBps": one,
        "host_cpus": len(os.sched_getaffinity(0)),
        "cpu_model": cpu_model,
        "gpu_results_match_oracle_on_sample": verified,
    }
    if parallel is not None:
        out["value"] = parallel["value"]
        out["cores"] = parallel["workers"]
        out["sample"] = (f"encode + recovery of each stripe's pair on the first {64 * parallel['workers']} "
                         f"stripes of the workload, NumPy oracle in {parallel['workers']} worker processes "
                         f"(one per core), {parallel['stripes']} stripes in {parallel['span_s']} s; "
                         f"one thread: {one} GB/s over the first {done} stripes ({spent:.1f} s)")
        out["parallel"] = parallel
    return out


def _oracle_worker(wid, nworkers, seconds, barrier, queue):
    """One worker of the parallel CPU-oracle run: generates its share of the
    workload's stripes (untimed), waits for the others, then runs the oracle's
    encode + recovery over them, round after round, for about `seconds`."""
    import datagen
    from oracle import zp_raid as zp
    er = datagen.erasures(SEED, NSTRIPES, K, "any")
    mine = list(range(wid, min(NSTRIPES, 64 * nworkers), nworkers))
    data = [(datagen.stripe_data(SEED, s, K, P, W), tuple(int(v) for v in er[s])) for s in mine]
    barrier.wait()
    t0 = time.time()
    done = 0
    while time.time() - t0 < seconds:
        for d, e in data:
            stripe = zp.encode_stripe(d, P)
            bad = stripe.copy()
            bad[list(e)] = 0
            zp.recover(bad, P, e)
            done += 1
    t1 = time.time()
    queue.put((done, t0, t1))


def cpu_oracle_parallel(seconds: float):
    """The CPU oracle on every core of this process's CPU set, at most 16 (the
    host share of one GPU), one worker process each, started before anything
    touches the GPU.  Each worker runs encode + recovery of its own stripes of
    the workload for about `seconds`; the rate is the user bytes of all
    workers over the span from the first start to the last end."""
    import multiprocessing as mp
    n = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")
    barrier, queue = ctx.Barrier(n), ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker, args=(i, n, seconds, barrier, queue)) for i in range(n)]
    for pr in procs:
        pr.start()
    got = [queue.get(timeout=600) for _ in procs]
    for pr in procs:
        pr.join()
    user = K * (P - 1) * W
    stripes = sum(g[0] for g in got)
    span = max(g[2] for g in got) - min(g[1] for g in got)
    return {"value": round(2 * user * stripes / span / 1e9, 6), "workers": n, "stripes": stripes,
            "span_s": round(span, 3)}


def extras(reps, stream):
    """Comparison and second-geometry measurements (not part of `value`)."""
    import torch

    import datagen
    import paper_cs_0611109_amd as r
    out = {}

    # GF(256) Reed-Solomon P+Q on the bytes of the main workload's geometry.
    b = r.StripeBatch.empty(P, K, W, NSTRIPES)
    b.tensor[:, :K].random_(0, 256)
    ms = time_launches(lambda: b.rs_encode(), reps, stream)
    mean = sum(ms) / len(ms)
    out["rs_gf256_encode"] = {
        "GBps_user": round(b.user_bytes / (mean / 1e3) / 1e9, 1),
        "hbm_frac": round((K + 2) * b.strip_stride * NSTRIPES / (mean / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
        "ms_p50": round(pct(ms, 50), 4), "ms_p99": round(pct(ms, 99), 4),
    }
    zp_ms = time_launches(lambda: b.encode(), reps, stream)
    out["zp_encode_same_bytes_ms_p50"] = round(pct(zp_ms, 50), 4)
    # Recovery by case, RS against Z_p on the same geometry (the shape of the
    # paper's DD / DP / PQ reconstruction table; timings do not depend on the
    # byte values).
    cmp_ = {}
    for kind in ("dd", "dp", "dq", "pq"):
        er = torch.from_numpy(datagen.erasures(2, NSTRIPES, K, kind)).to("cuda:0")
        rs_ms = time_launches(lambda: b.rs_recover(er), reps, stream)
        zp_ms = time_launches(lambda: b.recover(er), reps, stream)
        cmp_[kind] = {"rs_ms_p50": round(pct(rs_ms, 50), 4), "zp_ms_p50": round(pct(zp_ms, 50), 4),
                      "rs_GBps_user": round(b.user_bytes / (pct(rs_ms, 50) / 1e3) / 1e9, 1),
                      "zp_GBps_user": round(b.user_bytes / (pct(zp_ms, 50) / 1e3) / 1e9, 1)}
    cmp_["paper_p4_time_units"] = {"dd": {"rs": 2917, "z17": 2711}, "dp": {"rs": 2771, "z17": 1274},
                                   "pq": {"rs": 905, "z17": 809}}
    out["rs_vs_zp_recovery"] = cmp_
    del b
    torch.cuda.empty_cache()

    # The remaining figures are independent: one that fails is recorded as
    # such and the others are still measured.
    for name, fn in (("extended_q_parity", lambda: extended(reps, stream)),
                     ("small_write_update", lambda: small_writes(reps, stream)),
                     ("z17_horizontal_interop", lambda: z17_interop(reps, stream)),
                     ("batched_20000_mixed", lambda: batched_mixed(reps, stream)),
                     ("served_poisson", served_poisson),
                     ("served_sustained_saturation", served_sustained)):
        try:
            out[name] = fn()
        except Exception as e:  # noqa: BLE001 - reported in the JSON line
            log(f"{name} failed: {e}")
            out[name] = {"error": str(e)}
        torch.cuda.empty_cache()
    return out


P3, K3, W3, N3, SEED3 = 29, 28, 1024, 8192, 3
CONFIG3_ROLES = ("dd", "dp", "dq", "encode")


def config3(reps, stream):
    """Recovery at p = 29, k = 28, 1 KiB rows, 8192 stripes (6.125 GiB of user
    data): per-stripe pairs of one class per launch (dd: two data strips
    uniform over the 378 pairs; dp / dq: a data strip uniform over the 28,
    plus P / Q), and the encode of the same stripes.  Per role: user GB/s,
    fraction of HBM peak over the algorithmic bytes, and a roofline object
    (HIP-event mean launch duration; HBM bytes from the committed counter
    summary when it was taken on the current kernel sources)."""
    import torch

    import datagen
    import paper_cs_0611109_amd as r
    b = r.StripeBatch.empty(P3, K3, W3, N3)
    b.tensor[:, :K3].random_(0, 256)
    b.encode()
    alg = (K3 + 2) * b.strip_stride * N3
    res = {"workload": f"Z_p-RAID recovery, p={P3} k={K3} W={W3} B x {N3} stripes, one erasure class per launch",
           "user_bytes_per_launch": b.user_bytes, "algorithmic_bytes_per_launch": alg}
    bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    for role in CONFIG3_ROLES:
        if role == "encode":
            ms = time_launches(lambda: b.encode(), reps, stream)
            op = 0
        else:
            er = torch.from_numpy(datagen.erasures(SEED3, N3, K3, role)).to("cuda:0")
            ms = time_launches(lambda: b.recover(er, bad), reps, stream)
            op = 1
        mean = sum(ms) / len(ms)
        vec, unroll, threads, split, order = r.raid6c_tune_get(P3, op, W3)
        kname = _kernel_name(P3, op, vec, unroll, split)
        achieved = alg / (mean / 1e3) / 1e9
        res[role] = {
            "GBps_user": round(b.user_bytes / (mean / 1e3) / 1e9, 1),
            "hbm_frac": round(achieved / HBM_PEAK_GBPS, 4),
            "ms_p50": round(pct(ms, 50), 4), "ms_p99": round(pct(ms, 99), 4),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBPS, 4),
                         "traffic": lookup_traffic(kname, (vec, unroll, threads, split, order), alg, role),
                         "kernel": kname, "avg_launch_ms": round(mean, 4),
                         "launch": {"vec": vec, "unroll": unroll, "threads": threads, "split": split,
                                    "order": order}},
        }
    torch.cuda.synchronize()
    if int(bad.item()) != 0:
        raise RuntimeError("p = 29 recovery rejected erasure entries")
    del b
    torch.cuda.empty_cache()
    return res


def _kernel_name(p, op, vec, unroll, split, ext=False):
    """Name (as the profiler shows it) of the strided Z_p kernel a launch
    configuration selects, for rows on 128-byte lines."""
    e = "true" if ext else "false"
    if split > 1:
        return f"zp_split_kernel<{p},{vec},{unroll},{split},{e},{LOAD_POLICY_STREAM}>"
    kind = "encode" if op in (0, 2) else "recover"
    return f"zp_{kind}_kernel<{p},{vec},{unroll},{e},{LOAD_POLICY_STREAM}>"


def config1_latency(reps, stream):
    """p = 5, k = 4, W = 64 B, 1024 stripes (1 MiB of user data: cache-resident,
    launch-bound): per-launch latency of the encode and of the recovery of each
    of the 15 strip pairs among the 6 strips (the same pair on every stripe).
    kernel_ms: HIP events around the launch on its stream; call_ms: host time
    from the call to the end of a stream synchronize."""
    import torch

    import paper_cs_0611109_amd as r
    b = r.StripeBatch.empty(5, 4, 64, 1024)
    b.tensor[:, :4].random_(0, 256)
    b.encode()
    ops = [("encode", None)] + [(f"{a},{c}", (a, c)) for a in range(6) for c in range(a + 1, 6)]
    per, allk, allc = {}, [], []
    for name, pair in ops:
        if pair is None:
            fn = b.encode
        else:
            er = torch.tensor([pair] * 1024, dtype=torch.int32, device="cuda:0")
            fn = (lambda er=er: b.recover(er))
        kms = time_launches(fn, reps, stream)
        cms = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            stream.synchronize()
            cms.append((time.perf_counter() - t0) * 1e3)
        allk += kms
        allc += cms
        per[name] = {"kernel_ms_p50": round(pct(kms, 50), 4), "kernel_ms_p99": round(pct(kms, 99), 4),
                     "call_ms_p50": round(pct(cms, 50), 4), "call_ms_p99": round(pct(cms, 99), 4)}
    del b
    return {"workload": "p=5 k=4 W=64 B x 1024 stripes; encode + each of the 15 pairs", "launches_per_op": reps,
            "kernel_ms_p50": round(pct(allk, 50), 4), "kernel_ms_p99": round(pct(allk, 99), 4),
            "call_ms_p50": round(pct(allc, 50), 4), "call_ms_p99": round(pct(allc, 99), 4), "by_op": per}


def extended(reps, stream):
    """Extended Q parity (Section 3.3, k = 2p-1 data strips): encode, and
    recovery of a pair uniform over all pairs and of each class that the
    plain code does not have (plain + extended data, which takes the
    trinomial inverse; two extended data strips; extended data + P / Q).
    Bytes moved per launch (k+2)(p-1)W per stripe, as for the plain code."""
    import torch

    import datagen
    import paper_cs_0611109_amd as r
    out = {}
    for p, w, n in ((13, 4096, 2048), (29, 1024, 4096)):
        k = 2 * p - 1
        b = r.StripeBatch.empty(p, k, w, n)
        b.tensor[:, :k].random_(0, 256)
        moved = (k + 2) * b.strip_stride * n

        def entry(ms):
            mean = sum(ms) / len(ms)
            return {"GBps_user": round(b.user_bytes / (mean / 1e3) / 1e9, 1),
                    "hbm_frac": round(moved / (mean / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                    "ms_p50": round(pct(ms, 50), 4)}

        res = {"encode": entry(time_launches(lambda: b.encode(), reps, stream))}
        kinds = [("any", datagen.erasures(6, n, k, "any"))]
        kinds += [(kd, datagen.erasures_extended(6, n, k, p, kd)) for kd in datagen.EXTENDED_ERASURE_KINDS]
        for kd, er_host in kinds:
            er = torch.from_numpy(er_host).to("cuda:0")
            res[kd] = entry(time_launches(lambda: b.recover(er), reps, stream))
        out[f"p{p}_k{k}_w{w}_x{n}"] = res
        del b
        torch.cuda.empty_cache()
    return out


def small_writes(reps, stream):
    """One data strip per stripe replaced, P and Q updated from the change
    (7 strips moved per stripe), on the main workload's geometry; against a
    re-encode of the whole batch ((k+2) strips per stripe)."""
    import torch

    import datagen
    import paper_cs_0611109_amd as r
    b = r.StripeBatch.empty(P, K, W, NSTRIPES)
    b.tensor.random_(0, 256)
    src = torch.empty((NSTRIPES, P - 1, W), dtype=torch.uint8, device="cuda:0")
    src.random_(0, 256)
    d = datagen.Draws(7, datagen.TAG_ERASURE, 99)
    targets = torch.tensor([d.below(K) for _ in range(NSTRIPES)], dtype=torch.int32, device="cuda:0")
    ms = time_launches(lambda: b.update(targets, src), reps, stream)
    enc = time_launches(lambda: b.encode(), reps, stream)
    mean, emean = sum(ms) / len(ms), sum(enc) / len(enc)
    moved = 7 * b.strip_stride * NSTRIPES
    out = {"stripes": NSTRIPES, "new_bytes": b.strip_stride * NSTRIPES,
           "GBps_new_data": round(b.strip_stride * NSTRIPES / (mean / 1e3) / 1e9, 1),
           "hbm_frac": round(moved / (mean / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
           "ms_p50": round(pct(ms, 50), 4), "reencode_ms_p50": round(pct(enc, 50), 4),
           "speedup_vs_reencode": round(emean / mean, 3)}
    del b, src
    torch.cuda.empty_cache()
    return out


def z17_interop(reps, stream):
    """Conversion between the paper's horizontal Z_17 layout (one codeword per
    int16) and vertical strips: 2 GiB of strips each way; bytes moved = read
    + written."""
    import torch

    import paper_cs_0611109_amd as r
    w, count = 4096, 16384                         # 16384 strips of 64 KiB
    h = torch.empty((count, 8 * w), dtype=torch.int16, device="cuda:0")
    h.random_(-32768, 32767)
    v = torch.empty((count, 16, w), dtype=torch.uint8, device="cuda:0")
    moved = 2 * 16 * w * count
    to_v = time_launches(lambda: r.raid6c_z17_to_vertical(h, w, count, v), reps, stream)
    to_h = time_launches(lambda: r.raid6c_z17_to_horizontal(v, w, count, h), reps, stream)
    out = {}
    for name, ms in (("to_vertical", to_v), ("to_horizontal", to_h)):
        mean = sum(ms) / len(ms)
        out[name] = {"GBps_moved": round(moved / (mean / 1e3) / 1e9, 1),
                     "hbm_frac": round(moved / (mean / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                     "ms_p50": round(pct(ms, 50), 4)}
    del h, v
    torch.cuda.empty_cache()
    return out


def _stage_served(reqs):
    """Device buffers for a request stream (payloads of random bytes, outputs
    of the reads) and the C request array that points into them."""
    import torch

    import paper_cs_0611109_amd as r
    pay_off, out_off, pp, po = {}, {}, 0, 0
    for q in reqs:
        strip = (q.p - 1) * q.row_bytes
        if q.kind == "write":
            pay_off[q.index] = pp
            pp += q.k * strip
        else:
            out_off[q.index] = po
            po += 2 * strip
    pay = torch.empty(pp, dtype=torch.uint8, device="cuda:0")
    pay.random_(0, 256)
    outb = torch.empty(max(po, 16), dtype=torch.uint8, device="cuda:0")
    creq = []
    for q in reqs:
        if q.kind == "write":
            creq.append(r.raid6c_request(r.RAID6C_REQ_WRITE, q.p, q.k, -1, -1, q.row_bytes, q.index,
                                         pay.data_ptr() + pay_off[q.index], None, q.index))
        else:
            creq.append(r.raid6c_request(r.RAID6C_REQ_READ, 0, 0, q.e0, q.e1, 0, q.target, None,
                                         outb.data_ptr() + out_off[q.index], q.index))
    arr = (r.raid6c_request * len(reqs))(*creq)
    torch.cuda.synchronize()
    return arr, pay, outb, pay_off, out_off


def served_sustained(n=16000, seed=6):
    """The served path's sustained rate: a burst of n requests of the same
    stream recipe, all due at t = 0, into a 16 GiB store (the resident
    stripes take about 6.5 GB, so nothing is evicted), three runs after an
    untimed warm-up.  A 4000-request burst lasts about 1.4 ms, much of it
    filling and draining the slots; this one lasts about 4.5 ms."""
    import torch

    import datagen
    import paper_cs_0611109_amd as r
    reqs = datagen.serve_requests(seed, n, qps=1.0)
    arr, pay, outb, _, _ = _stage_served(reqs)
    # Untimed warm-up (the first launch of each kernel in a process loads it).
    srv = r.raid6c_server_create(16 << 30, max_inflight=SERVE_INFLIGHT, max_batch=SERVE_MAX_BATCH)
    try:
        r.raid6c_server_replay(srv, arr[:400], [0.0] * 400)
    finally:
        r.raid6c_server_destroy(srv)
    runs = []
    for _ in range(3):
        srv = r.raid6c_server_create(16 << 30, max_inflight=SERVE_INFLIGHT, max_batch=SERVE_MAX_BATCH)
        try:
            comps = r.raid6c_server_replay(srv, arr, [0.0] * n)
            st = r.raid6c_server_get_stats(srv)
        finally:
            r.raid6c_server_destroy(srv)
        span = (max(c.complete_ns for c in comps) - min(c.arrival_ns for c in comps)) / 1e9
        runs.append({"GBps_user": round(st.user_bytes / span / 1e9, 1), "requests_per_s": round(n / span, 1),
                     "span_ms": round(span * 1e3, 3), "batches": st.batches,
                     "failed": sum(c.status != r.RAID6C_ST_OK for c in comps),
                     "host_admit_ns_per_request": round(st.admit_ns / max(1, st.completed), 1),
                     "host_launch_us_per_batch": round(st.launch_ns / 1e3 / max(1, st.batches), 1)})
    del pay, outb
    torch.cuda.empty_cache()
    best = max(runs, key=lambda x: x["GBps_user"])
    return {"requests": n, "writes": sum(q.kind == "write" for q in reqs), "runs": runs,
            "GBps_user_median": sorted(x["GBps_user"] for x in runs)[1], "best": best}


def served_poisson(n=4000, seed=5):
    """Open-loop Poisson stream of writes (60%) and degraded reads (40%, one or
    two erased strips) on p in {11,13,29,37}, k = p-1, payloads log-uniform over
    4 KiB..4 MiB, pre-staged in device memory, 8 GiB stripe store (the
    resident stripes take about 1.8 GB).  First the
    saturation rate R of the per-request plain path (all requests at t=0), then
    both paths at 0.8 R: p50/p99 latency (completion - scheduled arrival) and
    user GB/s."""
    import torch

    import datagen
    import paper_cs_0611109_amd as r
    reqs = datagen.serve_requests(seed, n, qps=1.0)
    arr, pay, outb, pay_off, out_off = _stage_served(reqs)
    base_t = [q.arrival_s for q in reqs]
    # A seeded sample of requests whose results are copied to the host after
    # every run, for the oracle check of the CPU-baseline leg; the payloads
    # they depend on too.
    d = datagen.Draws(seed, datagen.TAG_POISON, 7)
    sample = sorted({d.below(n) for _ in range(SERVE_SAMPLE)})
    need = {i if reqs[i].kind == "write" else reqs[i].target for i in sample}
    payloads = {}
    for i in need:
        q = reqs[i]
        nb = q.k * (q.p - 1) * q.row_bytes
        payloads[i] = pay[pay_off[i]:pay_off[i] + nb].cpu().numpy().reshape(q.k, q.p - 1, q.row_bytes)
    _SERVED_SAMPLES.clear()

    def grab(name, srv, comps):
        got = []
        for i in sample:
            q = reqs[i]
            if comps[i].status != r.RAID6C_ST_OK:
                got.append((i, None))
                continue
            strip = (q.p - 1) * q.row_bytes
            if q.kind == "write":
                base, stride = r.raid6c_server_stripe(srv, i)
                got.append((i, _device_bytes(base, (q.k + 2) * stride)))
            else:
                ne = 2 if q.e1 >= 0 else 1
                got.append((i, outb[out_off[i]:out_off[i] + ne * strip].cpu().numpy()))
        _SERVED_SAMPLES.append((name, got))

    def run(plain, times, name):
        srv = r.raid6c_server_create(8 << 30, max_inflight=SERVE_INFLIGHT, max_batch=SERVE_MAX_BATCH, plain=plain)
        try:
            comps = r.raid6c_server_replay(srv, arr, times)
            st = r.raid6c_server_get_stats(srv)
            if name is not None:
                grab(name, srv, comps)
        finally:
            r.raid6c_server_destroy(srv)
        bad = sum(c.status != r.RAID6C_ST_OK for c in comps)
        lat = [(c.complete_ns - c.arrival_ns) / 1e6 for c in comps]
        span = (max(c.complete_ns for c in comps) - min(c.arrival_ns for c in comps)) / 1e9
        return {"p50_ms": round(pct(lat, 50), 4), "p99_ms": round(pct(lat, 99), 4),
                "GBps_user": round(st.user_bytes / span / 1e9, 1), "requests_per_s": round(n / span, 1),
                "batches": st.batches, "failed": bad,
                "host_admit_ns_per_request": round(st.admit_ns / max(1, st.completed), 1),
                "host_launch_us_per_batch": round(st.launch_ns / 1e3 / max(1, st.batches), 1)}

    zero = [0.0] * n
    # Untimed warm-up of both paths (the first launch of each kernel loads it).
    for plain in (True, False):
        for times in (zero, [t / 50000.0 for t in base_t[:400]]):
            srv = r.raid6c_server_create(8 << 30, max_inflight=SERVE_INFLIGHT, max_batch=SERVE_MAX_BATCH, plain=plain)
            try:
                r.raid6c_server_replay(srv, arr[:len(times)], times)
            finally:
                r.raid6c_server_destroy(srv)
    sat_plain = run(True, zero, "saturation_plain")
    sat_served = run(False, zero, "saturation_served")
    rate = 0.8 * sat_plain["requests_per_s"]
    times = [t / rate for t in base_t]
    high = 4.0 * sat_plain["requests_per_s"]
    _SERVED_SAMPLES.append(("payloads", (reqs, payloads)))
    out = {"requests": n, "writes": sum(q.kind == "write" for q in reqs),
           "saturation_plain": sat_plain, "saturation_served": sat_served,
           "qps": round(rate, 1), "served_at_qps": run(False, times, "served_at_qps"),
           "plain_at_qps": run(True, times, "plain_at_qps"),
           "qps_4x_plain_saturation": round(high, 1),
           "served_at_4x": run(False, [t / high for t in base_t], "served_at_4x"),
           "verified_against_oracle": None}
    # Latency against load, from the plain path's saturation rate R up to
    # the served path's own saturation (about 60 R).
    sweep = []
    for mult in SERVE_SWEEP:
        q_ = mult * sat_plain["requests_per_s"]
        res = run(False, [t / q_ for t in base_t], None)
        sweep.append({"x_plain_saturation": mult, "qps": round(q_, 1),
                      **{k: res[k] for k in ("p50_ms", "p99_ms", "GBps_user", "requests_per_s", "batches",
                                             "failed")}})
    out["sweep"] = sweep
    return out


# Server configuration of the served runs: one slot per hardware queue of
# the process (4), up to 1024 requests per batch (at 0.8 R batches hold one
# or two requests; a backlog is taken in large batches).
SERVE_INFLIGHT, SERVE_MAX_BATCH = 4, 1024
# Offered loads of the served sweep, in multiples of the plain path's
# saturation rate.
SERVE_SWEEP = (1, 2, 8, 16, 32, 64)

# (run name, [(request index, host bytes or None)]) of the last served_poisson
# call, and ("payloads", (requests, {write index: data strips})).
_SERVED_SAMPLES = []
SERVE_SAMPLE = 32


def _device_bytes(addr, n):
    """n bytes at a raw device address (inside the server's store), on the host."""
    import ctypes

    import numpy as np
    import torch
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    out = np.empty(n, dtype=np.uint8)
    torch.cuda.synchronize()
    if hip.hipMemcpy(out.ctypes.data, ctypes.c_void_p(addr), n, 2) != 0:   # device to host
        raise RuntimeError("hipMemcpy from the stripe store failed")
    return out


def verify_served_samples():
    """Oracle check of the served_poisson sample (part of the CPU-baseline
    leg): every sampled write's stored stripe equals the oracle's encode of
    its payload, and every sampled degraded read's rebuilt strips equal the
    oracle's strips of the stripe it read."""
    import numpy as np

    from oracle import zp_raid as zp
    runs = [x for x in _SERVED_SAMPLES if x[0] != "payloads"]
    pl = [x[1] for x in _SERVED_SAMPLES if x[0] == "payloads"]
    if not runs or not pl:
        return None
    reqs, payloads = pl[0]
    want = {i: zp.encode_stripe(d, reqs[i].p) for i, d in payloads.items()}
    checked, bad, skipped = 0, [], 0
    for name, got in runs:
        for i, buf in got:
            q = reqs[i]
            if buf is None:
                skipped += 1
                continue
            if q.kind == "write":
                ok = np.array_equal(buf.reshape(want[i].shape), want[i])
            else:
                w = want[q.target]
                es = sorted(e for e in (q.e0, q.e1) if e >= 0)
                ok = np.array_equal(buf.reshape(len(es), q.p - 1, q.row_bytes), w[es])
            checked += 1
            if not ok:
                bad.append((name, i))
    return {"checked": checked, "not_completed_ok": skipped, "mismatches": len(bad), "match": not bad and skipped == 0,
            "sample": f"{SERVE_SAMPLE} seeded request draws per run, {len(runs)} runs; writes: the stored stripe "
                      "(data + P + Q), reads: the rebuilt strips"}


def batched_mixed(reps, stream):
    """20,000 stripes of mixed geometry (p from {5,11,13,19,29,37,53}, k
    uniform in [2, p-1], rows log-uniform over 512 B..64 KiB; 60% encode, 40%
    two-erasure recovery): one plan run (a HIP graph: one job-list grid per
    prime, or one persistent kernel, whichever the autotuner picks) against
    the same jobs as 20,000 plain launches on one stream."""
    import torch

    import datagen
    import paper_cs_0611109_amd as r
    jobs = datagen.batch_jobs(4, 20000)
    offs, pos = [], 0
    for j in jobs:
        offs.append(pos)
        pos += (j.k + 2) * (j.p - 1) * j.row_bytes
    buf = torch.empty(pos, dtype=torch.uint8, device="cuda:0")
    buf.random_(0, 256)
    base = buf.data_ptr()
    cj = []
    for j, off in zip(jobs, offs):
        strip = (j.p - 1) * j.row_bytes
        op = r.RAID6C_JOB_ENCODE if j.op == "encode" else r.RAID6C_JOB_RECOVER
        cj.append(r.raid6c_job(op, j.p, j.k, j.e0, j.e1, j.row_bytes, strip, base + off))
    arr = (r.raid6c_job * len(cj))(*cj)
    plan = r.raid6c_plan_create(arr)
    try:
        info = r.raid6c_plan_stats(plan)
        tuned_ms = r.raid6c_plan_autotune(plan, reps=2)
        sched = r.raid6c_plan_get_schedule(plan)
        plan_ms = time_launches(lambda: r.raid6c_plan_run(plan), reps, stream)
        # Both execution modes on their own, for the record (the persistent
        # kernel with 8 single-wave work-groups per CU, one item per pop).
        modes = {}
        for name, cand in (("grouped_chained", (8, 4, 0, 2)), ("grouped_side_by_side", (8, 4, 0, 1)),
                           ("persistent", (8, 1, 0, 0))):
            r.raid6c_plan_set_schedule(plan, *cand)
            ms_m = time_launches(lambda: r.raid6c_plan_run(plan), max(3, reps // 2), stream)
            modes[name] = round(sum(ms_m) / len(ms_m), 3)
        r.raid6c_plan_set_schedule(plan, sched.waves_per_cu, sched.chunk, sched.order, sched.grouped)
        plain_ms = time_launches(lambda: r.raid6c_run_jobs(arr), max(3, reps // 5), stream)
    finally:
        r.raid6c_plan_destroy(plan)
    del buf
    torch.cuda.empty_cache()
    pm = sum(plan_ms) / len(plan_ms)
    qm = sum(plain_ms) / len(plain_ms)
    return {
        "stripes": len(jobs), "bytes_moved": info.bytes_moved, "user_bytes": info.user_bytes,
        "work_items": info.nitems,
        "plan_ms_mean": round(pm, 3), "plan_ms_p50": round(pct(plan_ms, 50), 3),
        "plan_ms_p99": round(pct(plan_ms, 99), 3),
        "plan_GBps_user": round(info.user_bytes / (pm / 1e3) / 1e9, 1),
        "plan_hbm_frac": round(info.bytes_moved / (pm / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
        "plain_launches_ms_mean": round(qm, 3),
        "plain_GBps_user": round(info.user_bytes / (qm / 1e3) / 1e9, 1),
        "speedup_vs_plain": round(qm / pm, 3),
        "schedule": {"waves_per_cu": sched.waves_per_cu, "chunk": sched.chunk, "order": sched.order,
                     "grouped": sched.grouped},
        "autotune_best_ms": round(tuned_ms, 3),
        "mode_ms_mean": modes,
    }


def copy_ceiling(stream, nbytes=2 << 30, reps=10):
    """The bandwidth a plain device-to-device copy reaches (the runtime's own
    copy kernel, read and write 1:1), as context for the roofline: the Z_p
    kernels read 6 to 14 bytes per byte written."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    a.random_(0, 256)
    b = torch.empty_like(a)
    ms = time_launches(lambda: b.copy_(a), reps, stream)
    med = pct(ms, 50)
    del a, b
    torch.cuda.empty_cache()
    moved = 2 * nbytes
    return {"kind": "device-to-device copy, 2 GiB each way", "ms_p50": round(med, 4),
            "GBps_moved": round(moved / (med / 1e3) / 1e9, 1),
            "frac_of_peak": round(moved / (med / 1e3) / 1e9 / HBM_PEAK_GBPS, 4)}


def copy_probe(stream, nbytes=1 << 30, reps=3):
    """Plain device copies of a known size (to scale HBM byte counters)."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    a.random_(0, 256)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# rocprofv3 summaries.  The three runs below (from the repository root, on one
# MI355X) produce the CSV folders that --summarize turns into the committed
# text summaries and the traffic table read by lookup_traffic().
PROFILE_CMDS = {
    "stats": "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_stats -o run -- "
             "python -u bench.py --steps 10 --warmup 2 --no-cpu-baseline --no-extras",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof_fetch -o run -- "
             "python -u bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-extras --copy-probe",
    "write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof_write -o run -- "
             "python -u bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-extras --copy-probe",
}
WORKLOAD_TAG = f"zp_p{P}_k{K}_w{W}_x{NSTRIPES}"
# The plan workload (20,000 mixed stripes) profiled on its own: the job-list
# kernel of each prime, grouped schedule.
PLAN_PROFILE_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_plan -o run -- "
                    "python -u bench.py --plan-profile 10")
PLAN_SEED, PLAN_STRIPES = 4, 20000
# Rows on 128-byte lines against rows 16 bytes past them: strided encode at
# p = 53, k = 26 (tuned configuration of the row-size bucket), HBM byte counters.
ROWS_PROBE = ((2048, 503), (2064, 499), (13312, 77), (13328, 77))   # (row bytes, stripes)
ROWS_PROBE_CMDS = {c: f"rocprofv3 --pmc {c} --output-format csv -d gpurun_out/prof_rows_{c.split('_')[0].lower()} "
                      "-o run -- python -u bench.py --rows-probe" for c in ("FETCH_SIZE", "WRITE_SIZE")}


PLAN_PMC_CMDS = {c: f"rocprofv3 --pmc {c} --output-format csv -d gpurun_out/prof_plan_{c.split('_')[0].lower()} "
                    "-o run -- python -u bench.py --plan-profile 3 --copy-probe" for c in ("FETCH_SIZE", "WRITE_SIZE")}


def plan_jobs_bytes(split=False):
    """Per prime: the algorithmic bytes (k+2)(p-1)W of the plan workload; with
    `split`, (read, written) = (k(p-1)W, 2(p-1)W) per prime (an encode reads
    the k data strips and writes P, Q; a two-erasure recovery reads the k
    surviving strips and writes the 2 erased ones)."""
    import datagen
    out = {}
    for j in datagen.batch_jobs(PLAN_SEED, PLAN_STRIPES):
        strip = (j.p - 1) * j.row_bytes
        if split:
            rd, wr = out.get(j.p, (0, 0))
            out[j.p] = (rd + j.k * strip, wr + 2 * strip)
        else:
            out[j.p] = out.get(j.p, 0) + (j.k + 2) * strip
    return out


def summarize_plan_counters(fetch_dir: str, write_dir: str, out_dir: str = None) -> dict:
    """HBM bytes per run of each prime's job-list grid in the PLAN_PMC_CMDS runs
    against the bytes its jobs read and write (host-only)."""
    import re
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    alg = plan_jobs_bytes(split=True)

    def read(d, counter):
        per, copies = {}, []
        for r_ in _read_csv(os.path.join(d, "run_counter_collection.csv")):
            if r_["Counter_Name"] != counter:
                continue
            v = float(r_["Counter_Value"])
            if "copyBuffer" in r_["Kernel_Name"]:
                if v > 100000:
                    copies.append(v)
                continue
            m = re.search(r"zp_group_kernel<(\d+)>", r_["Kernel_Name"])
            if m:
                per.setdefault(int(m.group(1)), []).append((int(r_["Dispatch_Id"]), v))
        if not copies or set(per) != set(alg):
            raise RuntimeError(f"{d}: expected the grids of primes {sorted(alg)} and the probe copies")
        scale = 2**30 / (sum(copies) / len(copies) * 1024)
        # the first run warms up; average the others
        return {p: sum(v for _, v in sorted(x)[1:]) / max(1, len(x) - 1) * 1024 * scale for p, x in per.items()}, scale

    fetch, fs = read(fetch_dir, "FETCH_SIZE")
    write, ws = read(write_dir, "WRITE_SIZE")
    lines = ["# rocprofv3 HBM byte counters: plan of 20,000 mixed stripes (p from {5,11,13,19,29,37,53},",
             "# k uniform in [2, p-1], rows log-uniform over 512 B..64 KiB rounded to 16 B, 60% encode / 40%",
             "# two-erasure recovery; 7 in 8 jobs have rows off 128-byte lines), default schedule",
             "# commands (one counter per run, from the repository root, on one MI355X):",
             "#   " + PLAN_PMC_CMDS["FETCH_SIZE"], "#   " + PLAN_PMC_CMDS["WRITE_SIZE"],
             f"# counters scaled by 1 GiB probe copies in the same runs: fetch x{fs:.4f}, write x{ws:.4f};",
             "# per prime: the mean over the runs after the first; read / written = the bytes the jobs must",
             "# read (k surviving or data strips) and write (2 strips)", "",
             f"{'grid':<22}{'read_B':>14}{'fetched_B':>14}{'fetch/read':>11}{'written_B':>13}{'wrote_B':>13}{'ratio':>8}"]
    table = {}
    trd = twr = tf = tw = 0
    for p in sorted(alg, reverse=True):
        rd, wr = alg[p]
        f, w = fetch[p], write[p]
        trd, twr, tf, tw = trd + rd, twr + wr, tf + f, tw + w
        lines.append(f"{'zp_group_kernel<%d>' % p:<22}{rd:>14}{f:>14.0f}{f / rd:>11.4f}{wr:>13}{w:>13.0f}{w / wr:>8.4f}")
        table[p] = {"fetch_over_read": round(f / rd, 4), "write_over_written": round(w / wr, 4)}
    lines.append(f"{'all':<22}{trd:>14}{tf:>14.0f}{tf / trd:>11.4f}{twr:>13}{tw:>13.0f}{tw / twr:>8.4f}")
    lines.append(f"\nHBM bytes per run: {tf + tw:.0f} against {trd + twr} algorithmic ({(tf + tw) / (trd + twr):.4f}x)")
    table["all"] = {"fetch_over_read": round(tf / trd, 4), "write_over_written": round(tw / twr, 4),
                    "hbm_over_algorithmic": round((tf + tw) / (trd + twr), 4)}
    with open(os.path.join(out_dir, "zp_group_kernel_plan_mixed_x20000_hbm_bytes.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return table


def plan_profile(runs):
    """Run the 20,000-stripe plan `runs` times under the default schedule
    (per-prime job-list grids one after another; nothing else is launched but
    the input fill), for the profiler."""
    import torch

    import datagen
    import paper_cs_0611109_amd as r
    jobs = datagen.batch_jobs(PLAN_SEED, PLAN_STRIPES)
    offs, pos = [], 0
    for j in jobs:
        offs.append(pos)
        pos += (j.k + 2) * (j.p - 1) * j.row_bytes
    buf = torch.empty(pos, dtype=torch.uint8, device="cuda:0")
    buf.random_(0, 256)
    base = buf.data_ptr()
    cj = []
    for j, off in zip(jobs, offs):
        op = r.RAID6C_JOB_ENCODE if j.op == "encode" else r.RAID6C_JOB_RECOVER
        cj.append(r.raid6c_job(op, j.p, j.k, j.e0, j.e1, j.row_bytes, (j.p - 1) * j.row_bytes, base + off))
    plan = r.raid6c_plan_create((r.raid6c_job * len(cj))(*cj))
    try:
        r.raid6c_plan_set_schedule(plan, 8, 4, 0, 2)
        ms = time_launches(lambda: r.raid6c_plan_run(plan), runs, torch.cuda.current_stream())
    finally:
        r.raid6c_plan_destroy(plan)
    return {"plan_runs": runs, "plan_ms_mean": round(sum(ms) / len(ms), 3)}


SERVE_PROFILE_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_serve -o run -- "
                     "python -u bench.py --serve-profile 3")


def serve_profile(runs):
    """The served stream's 4000 requests, all due at t = 0, replayed `runs`
    times into a fresh server each (after one untimed warm-up replay), for
    the profiler: the saturated case, where batches overlap most."""
    import time

    import datagen
    import paper_cs_0611109_amd as r
    reqs = datagen.serve_requests(5, 4000, qps=1.0)
    arr, pay, outb, _, _ = _stage_served(reqs)
    out = []
    for i in range(runs + 1):
        srv = r.raid6c_server_create(8 << 30, max_inflight=SERVE_INFLIGHT, max_batch=SERVE_MAX_BATCH)
        try:
            comps = r.raid6c_server_replay(srv, arr, [0.0] * len(reqs))
            st = r.raid6c_server_get_stats(srv)
        finally:
            r.raid6c_server_destroy(srv)
        span = (max(c.complete_ns for c in comps) - min(c.arrival_ns for c in comps)) / 1e9
        if i > 0:
            out.append({"GBps_user": round(st.user_bytes / span / 1e9, 1), "batches": st.batches,
                        "failed": sum(c.status != r.RAID6C_ST_OK for c in comps)})
        time.sleep(0.02)   # a gap that separates the runs in the trace
    del pay, outb
    return {"serve_runs": out, "user_bytes_per_run": sum(q.k * (q.p - 1) * q.row_bytes for q in reqs)}


def summarize_serve_profile(stats_dir: str, out_dir: str = None) -> dict:
    """Summary of a SERVE_PROFILE_CMD run (host-only): per run, the span
    from the first grid's start to the last grid's end, the time the GPU had
    a grid running, and per kernel the grids and their mean duration."""
    import re
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    import datagen
    reqs = datagen.serve_requests(5, 4000, qps=1.0)
    user = sum(q.k * (q.p - 1) * q.row_bytes for q in reqs)
    rows = [t for t in _read_csv(os.path.join(stats_dir, "run_kernel_trace.csv")) if "zp_" in t["Kernel_Name"]]
    rows.sort(key=lambda t: int(t["Start_Timestamp"]))
    runs = [[rows[0]]]
    for a, b in zip(rows, rows[1:]):
        if int(b["Start_Timestamp"]) - int(a["End_Timestamp"]) > 3_000_000:
            runs.append([])
        runs[-1].append(b)
    runs = runs[1:]                    # the first is the warm-up replay
    if not runs:
        raise RuntimeError(f"{stats_dir}: no timed replay found after the warm-up")

    def name(k):
        m = re.search(r"(zp_\w+_kernel)(<(\d+)>)?", k)
        return m.group(1) + (f"<{m.group(3)}>" if m.group(3) else "")

    lines = ["# rocprofv3 kernel trace: served stream, 4000 requests (60% writes, 40% degraded reads; p from "
             "{11,13,29,37}, k = p-1,",
             "# payloads log-uniform over 4 KiB..4 MiB) all due at t = 0 (saturation), 4 slots, up to 1024 "
             "requests per batch",
             "# command (from the repository root, on one MI355X):", "#   " + SERVE_PROFILE_CMD,
             "# source: run_kernel_trace.csv; runs separated by idle gaps; the first (warm-up) run is left out",
             f"# user data per run: {user} B", ""]
    res = {"runs": []}
    per_kernel = {}
    for i, run in enumerate(runs):
        t0 = min(int(t["Start_Timestamp"]) for t in run)
        t1 = max(int(t["End_Timestamp"]) for t in run)
        busy, cur = 0, None
        for t in sorted(run, key=lambda t: int(t["Start_Timestamp"])):
            s_, e_ = int(t["Start_Timestamp"]), int(t["End_Timestamp"])
            if cur is None or s_ > cur[1]:
                if cur:
                    busy += cur[1] - cur[0]
                cur = [s_, e_]
            else:
                cur[1] = max(cur[1], e_)
        busy += cur[1] - cur[0]
        streams = {t["Stream_Id"] for t in run}
        lines.append(f"run {i + 1}: {len(run)} grids on {len(streams)} streams; span {(t1 - t0) / 1e3:.1f} us, "
                     f"a grid running {busy / (t1 - t0):.1%} of it; {user / (t1 - t0):.1f} GB/s of user data "
                     "over the span")
        res["runs"].append({"grids": len(run), "span_us": round((t1 - t0) / 1e3, 1),
                            "busy_frac": round(busy / (t1 - t0), 4), "GBps_user": round(user / (t1 - t0), 1)})
        for t in run:
            per_kernel.setdefault(name(t["Kernel_Name"]), []).append(
                (int(t["End_Timestamp"]) - int(t["Start_Timestamp"]),
                 int(t["Grid_Size_X"]) // max(1, int(t["Workgroup_Size_X"]))))
    lines += ["", f"{'kernel':<34}{'grids':>7}{'mean_us':>10}{'mean_wgs':>10}"]
    for k in sorted(per_kernel, key=lambda k: -sum(d for d, _ in per_kernel[k])):
        v = per_kernel[k]
        lines.append(f"{k:<34}{len(v):>7}{sum(d for d, _ in v) / len(v) / 1e3:>10.1f}"
                     f"{sum(g for _, g in v) / len(v):>10.0f}")
        res[k] = {"grids": len(v), "mean_us": round(sum(d for d, _ in v) / len(v) / 1e3, 1)}
    with open(os.path.join(out_dir, "zp_group_served_poisson_x4000_kernel_stats.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return res


P29_PROFILE_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_p29 -o run -- "
                   "python -u bench.py --p29-profile")
P29_ROLES = ("encode", "dd", "dp", "dq")


P29_PMC_CMDS = {c: f"rocprofv3 --pmc {c} --output-format csv -d gpurun_out/prof_p29_{c.split('_')[0].lower()} "
                   "-o run -- python -u bench.py --p29-profile --copy-probe" for c in ("FETCH_SIZE", "WRITE_SIZE")}


def p29_profile(stream, reps=10):
    """p = 29, k = 28, 1 KiB rows, 8192 stripes: `reps` launches (after one
    warm-up) of the encode and of the recovery of each erasure class, in
    P29_ROLES order, for the profiler (the erasure draws of config3)."""
    import torch

    import datagen
    import paper_cs_0611109_amd as r
    p3, k3, w3, n3 = 29, 28, 1024, 8192
    b = r.StripeBatch.empty(p3, k3, w3, n3)
    b.tensor[:, :k3].random_(0, 256)
    out = {"encode": time_launches(lambda: b.encode(), reps, stream)}
    for kind in P29_ROLES[1:]:
        er = torch.from_numpy(datagen.erasures(3, n3, k3, kind)).to("cuda:0")
        out[kind] = time_launches(lambda: b.recover(er), reps, stream)
    return {k: round(sum(v) / len(v), 4) for k, v in out.items()}


def summarize_p29_profile(stats_dir: str, out_dir: str = None) -> dict:
    """Per-role kernel durations of a P29_PROFILE_CMD run (host-only)."""
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    alg = 30 * 28 * 1024 * 8192
    trace = [t for t in _read_csv(os.path.join(stats_dir, "run_kernel_trace.csv"))
             if _short_name(t["Kernel_Name"]).startswith("zp_")]
    trace.sort(key=lambda t: int(t["Start_Timestamp"]))
    per = len(trace) // len(P29_ROLES)
    if per * len(P29_ROLES) != len(trace) or per < 2:
        raise RuntimeError(f"{stats_dir}: {len(trace)} Z_p launches, expected a multiple of {len(P29_ROLES)}")
    lines = ["# rocprofv3 kernel trace: p=29, k=28, W=1024 B rows, 8192 stripes; encode, then recovery with",
             "# per-stripe pairs of one class (dd: two data strips, dp: data + P, dq: data + Q), seed 3;",
             "# launch configurations from paper_cs_0611109_amd/tuned_mi355x.json",
             "# command (from the repository root, on one MI355X):", "#   " + P29_PROFILE_CMD,
             f"# source: run_kernel_trace.csv; {per} launches per role, the first a warm-up (not averaged);",
             f"# algorithmic bytes per launch (k+2)(p-1)W x stripes = {alg} B", "",
             f"{'role':<8}{'kernel':<40}{'avg_ns':>11}{'GB/s':>9}{'frac':>8}"]
    table = {}
    for i, role in enumerate(P29_ROLES):
        grp = trace[i * per:(i + 1) * per][1:]
        ns = sum(int(t["End_Timestamp"]) - int(t["Start_Timestamp"]) for t in grp) / len(grp)
        name = _short_name(grp[0]["Kernel_Name"])
        table[role] = {"kernel": name, "avg_ns": round(ns), "frac": round(alg / ns / HBM_PEAK_GBPS, 4)}
        lines.append(f"{role:<8}{name:<40}{ns:>11.0f}{alg / ns:>9.1f}{alg / ns / HBM_PEAK_GBPS:>8.4f}")
    with open(os.path.join(out_dir, "zp_p29_k28_w1024_x8192_kernel_stats.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return table


def summarize_p29_counters(fetch_dir: str, write_dir: str, out_dir: str = None) -> dict:
    """HBM bytes per launch of the P29_PMC_CMDS runs against the algorithmic
    bytes, per role, and their entries in the traffic table (host-only)."""
    import re
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    alg = (K3 + 2) * (P3 - 1) * W3 * N3

    def read(d, counter):
        zp, copies, wg = [], [], {}
        for r_ in _read_csv(os.path.join(d, "run_counter_collection.csv")):
            if r_["Counter_Name"] != counter:
                continue
            v = float(r_["Counter_Value"])
            if "copyBuffer" in r_["Kernel_Name"]:
                if v > 100000:
                    copies.append(v)
                continue
            n = _short_name(r_["Kernel_Name"])
            if n.startswith("zp_"):
                zp.append((int(r_["Dispatch_Id"]), v, n))
                wg[n] = int(r_["Workgroup_Size"])
        zp.sort()
        if not copies or len(zp) % len(P29_ROLES) != 0:
            raise RuntimeError(f"{d}: {len(zp)} Z_p launches, expected a multiple of {len(P29_ROLES)}, and probe copies")
        return zp, 2**30 / (sum(copies) / len(copies) * 1024), wg

    fetch, fs, wg = read(fetch_dir, "FETCH_SIZE")
    write, ws, _ = read(write_dir, "WRITE_SIZE")
    per = len(fetch) // len(P29_ROLES)
    lines = ["# rocprofv3 HBM byte counters: p=29, k=28, W=1024 B rows, 8192 stripes; encode, then recovery",
             "# with per-stripe pairs of one class (dd, dp, dq; seed 3); launch configurations from",
             "# paper_cs_0611109_amd/tuned_mi355x.json",
             "# commands (one counter per run, from the repository root, on one MI355X):",
             "#   " + P29_PMC_CMDS["FETCH_SIZE"], "#   " + P29_PMC_CMDS["WRITE_SIZE"],
             f"# counters scaled by 1 GiB probe copies in the same runs: fetch x{fs:.4f}, write x{ws:.4f};",
             f"# {per} launches per role (the first a warm-up, not averaged); algorithmic bytes per launch",
             f"# (k+2)(p-1)W x stripes = {alg} B", "",
             f"{'role':<8}{'kernel':<40}{'fetch_KiB':>11}{'write_KiB':>11}{'hbm_B':>13}{'ratio':>9}"]
    path = os.path.join(out_dir, "traffic.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    digest = source_digest()
    import paper_cs_0611109_amd as r
    from paper_cs_0611109_amd import autotune as at
    at.load_cache()
    res = {}
    for i, role in enumerate(P29_ROLES):
        f = [v for _, v, _ in fetch[i * per:(i + 1) * per][1:]]
        w = [v for _, v, _ in write[i * per:(i + 1) * per][1:]]
        name = fetch[i * per][2]
        fk, wk = sum(f) / len(f), sum(w) / len(w)
        hbm = int(round(fk * 1024 * fs + wk * 1024 * ws))
        lines.append(f"{role:<8}{name:<40}{fk:>11.0f}{wk:>11.0f}{hbm:>13}{hbm / alg:>9.5f}")
        m = re.match(r"zp_(\w+)_kernel<(\d+), (\d+), (\d+), (\w+)(?:, \w+)*>", name)
        split = int(m.group(5)) if m.group(1) == "split" else 1
        op = 0 if role == "encode" else 1
        cfg = list(r.raid6c_tune_get(P3, op, W3))
        key = f"{name.replace(', ', ',')} {role}"
        table[key] = {"source_sha256": digest, "config": cfg, "algorithmic_bytes": alg, "hbm_bytes_per_launch": hbm,
                      "fetch_kib": round(fk), "write_kib": round(wk), "fetch_scale": round(fs, 4),
                      "write_scale": round(ws, 4), "summary": "profiles/zp_p29_k28_w1024_x8192_hbm_bytes.txt",
                      "workgroup": wg.get(name), "split": split}
        res[role] = {"kernel": name, "ratio": round(hbm / alg, 5)}
    with open(os.path.join(out_dir, "zp_p29_k28_w1024_x8192_hbm_bytes.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1)
    return res


def rows_probe(stream):
    """Four launches (one warm-up) of the strided encode per ROWS_PROBE row
    size, then the 1 GiB copies that scale the byte counters."""
    import paper_cs_0611109_amd as r
    out = {}
    for w, n in ROWS_PROBE:
        b = r.StripeBatch.empty(53, 26, w, n)
        b.tensor[:, :26].random_(0, 256)
        ms = time_launches(lambda: b.encode(), 3, stream)
        moved = 28 * b.strip_stride * n
        out[w] = round(moved / (sum(ms) / len(ms) / 1e3) / 1e9 / HBM_PEAK_GBPS, 4)
        del b
    copy_probe(stream)
    return {"hbm_frac_by_row_bytes": out}


def summarize_rows_probe(fetch_dir: str, write_dir: str, out_dir: str = None) -> dict:
    """HBM bytes per launch of the ROWS_PROBE encodes against the bytes they
    read and write (host-only)."""
    out_dir = out_dir or os.path.join(ROOT, "profiles")

    def read(d, counter):
        zp, copies = [], []
        for r_ in _read_csv(os.path.join(d, "run_counter_collection.csv")):
            if r_["Counter_Name"] != counter:
                continue
            v = float(r_["Counter_Value"])
            if "copyBuffer" in r_["Kernel_Name"] and v > 100000:
                copies.append(v)
            elif _short_name(r_["Kernel_Name"]).startswith("zp_"):
                zp.append((int(r_["Dispatch_Id"]), v, _short_name(r_["Kernel_Name"])))
        zp.sort()
        if not copies or len(zp) != 4 * len(ROWS_PROBE):
            raise RuntimeError(f"{d}: expected {4 * len(ROWS_PROBE)} encode launches and the probe copies")
        return zp, 2**30 / (sum(copies) / len(copies) * 1024)

    fetch, fs = read(fetch_dir, "FETCH_SIZE")
    write, ws = read(write_dir, "WRITE_SIZE")
    lines = ["# rocprofv3 HBM byte counters: strided encode, p=53 k=26, rows on 128-byte lines (2048, 13312 B)",
             "# and 16 bytes past them (2064, 13328 B); tuned configuration of each row-size bucket",
             "# commands (one counter per run, from the repository root, on one MI355X):",
             "#   " + ROWS_PROBE_CMDS["FETCH_SIZE"], "#   " + ROWS_PROBE_CMDS["WRITE_SIZE"],
             "# counters scaled by 1 GiB probe copies in the same runs: "
             f"fetch x{fs:.4f}, write x{ws:.4f}; four launches per row size (one warm-up), averaged", "",
             f"{'row_bytes':>10}{'stripes':>9}  {'kernel':<36}{'read_B':>13}{'fetched_B':>13}{'fetch/read':>11}"
             f"{'written_B':>13}{'wrote_B':>13}{'ratio':>7}"]
    table = {}
    for i, (w, n) in enumerate(ROWS_PROBE):
        f = sum(v for _, v, _ in fetch[4 * i:4 * i + 4]) / 4 * 1024 * fs
        wr = sum(v for _, v, _ in write[4 * i:4 * i + 4]) / 4 * 1024 * ws
        rd = 26 * 52 * w * n
        wt = 2 * 52 * w * n
        name = fetch[4 * i][2]
        table[w] = {"kernel": name, "fetch_over_read": round(f / rd, 4), "write_over_written": round(wr / wt, 4)}
        lines.append(f"{w:>10}{n:>9}  {name:<36}{rd:>13}{f:>13.0f}{f / rd:>11.4f}{wt:>13}{wr:>13.0f}{wr / wt:>7.4f}")
    with open(os.path.join(out_dir, "zp_encode_kernel_rows_off_lines_p53_hbm_bytes.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return table


def summarize_plan_profile(stats_dir: str, out_dir: str = None) -> dict:
    """Summary of a PLAN_PROFILE_CMD run (host-only): the span of each plan run
    (first grid start to last grid end, from the kernel trace; the per-prime
    grids overlap in time) against the algorithmic bytes, and per-prime grid
    durations."""
    import re
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    alg = plan_jobs_bytes()
    total = sum(alg.values())
    trace = [t for t in _read_csv(os.path.join(stats_dir, "run_kernel_trace.csv"))
             if re.search(r"zp_group_kernel<\d+>", t["Kernel_Name"])]
    trace.sort(key=lambda t: int(t["Start_Timestamp"]))
    per_run = len(alg)
    runs = [trace[i:i + per_run] for i in range(0, len(trace) - per_run + 1, per_run)]
    spans = [(max(int(t["End_Timestamp"]) for t in g) - min(int(t["Start_Timestamp"]) for t in g)) for g in runs]
    spans = spans[1:] if len(spans) > 1 else spans           # the first run warms up
    span = sum(spans) / len(spans)
    lines = ["# rocprofv3 kernel trace: plan of 20,000 mixed stripes (p from {5,11,13,19,29,37,53},",
             "# k uniform in [2, p-1], rows log-uniform over 512 B..64 KiB, 60% encode / 40% two-erasure",
             "# recovery), default schedule: one job-list grid per prime, chained in one graph (one after another)",
             "# command (from the repository root, on one MI355X):", "#   " + PLAN_PROFILE_CMD,
             "# source: run_kernel_trace.csv; algorithmic bytes (k+2)(p-1)W summed over the stripes", "",
             f"plan runs timed: {len(spans)} (after one warm-up run)",
             f"span per run (first grid start to last grid end): {span / 1e6:.3f} ms",
             f"algorithmic bytes per run: {total} B -> {total / span:.1f} GB/s = "
             f"{total / span / HBM_PEAK_GBPS:.4f} of the 8 TB/s HBM peak", "",
             "per-prime grids (chained: each grid runs alone, so its duration is its share of the run):",
             f"{'kernel':<24}{'avg_ns':>11}{'alg_bytes':>14}"]
    table = {"span_ns": round(span), "alg_bytes": total, "frac": round(total / span / HBM_PEAK_GBPS, 4)}
    for p in sorted(alg, reverse=True):
        ns = [int(t["End_Timestamp"]) - int(t["Start_Timestamp"]) for g in runs[1:] or runs for t in g
              if f"zp_group_kernel<{p}>" in t["Kernel_Name"]]
        avg = sum(ns) / len(ns) if ns else 0.0
        lines.append(f"{'zp_group_kernel<%d>' % p:<24}{avg:>11.0f}{alg[p]:>14}")
        table[p] = {"avg_ns": round(avg), "alg_bytes": alg[p]}
    with open(os.path.join(out_dir, "zp_group_kernel_plan_mixed_x20000_kernel_stats.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return table


def _short_name(name: str) -> str:
    import re
    m = re.search(r"(zp_\w+_kernel<[^>]*>)", name)
    if m:
        return m.group(1)
    if "direct_copy_kernel" in name:
        return "torch direct_copy (host->device staging of the input)"
    if "FillFunctor" in name or "fill_kernel" in name:
        return "torch fill"
    return name[:60]


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def summarize_profiles(stats_dir: str, fetch_dir: str, write_dir: str, out_dir: str = None) -> dict:
    """Turn the three rocprofv3 runs of PROFILE_CMDS into the kernel-statistics
    and HBM-byte summaries and the traffic table (host-only; no GPU)."""
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    strip = (P - 1) * W
    alg = (K + 2) * strip * NSTRIPES
    head = (f"workload: p={P}, k={K}, W={W} B rows, {NSTRIPES} stripes "
            f"({K * strip * NSTRIPES / 2**30:.2f} GiB user data); one step = one encode launch + one "
            f"recovery launch (per-stripe pair uniform over the {(K + 2) * (K + 1) // 2} strip pairs); "
            "launch configurations from paper_cs_0611109_amd/tuned_mi355x.json")

    rows = _read_csv(os.path.join(stats_dir, "run_kernel_stats.csv"))
    lines = ["# rocprofv3 kernel statistics: Z_p-RAID encode + two-erasure recovery", "# " + head,
             "# command (from the repository root, on one MI355X):", "#   " + PROFILE_CMDS["stats"],
             "# source: run_kernel_stats.csv (durations in ns)", "",
             f"{'kernel':<56}{'calls':>6}{'avg_ns':>11}{'min_ns':>10}{'max_ns':>10}{'pct':>7}"]
    avg = {}
    for r_ in rows:
        n = _short_name(r_["Name"])
        lines.append(f"{n:<56}{int(r_['Calls']):>6}{float(r_['AverageNs']):>11.0f}{int(r_['MinNs']):>10}"
                     f"{int(r_['MaxNs']):>10}{float(r_['Percentage']):>7.2f}")
        if n.startswith("zp_"):
            avg[n] = float(r_["AverageNs"])
    lines += ["", f"algorithmic bytes per launch (both kernels): (k+2)(p-1)W x stripes = {alg} B"]
    for n, ns in avg.items():
        gbs = alg / ns
        lines.append(f"{n}: {gbs:.1f} GB/s = {gbs / HBM_PEAK_GBPS:.4f} of the 8 TB/s HBM peak")
    # Every step launches the encode, then the recovery; when both use the
    # same kernel the per-role figures come from the dispatch order.
    trace = [t for t in _read_csv(os.path.join(stats_dir, "run_kernel_trace.csv"))
             if _short_name(t["Kernel_Name"]).startswith("zp_")]
    trace.sort(key=lambda t: int(t["Start_Timestamp"]))
    if trace and len(trace) % 2 == 0:
        lines += ["", "per role (source: run_kernel_trace.csv, dispatches alternate encode, recovery):"]
        for role, sub in (("encode", trace[0::2]), ("recovery", trace[1::2])):
            ns = [int(t["End_Timestamp"]) - int(t["Start_Timestamp"]) for t in sub]
            mean = sum(ns) / len(ns)
            lines.append(f"{role:<9} {_short_name(sub[0]['Kernel_Name'])}: {len(ns)} launches, avg {mean:.0f} ns, "
                         f"{alg / mean:.1f} GB/s = {alg / mean / HBM_PEAK_GBPS:.4f} of peak")
    with open(os.path.join(out_dir, f"{WORKLOAD_TAG}_kernel_stats.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")

    def per_kernel(d, counter):
        got, wg, copies = {}, {}, []
        for r_ in _read_csv(os.path.join(d, "run_counter_collection.csv")):
            if r_["Counter_Name"] != counter:
                continue
            v = float(r_["Counter_Value"])
            if "copyBuffer" in r_["Kernel_Name"]:
                if v > 100000:          # the 1 GiB probe copies, not small staging copies
                    copies.append(v)
                continue
            n = _short_name(r_["Kernel_Name"])
            if n.startswith("zp_"):
                got.setdefault(n, []).append(v)
                wg[n] = int(r_["Workgroup_Size"])
        if len(copies) < 1:
            raise RuntimeError(f"{d}: no 1 GiB probe copy found (run with --copy-probe)")
        return {n: sum(v) / len(v) for n, v in got.items()}, wg, sum(copies) / len(copies)

    fetch, wg, cf = per_kernel(fetch_dir, "FETCH_SIZE")
    write, _, cw = per_kernel(write_dir, "WRITE_SIZE")
    fs, ws = 2**30 / (cf * 1024), 2**30 / (cw * 1024)
    lines = [f"# rocprofv3 HBM byte counters: Z_p-RAID kernels, p={P} k={K} W={W} B x {NSTRIPES} stripes",
             "# commands (one counter per run, from the repository root, on one MI355X):",
             "#   " + PROFILE_CMDS["fetch"], "#   " + PROFILE_CMDS["write"],
             "# --copy-probe adds three plain 1 GiB device-to-device copies (the runtime's copyBuffer",
             "# kernel) whose counter readings give the scale from counter KiB to bytes moved.", "",
             f"copy_1GiB FETCH_SIZE avg {cf:.0f} KiB -> fetch scale {fs:.4f} (bytes per counted byte)",
             f"copy_1GiB WRITE_SIZE avg {cw:.0f} KiB -> write scale {ws:.4f}", ""]
    table, digest = {}, source_digest()
    import re

    # The work-group order is not part of a kernel's name: take it from the
    # configurations the profiled run used (the committed tuning cache).
    import paper_cs_0611109_amd as r
    from paper_cs_0611109_amd import autotune as at
    at.load_cache()
    orders = {}
    for op in (0, 1):
        v, u, t, sp, o = r.raid6c_tune_get(P, op, W)
        orders[(v, u, t, sp)] = o
    for n in sorted(fetch):
        if n not in write:
            continue
        hbm = int(round(fetch[n] * 1024 * fs + write[n] * 1024 * ws))
        lines.append(f"{n}: FETCH_SIZE {fetch[n]:.0f} KiB, WRITE_SIZE {write[n]:.0f} KiB per launch -> "
                     f"{hbm} B scaled HBM traffic; algorithmic {alg} B; ratio {hbm / alg:.5f}")
        m = re.match(r"zp_(\w+)_kernel<(\d+), (\d+), (\d+), (\w+)(?:, \w+)*>", n)
        split = int(m.group(5)) if m.group(1) == "split" else 1
        key = n.replace(", ", ",")
        cfg = (int(m.group(3)), int(m.group(4)), wg[n], split)
        table[key] = {"source_sha256": digest, "config": [*cfg, orders.get(cfg, 0)],
                      "algorithmic_bytes": alg, "hbm_bytes_per_launch": hbm,
                      "fetch_kib": round(fetch[n]), "write_kib": round(write[n]),
                      "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
                      "summary": f"profiles/{WORKLOAD_TAG}_hbm_bytes.txt"}
    with open(os.path.join(out_dir, f"{WORKLOAD_TAG}_hbm_bytes.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(out_dir, "traffic.json"), "w") as f:
        json.dump(table, f, indent=1)
    return table


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="time every launch configuration for this geometry first (else use the tuning cache)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run plain 1 GiB device copies (for scaling HBM byte counters)")
    ap.add_argument("--summarize", nargs=3, metavar=("STATS_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write the profiles/ summaries from the three rocprofv3 runs (no GPU needed)")
    ap.add_argument("--plan-profile", type=int, metavar="RUNS",
                    help="only run the 20,000-stripe plan RUNS times (for the profiler)")
    ap.add_argument("--summarize-plan-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the profiles/ HBM-byte summary of the two plan counter runs (no GPU needed)")
    ap.add_argument("--summarize-plan", metavar="STATS_DIR",
                    help="write the profiles/ summary of a --plan-profile run (no GPU needed)")
    ap.add_argument("--p29-profile", action="store_true",
                    help="only the p = 29 encode and recoveries (for the profiler)")
    ap.add_argument("--summarize-p29", metavar="STATS_DIR",
                    help="write the profiles/ summary of a --p29-profile run (no GPU needed)")
    ap.add_argument("--summarize-p29-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the profiles/ HBM-byte summary of the two --p29-profile counter runs (no GPU needed)")
    ap.add_argument("--serve-profile", type=int, metavar="RUNS",
                    help="only the saturated served stream, RUNS replays after a warm-up (for the profiler)")
    ap.add_argument("--summarize-serve", metavar="STATS_DIR",
                    help="write the profiles/ summary of a --serve-profile run (no GPU needed)")
    ap.add_argument("--config", type=int, choices=(1, 2, 3, 4, 5),
                    help="measure one workload only and print its JSON object: 1 launch latency at p=5, "
                         "2 the headline step (no extras), 3 p=29 recovery by class, 4 the 20,000-stripe plan, "
                         "5 the served stream")
    ap.add_argument("--rows-probe", action="store_true",
                    help="only the encodes of rows on / off 128-byte lines (for the byte counters)")
    ap.add_argument("--summarize-rows", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the profiles/ summary of the two --rows-probe counter runs (no GPU needed)")
    args = ap.parse_args()
    if args.summarize:
        print(json.dumps(summarize_profiles(*args.summarize), indent=1))
        return
    if args.summarize_plan_counters:
        print(json.dumps(summarize_plan_counters(*args.summarize_plan_counters), indent=1))
        return
    if args.summarize_plan:
        print(json.dumps(summarize_plan_profile(args.summarize_plan), indent=1))
        return
    if args.summarize_rows:
        print(json.dumps(summarize_rows_probe(*args.summarize_rows), indent=1))
        return
    if args.summarize_p29_counters:
        print(json.dumps(summarize_p29_counters(*args.summarize_p29_counters), indent=1))
        return
    if args.summarize_p29:
        print(json.dumps(summarize_p29_profile(args.summarize_p29), indent=1))
        return
    if args.summarize_serve:
        print(json.dumps(summarize_serve_profile(args.summarize_serve), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (stripes are independent, "
              "so more GPUs would each take a share of the stripes, with no communication between them).",
              file=sys.stderr)
        sys.exit(2)
    # The CPU oracle over every core runs first, in worker processes started
    # before torch is imported and before anything touches the GPU.
    parallel = None
    if args.config == 2:
        args.no_extras = True
    if not (args.no_cpu_baseline or args.plan_profile or args.p29_profile or args.rows_probe or
            args.serve_profile or args.config not in (None, 2)):
        log("cpu baseline: oracle on every core (worker processes, before the GPU is touched)")
        parallel = cpu_oracle_parallel(max(1.0, args.cpu_seconds / 8))

    import torch

    import datagen
    import paper_cs_0611109_amd as r
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    r.load()
    stream = torch.cuda.current_stream()
    if args.plan_profile:
        res = plan_profile(args.plan_profile)
        if args.copy_probe:
            copy_probe(stream)
        print(json.dumps(res), flush=True)
        return
    if args.p29_profile:
        from paper_cs_0611109_amd import autotune as at
        at.load_cache()
        res = p29_profile(stream)
        if args.copy_probe:
            copy_probe(stream)
        print(json.dumps(res), flush=True)
        return
    if args.rows_probe:
        from paper_cs_0611109_amd import autotune as at
        at.load_cache()
        print(json.dumps(rows_probe(stream)), flush=True)
        return
    if args.serve_profile:
        print(json.dumps(serve_profile(args.serve_profile)), flush=True)
        return
    if args.config not in (None, 2):
        from paper_cs_0611109_amd import autotune as at
        at.load_cache()
        if args.config == 1:
            res = config1_latency(50, stream)
        elif args.config == 3:
            res = config3(max(20, args.steps), stream)
        elif args.config == 4:
            res = batched_mixed(max(10, args.steps // 2), stream)
        else:
            res = {"served_poisson": served_poisson(), "served_sustained_saturation": served_sustained()}
        print(json.dumps({"config": args.config, "result": res}), flush=True)
        return

    log(f"allocating and filling p={P} k={K} W={W} x {NSTRIPES} stripes")
    batch = r.StripeBatch.empty(P, K, W, NSTRIPES)
    fill_batch(batch, SEED)
    er_host = datagen.erasures(SEED, NSTRIPES, K, "any")
    er = torch.from_numpy(er_host).to("cuda:0")
    bad = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()

    from paper_cs_0611109_amd import autotune as at
    tuned = {"cache_entries": at.load_cache()}
    if args.autotune:
        log("autotuning the launch configuration for this geometry (outside the timed region)")
        tuned["encode_ms"] = round(batch.autotune(0, reps=5), 4)
        tuned["recover_ms"] = round(batch.autotune(1, er, reps=5), 4)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        batch.encode()
        if ev is not None:
            ev[1].record(stream)
        batch.recover(er, bad)
        if ev is not None:
            ev[2].record(stream)

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if int(bad.item()) != 0:
        raise RuntimeError("recovery rejected erasure entries")
    enc_ms = [e[0].elapsed_time(e[1]) for e in evs]
    rec_ms = [e[1].elapsed_time(e[2]) for e in evs]
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    user = batch.user_bytes
    alg_bytes = (K + 2) * batch.strip_stride * NSTRIPES           # per launch, encode and recovery alike
    enc_mean = sum(enc_ms) / len(enc_ms)
    rec_mean = sum(rec_ms) / len(rec_ms)
    value = 2 * user / (ms_per_step / 1e3) / 1e9

    dom = "recover" if rec_mean >= enc_mean else "encode"
    dom_ms = rec_mean if dom == "recover" else enc_mean
    vec, unroll, threads, split, order = r.raid6c_tune_get(P, 1 if dom == "recover" else 0, W)
    if split > 1:
        kname = f"zp_split_kernel<{P},{vec},{unroll},{split},false,{LOAD_POLICY_STREAM}>"
    else:
        kname = f"zp_{dom}_kernel<{P},{vec},{unroll},false,{LOAD_POLICY_STREAM}>"
    achieved = alg_bytes / (dom_ms / 1e3) / 1e9
    traffic = lookup_traffic(kname, (vec, unroll, threads, split, order), alg_bytes)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": kname, "launch": {"vec": vec, "unroll": unroll, "threads": threads, "split": split,
                                                  "order": order},
                "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_ms": round(dom_ms, 4)}
    log(f"value {value:.1f} GB/s; encode {enc_mean:.3f} ms, recovery {rec_mean:.3f} ms per launch")

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded uniform random bytes)",
        "config": {"workload": "Z_p-RAID encode + two-erasure recovery, p=13 k=12 W=4096 B x 4096 stripes",
                   "p": P, "k": K, "row_bytes": W, "nstripes": NSTRIPES,
                   "user_bytes_per_pass": user, "passes_per_step": 2,
                   "erasures": "per-stripe pair uniform over all 91 strip pairs", "parallelism": "single GPU"},
        "encode": {"GBps_user": round(user / (enc_mean / 1e3) / 1e9, 1),
                   "hbm_frac": round(alg_bytes / (enc_mean / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                   "ms_p50": round(pct(enc_ms, 50), 4), "ms_p99": round(pct(enc_ms, 99), 4),
                   "launch": dict(zip(("vec", "unroll", "threads", "split", "order"), r.raid6c_tune_get(P, 0, W)))},
        "recover_2": {"GBps_user": round(user / (rec_mean / 1e3) / 1e9, 1),
                      "hbm_frac": round(alg_bytes / (rec_mean / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                      "ms_p50": round(pct(rec_ms, 50), 4), "ms_p99": round(pct(rec_ms, 99), 4),
                      "launch": dict(zip(("vec", "unroll", "threads", "split", "order"),
                                         r.raid6c_tune_get(P, 1, W)))},
        "roofline": roofline,
        "autotune": tuned,
    }
    # The paper's own speeds, quoted (not re-run), with the processor it names.
    result["paper_reference"] = {
        "processor": "2.8 GHz Intel Pentium 4",
        "syndrome_generation_MBps": {"linux_rs_sse2x2": 2702, "z17_sse2x2": 3160},
        "source": "Section 4.5, syndrome-generation speed table (fastest routines)",
        "this_encode_over_paper_z17": round(result["encode"]["GBps_user"] * 1e3 / 3160, 1)}
    if not args.no_extras:
        log("HBM ceiling of a plain device copy")
        result["hbm_ceiling"] = copy_ceiling(stream)
        log(f"recovery at p={P3} k={K3} W={W3} x {N3} stripes, by erasure class")
        result["recover_config3"] = config3(max(20, args.steps), stream)
        log("launch latency at p=5 k=4 W=64 x 1024 stripes")
        result["latency_config1"] = config1_latency(50, stream)
        log("extras: GF(256) RS comparison, extended parity, small writes, Z17 layout, plans, server")
        result["extras"] = extras(max(10, args.steps // 2), stream)
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle for about {args.cpu_seconds:.0f} s")
        result["cpu_baseline"] = cpu_baseline(batch, er_host, args.cpu_seconds, parallel)
        served = result.get("extras", {}).get("served_poisson")
        if isinstance(served, dict) and "error" not in served:
            log("cpu baseline: oracle check of the served sample")
            served["verified_against_oracle"] = verify_served_samples()
            result["cpu_baseline"]["served_sample_matches_oracle"] = (served["verified_against_oracle"] or {}).get("match")
    else:
        result["cpu_baseline"] = None
    if args.copy_probe:
        copy_probe(stream)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

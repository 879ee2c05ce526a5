"""Host-side logic of bench.py, on the CPU: the one-GPU refusal, the lookup
of measured HBM traffic in the committed table, the turning of rocprofv3
counter readings into bytes (scaled by the plain copies of known size that
the counter runs include), and the summary of a served kernel trace."""

import csv
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "measures one GPU" in out.stderr


def test_committed_traffic_is_found_only_for_its_own_source_and_launch():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        table = json.load(f)
    assert table
    for key, e in table.items():
        kernel, _, role = key.partition(" ")
        role = role or None
        got = bench.lookup_traffic(kernel, e["config"], e["algorithmic_bytes"], role)
        if e["source_sha256"] != bench.source_digest():
            assert got is None
            continue
        assert got == e["hbm_bytes_per_launch"]
        other = list(e["config"])
        other[2] = 64 if other[2] != 64 else 128                # another work-group size
        assert bench.lookup_traffic(kernel, other, e["algorithmic_bytes"], role) is None
        assert bench.lookup_traffic(kernel, e["config"], e["algorithmic_bytes"] + 1, role) is None


def _write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_counter_summary_scales_by_the_probe_copies(tmp_path):
    """Two kernels, each read at a known byte count; the 1 GiB copies read
    half of what they move on FETCH_SIZE and all of it on WRITE_SIZE, as the
    counters do on this GPU, so the scales must come out as 2 and 1."""
    pytest.importorskip("torch")
    alg = (bench.K + 2) * (bench.P - 1) * bench.W * bench.NSTRIPES
    enc = "void raid6c::zp_split_kernel<13, 2, 4, 4, false, 2>(raid6c::ZpArgs)"
    rec = "void raid6c::zp_split_kernel<13, 2, 1, 4, false, 2>(raid6c::ZpArgs)"
    copy = "__amd_rocclr_copyBuffer"
    stats, fetch, write = tmp_path / "stats", tmp_path / "fetch", tmp_path / "write"
    for d in (stats, fetch, write):
        d.mkdir()
    _write_csv(stats / "run_kernel_stats.csv",
               [{"Name": enc, "Calls": 2, "AverageNs": 450000, "MinNs": 449000, "MaxNs": 451000, "Percentage": 48},
                {"Name": rec, "Calls": 2, "AverageNs": 480000, "MinNs": 479000, "MaxNs": 481000, "Percentage": 52}])
    trace = []
    t = 1000
    for name, ns in ((enc, 450000), (rec, 480000), (enc, 450000), (rec, 480000)):
        trace.append({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + ns})
        t += ns + 1000
    _write_csv(stats / "run_kernel_trace.csv", trace)
    # Counter readings in KiB: the kernels fetch 12/14 and write 2/14 of the
    # algorithmic bytes, plus 1% more fetched by the recovery.
    enc_f, enc_w = alg * 12 / 14, alg * 2 / 14
    rec_f, rec_w = enc_f * 1.01, enc_w

    def rows(counter, enc_bytes, rec_bytes, scale):
        out = [{"Counter_Name": counter, "Counter_Value": (1 << 30) / scale / 1024, "Kernel_Name": copy,
                "Workgroup_Size": 256} for _ in range(3)]
        out += [{"Counter_Name": counter, "Counter_Value": enc_bytes / scale / 1024, "Kernel_Name": enc,
                 "Workgroup_Size": 256},
                {"Counter_Name": counter, "Counter_Value": rec_bytes / scale / 1024, "Kernel_Name": rec,
                 "Workgroup_Size": 256}]
        return out

    _write_csv(fetch / "run_counter_collection.csv", rows("FETCH_SIZE", enc_f, rec_f, 2.0))
    _write_csv(write / "run_counter_collection.csv", rows("WRITE_SIZE", enc_w, rec_w, 1.0))
    table = bench.summarize_profiles(str(stats), str(fetch), str(write), out_dir=str(tmp_path))
    e = table["zp_split_kernel<13,2,4,4,false,2>"]
    assert e["fetch_scale"] == pytest.approx(2.0) and e["write_scale"] == pytest.approx(1.0)
    assert e["hbm_bytes_per_launch"] == pytest.approx(alg, rel=1e-6)
    r = table["zp_split_kernel<13,2,1,4,false,2>"]
    assert r["hbm_bytes_per_launch"] == pytest.approx(rec_f + rec_w, rel=1e-6)
    assert e["config"][:4] == [2, 4, 256, 4] and r["config"][:4] == [2, 1, 256, 4]
    assert (tmp_path / "traffic.json").exists()
    text = (tmp_path / f"{bench.WORKLOAD_TAG}_kernel_stats.txt").read_text()
    assert "encode    zp_split_kernel<13, 2, 4, 4, false, 2>: 2 launches, avg 450000 ns" in text


def test_served_trace_summary_splits_runs_and_measures_busy_time(tmp_path):
    """A warm-up run and two timed runs of grids, separated by idle gaps:
    the warm-up is left out, and the busy fraction counts overlapping grids
    once."""
    k37 = "void raid6c::(anonymous namespace)::zp_group_lat_kernel<37>(raid6c::GroupArgs)"
    km = "void raid6c::(anonymous namespace)::zp_group_multi_kernel(raid6c::GroupArgs)"
    rows = []

    def grid(name, s, e, stream):
        rows.append({"Kernel_Name": name, "Start_Timestamp": s, "End_Timestamp": e, "Stream_Id": stream,
                     "Grid_Size_X": 256 * 100, "Workgroup_Size_X": 256})

    grid(k37, 0, 50_000, 1)                                  # warm-up run
    base = 10_000_000
    grid(k37, base, base + 100_000, 1)                       # run 1: two overlapping grids, then a gap
    grid(km, base + 50_000, base + 200_000, 2)
    grid(km, base + 300_000, base + 400_000, 1)
    base = 20_000_000
    grid(km, base, base + 100_000, 3)                        # run 2: one grid
    (tmp_path / "t").mkdir()
    _write_csv(tmp_path / "t" / "run_kernel_trace.csv", rows)
    res = bench.summarize_serve_profile(str(tmp_path / "t"), out_dir=str(tmp_path))
    assert [r["grids"] for r in res["runs"]] == [3, 1]
    assert res["runs"][0]["span_us"] == 400.0 and res["runs"][0]["busy_frac"] == 0.75
    assert res["runs"][1]["busy_frac"] == 1.0
    assert res["zp_group_multi_kernel"]["grids"] == 3 and res["zp_group_lat_kernel<37>"]["grids"] == 1

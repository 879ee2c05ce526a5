"""Autotuner front end and its cache file.

The library picks a launch configuration (vector width, strip batching,
work-group size) per (p, operation, row-size bucket) from a process-wide
table.  `tune()` fills the table by timing every built configuration on
synthetic stripes of the given geometries (raid6c_autotune_n); the result
can be saved as JSON and loaded at start-up with `load_cache()`.  Like the
kernel's algorithm-selection benchmark that picks the fastest routine at boot,
this changes speed only, never results.

    python -m paper_cs_0611109_amd.autotune --out tuned.json 13,12,4096,4096 29,28,1024,8192,dd+dp+dq

A geometry is ``p,k,row_bytes,nstripes`` with an optional fifth field naming
the erasure classes the recovery is scored on: ``any`` (a pair uniform over
all strip pairs of each stripe, the default) or classes joined by ``+``
(the stripes split into equal consecutive blocks, one class each, e.g.
``dd+dp+dq``).  Each configuration's score is the median of ``reps``
launches timed one by one.
"""

from __future__ import annotations

import argparse
import json
import os
import sys

from . import _lib

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def load_cache(path: str = DEFAULT_CACHE) -> int:
    """Apply every entry of a cache file; returns the number applied (0 when
    the file does not exist)."""
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    n = 0
    for e in data.get("entries", []):
        _lib.raid6c_tune_set(e["p"], e["op"], e["row_bytes"], e["vec"], e["unroll"], e["threads"],
                             e.get("split", 1), e.get("order", 0))
        n += 1
    return n


def erasure_mix(seed: int, n: int, k: int, classes: str):
    """Per-stripe erasure pairs for tuning: one class for all stripes, or
    consecutive blocks of the classes joined by '+'."""
    import numpy as np

    import datagen
    kinds = classes.split("+")
    edges = [n * i // len(kinds) for i in range(len(kinds) + 1)]
    return np.concatenate([datagen.erasures(seed + i, edges[i + 1] - edges[i], k, kd)
                           for i, kd in enumerate(kinds)], axis=0)


def tune(geoms, reps: int = 20, seed: int = 1):
    """Autotune encode and recovery for each (p, k, row_bytes, nstripes[,
    classes]); returns cache entries."""
    import torch

    from .layout import StripeBatch
    entries = []
    for g in geoms:
        p, k, w, n = g[:4]
        classes = g[4] if len(g) > 4 else "any"
        b = StripeBatch.empty(p, k, w, n)
        b.tensor.random_(0, 256)
        er = torch.from_numpy(erasure_mix(seed, n, k, classes)).to(b.tensor.device)
        for op in (0, 1):
            ms = b.autotune(op, er if op == 1 else None, reps=reps)
            slot = op + (2 if k > p else 0)        # the extended Q parity has its own entries
            vec, unroll, threads, split, order = _lib.raid6c_tune_get(p, slot, w)
            moved = (k + 2) * b.strip_stride * n
            entries.append({"p": p, "op": slot, "row_bytes": w, "vec": vec, "unroll": unroll, "threads": threads,
                            "split": split, "order": order, "k": k, "nstripes": n,
                            "erasures": classes if op == 1 else None, "reps": reps, "ms_median": round(ms, 4),
                            "GBps_moved": round(moved / (ms / 1e3) / 1e9, 1)})
            print(f"p={p} k={k} W={w} n={n} op={slot}: vec={vec} unroll={unroll} threads={threads} split={split} "
                  f"order={order} {ms:.4f} ms {moved / (ms / 1e3) / 1e9:.0f} GB/s", file=sys.stderr, flush=True)
        del b
        torch.cuda.empty_cache()
    return entries


def save_cache(entries, path: str, command: str = "") -> None:
    import torch
    with open(path, "w") as f:
        json.dump({"device": torch.cuda.get_device_name(0), "command": command, "entries": entries}, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser(description="autotune libraid6c launch configurations")
    ap.add_argument("geoms", nargs="+", help="p,k,row_bytes,nstripes[,classes]")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    args = ap.parse_args(argv)
    geoms = []
    for g in args.geoms:
        f = g.split(",")
        geoms.append(tuple(int(x) for x in f[:4]) + tuple(f[4:5]))
    cmd = "python -m paper_cs_0611109_amd.autotune " + " ".join(a for a in (argv or sys.argv[1:]) if a != args.out)
    cmd = cmd.replace("--out ", "")
    save_cache(tune(geoms, args.reps), args.out, cmd)


if __name__ == "__main__":
    main()

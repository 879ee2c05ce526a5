"""Autotuner front end and its cache file.

The library picks a launch configuration (vector width, strip batching,
work-group size) per (p, operation, row-size bucket) from a process-wide
table.  `tune()` fills the table by timing every built configuration on
synthetic stripes of the given geometries (raid6c_autotune_n); the result
can be saved as JSON and loaded at start-up with `load_cache()`.  Like the
kernel's algorithm-selection benchmark that picks the fastest routine at boot,
this changes speed only, never results.

    python -m paper_cs_0611109_amd.autotune --out tuned.json 13,12,4096,4096 29,28,1024,8192
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


def tune(geoms, reps: int = 5, seed: int = 1):
    """Autotune encode and recovery (uniform random erasure pairs) for each
    (p, k, row_bytes, nstripes); returns cache entries."""
    import torch

    import datagen
    from .layout import StripeBatch
    entries = []
    for (p, k, w, n) in geoms:
        b = StripeBatch.empty(p, k, w, n)
        b.tensor.random_(0, 256)
        er = torch.from_numpy(datagen.erasures(seed, n, k, "any")).to(b.tensor.device)
        for op in (0, 1):
            ms = b.autotune(op, er if op == 1 else None, reps=reps)
            slot = op + (2 if k > p else 0)        # the extended Q parity has its own entries
            vec, unroll, threads, split, order = _lib.raid6c_tune_get(p, slot, w)
            moved = (k + 2) * b.strip_stride * n
            entries.append({"p": p, "op": slot, "row_bytes": w, "vec": vec, "unroll": unroll, "threads": threads,
                            "split": split, "order": order, "k": k, "nstripes": n, "ms": round(ms, 4),
                            "GBps_moved": round(moved / (ms / 1e3) / 1e9, 1)})
            print(f"p={p} k={k} W={w} n={n} op={slot}: vec={vec} unroll={unroll} threads={threads} split={split} "
                  f"order={order} {ms:.4f} ms {moved / (ms / 1e3) / 1e9:.0f} GB/s", file=sys.stderr, flush=True)
        del b
        torch.cuda.empty_cache()
    return entries


def save_cache(entries, path: str) -> None:
    import torch
    with open(path, "w") as f:
        json.dump({"device": torch.cuda.get_device_name(0), "entries": entries}, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser(description="autotune libraid6c launch configurations")
    ap.add_argument("geoms", nargs="+", help="p,k,row_bytes,nstripes")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    args = ap.parse_args(argv)
    geoms = [tuple(int(x) for x in g.split(",")) for g in args.geoms]
    save_cache(tune(geoms, args.reps), args.out)


if __name__ == "__main__":
    main()

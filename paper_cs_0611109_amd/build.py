"""Build libraid6c.so in-tree with hipcc for gfx950.

The Z_p kernel source is compiled six times per supported prime
(-DRAID6C_P=p, -DRAID6C_VARIANT=0..5: plain, extended Q parity, split-K,
plan job list, plan job list with extended Q parity, the server's job list
for small batches), in parallel, then everything is linked into
``paper_cs_0611109_amd/libraid6c.so``.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libraid6c.so")

PRIMES = (3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61)
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

CFLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]

# Plain (non-templated-per-prime) sources.
SOURCES = ["raid6c_api.hip", "tune.hip", "rs_kernels.hip", "update.hip", "layout.hip", "batch.hip", "serve.hip",
           "noalloc.hip", "zp_multi.hip"]


def _units(build_dir):
    units = []
    for src in SOURCES:
        units.append((os.path.join(CSRC, src), os.path.join(build_dir, src.replace(".hip", ".o")), []))
    for p in PRIMES:
        for variant, suffix in ((0, ""), (1, "_ext"), (2, "_split"), (3, "_group"), (4, "_group_ext"),
                                (5, "_group_lat")):
            units.append((os.path.join(CSRC, "zp_kernels.hip"),
                          os.path.join(build_dir, f"zp_kernels_p{p}{suffix}.o"),
                          [f"-DRAID6C_P={p}", f"-DRAID6C_VARIANT={variant}"]))
    return units


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(ln for ln in r.stdout.splitlines() if "packed-fp32-ops" not in ln)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out, flush=True)


def build(verbose: bool = False, jobs: int | None = None, out: str = LIB, build_dir: str = BUILD,
          defines=()) -> str:
    """Compile every source for gfx950 and link libraid6c.so; returns its path.

    ``out``, ``build_dir`` and ``defines`` (extra -D flags) allow building
    variants elsewhere, e.g. for tuning experiments."""
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = _units(build_dir)
    dflags = [f"-D{d}" for d in defines]

    def compile_one(u):
        src, obj, extra = u
        _run([HIPCC, *CFLAGS, *dflags, *extra, "-I", CSRC, "-c", src, "-o", obj], verbose)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as pool:
        objs = list(pool.map(compile_one, units))
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

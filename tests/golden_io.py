"""Readers for the small text fixtures under tests/golden (values printed in the paper)."""

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def sections(name):
    """Split a fixture into ``{section: [lines]}`` (lines before any header go to '')."""
    out, cur = {"": []}, ""
    for line in _lines(name):
        if line.startswith("[") and line.endswith("]"):
            cur = line[1:-1]
            out[cur] = []
        else:
            out[cur].append(line)
    return out


def matrix(lines):
    return np.array([[int(v) for v in ln.split()] for ln in lines], dtype=np.uint8)


def equations(lines):
    """``a = b + c + d`` lines as ``{a: [b, c, d]}``."""
    eqs = {}
    for ln in lines:
        lhs, rhs = ln.split("=")
        eqs[lhs.strip()] = [t.strip() for t in rhs.split("+")]
    return eqs

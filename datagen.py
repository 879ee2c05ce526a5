"""Seeded synthetic inputs for the cyclic-group RAID-6 tests and benchmark.

This module holds none of the code's arithmetic.  It only produces bytes,
erasure choices, stripe geometries and arrival times, and it serves both the
CPU oracle (through the tests and the benchmark) and the GPU library.

Every stream is counter based: a Philox4x64-10 generator keyed by
``(seed, stream tag, index)``.  Any one stripe can therefore be regenerated on
the host without generating the stripes before it, which is how full-size GPU
runs are checked on sampled stripes.

Integer draws use explicit rejection sampling on raw 64-bit words, so the
results do not depend on a library's choice of mapping.
"""

from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

# Stream tags: independent streams for independent purposes.
TAG_DATA = 1
TAG_ERASURE = 2
TAG_GEOMETRY = 3
TAG_ARRIVAL = 4
TAG_POISON = 5

_MASK64 = (1 << 64) - 1


def _philox(seed: int, tag: int, index: int) -> np.random.Philox:
    if seed < 0 or tag < 0 or index < 0:
        raise ValueError("seed, tag and index must be non-negative")
    if tag >= (1 << 16) or index >= (1 << 48):
        raise ValueError("tag or index out of range")
    key = np.array([seed & _MASK64, (tag << 48) | index], dtype=np.uint64)
    return np.random.Philox(key=key)


def random_bytes(seed: int, tag: int, index: int, n: int) -> np.ndarray:
    """``n`` uniform random bytes from stream ``(seed, tag, index)``."""
    if n < 0:
        raise ValueError("n must be non-negative")
    words = _philox(seed, tag, index).random_raw((n + 7) // 8)
    return words.astype("<u8", copy=False).view(np.uint8)[:n].copy()


def stripe_data(seed: int, stripe: int, k: int, p: int, row_bytes: int) -> np.ndarray:
    """The ``k`` data strips of one stripe: shape ``(k, p-1, row_bytes)``, uint8."""
    n = k * (p - 1) * row_bytes
    return random_bytes(seed, TAG_DATA, stripe, n).reshape(k, p - 1, row_bytes)


def fill_stripes(seed: int, first: int, count: int, k: int, p: int, row_bytes: int,
                 out: np.ndarray | None = None, threads: int = 8) -> np.ndarray:
    """Data strips of stripes ``first .. first+count-1``: ``(count, k, p-1, row_bytes)``.

    Stripe ``s`` always holds the same bytes, whatever ``first`` and ``count``.
    """
    shape = (count, k, p - 1, row_bytes)
    if out is None:
        out = np.empty(shape, dtype=np.uint8)
    elif out.shape != shape or out.dtype != np.uint8:
        raise ValueError("out has the wrong shape or dtype")

    def one(i: int) -> None:
        out[i] = stripe_data(seed, first + i, k, p, row_bytes)

    if threads <= 1 or count < 4:
        for i in range(count):
            one(i)
    else:
        with ThreadPoolExecutor(max_workers=threads) as pool:
            list(pool.map(one, range(count)))
    return out


def poison(shape, seed: int = 0xA5, index: int = 0) -> np.ndarray:
    """Random bytes used to overwrite erased strips before a recovery."""
    n = int(np.prod(shape))
    return random_bytes(seed, TAG_POISON, index, n).reshape(shape)


class Draws:
    """Deterministic scalar draws from one counter-based stream."""

    def __init__(self, seed: int, tag: int, index: int = 0):
        self._bg = _philox(seed, tag, index)
        self._buf = np.empty(0, dtype=np.uint64)
        self._pos = 0

    def raw(self) -> int:
        if self._pos == len(self._buf):
            self._buf = self._bg.random_raw(4096)
            self._pos = 0
        v = int(self._buf[self._pos])
        self._pos += 1
        return v

    def below(self, n: int) -> int:
        """Uniform integer in ``[0, n)`` by rejection of the top partial block."""
        if n <= 0:
            raise ValueError("n must be positive")
        limit = ((1 << 64) // n) * n
        while True:
            v = self.raw()
            if v < limit:
                return v % n

    def between(self, lo: int, hi: int) -> int:
        """Uniform integer in ``[lo, hi]``."""
        return lo + self.below(hi - lo + 1)

    def unit(self) -> float:
        """Uniform float in ``[0, 1)`` from the top 53 bits."""
        return (self.raw() >> 11) * (1.0 / (1 << 53))

    def log_uniform(self, lo: float, hi: float) -> float:
        return math.exp(math.log(lo) + self.unit() * (math.log(hi) - math.log(lo)))

    def exponential(self, rate: float) -> float:
        return -math.log1p(-self.unit()) / rate


ERASURE_KINDS = ("any", "dd", "dp", "dq", "pq", "d", "p", "q", "any1")


def erasures(seed: int, nstripes: int, k: int, kind: str) -> np.ndarray:
    """Per-stripe erased strip indices, shape ``(nstripes, 2)`` int32.

    Strip indices: ``0..k-1`` data, ``k`` = P, ``k+1`` = Q.  Pairs are sorted
    (``e0 < e1``).  Kinds:

    * ``any``: a pair uniform over all ``C(k+2, 2)`` pairs of the stripe.
    * ``dd``: two data strips, uniform over the ``C(k, 2)`` pairs (needs k >= 2).
    * ``dp`` / ``dq``: one data strip, uniform, plus P / Q.
    * ``pq``: P and Q.
    * ``d``, ``p``, ``q``, ``any1``: a single erasure, stored as ``(e, -1)``.
    """
    if kind not in ERASURE_KINDS:
        raise ValueError(f"unknown erasure kind {kind!r}")
    d = Draws(seed, TAG_ERASURE, ERASURE_KINDS.index(kind))
    out = np.empty((nstripes, 2), dtype=np.int32)
    n = k + 2
    for s in range(nstripes):
        if kind == "any":
            a = d.below(n)
            b = d.below(n - 1)
            b += b >= a
            pair = (min(a, b), max(a, b))
        elif kind == "dd":
            if k < 2:
                raise ValueError("dd needs k >= 2")
            a = d.below(k)
            b = d.below(k - 1)
            b += b >= a
            pair = (min(a, b), max(a, b))
        elif kind == "dp":
            pair = (d.below(k), k)
        elif kind == "dq":
            pair = (d.below(k), k + 1)
        elif kind == "pq":
            pair = (k, k + 1)
        elif kind == "d":
            pair = (d.below(k), -1)
        elif kind == "p":
            pair = (k, -1)
        elif kind == "q":
            pair = (k + 1, -1)
        else:  # any1
            pair = (d.below(n), -1)
        out[s] = pair
    return out


EXTENDED_ERASURE_KINDS = ("dd_mixed", "dd_ext", "dp_ext", "dq_ext")


def erasures_extended(seed: int, nstripes: int, k: int, p: int, kind: str) -> np.ndarray:
    """Erasure pairs of one class of a stripe with extended Q parity
    (``p < k <= 2p-1``; strips ``t >= p`` are the extended ones), shape
    ``(nstripes, 2)`` int32, sorted:

    * ``dd_mixed``: data ``x < p`` and extended data ``y >= p``, uniform.
    * ``dd_ext``: two extended data strips, uniform (needs ``k >= p+2``).
    * ``dp_ext`` / ``dq_ext``: an extended data strip, uniform, plus P / Q.
    """
    if kind not in EXTENDED_ERASURE_KINDS:
        raise ValueError(f"unknown extended erasure kind {kind!r}")
    if not p < k <= 2 * p - 1:
        raise ValueError("needs p < k <= 2p-1")
    d = Draws(seed, TAG_ERASURE, 64 + EXTENDED_ERASURE_KINDS.index(kind))
    m = k - p                         # extended strips p .. k-1
    out = np.empty((nstripes, 2), dtype=np.int32)
    for s in range(nstripes):
        if kind == "dd_mixed":
            pair = (d.below(p), p + d.below(m))
        elif kind == "dd_ext":
            if m < 2:
                raise ValueError("dd_ext needs two extended strips")
            a = d.below(m)
            b = d.below(m - 1)
            b += b >= a
            pair = (p + min(a, b), p + max(a, b))
        elif kind == "dp_ext":
            pair = (p + d.below(m), k)
        else:
            pair = (p + d.below(m), k + 1)
        out[s] = pair
    return out


# ---------------------------------------------------------------------------
# Mixed-geometry workloads (batched and served forms)
# ---------------------------------------------------------------------------

BATCH_PRIMES = (5, 11, 13, 19, 29, 37, 53)
SERVE_PRIMES = (11, 13, 29, 37)


@dataclass(frozen=True)
class StripeJob:
    """One stripe of a mixed batch.

    ``op`` is ``"encode"`` or ``"recover"``.  ``e0, e1`` are the erased strips
    of a recovery (``e1 = -1`` for a single erasure), else ``-1, -1``.
    """
    p: int
    k: int
    row_bytes: int
    op: str
    e0: int
    e1: int
    index: int


def _round16(x: float) -> int:
    return max(16, int(math.ceil(x / 16.0)) * 16)


def batch_jobs(seed: int, n: int, primes=BATCH_PRIMES, w_lo: int = 512, w_hi: int = 65536,
               encode_frac: float = 0.6) -> list[StripeJob]:
    """Mixed stripes: p uniform over ``primes``, k uniform in [2, p-1], row size
    log-uniform over [w_lo, w_hi] rounded up to a multiple of 16, a fraction
    ``encode_frac`` encodes and the rest two-erasure recoveries with the pair
    uniform over all C(k+2, 2) strip pairs."""
    d = Draws(seed, TAG_GEOMETRY, 0)
    jobs = []
    for i in range(n):
        p = primes[d.below(len(primes))]
        k = d.between(2, p - 1)
        w = min(w_hi, _round16(d.log_uniform(w_lo, w_hi)))
        if d.unit() < encode_frac:
            jobs.append(StripeJob(p, k, w, "encode", -1, -1, i))
        else:
            a = d.below(k + 2)
            b = d.below(k + 1)
            b += b >= a
            jobs.append(StripeJob(p, k, w, "recover", min(a, b), max(a, b), i))
    return jobs


@dataclass(frozen=True)
class Request:
    """One request of a served stream.

    ``kind`` is ``"write"`` (encode a new stripe) or ``"read"`` (degraded read
    of a resident stripe: recover ``e0`` and, if ``e1 >= 0``, ``e1``).
    ``target`` is, for a read, the index of the earlier write it reads.
    """
    index: int
    arrival_s: float
    kind: str
    p: int
    k: int
    row_bytes: int
    payload: int
    e0: int
    e1: int
    target: int


def serve_requests(seed: int, n: int, qps: float, primes=SERVE_PRIMES, pay_lo: int = 4096,
                   pay_hi: int = 4 << 20, write_frac: float = 0.6,
                   warm_writes: int = 16) -> list[Request]:
    """An open-loop Poisson request stream.

    Writes carry a payload log-uniform over [pay_lo, pay_hi] bytes on a stripe
    with p uniform over ``primes`` and k = p-1; the row size is the smallest
    multiple of 16 that holds the payload.  Reads target a uniformly chosen
    earlier write and erase one or two strips (50/50), at least one of them a
    data strip.  The first ``warm_writes`` requests are writes.
    """
    d = Draws(seed, TAG_ARRIVAL, 0)
    t = 0.0
    out: list[Request] = []
    writes: list[int] = []
    for i in range(n):
        t += d.exponential(qps)
        is_write = i < warm_writes or not writes or d.unit() < write_frac
        if is_write:
            p = primes[d.below(len(primes))]
            k = p - 1
            payload = int(d.log_uniform(pay_lo, pay_hi))
            w = _round16(payload / (k * (p - 1)))
            out.append(Request(i, t, "write", p, k, w, payload, -1, -1, -1))
            writes.append(i)
        else:
            tgt = writes[d.below(len(writes))]
            src = out[tgt]
            k = src.k
            e0 = d.below(k)
            if d.unit() < 0.5:
                e1 = -1
            else:
                e1 = d.below(k + 1)
                e1 += e1 >= e0
                e0, e1 = min(e0, e1), max(e0, e1)
            out.append(Request(i, t, "read", src.p, k, src.row_bytes, src.payload, e0, e1, tgt))
    return out

"""Device layout of many stripes of one geometry in a single torch tensor.

A batch is a contiguous uint8 tensor of shape ``(nstripes, k+2, p-1, W)``:
stripe ``s`` at byte ``s*(k+2)*(p-1)*W``, strip ``j`` of it at
``j*(p-1)*W`` (data 0..k-1, then P, then Q), row ``r`` at ``r*W``.  These
are the strides the strided entry points take.
"""

from __future__ import annotations

from dataclasses import dataclass

from . import _lib


@dataclass
class StripeBatch:
    p: int
    k: int
    row_bytes: int
    nstripes: int
    tensor: object  # torch.Tensor (uint8, device)

    @classmethod
    def empty(cls, p: int, k: int, row_bytes: int, nstripes: int, device="cuda"):
        import torch
        t = torch.empty((nstripes, k + 2, p - 1, row_bytes), dtype=torch.uint8, device=device)
        return cls(p, k, row_bytes, nstripes, t)

    @property
    def strip_stride(self) -> int:
        return (self.p - 1) * self.row_bytes

    @property
    def stripe_stride(self) -> int:
        return (self.k + 2) * self.strip_stride

    @property
    def user_bytes(self) -> int:
        return self.nstripes * self.k * self.strip_stride

    def encode(self, stream=None, first: int = 0, count: int | None = None):
        n = self.nstripes - first if count is None else count
        base = self.tensor.data_ptr() + first * self.stripe_stride
        return _lib.raid6c_encode_n(self.p, self.k, self.row_bytes, base, self.strip_stride,
                                    self.stripe_stride, n, stream)

    def recover(self, erasures, bad_count=None, stream=None, first: int = 0, count: int | None = None):
        """``erasures``: device int32 tensor ``(nstripes, 2)`` of erased strip pairs."""
        n = self.nstripes - first if count is None else count
        base = self.tensor.data_ptr() + first * self.stripe_stride
        eptr = erasures.data_ptr() + first * 8
        return _lib.raid6c_recover_n(self.p, self.k, self.row_bytes, base, self.strip_stride,
                                     self.stripe_stride, n, eptr, bad_count, stream)

    def autotune(self, op: int, erasures=None, reps: int = 20, stream=None) -> float:
        """Record the fastest launch configuration for this geometry (op 0 encode, 1 recovery)."""
        return _lib.raid6c_autotune_n(self.p, self.k, self.row_bytes, self.tensor.data_ptr(), self.strip_stride,
                                      self.stripe_stride, self.nstripes, op, erasures, reps, stream)

    def update(self, targets, src, src_stride=None, bad_count=None, stream=None):
        """Small writes: stripe s replaces data strip targets[s] (device int32)
        with the strip at ``src`` + s*src_stride; P and Q follow."""
        ss = self.strip_stride if src_stride is None else src_stride
        return _lib.raid6c_update_n(self.p, self.k, self.row_bytes, self.tensor.data_ptr(), self.strip_stride,
                                    self.stripe_stride, self.nstripes, targets, src, ss, bad_count, stream)

    def rs_encode(self, stream=None):
        """Reed-Solomon GF(256) P+Q over the same bytes (each strip a byte vector)."""
        return _lib.raid6c_rs_encode_n(self.k, self.strip_stride, self.tensor.data_ptr(), self.strip_stride,
                                       self.stripe_stride, self.nstripes, stream)

    def rs_recover(self, erasures, bad_count=None, stream=None):
        """Reed-Solomon recovery of the per-stripe erasures (device int32 (n, 2))."""
        return _lib.raid6c_rs_recover_n(self.k, self.strip_stride, self.tensor.data_ptr(), self.strip_stride,
                                        self.stripe_stride, self.nstripes, erasures, bad_count, stream)

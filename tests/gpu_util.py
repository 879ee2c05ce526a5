"""Helpers of the GPU tests: device set-up that fails loudly, host<->device copies."""

import numpy as np
import pytest


def device():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_cs_0611109_amd as r
    r.load()          # raises when libraid6c.so is missing: no fallback
    return torch.device("cuda:0")


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def to_host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def log(msg: str) -> None:
    print(msg, flush=True)

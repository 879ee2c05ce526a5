"""GPU parity of the conversion between the paper's horizontal Z_17 layout
(Section 4.5, one codeword per int16) and the vertical layout, and of the
pipeline convert -> encode -> convert back against the paper's packed
encode routine in the oracle."""

import numpy as np
import pytest

import datagen
import paper_cs_0611109_amd as r
from gpu_util import device, log, to_dev, to_host
from oracle import z17_layout as z

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _dev():
    device()


def _words(n_strips, w, seed):
    return datagen.random_bytes(seed, 9, 0, n_strips * 16 * w).view(np.uint16).reshape(n_strips, 8 * w)


@pytest.mark.parametrize("w,count", [(16, 1), (48, 3), (4096 + 16, 2), (1024, 64)])
def test_conversion_matches_oracle(w, count):
    import torch
    log(f"z17 conversion W={w} count={count}")
    words = _words(count, w, seed=w + count)
    want_v = z.to_vertical(words)                                  # (count, 16, w)
    out_v = torch.empty((count, 16, w), dtype=torch.uint8, device="cuda:0")
    out_v.fill_(0x5A)
    r.raid6c_z17_to_vertical(to_dev(words.view(np.int16)), w, count, out_v)
    assert np.array_equal(to_host(out_v), want_v)
    # 4 KiB past the output must stay untouched (the last work-group may be
    # partial).
    guard = 2048
    out_g = torch.empty(count * 8 * w + guard, dtype=torch.int16, device="cuda:0")
    out_g.fill_(0x5A5A)
    out_h = out_g[:count * 8 * w].view(count, 8 * w)
    r.raid6c_z17_to_horizontal(out_v, w, count, out_h)
    got = to_host(out_g).view(np.uint16)
    assert np.array_equal(got[:count * 8 * w].reshape(count, 8 * w), words)
    assert np.all(got[count * 8 * w:] == 0x5A5A)


def test_pipeline_equals_packed_encode():
    # Horizontal data strips -> vertical -> Z_17 encode on the GPU -> P, Q back
    # to horizontal == the Section 4.5 loop on the packed words.
    import torch
    k, w, n = 16, 1024, 8
    words = _words(n * k, w, seed=77).reshape(n, k, 8 * w)
    P, Q = z.encode_packed(words)
    stripes = torch.empty((n, k + 2, 16, w), dtype=torch.uint8, device="cuda:0")
    stripes.fill_(0xEE)
    hw = to_dev(words.view(np.int16))
    for s in range(n):
        r.raid6c_z17_to_vertical(hw[s], w, k, stripes[s, :k])
    r.raid6c_encode_n(17, k, w, stripes, 16 * w, (k + 2) * 16 * w, n)
    back = torch.empty((n, 2, 8 * w), dtype=torch.int16, device="cuda:0")
    for s in range(n):
        r.raid6c_z17_to_horizontal(stripes[s, k:], w, 2, back[s])
    got = to_host(back).view(np.uint16)
    assert np.array_equal(got[:, 0], P) and np.array_equal(got[:, 1], Q)

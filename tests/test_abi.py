"""Host-side checks of the C ABI: every declared symbol is exported, and bad
arguments are rejected before any device work (no GPU needed)."""

import ctypes
import os
import re

import pytest

import paper_cs_0611109_amd as r

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "raid6c.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(raid6c_\w+)\s*\(", text)))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ["raid6c_encode", "raid6c_recover_1", "raid6c_recover_2", "raid6c_encode_n",
              "raid6c_recover_n", "raid6c_rs_encode_n", "raid6c_strerror"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(r.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_cs_0611109_amd import _lib
    missing = [n for n in declared_functions() if n not in _lib.SIGNATURES]
    assert not missing, missing


def test_prime_support():
    assert r.raid6c_max_prime() >= 53
    for p in range(0, 80):
        odd_prime = p >= 3 and p % 2 == 1 and all(p % d for d in range(3, int(p ** 0.5) + 1, 2))
        assert r.raid6c_is_supported_prime(p) == (odd_prime and p <= r.raid6c_max_prime())
        assert (r.raid6c_vec_mask(p) != 0) == r.raid6c_is_supported_prime(p)


def test_max_data_strips_follows_theorem_333():
    # 2p-1 data strips exactly where the extended cone exists (the oracle's
    # reading of Theorem 3.3.3): every supported prime but 3, 7 and 31.
    from oracle import ring
    for p in range(3, r.raid6c_max_prime() + 1, 2):
        if not r.raid6c_is_supported_prime(p):
            continue
        want = 2 * p - 1 if ring.extension_ok(p) else p
        assert r.raid6c_max_data_strips(p) == want, p
    assert [p for p in range(3, 62, 2) if r.raid6c_is_supported_prime(p) and r.raid6c_max_data_strips(p) == p] \
        == [3, 7, 31]
    _err(r.raid6c_max_data_strips, 9)
    _err(r.raid6c_max_data_strips, 67, code=r.RAID6C_E_UNSUPPORTED)


def _err(fn, *args, code=r.RAID6C_E_ARG, **kw):
    with pytest.raises(r.Raid6cError) as ei:
        fn(*args, **kw)
    assert ei.value.code == code, str(ei.value)
    assert r.raid6c_last_error()


FAKE = 1 << 40  # a 16-byte-aligned address that is never dereferenced


def test_encode_n_argument_checks():
    ok = dict(p=5, k=4, row_bytes=64, base=FAKE, strip_stride=256, stripe_stride=6 * 256, nstripes=2, stream=0)

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return r.raid6c_encode_n(a["p"], a["k"], a["row_bytes"], a["base"], a["strip_stride"],
                                 a["stripe_stride"], a["nstripes"], stream=a["stream"])

    _err(call, p=9)
    _err(call, p=2)
    _err(call, p=67, code=r.RAID6C_E_UNSUPPORTED)
    _err(call, k=0)
    _err(call, k=10, stripe_stride=12 * 256)      # k > 2p-1
    _err(call, p=7, k=8, row_bytes=16, strip_stride=96, stripe_stride=10 * 96)   # p = 7: no extended parity
    _err(call, row_bytes=0)
    _err(call, row_bytes=24)
    _err(call, base=0)
    _err(call, base=FAKE + 8)
    _err(call, strip_stride=255)
    _err(call, strip_stride=240)
    _err(call, stripe_stride=6 * 256 - 16)
    _err(call, row_bytes=1 << 29, strip_stride=4 << 29, stripe_stride=24 << 29)   # strip >= 2 GiB
    assert call(nstripes=0) == 0          # empty call: no device work


def test_recover_argument_checks():
    strips = [FAKE + i * 4096 for i in range(6)]
    _err(r.raid6c_recover_2, 5, 4, 64, strips, 1, 1, stream=0)
    _err(r.raid6c_recover_2, 5, 4, 64, strips, 0, 6, stream=0)
    _err(r.raid6c_recover_2, 5, 4, 64, strips, -1, 2, stream=0)
    _err(r.raid6c_recover_1, 5, 4, 64, strips, 6, stream=0)
    _err(r.raid6c_recover_1, 5, 4, 64, strips, -1, stream=0)
    overlapping = [FAKE + i * 128 for i in range(6)]          # strips are 256 bytes
    _err(r.raid6c_recover_2, 5, 4, 64, overlapping, 0, 1, stream=0)
    misaligned = list(strips)
    misaligned[3] += 4
    _err(r.raid6c_recover_1, 5, 4, 64, misaligned, 0, stream=0)
    _err(r.raid6c_recover_n, 5, 4, 64, FAKE, 256, 1536, 4, 0, stream=0)       # NULL erasures
    _err(r.raid6c_recover_n, 5, 4, 64, FAKE, 256, 1536, 4, FAKE + 2, stream=0)


def test_encode_single_argument_checks():
    data = [FAKE + i * 4096 for i in range(4)]
    _err(r.raid6c_encode, 5, 4, 64, data, FAKE + 4 * 4096, FAKE + 4 * 4096, stream=0)   # P == Q
    _err(r.raid6c_encode, 5, 4, 64, data, 0, FAKE + 5 * 4096, stream=0)
    _err(r.raid6c_encode, 7, 4, 64, data[:3] + [FAKE + 2 * 4096 + 64], FAKE + 4 * 4096, FAKE + 5 * 4096,
         stream=0)


def test_update_argument_checks():
    strips = [FAKE + i * 4096 for i in range(6)]
    new = FAKE + 100 * 4096
    _err(r.raid6c_update, 5, 4, 64, strips, 4, new, stream=0)            # t = P
    _err(r.raid6c_update, 5, 4, 64, strips, -1, new, stream=0)
    _err(r.raid6c_update, 5, 4, 64, strips, 1, strips[4] + 64, stream=0)   # new overlaps P
    _err(r.raid6c_update, 5, 4, 64, strips, 1, 0, stream=0)
    _err(r.raid6c_update, 5, 4, 24, strips, 1, new, stream=0)
    _err(r.raid6c_update_n, 5, 4, 64, FAKE, 256, 1536, 4, 0, new, 256, stream=0)        # NULL targets
    _err(r.raid6c_update_n, 5, 4, 64, FAKE, 256, 1536, 4, FAKE + 2, new, 256, stream=0)
    _err(r.raid6c_update_n, 5, 4, 64, FAKE, 256, 1536, 4, FAKE, 0, 256, stream=0)       # NULL src
    _err(r.raid6c_update_n, 5, 4, 64, FAKE, 256, 1536, 4, FAKE, new, 128, stream=0)     # src stride
    assert r.raid6c_update_n(5, 4, 64, FAKE, 256, 1536, 0, 0, 0, 0, stream=0) == 0      # empty call


def test_z17_argument_checks():
    _err(r.raid6c_z17_to_vertical, FAKE, 24, 1, FAKE + (1 << 20), stream=0)          # row bytes
    _err(r.raid6c_z17_to_vertical, FAKE + 8, 64, 1, FAKE + (1 << 20), stream=0)      # alignment
    _err(r.raid6c_z17_to_vertical, FAKE, 64, 4, FAKE + 1024, stream=0)               # overlap
    _err(r.raid6c_z17_to_horizontal, 0, 64, 1, FAKE, stream=0)
    assert r.raid6c_z17_to_vertical(FAKE, 64, 0, FAKE, stream=0) == 0                 # empty call


def test_rs_argument_checks():
    _err(r.raid6c_rs_encode_n, 0, 64, FAKE, 64, 64 * 4, 1, stream=0)
    _err(r.raid6c_rs_encode_n, 256, 64, FAKE, 64, 64 * 258, 1, stream=0)
    _err(r.raid6c_rs_encode_n, 4, 40, FAKE, 48, 48 * 6, 1, stream=0)
    _err(r.raid6c_rs_encode_n, 4, 64, FAKE, 48, 64 * 6, 1, stream=0)
    assert r.raid6c_rs_encode_n(4, 64, FAKE, 64, 64 * 6, 0, stream=0) == 0


def test_tuning_table():
    r.raid6c_tune_clear()
    d0 = r.raid6c_tune_get(13, 0, 4096)
    assert d0[0] in (1, 2, 4) and d0[1] in (1, 2, 4) and d0[2] in (64, 128, 256) and d0[3] in (1, 2, 4)
    assert d0[4] in (0, 1)
    r.raid6c_tune_set(13, 0, 4096, 1, 2, 128)
    assert r.raid6c_tune_get(13, 0, 4096) == (1, 2, 128, 1, 0)
    assert r.raid6c_tune_get(13, 0, 4096 + 2048) == (1, 2, 128, 1, 0)     # same power-of-two bucket
    assert r.raid6c_tune_get(13, 0, 8192) == d0 or r.raid6c_tune_get(13, 0, 8192) != (1, 2, 128, 1, 0)
    r.raid6c_tune_set(13, 1, 4096, 2, 1, 256, 4, 1)
    assert r.raid6c_tune_get(13, 1, 4096) == (2, 1, 256, 4, 1)
    # the extended-parity slots are separate entries
    r.raid6c_tune_set(13, 3, 4096, 1, 1, 64)
    assert r.raid6c_tune_get(13, 3, 4096) == (1, 1, 64, 1, 0)
    assert r.raid6c_tune_get(13, 1, 4096) == (2, 1, 256, 4, 1)
    r.raid6c_tune_clear()
    assert r.raid6c_tune_get(13, 0, 4096) == d0
    _err(r.raid6c_tune_set, 9, 0, 64, 1, 1, 64)
    _err(r.raid6c_tune_set, 53, 0, 64, 4, 1, 64)     # vec 4 not built for large p
    _err(r.raid6c_tune_set, 53, 0, 64, 2, 2, 64)     # (2*53-1)*2 + 2*52*2 = 418 registers > 400
    _err(r.raid6c_tune_set, 13, 4, 64, 1, 1, 64)      # op 0..3
    _err(r.raid6c_tune_set, 13, 0, 64, 1, 1, 96)
    _err(r.raid6c_tune_set, 13, 0, 64, 1, 3, 64)
    _err(r.raid6c_tune_set, 13, 0, 64, 2, 1, 128, 4)   # split 4 needs 256 threads
    _err(r.raid6c_tune_set, 13, 0, 64, 2, 1, 256, 3)   # no split 3
    _err(r.raid6c_tune_set, 61, 0, 64, 1, 1, 256, 4)   # partials of 4 waves exceed 64 KiB of LDS at p = 61
    _err(r.raid6c_tune_set, 13, 0, 64, 1, 1, 64, 1, 3)  # order 0, 1 or 2


def test_built_configurations():
    for p in range(3, r.raid6c_max_prime() + 1):
        if not r.raid6c_is_supported_prime(p):
            assert r.raid6c_unroll_mask(p, 1) == 0
            assert r.raid6c_split_mask(p, 1) == 0
            continue
        assert r.raid6c_unroll_mask(p, 1) & 1            # (vec 1, unroll 1) always built
        for v in (1, 2, 4):
            m = r.raid6c_unroll_mask(p, v)
            assert (m != 0) <= bool(r.raid6c_vec_mask(p) & v)
            # (vec, unroll) is built when its registers ((2p-1)v accumulators and
            # unroll*(p-1)*v loads) fit in a 400-VGPR budget
            for u in (1, 2, 4):
                fits = (2 * p - 1) * v + u * (p - 1) * v <= 400
                assert bool(m & u) == (fits and bool(r.raid6c_vec_mask(p) & v)), (p, v, u)
            # split s is built exactly when s waves' partials (2p-1 rows of 64*v dwords) fit in 64 KiB
            for sp in (2, 4):
                fits = sp * (2 * p - 1) * 64 * v * 4 <= 65536
                assert bool(r.raid6c_split_mask(p, v) & sp) == (fits and m != 0), (p, v, sp)
        v, u, t, sp, order = r.raid6c_tune_get(p, 1, 1024)
        assert order in (0, 1, 2)
        assert r.raid6c_unroll_mask(p, v) & u
        assert sp == 1 or (r.raid6c_split_mask(p, v) & sp and t == 64 * sp)

def test_plan_rejects_bad_jobs_before_device_work():
    J = r.raid6c_job
    good = J(0, 5, 4, -1, -1, 64, 256, FAKE)
    cases = [
        J(0, 9, 4, -1, -1, 64, 256, FAKE),            # not prime
        J(0, 5, 10, -1, -1, 64, 256, FAKE),           # k > 2p-1
        J(0, 5, 4, -1, -1, 24, 256, FAKE),            # row bytes
        J(0, 5, 4, -1, -1, 64, 255, FAKE),            # stride
        J(0, 5, 4, -1, -1, 64, 256, FAKE + 8),        # alignment
        J(1, 5, 4, 2, 2, 64, 256, FAKE),              # equal erasures
        J(1, 5, 4, -1, -1, 64, 256, FAKE),            # recover without erasure
        J(3, 5, 4, -1, -1, 64, 256, FAKE),            # unknown op
    ]
    for bad in cases:
        _err(r.raid6c_plan_create, [bad])
        _err(r.raid6c_plan_create, [good, bad])
    _err(r.raid6c_plan_create, [J(0, 67, 4, -1, -1, 64, 66 * 64, FAKE)], code=r.RAID6C_E_UNSUPPORTED)
    # k > p only where the prime has the extended Q parity (7 fails Theorem 3.3.3)
    _err(r.raid6c_plan_create, [J(0, 7, 8, -1, -1, 64, 384, FAKE)])
    # two jobs sharing bytes
    _err(r.raid6c_plan_create, [J(0, 5, 4, -1, -1, 64, 256, FAKE), J(0, 5, 4, -1, -1, 64, 256, FAKE + 1024)])


def test_noalloc_rejects_bad_calls_before_device_work():
    J = r.raid6c_job
    good = J(0, 5, 4, -1, -1, 64, 256, FAKE)
    for bad in (J(0, 9, 4, -1, -1, 64, 256, FAKE), J(0, 5, 10, -1, -1, 64, 256, FAKE),
                J(0, 7, 8, -1, -1, 64, 384, FAKE), J(1, 5, 4, 2, 2, 64, 256, FAKE)):
        _err(r.raid6c_run_jobs_noalloc, [good, bad], stream=0)
    _err(r.raid6c_run_jobs_noalloc, [good] * (r.RAID6C_NOALLOC_MAX_JOBS + 1), stream=0)
    wide = J(0, 3, 1, -1, -1, 65536, 2 * 65536, FAKE)                   # 128 tiles of 512 bytes
    _err(r.raid6c_run_jobs_noalloc, [wide] * (r.RAID6C_NOALLOC_MAX_ITEMS // 128 + 1), stream=0)
    assert r.raid6c_run_jobs_noalloc([], stream=0) == 0


def test_server_rejects_bad_configurations_before_device_work():
    # Checked before the store is allocated: no device is touched.
    _err(r.raid6c_server_create, 1024)                                   # store below 4096 bytes
    _err(r.raid6c_server_create, 1 << 20, max_inflight=0)
    _err(r.raid6c_server_create, 1 << 20, max_inflight=65)
    _err(r.raid6c_server_create, 1 << 20, max_batch=0)
    _err(r.raid6c_server_create, 1 << 20, max_batch=65537)
    _err(r.raid6c_server_create, 1 << 20, waves_per_cu=33)
    cfg = r.raid6c_server_config(1 << 20, 4, 64, 0, 0, 2)             # persistent must be 0 or 1
    out = ctypes.c_void_p()
    assert r.load().raid6c_server_create(ctypes.byref(cfg), ctypes.byref(out)) == r.RAID6C_E_ARG
    assert not out.value and r.raid6c_last_error()


def test_built_in_launch_rule():
    # With no tuned entry: split-K with vec 2 where built and the row holds a
    # tile; above p = 31 vec 2, one strip per batch, on rows of whole
    # 512-byte tiles (largest work-group whose tile divides the row);
    # otherwise the most loads in flight, up to 256 threads as the row allows.
    r.raid6c_tune_clear()
    assert r.raid6c_tune_get(13, 1, 4096) == (2, 1, 256, 4, 0)
    assert r.raid6c_tune_get(29, 0, 1024) == (2, 1, 128, 2, 0)
    assert r.raid6c_tune_get(53, 0, 2048) == (2, 1, 256, 1, 0)
    assert r.raid6c_tune_get(53, 1, 512) == (2, 1, 64, 1, 0)
    assert r.raid6c_tune_get(37, 0, 1024) == (2, 1, 128, 1, 0)
    assert r.raid6c_tune_get(53, 3, 13312) == (2, 1, 128, 1, 0)      # extended slots follow the same rule
    v, u, t, sp, o = r.raid6c_tune_get(53, 0, 2064)                   # ragged last tile: not vec 2
    assert v == 1 and sp == 1 and t == 256
    v, u, t, sp, o = r.raid6c_tune_get(61, 0, 16)                     # 4 lanes of work: one wave
    assert sp == 1 and t == 64

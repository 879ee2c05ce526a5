"""ctypes binding of libraid6c.so (the C ABI declared in include/raid6c.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Device buffers are passed as integers (device
addresses) or as torch tensors, streams as ``hipStream_t`` integers or torch
streams; ``None`` selects torch's current stream on the current device.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libraid6c.so")

RAID6C_OK = 0
RAID6C_E_ARG = -1
RAID6C_E_UNSUPPORTED = -2
RAID6C_E_HIP = -3
RAID6C_E_NOMEM = -4
RAID6C_E_STATE = -5

_c_int, _c_size, _vp = ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p
_i32p = ctypes.c_void_p

# name -> (restype, argtypes); mirrors include/raid6c.h.
SIGNATURES = {
    "raid6c_max_prime": (_c_int, []),
    "raid6c_is_supported_prime": (_c_int, [_c_int]),
    "raid6c_max_data_strips": (_c_int, [_c_int]),
    "raid6c_strerror": (ctypes.c_char_p, [_c_int]),
    "raid6c_last_error": (ctypes.c_char_p, []),
    "raid6c_encode": (_c_int, [_c_int, _c_int, _c_size, ctypes.POINTER(_vp), _vp, _vp, _vp]),
    "raid6c_recover_1": (_c_int, [_c_int, _c_int, _c_size, ctypes.POINTER(_vp), _c_int, _vp]),
    "raid6c_recover_2": (_c_int, [_c_int, _c_int, _c_size, ctypes.POINTER(_vp), _c_int, _c_int, _vp]),
    "raid6c_encode_n": (_c_int, [_c_int, _c_int, _c_size, _vp, _c_size, _c_size, _c_size, _vp]),
    "raid6c_recover_n": (_c_int, [_c_int, _c_int, _c_size, _vp, _c_size, _c_size, _c_size, _i32p, _i32p, _vp]),
    "raid6c_rs_encode_n": (_c_int, [_c_int, _c_size, _vp, _c_size, _c_size, _c_size, _vp]),
    "raid6c_rs_recover_n": (_c_int, [_c_int, _c_size, _vp, _c_size, _c_size, _c_size, _vp, _vp, _vp]),
    "raid6c_rs_set_config": (_c_int, [_c_int, _c_int, _c_int]),
    "raid6c_z17_to_vertical": (_c_int, [_vp, _c_size, _c_size, _vp, _vp]),
    "raid6c_z17_to_horizontal": (_c_int, [_vp, _c_size, _c_size, _vp, _vp]),
    "raid6c_update": (_c_int, [_c_int, _c_int, _c_size, _vp, _c_int, _vp, _vp]),
    "raid6c_update_n": (_c_int, [_c_int, _c_int, _c_size, _vp, _c_size, _c_size, _c_size, _vp, _vp, _c_size, _vp,
                                 _vp]),
    "raid6c_write": (_c_int, [_c_int, _c_int, _c_size, _vp, _c_size, ctypes.POINTER(_vp), _vp]),
    "raid6c_read_degraded": (_c_int, [_c_int, _c_int, _c_size, ctypes.POINTER(_vp), _c_int, _c_int, _vp, _vp]),
    "raid6c_vec_mask": (_c_int, [_c_int]),
    "raid6c_unroll_mask": (_c_int, [_c_int, _c_int]),
    "raid6c_tune_set": (_c_int, [_c_int, _c_int, _c_size, _c_int, _c_int, _c_int, _c_int, _c_int]),
    "raid6c_split_mask": (_c_int, [_c_int, _c_int]),
    "raid6c_tune_get": (_c_int, [_c_int, _c_int, _c_size, ctypes.POINTER(_c_int), ctypes.POINTER(_c_int),
                                 ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), ctypes.POINTER(_c_int)]),
    "raid6c_tune_clear": (None, []),
    "raid6c_autotune_n": (_c_int, [_c_int, _c_int, _c_size, _vp, _c_size, _c_size, _c_size, _c_int, _vp, _c_int,
                                   _vp, ctypes.POINTER(ctypes.c_float)]),
    "raid6c_plan_create": (_c_int, [_vp, _c_size, _vp]),
    "raid6c_plan_run": (_c_int, [_vp, _vp]),
    "raid6c_plan_get_schedule": (_c_int, [_vp, _vp]),
    "raid6c_plan_set_schedule": (_c_int, [_vp, _vp]),
    "raid6c_plan_stats": (_c_int, [_vp, _vp]),
    "raid6c_plan_autotune": (_c_int, [_vp, _vp, _c_int, ctypes.POINTER(ctypes.c_float)]),
    "raid6c_plan_destroy": (_c_int, [_vp]),
    "raid6c_run_jobs": (_c_int, [_vp, _c_size, _vp]),
    "raid6c_run_jobs_noalloc": (_c_int, [_vp, _c_size, _vp]),
    "raid6c_server_create": (_c_int, [_vp, _vp]),
    "raid6c_server_submit": (_c_int, [_vp, _vp, _c_size]),
    "raid6c_server_poll": (_c_int, [_vp, _vp, _c_size, ctypes.POINTER(_c_size)]),
    "raid6c_server_wait_idle": (_c_int, [_vp]),
    "raid6c_server_replay": (_c_int, [_vp, _vp, _vp, _c_size, _vp]),
    "raid6c_server_get_stats": (_c_int, [_vp, _vp]),
    "raid6c_server_stripe": (_c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_uint64)]),
    "raid6c_server_destroy": (_c_int, [_vp]),
}



class raid6c_job(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("p", ctypes.c_int32), ("k", ctypes.c_int32),
                ("e0", ctypes.c_int32), ("e1", ctypes.c_int32), ("row_bytes", ctypes.c_uint32),
                ("strip_stride", ctypes.c_uint64), ("base", ctypes.c_void_p)]


class raid6c_schedule(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_int32), ("chunk", ctypes.c_int32), ("order", ctypes.c_int32),
                ("grouped", ctypes.c_int32)]


class raid6c_plan_info(ctypes.Structure):
    _fields_ = [("njobs", ctypes.c_uint64), ("nitems", ctypes.c_uint64), ("bytes_moved", ctypes.c_uint64),
                ("user_bytes", ctypes.c_uint64), ("max_p", ctypes.c_int32), ("grid", ctypes.c_int32)]


class raid6c_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("p", ctypes.c_int32), ("k", ctypes.c_int32), ("e0", ctypes.c_int32),
                ("e1", ctypes.c_int32), ("row_bytes", ctypes.c_uint32), ("stripe_id", ctypes.c_uint64),
                ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("tag", ctypes.c_uint64)]


class raid6c_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("arrival_ns", ctypes.c_uint64), ("launch_ns", ctypes.c_uint64), ("complete_ns", ctypes.c_uint64)]


class raid6c_server_config(ctypes.Structure):
    _fields_ = [("store_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("plain", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32), ("persistent", ctypes.c_int32)]


class raid6c_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("evictions", ctypes.c_uint64), ("user_bytes", ctypes.c_uint64), ("resident", ctypes.c_uint64),
                ("store_used", ctypes.c_uint64), ("table_grows", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64),
                ("launch_ns", ctypes.c_uint64)]


RAID6C_REQ_WRITE = 0
RAID6C_REQ_READ = 1
RAID6C_ST_OK = 0
RAID6C_ST_NOT_RESIDENT = 1
RAID6C_ST_TOO_LARGE = 2
RAID6C_ST_INVALID = 3
RAID6C_ST_DUPLICATE = 4

RAID6C_JOB_ENCODE = 0
RAID6C_JOB_RECOVER = 1
RAID6C_ORDER_LARGEST_FIRST = 0
RAID6C_ORDER_BY_PRIME = 1
RAID6C_ORDER_SUBMITTED = 2

_lib = None


class Raid6cError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} (code {code})")
        self.code = code


def load(path: str = LIB_PATH):
    """Load the library (once) and declare the signatures.  Raises when the
    library has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_cs_0611109_amd/build.py`")
    # PyTorch carries its own HIP runtime.  Loading it first makes the
    # library bind to that same runtime (same soname), so the process has one
    # HIP runtime and one view of the device; loaded the other way round, the
    # library's runtime can report no device at all.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    raise TypeError(f"cannot take a device address of {type(x).__name__}")


def _stream(s) -> int | None:
    if s is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(s, int):
        return s
    if hasattr(s, "cuda_stream"):
        return int(s.cuda_stream)
    raise TypeError("stream must be None, an int handle or a torch stream")


def _check(rc: int) -> int:
    if rc != RAID6C_OK:
        lib = load()
        msg = (lib.raid6c_last_error() or b"").decode() or lib.raid6c_strerror(rc).decode()
        raise Raid6cError(rc, msg)
    return rc


def _ptr_array(items):
    arr = (_vp * len(items))()
    for i, it in enumerate(items):
        arr[i] = _ptr(it)
    return arr


def raid6c_max_prime() -> int:
    return load().raid6c_max_prime()


def raid6c_is_supported_prime(p: int) -> bool:
    return bool(load().raid6c_is_supported_prime(p))


def raid6c_max_data_strips(p: int) -> int:
    """2p-1 where the extended Q parity exists (Theorem 3.3.3), else p."""
    rc = load().raid6c_max_data_strips(p)
    if rc < 0:
        _check(rc)
    return rc


def raid6c_strerror(code: int) -> str:
    return load().raid6c_strerror(code).decode()


def raid6c_last_error() -> str:
    return (load().raid6c_last_error() or b"").decode()


def raid6c_encode(p, k, row_bytes, data, P, Q, stream=None):
    """``data``: sequence of k device strips; ``P``, ``Q``: device strips."""
    return _check(load().raid6c_encode(p, k, row_bytes, _ptr_array(list(data)), _ptr(P), _ptr(Q),
                                       _stream(stream)))


def raid6c_recover_1(p, k, row_bytes, strips, e, stream=None):
    """``strips``: sequence of k+2 device strips (D_0..D_{k-1}, P, Q)."""
    return _check(load().raid6c_recover_1(p, k, row_bytes, _ptr_array(list(strips)), e, _stream(stream)))


def raid6c_recover_2(p, k, row_bytes, strips, e0, e1, stream=None):
    return _check(load().raid6c_recover_2(p, k, row_bytes, _ptr_array(list(strips)), e0, e1,
                                          _stream(stream)))


def raid6c_write(p, k, row_bytes, src, src_strip_stride, strips, stream=None):
    """Copy a payload of k strips into ``strips[:k]`` and write P, Q (``strips[k:]``)."""
    return _check(load().raid6c_write(p, k, row_bytes, _ptr(src), src_strip_stride, _ptr_array(list(strips)),
                                      _stream(stream)))


def raid6c_read_degraded(p, k, row_bytes, strips, e0, e1, out, stream=None):
    """Rebuild erased strips into ``out`` (ascending strip order) without writing the stripe."""
    return _check(load().raid6c_read_degraded(p, k, row_bytes, _ptr_array(list(strips)), e0, e1, _ptr(out),
                                              _stream(stream)))


def raid6c_encode_n(p, k, row_bytes, base, strip_stride, stripe_stride, nstripes, stream=None):
    return _check(load().raid6c_encode_n(p, k, row_bytes, _ptr(base), strip_stride, stripe_stride,
                                         nstripes, _stream(stream)))


def raid6c_recover_n(p, k, row_bytes, base, strip_stride, stripe_stride, nstripes, erasures,
                     bad_count=None, stream=None):
    """``erasures``: device int32 array of 2*nstripes entries (second = -1 for one erasure)."""
    return _check(load().raid6c_recover_n(p, k, row_bytes, _ptr(base), strip_stride, stripe_stride,
                                          nstripes, _ptr(erasures), _ptr(bad_count), _stream(stream)))


def raid6c_rs_encode_n(k, strip_bytes, base, strip_stride, stripe_stride, nstripes, stream=None):
    return _check(load().raid6c_rs_encode_n(k, strip_bytes, _ptr(base), strip_stride, stripe_stride,
                                            nstripes, _stream(stream)))


def raid6c_rs_recover_n(k, strip_bytes, base, strip_stride, stripe_stride, nstripes, erasures,
                        bad_count=None, stream=None):
    return _check(load().raid6c_rs_recover_n(k, strip_bytes, _ptr(base), strip_stride, stripe_stride, nstripes,
                                             _ptr(erasures), _ptr(bad_count), _stream(stream)))


def raid6c_z17_to_vertical(words, row_bytes, count, strips, stream=None):
    """Horizontal Z_17 strips (one codeword per uint16) -> vertical strips."""
    return _check(load().raid6c_z17_to_vertical(_ptr(words), row_bytes, count, _ptr(strips), _stream(stream)))


def raid6c_z17_to_horizontal(strips, row_bytes, count, words, stream=None):
    return _check(load().raid6c_z17_to_horizontal(_ptr(strips), row_bytes, count, _ptr(words), _stream(stream)))


def raid6c_update(p, k, row_bytes, strips, t, new_strip, stream=None):
    """Small write: strip t of one stripe becomes ``new_strip``; P and Q follow."""
    return _check(load().raid6c_update(p, k, row_bytes, _ptr_array(list(strips)), t, _ptr(new_strip),
                                       _stream(stream)))


def raid6c_update_n(p, k, row_bytes, base, strip_stride, stripe_stride, nstripes, targets, src, src_stride,
                    bad_count=None, stream=None):
    return _check(load().raid6c_update_n(p, k, row_bytes, _ptr(base), strip_stride, stripe_stride, nstripes,
                                         _ptr(targets), _ptr(src), src_stride, _ptr(bad_count), _stream(stream)))


def raid6c_rs_set_config(vec: int, unroll: int, threads: int) -> int:
    return _check(load().raid6c_rs_set_config(vec, unroll, threads))


def raid6c_vec_mask(p: int) -> int:
    return load().raid6c_vec_mask(p)


def raid6c_unroll_mask(p: int, vec: int) -> int:
    return load().raid6c_unroll_mask(p, vec)


def raid6c_split_mask(p: int, vec: int) -> int:
    return load().raid6c_split_mask(p, vec)


def raid6c_tune_set(p, op, row_bytes, vec, unroll, threads, split=1, order=0):
    return _check(load().raid6c_tune_set(p, op, row_bytes, vec, unroll, threads, split, order))


def raid6c_tune_get(p, op, row_bytes):
    """(vec, unroll, threads, split, order) a call with these arguments would use."""
    v, u, t, sp, o = _c_int(), _c_int(), _c_int(), _c_int(), _c_int()
    _check(load().raid6c_tune_get(p, op, row_bytes, ctypes.byref(v), ctypes.byref(u), ctypes.byref(t),
                                  ctypes.byref(sp), ctypes.byref(o)))
    return v.value, u.value, t.value, sp.value, o.value


def raid6c_tune_clear():
    load().raid6c_tune_clear()


def raid6c_plan_create(jobs) -> int:
    """``jobs``: sequence of raid6c_job (or a ctypes array of them).  Returns
    the plan handle (an int); free it with raid6c_plan_destroy."""
    arr = jobs if isinstance(jobs, ctypes.Array) else (raid6c_job * len(jobs))(*jobs)
    out = _vp()
    _check(load().raid6c_plan_create(ctypes.cast(arr, _vp) if len(arr) else None, len(arr), ctypes.byref(out)))
    return out.value


def raid6c_plan_run(plan, stream=None):
    return _check(load().raid6c_plan_run(plan, _stream(stream)))


def raid6c_plan_get_schedule(plan) -> raid6c_schedule:
    s = raid6c_schedule()
    _check(load().raid6c_plan_get_schedule(plan, ctypes.byref(s)))
    return s


def raid6c_plan_set_schedule(plan, waves_per_cu, chunk, order, grouped=0):
    s = raid6c_schedule(waves_per_cu, chunk, order, grouped)
    return _check(load().raid6c_plan_set_schedule(plan, ctypes.byref(s)))


def raid6c_plan_stats(plan) -> raid6c_plan_info:
    i = raid6c_plan_info()
    _check(load().raid6c_plan_stats(plan, ctypes.byref(i)))
    return i


def raid6c_plan_autotune(plan, stream=None, reps=3) -> float:
    ms = ctypes.c_float()
    _check(load().raid6c_plan_autotune(plan, _stream(stream), reps, ctypes.byref(ms)))
    return ms.value


def raid6c_plan_destroy(plan):
    return _check(load().raid6c_plan_destroy(plan))


def raid6c_run_jobs(jobs, stream=None):
    """Every job as its own plain launch (the per-request path)."""
    arr = jobs if isinstance(jobs, ctypes.Array) else (raid6c_job * len(jobs))(*jobs)
    return _check(load().raid6c_run_jobs(ctypes.cast(arr, _vp) if len(arr) else None, len(arr), _stream(stream)))


def raid6c_run_jobs_noalloc(jobs, stream=None):
    """The jobs as a plan's grouped schedule runs them, tables staged in the
    library's fixed device array (nothing allocated)."""
    arr = jobs if isinstance(jobs, ctypes.Array) else (raid6c_job * len(jobs))(*jobs)
    return _check(load().raid6c_run_jobs_noalloc(ctypes.cast(arr, _vp) if len(arr) else None, len(arr),
                                                 _stream(stream)))


RAID6C_NOALLOC_MAX_JOBS = 4096
RAID6C_NOALLOC_MAX_ITEMS = 262144


def raid6c_autotune_n(p, k, row_bytes, base, strip_stride, stripe_stride, nstripes, op, erasures=None, reps=20,
                      stream=None) -> float:
    """Pick and record the configuration with the smallest median launch time;
    returns that median in ms."""
    ms = ctypes.c_float()
    _check(load().raid6c_autotune_n(p, k, row_bytes, _ptr(base), strip_stride, stripe_stride, nstripes, op,
                                    _ptr(erasures), reps, _stream(stream), ctypes.byref(ms)))
    return ms.value


def raid6c_server_create(store_bytes, max_inflight=4, max_batch=256, plain=False, waves_per_cu=0,
                         persistent=False) -> int:
    cfg = raid6c_server_config(store_bytes, max_inflight, max_batch, 1 if plain else 0, waves_per_cu,
                               1 if persistent else 0)
    out = _vp()
    _check(load().raid6c_server_create(ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def raid6c_server_submit(server, reqs):
    arr = reqs if isinstance(reqs, ctypes.Array) else (raid6c_request * len(reqs))(*reqs)
    return _check(load().raid6c_server_submit(server, ctypes.cast(arr, _vp) if len(arr) else None, len(arr)))


def raid6c_server_poll(server, cap=4096):
    out = (raid6c_completion * cap)()
    n = _c_size()
    _check(load().raid6c_server_poll(server, ctypes.cast(out, _vp), cap, ctypes.byref(n)))
    return list(out[:n.value])


def raid6c_server_wait_idle(server):
    return _check(load().raid6c_server_wait_idle(server))


def raid6c_server_replay(server, reqs, arrival_s):
    """Open-loop replay; returns the completions in request order."""
    n = len(reqs)
    arr = reqs if isinstance(reqs, ctypes.Array) else (raid6c_request * n)(*reqs)
    times = (ctypes.c_double * n)(*arrival_s)
    out = (raid6c_completion * n)()
    _check(load().raid6c_server_replay(server, ctypes.cast(arr, _vp), ctypes.cast(times, _vp), n,
                                       ctypes.cast(out, _vp)))
    return list(out)


def raid6c_server_get_stats(server) -> raid6c_server_stats:
    st = raid6c_server_stats()
    _check(load().raid6c_server_get_stats(server, ctypes.byref(st)))
    return st


def raid6c_server_stripe(server, stripe_id):
    """(device address of strip 0, strip stride) of a resident stripe."""
    base, stride = _vp(), ctypes.c_uint64()
    _check(load().raid6c_server_stripe(server, stripe_id, ctypes.byref(base), ctypes.byref(stride)))
    return base.value, stride.value


def raid6c_server_destroy(server):
    return _check(load().raid6c_server_destroy(server))

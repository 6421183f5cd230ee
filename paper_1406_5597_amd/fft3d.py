"""Python binding of libfft3d: the C entry points under the same names.

Argument marshalling only -- every step of the transforms runs in the HIP
kernels of ``libfft3d.so``.  Arrays are torch tensors on the GPU (or raw
device addresses as ints); streams are torch streams, raw ``hipStream_t``
ints, or None for torch's current stream.  If the library is not built this
module raises on import: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfft3d.so")

FFT3D_F32 = 0
FFT3D_F64 = 1
FFT3D_OK = 0
FFT3D_ERR_INVALID_ARG = -1
FFT3D_ERR_UNSUPPORTED = -2
FFT3D_ERR_NOMEM = -3
FFT3D_ERR_HIP = -4
FFT3D_ERR_BUDGET = -5
FFT3D_ERR_ALIGN = -6
FFT3D_ERR_BUSY = -7
FFT3D_R2C = 0
FFT3D_C2R = 1
FFT3D_ROUNDTRIP = 2
FFT3D_PLAN_HOST_ONLY = 1
FFT3D_PLAN_COOP_PLANE = 2
FFT3D_PLAN_TUNED = 4
FFT3D_TUNE_FUSED = 1
FFT3D_TUNE_SPLIT = 2
FFT3D_TUNE_COOP = 3
FFT3D_PASS_PLANE_R2C = 0
FFT3D_PASS_N1_FWD = 1
FFT3D_PASS_N0_FWD = 2
FFT3D_PASS_N0_INV = 3
FFT3D_PASS_N1_INV = 4
FFT3D_PASS_PLANE_C2R = 5
FFT3D_PASS_SWAP01 = 6
FFT3D_PASS_SWAP10 = 7
FFT3D_PASS_N0T_FWD = 8
FFT3D_PASS_N0T_INV = 9
FFT3D_BATCH_SEQUENTIAL = 2
FFT3D_BATCH_DIRECT = 4
FFT3D_SERVER_NO_DEVICE = 1
FFT3D_SERVER_MAX_COMP = 8

# Every symbol include/fft3d.h declares.
EXPORTS = (
    "fft3d_version", "fft3d_batch_submit_static", "fft3d_plan", "fft3d_plan_ex", "fft3d_plan_destroy", "fft3d_work_bytes",
    "fft3d_real_bytes", "fft3d_complex_bytes", "fft3d_r2c", "fft3d_c2r", "fft3d_batch_submit",
    "fft3d_strerror", "fft3d_last_error", "fft3d_plan_describe", "fft3d_plan_twiddles",
    "fft3d_exchange_block", "fft3d_run_pass", "fft3d_batch_submit_ex", "fft3d_batch_create",
    "fft3d_batch_launch", "fft3d_batch_status", "fft3d_batch_describe", "fft3d_batch_destroy",
    "fft3d_server_create", "fft3d_server_submit", "fft3d_server_wait", "fft3d_server_result",
    "fft3d_server_release", "fft3d_server_stats", "fft3d_server_destroy", "fft3d_r2c_transposed",
    "fft3d_c2r_transposed", "fft3d_r2c_pruned", "fft3d_c2r_pruned", "fft3d_r2c_inplace", "fft3d_c2r_inplace",
    "fft3d_init", "fft3d_batch_submit_checked", "fft3d_batch_check", "fft3d_plan_tuned", "fft3d_autotune",
    "fft3d_tune_lookup", "fft3d_tune_save", "fft3d_tune_load", "fft3d_batch_create_tuned", "fft3d_batch_autotune",
)


class Fft3dError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (_strerror(code), code, message))
        self.code = code


class BatchItem(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("dir", ctypes.c_int), ("in_", ctypes.c_void_p),
                ("mid", ctypes.c_void_p), ("out", ctypes.c_void_p), ("work", ctypes.c_void_p)]


# the scalar fields of fft3d_tuning; the struct holds radix[3][8] between
# coop_w and rows_rpw_inv
TUNING_FIELDS = ("plane", "rows_rpw", "n1_w", "n0_w", "n0_group", "walk", "coop_lag", "coop_rpw", "coop_w",
                 "rows_rpw_inv", "cols_pipe")


class Tuning(ctypes.Structure):
    """fft3d_tuning: every field 0 keeps the plan's rule."""
    _fields_ = [(n, ctypes.c_int32) for n in TUNING_FIELDS[:9]] + [("radix", (ctypes.c_int32 * 8) * 3)] + \
        [(n, ctypes.c_int32) for n in TUNING_FIELDS[9:]]

    @classmethod
    def from_dict(cls, d: dict) -> "Tuning":
        t = cls()
        for k, v in (d or {}).items():
            if k == "radix":
                for a, lst in enumerate(v):
                    for i, r in enumerate(lst):
                        t.radix[a][i] = int(r)
            elif k in TUNING_FIELDS:
                setattr(t, k, int(v))
            else:
                raise ValueError("unknown tuning field %r" % k)
        return t

    def to_dict(self) -> dict:
        d = {k: int(getattr(self, k)) for k in TUNING_FIELDS}
        d["radix"] = [[int(r) for r in self.radix[a] if r] for a in range(3)]
        return d


class BatchTuning(ctypes.Structure):
    """fft3d_batch_tuning: every field 0 keeps the rule."""
    _fields_ = [(n, ctypes.c_int32) for n in ("mode", "lag", "widen", "wg_per_cu", "spin_limit")]

    def to_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k in ("mode", "lag", "widen", "wg_per_cu", "spin_limit")}


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("nstreams", ctypes.c_int), ("batch_points", ctypes.c_int64),
                ("max_batch_items", ctypes.c_int), ("flags", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int64), ("n1", ctypes.c_int64), ("n2", ctypes.c_int64), ("dtype", ctypes.c_int),
                ("dir", ctypes.c_int), ("ncomp", ctypes.c_int), ("in_", ctypes.c_void_p * FFT3D_SERVER_MAX_COMP)]


class ServerCounters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "admitted", "completed", "released", "waiting",
                                              "in_flight", "batched_launches", "single_launches")] + \
               [(n, ctypes.c_size_t) for n in ("reserved_bytes", "peak_reserved_bytes", "budget_bytes")]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfft3d.so is not built (run `python -m paper_1406_5597_amd.build` "
                          "or __graft_entry__.build()); there is no fallback")
    L = ctypes.CDLL(LIB_PATH)
    i64, vp, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    sig = {
        "fft3d_version": (ctypes.c_int, []),
        "fft3d_init": (ctypes.c_int, []),
        "fft3d_batch_submit_checked": (ctypes.c_int, [ctypes.POINTER(BatchItem), ctypes.c_int, vp,
                                                      ctypes.POINTER(i64)]),
        "fft3d_batch_check": (ctypes.c_int, [i64]),
        "fft3d_plan_tuned": (ctypes.c_int, [i64, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Tuning),
                                            ctypes.POINTER(vp)]),
        "fft3d_autotune": (ctypes.c_int, [i64, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Tuning),
                                          ctypes.c_char_p, sz]),
        "fft3d_tune_lookup": (ctypes.c_int, [i64, i64, i64, ctypes.c_int, ctypes.POINTER(Tuning)]),
        "fft3d_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
        "fft3d_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
        "fft3d_batch_create_tuned": (ctypes.c_int, [ctypes.POINTER(BatchItem), ctypes.c_int, ctypes.c_int,
                                                    ctypes.POINTER(BatchTuning), ctypes.POINTER(vp)]),
        "fft3d_batch_autotune": (ctypes.c_int, [ctypes.POINTER(BatchItem), ctypes.c_int, ctypes.c_int,
                                                ctypes.POINTER(BatchTuning), ctypes.c_char_p, sz]),
        "fft3d_batch_submit_static": (ctypes.c_int, [ctypes.POINTER(BatchItem), ctypes.c_int, vp, vp]),
        "fft3d_plan": (ctypes.c_int, [i64, i64, i64, ctypes.c_int, ctypes.POINTER(vp)]),
        "fft3d_plan_ex": (ctypes.c_int, [i64, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]),
        "fft3d_plan_destroy": (ctypes.c_int, [vp]),
        "fft3d_work_bytes": (sz, [vp]),
        "fft3d_real_bytes": (sz, [vp]),
        "fft3d_complex_bytes": (sz, [vp]),
        "fft3d_r2c": (ctypes.c_int, [vp, vp, vp, vp]),
        "fft3d_c2r": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fft3d_batch_submit": (ctypes.c_int, [ctypes.POINTER(BatchItem), ctypes.c_int, vp]),
        "fft3d_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "fft3d_last_error": (ctypes.c_char_p, []),
        "fft3d_plan_describe": (ctypes.c_int, [vp, ctypes.c_char_p, sz]),
        "fft3d_plan_twiddles": (i64, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), i64]),
        "fft3d_exchange_block": (ctypes.c_int, [i64, i64, i64, i64, i64, ctypes.POINTER(i64)]),
        "fft3d_run_pass": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
        "fft3d_batch_submit_ex": (ctypes.c_int, [ctypes.POINTER(BatchItem), ctypes.c_int, ctypes.c_int, vp]),
        "fft3d_batch_create": (ctypes.c_int, [ctypes.POINTER(BatchItem), ctypes.c_int, ctypes.c_int,
                                              ctypes.POINTER(vp)]),
        "fft3d_batch_launch": (ctypes.c_int, [vp, vp]),
        "fft3d_batch_status": (ctypes.c_int, [vp]),
        "fft3d_batch_describe": (ctypes.c_int, [vp, ctypes.c_char_p, sz]),
        "fft3d_batch_destroy": (ctypes.c_int, [vp]),
        "fft3d_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]),
        "fft3d_server_submit": (ctypes.c_int, [vp, ctypes.POINTER(Request), ctypes.POINTER(i64)]),
        "fft3d_server_wait": (ctypes.c_int, [vp, i64, ctypes.c_double]),
        "fft3d_server_result": (ctypes.c_int, [vp, i64, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_double)]),
        "fft3d_server_release": (ctypes.c_int, [vp, i64]),
        "fft3d_server_stats": (ctypes.c_int, [vp, ctypes.POINTER(ServerCounters)]),
        "fft3d_server_destroy": (ctypes.c_int, [vp]),
        "fft3d_r2c_transposed": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fft3d_c2r_transposed": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fft3d_r2c_pruned": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(i64), vp]),
        "fft3d_r2c_inplace": (ctypes.c_int, [vp, vp, vp]),
        "fft3d_c2r_inplace": (ctypes.c_int, [vp, vp, vp]),
        "fft3d_c2r_pruned": (ctypes.c_int, [vp, vp, vp, vp, ctypes.POINTER(i64), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


def _strerror(code: int) -> str:
    return lib.fft3d_strerror(code).decode()


def fft3d_last_error() -> str:
    return lib.fft3d_last_error().decode()


def fft3d_strerror(code: int) -> str:
    return _strerror(code)


def _check(rc: int) -> int:
    if rc < 0:
        raise Fft3dError(rc, fft3d_last_error())
    return rc


def _addr(a) -> int:
    if a is None:
        return 0
    if isinstance(a, int):
        return a
    return a.data_ptr()


def _stream(s) -> int:
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def fft3d_version() -> int:
    return lib.fft3d_version()


def fft3d_init() -> None:
    """Set up the current device for batched launches (its batch ring)."""
    _check(lib.fft3d_init())


class Plan:
    """An fft3d plan; owns the C handle (destroyed on close / garbage collection)."""

    def __init__(self, n0: int, n1: int, n2: int, dtype: str = "f32", host_only: bool = False,
                 coop_plane: bool = False, tuning=None, tuned: bool = False):
        """tuning: None (the rule), a dict of fft3d_tuning fields or a Tuning;
        tuned: take the tuning from the process's tuning table (FFT3D_PLAN_TUNED)."""
        self.shape = (int(n0), int(n1), int(n2))
        self.dtype = dtype
        dt = {"f32": FFT3D_F32, "f64": FFT3D_F64}.get(dtype)
        if dt is None:
            raise ValueError("dtype must be 'f32' or 'f64'")
        h = ctypes.c_void_p()
        flags = (FFT3D_PLAN_HOST_ONLY if host_only else 0) | (FFT3D_PLAN_COOP_PLANE if coop_plane else 0) | \
                (FFT3D_PLAN_TUNED if tuned else 0)
        if tuning is None:
            _check(lib.fft3d_plan_ex(int(n0), int(n1), int(n2), dt, flags, ctypes.byref(h)))
        else:
            t = tuning if isinstance(tuning, Tuning) else Tuning.from_dict(tuning)
            _check(lib.fft3d_plan_tuned(int(n0), int(n1), int(n2), dt, flags, ctypes.byref(t), ctypes.byref(h)))
        self.handle = h.value

    @property
    def half_shape(self):
        n0, n1, n2 = self.shape
        return (n0, n1, n2 // 2 + 1)

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.fft3d_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def describe(self) -> dict:
        n = _check(lib.fft3d_plan_describe(self.handle, None, 0))
        buf = ctypes.create_string_buffer(n + 1)
        lib.fft3d_plan_describe(self.handle, buf, n + 1)
        return json.loads(buf.value.decode())

    def twiddles(self, which: int):
        import numpy as np
        n = _check(lib.fft3d_plan_twiddles(self.handle, which, None, 0))
        out = np.zeros(2 * max(n, 1), dtype=np.float64)
        lib.fft3d_plan_twiddles(self.handle, which, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n)
        return out[: 2 * n].view(np.complex128)

    @property
    def work_bytes(self) -> int:
        return lib.fft3d_work_bytes(self.handle)

    @property
    def real_bytes(self) -> int:
        return lib.fft3d_real_bytes(self.handle)

    @property
    def complex_bytes(self) -> int:
        return lib.fft3d_complex_bytes(self.handle)


def fft3d_plan(n0: int, n1: int, n2: int, dtype: str = "f32") -> Plan:
    return Plan(n0, n1, n2, dtype)


def fft3d_plan_ex(n0: int, n1: int, n2: int, dtype: str = "f32", flags: int = 0) -> Plan:
    return Plan(n0, n1, n2, dtype, host_only=bool(flags & FFT3D_PLAN_HOST_ONLY),
                coop_plane=bool(flags & FFT3D_PLAN_COOP_PLANE))


def fft3d_plan_tuned(n0: int, n1: int, n2: int, dtype: str = "f32", flags: int = 0, tuning=None) -> Plan:
    return Plan(n0, n1, n2, dtype, host_only=bool(flags & FFT3D_PLAN_HOST_ONLY),
                coop_plane=bool(flags & FFT3D_PLAN_COOP_PLANE), tuning=tuning if tuning is not None else {},
                tuned=bool(flags & FFT3D_PLAN_TUNED))


def _dt(dtype: str) -> int:
    dt = {"f32": FFT3D_F32, "f64": FFT3D_F64}.get(dtype)
    if dt is None:
        raise ValueError("dtype must be 'f32' or 'f64'")
    return dt


def fft3d_autotune(n0: int, n1: int, n2: int, dtype: str = "f32", effort: int = 0):
    """Time candidate tunings on the current device; returns (best tuning as a
    dict, the JSON report as a dict).  The winner also enters the process's
    tuning table."""
    return autotune((n0, n1, n2), dtype, effort)


def autotune(shape, dtype: str = "f32", effort: int = 0):
    """fft3d_autotune with the report: returns (tuning dict, report dict)."""
    n0, n1, n2 = (int(v) for v in shape)
    t = Tuning()
    cap = 1 << 22
    buf = ctypes.create_string_buffer(cap)
    n = _check(lib.fft3d_autotune(n0, n1, n2, _dt(dtype), int(effort), ctypes.byref(t), buf, cap))
    if n >= cap:
        raise RuntimeError("autotune report larger than %d bytes" % cap)
    return t.to_dict(), json.loads(buf.value.decode())


def fft3d_tune_lookup(n0: int, n1: int, n2: int, dtype: str = "f32"):
    """The table's tuning for the shape on this device's architecture, or None."""
    t = Tuning()
    return t.to_dict() if _check(lib.fft3d_tune_lookup(int(n0), int(n1), int(n2), _dt(dtype), ctypes.byref(t))) else None


def fft3d_tune_save(path: str) -> None:
    _check(lib.fft3d_tune_save(os.fsencode(path)))


def fft3d_tune_load(path: str) -> None:
    _check(lib.fft3d_tune_load(os.fsencode(path)))


def fft3d_plan_destroy(plan: Plan) -> None:
    plan.close()


def fft3d_work_bytes(plan: Plan) -> int:
    return plan.work_bytes


def fft3d_r2c(plan: Plan, x, X, stream=None) -> None:
    _check(lib.fft3d_r2c(plan.handle, _addr(x), _addr(X), _stream(stream)))


def fft3d_c2r(plan: Plan, X, y, work=None, stream=None) -> None:
    _check(lib.fft3d_c2r(plan.handle, _addr(X), _addr(y), _addr(work), _stream(stream)))


def _items(items):
    arr = (BatchItem * max(len(items), 1))()
    for i, (plan, d, a, m, o, w) in enumerate(items):
        arr[i] = BatchItem(plan.handle, d, _addr(a), _addr(m), _addr(o), _addr(w))
    return arr


def fft3d_r2c_transposed(plan: Plan, x, Xt, work, stream=None) -> None:
    _check(lib.fft3d_r2c_transposed(plan.handle, _addr(x), _addr(Xt), _addr(work), _stream(stream)))


def fft3d_c2r_transposed(plan: Plan, Xt, y, work, stream=None) -> None:
    _check(lib.fft3d_c2r_transposed(plan.handle, _addr(Xt), _addr(y), _addr(work), _stream(stream)))


def _kmax(kmax):
    if kmax is None:
        return None
    k = [int(v) for v in kmax]
    if len(k) != 3:
        raise ValueError("kmax: three cuts (K0, K1, K2)")
    return (ctypes.c_int64 * 3)(*k)


def fft3d_r2c_pruned(plan: Plan, x, X, kmax, stream=None) -> None:
    _check(lib.fft3d_r2c_pruned(plan.handle, _addr(x), _addr(X), _kmax(kmax), _stream(stream)))


def fft3d_c2r_pruned(plan: Plan, X, y, kmax, work=None, stream=None) -> None:
    _check(lib.fft3d_c2r_pruned(plan.handle, _addr(X), _addr(y), _addr(work), _kmax(kmax), _stream(stream)))


def fft3d_r2c_inplace(plan: Plan, buf, stream=None) -> None:
    _check(lib.fft3d_r2c_inplace(plan.handle, _addr(buf), _stream(stream)))


def fft3d_c2r_inplace(plan: Plan, buf, stream=None) -> None:
    _check(lib.fft3d_c2r_inplace(plan.handle, _addr(buf), _stream(stream)))


def fft3d_batch_submit(items, stream=None) -> None:
    """items: sequence of (plan, dir, in, mid, out, work) tuples; one batched launch."""
    _check(lib.fft3d_batch_submit(_items(items), len(items), _stream(stream)))


def fft3d_batch_submit_ex(items, flags: int = 0, stream=None) -> None:
    _check(lib.fft3d_batch_submit_ex(_items(items), len(items), int(flags), _stream(stream)))


def fft3d_batch_submit_checked(items, stream=None) -> int:
    """As fft3d_batch_submit; returns the token for fft3d_batch_check."""
    tok = ctypes.c_int64()
    _check(lib.fft3d_batch_submit_checked(_items(items), len(items), _stream(stream), ctypes.byref(tok)))
    return tok.value


def fft3d_batch_submit_static(items, status=None, stream=None) -> None:
    """As fft3d_batch_submit, through the library's static device scratch
    (no allocation); status: None or a one-int device tensor that receives the
    launch's error bits."""
    _check(lib.fft3d_batch_submit_static(_items(items), len(items), _addr(status), _stream(stream)))


def fft3d_batch_check(token: int) -> int:
    """Error bits of a finished batched launch (0 clean); raises Fft3dError
    (code FFT3D_ERR_BUSY) while it runs."""
    return _check(lib.fft3d_batch_check(int(token)))


class Batch:
    """A batch built once (task list on the device, hipGraph instantiated) and
    launched many times; owns the C handle.  Keeps the item tuples (and so the
    plans and tensors) alive as long as it lives."""

    def __init__(self, items, flags: int = 0, tuning=None):
        """tuning: None (the rule), a dict of fft3d_batch_tuning fields or a BatchTuning."""
        self.items = list(items)
        h = ctypes.c_void_p()
        if tuning is None:
            _check(lib.fft3d_batch_create(_items(self.items), len(self.items), int(flags), ctypes.byref(h)))
        else:
            bt = tuning if isinstance(tuning, BatchTuning) else BatchTuning(**{k: int(v) for k, v in tuning.items()})
            _check(lib.fft3d_batch_create_tuned(_items(self.items), len(self.items), int(flags), ctypes.byref(bt),
                                                ctypes.byref(h)))
        self.handle = h.value

    def launch(self, stream=None) -> None:
        _check(lib.fft3d_batch_launch(self.handle, _stream(stream)))

    def status(self) -> int:
        return _check(lib.fft3d_batch_status(self.handle))

    def describe(self) -> dict:
        n = _check(lib.fft3d_batch_describe(self.handle, None, 0))
        buf = ctypes.create_string_buffer(n + 1)
        lib.fft3d_batch_describe(self.handle, buf, n + 1)
        return json.loads(buf.value.decode())

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.fft3d_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fft3d_batch_create(items, flags: int = 0) -> Batch:
    return Batch(items, flags)


def fft3d_batch_create_tuned(items, flags: int = 0, tuning=None) -> Batch:
    return Batch(items, flags, tuning=tuning if tuning is not None else {})


def fft3d_batch_autotune(items, effort: int = 0):
    """Time launch shapes of the batch of these items (their outputs are
    overwritten); returns (best batch tuning dict, report dict)."""
    bt = BatchTuning()
    cap = 1 << 20
    buf = ctypes.create_string_buffer(cap)
    n = _check(lib.fft3d_batch_autotune(_items(items), len(items), int(effort), ctypes.byref(bt), buf, cap))
    if n >= cap:
        raise RuntimeError("batch autotune report larger than %d bytes" % cap)
    return bt.to_dict(), json.loads(buf.value.decode())


def fft3d_batch_launch(batch: Batch, stream=None) -> None:
    batch.launch(stream)


def fft3d_batch_status(batch: Batch) -> int:
    return batch.status()


def fft3d_batch_describe(batch: Batch) -> dict:
    return batch.describe()


def fft3d_batch_destroy(batch: Batch) -> None:
    batch.close()


def fft3d_run_pass(plan: Plan, pass_id: int, src, dst, stream=None) -> None:
    _check(lib.fft3d_run_pass(plan.handle, pass_id, _addr(src), _addr(dst), _stream(stream)))


def fft3d_plan_describe(plan: Plan) -> dict:
    return plan.describe()


def fft3d_plan_twiddles(plan: Plan, which: int):
    return plan.twiddles(which)


def fft3d_exchange_block(n0: int, ncols: int, p: int, src: int, dst: int):
    """(sender first, count, blocklen, stride), (receiver first, count, blocklen, stride)."""
    out = (ctypes.c_int64 * 8)()
    _check(lib.fft3d_exchange_block(n0, ncols, p, src, dst, out))
    v = list(out)
    return tuple(v[:4]), tuple(v[4:])


class Server:
    """A serving loop on the current device (see include/fft3d.h, "Serving"):
    submit r2c / c2r requests of 1..8 fields, wait, read the outputs (device
    addresses in the server's arena) and times, release."""

    def __init__(self, budget_bytes: int, nstreams: int = 0, batch_points: int = 0, max_batch_items: int = 0,
                 flags: int = 0):
        cfg = ServerConfig(int(budget_bytes), int(nstreams), int(batch_points), int(max_batch_items), int(flags))
        h = ctypes.c_void_p()
        _check(lib.fft3d_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h.value

    def submit(self, shape, dtype: str, direction: int, inputs) -> int:
        r = Request()
        r.n0, r.n1, r.n2 = (int(v) for v in shape)
        r.dtype = FFT3D_F32 if dtype == "f32" else FFT3D_F64
        r.dir = int(direction)
        r.ncomp = len(inputs)
        for i, a in enumerate(inputs):
            r.in_[i] = _addr(a)
        rid = ctypes.c_int64()
        _check(lib.fft3d_server_submit(self.handle, ctypes.byref(r), ctypes.byref(rid)))
        return rid.value

    def wait(self, rid: int, timeout: float = -1.0) -> bool:
        return _check(lib.fft3d_server_wait(self.handle, int(rid), float(timeout))) == 1

    def result(self, rid: int, ncomp: int):
        """(output device addresses, (t_arrive, t_admit, t_launch, t_done))."""
        out = (ctypes.c_void_p * ncomp)()
        times = (ctypes.c_double * 4)()
        _check(lib.fft3d_server_result(self.handle, int(rid), out, times))
        return [o for o in out], tuple(times)

    def release(self, rid: int) -> None:
        _check(lib.fft3d_server_release(self.handle, int(rid)))

    def stats(self) -> dict:
        c = ServerCounters()
        _check(lib.fft3d_server_stats(self.handle, ctypes.byref(c)))
        return {n: getattr(c, n) for n, _ in ServerCounters._fields_}

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.fft3d_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def fft3d_server_create(budget_bytes: int, **kw) -> Server:
    return Server(budget_bytes, **kw)


def fft3d_server_submit(server: Server, shape, dtype: str, direction: int, inputs) -> int:
    return server.submit(shape, dtype, direction, inputs)


def fft3d_server_wait(server: Server, rid: int, timeout: float = -1.0) -> bool:
    return server.wait(rid, timeout)


def fft3d_server_result(server: Server, rid: int, ncomp: int):
    return server.result(rid, ncomp)


def fft3d_server_release(server: Server, rid: int) -> None:
    server.release(rid)


def fft3d_server_stats(server: Server) -> dict:
    return server.stats()


def fft3d_server_destroy(server: Server) -> None:
    server.close()


_HIP = None


def copy_from_device(dst, src_addr: int, nbytes: int) -> None:
    """Copy nbytes from a raw device address into the device tensor dst
    (synchronous, for reading server outputs)."""
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.restype = ctypes.c_int
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    if nbytes > dst.numel() * dst.element_size():
        raise ValueError("destination too small")
    rc = _HIP.hipMemcpy(_addr(dst), int(src_addr), int(nbytes), 3)  # device to device
    if rc != 0:
        raise RuntimeError("hipMemcpy failed: %d" % rc)


# ------------------------------------------------------------ conveniences --

def torch_dtypes(dtype: str):
    import torch
    return (torch.float32, torch.complex64) if dtype == "f32" else (torch.float64, torch.complex128)


def empty_real(plan: Plan, device="cuda"):
    import torch
    return torch.empty(plan.shape, dtype=torch_dtypes(plan.dtype)[0], device=device)


def empty_complex(plan: Plan, device="cuda"):
    import torch
    return torch.empty(plan.half_shape, dtype=torch_dtypes(plan.dtype)[1], device=device)


def r2c(plan: Plan, x, X=None, stream=None):
    """Forward transform of the real GPU tensor x; returns X (allocated if None)."""
    if X is None:
        X = empty_complex(plan, x.device)
    _shape_check(plan, x, X)
    fft3d_r2c(plan, x, X, stream)
    return X


def c2r(plan: Plan, X, y=None, work=None, stream=None):
    """Inverse transform; X is preserved iff work is given."""
    if y is None:
        y = empty_real(plan, X.device)
    _shape_check(plan, y, X)
    fft3d_c2r(plan, X, y, work, stream)
    return y


def r2c_pruned(plan: Plan, x, kmax, X=None, stream=None):
    """Pruned forward transform: X holds the kept modes of the box kmax (its
    other elements are unspecified); X is allocated if None."""
    if X is None:
        X = empty_complex(plan, x.device)
    _shape_check(plan, x, X)
    fft3d_r2c_pruned(plan, x, X, kmax, stream)
    return X


def c2r_pruned(plan: Plan, X, kmax, y=None, work=None, stream=None):
    """Pruned inverse transform: reads only the kept modes of X; X is
    preserved iff work is given."""
    if y is None:
        y = empty_real(plan, X.device)
    _shape_check(plan, y, X)
    fft3d_c2r_pruned(plan, X, y, kmax, work, stream)
    return y


def _shape_check(plan: Plan, real, cplx) -> None:
    rd, cd = torch_dtypes(plan.dtype)
    if tuple(real.shape) != plan.shape or real.dtype != rd or not real.is_contiguous():
        raise ValueError("real array must be a contiguous %s tensor of shape %s" % (rd, plan.shape))
    if tuple(cplx.shape) != plan.half_shape or cplx.dtype != cd or not cplx.is_contiguous():
        raise ValueError("complex array must be a contiguous %s tensor of shape %s" % (cd, plan.half_shape))

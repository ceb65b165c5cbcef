"""Python binding of the C ABI in include/tm.h (ctypes).

Argument marshalling only: every step of the matcher runs in libtm.so's HIP
kernels.  torch supplies device memory and the current HIP stream; it does no
arithmetic here.  The library must be built (``python -m
paper_1509_04863_amd.build``); without it every call raises.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtm.so")

TM_OK, TM_ERR_INVALID, TM_ERR_NOMEM, TM_ERR_DEVICE, TM_ERR_UNSUPPORTED = range(5)
TM_I8, TM_F32, TM_BF16, TM_F16 = range(4)
TM_F_EXACT, TM_F_REAL, TM_F_ZERO_PAD, TM_F_FFT = 0x1, 0x2, 0x4, 0x8
TM_R_NOMATCH, TM_R_RESCORED, TM_R_NEAR_TIE, TM_R_EXACT = 0x1, 0x2, 0x4, 0x8

EXPORTS = ["tm_plan_params", "tm_plan_create", "tm_plan_destroy", "tm_plan_get_info", "tm_match",
           "tm_match_batch", "tm_match_intermediates", "tm_status_string", "tm_last_error",
           "tm_version", "tm_profile_enable", "tm_profile_read", "tm_server_create", "tm_server_submit",
           "tm_server_poll", "tm_server_wait", "tm_server_get_stats", "tm_server_destroy",
           "tm_admit_batches", "tm_match_many", "tm_profile_read_corr", "tm_match_noalloc",
           "tm_batch_create", "tm_batch_launch", "tm_batch_destroy"]


class PlanDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("k", ctypes.c_int32), ("m1", ctypes.c_int32),
                ("m2", ctypes.c_int32), ("fold_mult", ctypes.c_int32), ("x_dtype", ctypes.c_int32),
                ("t_dtype", ctypes.c_int32), ("fold_store", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("top_t", ctypes.c_int32), ("m3", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("m1", ctypes.c_int32), ("m2", ctypes.c_int32), ("l1", ctypes.c_int32),
                ("l2", ctypes.c_int32), ("fft_log2", ctypes.c_int32), ("exact", ctypes.c_int32),
                ("dual", ctypes.c_int32), ("fft_in_lds", ctypes.c_int32),
                ("fold_tiles", ctypes.c_int32), ("fold_segments", ctypes.c_int32),
                ("fold_bands", ctypes.c_int32), ("fft_global", ctypes.c_int32),
                ("corr_gemm", ctypes.c_int32), ("m3", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64), ("x_bytes", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("shift", ctypes.c_int64), ("m1_tilde", ctypes.c_int32),
                ("m2_tilde", ctypes.c_int32), ("n_candidates", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("peak1", ctypes.c_double),
                ("peak2", ctypes.c_double), ("score", ctypes.c_double),
                ("err_bound", ctypes.c_double), ("reserved", ctypes.c_int64)]


class ServerDesc(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_batch", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("peak_inflight_bytes", ctypes.c_int64),
                ("peak_held_bytes", ctypes.c_int64)]


assert ctypes.sizeof(Result) == 64 and ctypes.sizeof(PlanDesc) == 48
RESULT_BYTES = ctypes.sizeof(Result)

RESULT_DTYPE = np.dtype([("shift", "<i8"), ("m1_tilde", "<i4"), ("m2_tilde", "<i4"),
                         ("n_candidates", "<i4"), ("flags", "<u4"), ("peak1", "<f8"),
                         ("peak2", "<f8"), ("score", "<f8"), ("err_bound", "<f8"), ("reserved", "<i8")])


class TMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("tm status %d: %s" % (status, message))
        self.status = status


_LIB = None


def lib():
    """The loaded libtm.so (raises if it was not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtm.so is not built; run `python -m paper_1509_04863_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
        L.tm_plan_params.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(PlanInfo)]
        L.tm_plan_create.argtypes = [ctypes.POINTER(PlanDesc), vp, ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.tm_plan_destroy.argtypes = [vp]
        L.tm_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.tm_match.argtypes = [vp, vp, vp, vp]
        L.tm_match_batch.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp]
        L.tm_match_intermediates.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        for fn in ("tm_plan_params", "tm_plan_create", "tm_plan_destroy", "tm_plan_get_info",
                   "tm_match", "tm_match_batch", "tm_match_intermediates"):
            getattr(L, fn).restype = ctypes.c_int
        L.tm_status_string.argtypes = [ctypes.c_int]
        L.tm_status_string.restype = ctypes.c_char_p
        L.tm_last_error.argtypes = []
        L.tm_last_error.restype = ctypes.c_char_p
        L.tm_version.restype = ctypes.c_char_p
        L.tm_profile_enable.argtypes = [ctypes.c_int]
        L.tm_profile_enable.restype = ctypes.c_int
        L.tm_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int]
        L.tm_profile_read.restype = ctypes.c_int
        L.tm_profile_read_corr.argtypes = L.tm_profile_read.argtypes
        L.tm_profile_read_corr.restype = ctypes.c_int
        u64p, i64p = ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int64)
        L.tm_server_create.argtypes = [ctypes.POINTER(ServerDesc), ctypes.POINTER(vp)]
        L.tm_server_submit.argtypes = [vp, vp, vp, u64p]
        L.tm_server_poll.argtypes = [vp, ctypes.c_uint64, vp, i64p, ctypes.POINTER(ctypes.c_int)]
        L.tm_server_wait.argtypes = [vp, ctypes.c_uint64, vp, i64p]
        L.tm_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.tm_server_destroy.argtypes = [vp]
        L.tm_admit_batches.argtypes = [i32, i64p, ctypes.c_int64, i32, ctypes.POINTER(i32)]
        L.tm_match_many.argtypes = [vp, i32, ctypes.POINTER(vp), vp, vp]
        L.tm_match_many.restype = ctypes.c_int
        L.tm_match_noalloc.argtypes = [vp, vp, vp, vp]
        L.tm_match_noalloc.restype = ctypes.c_int
        L.tm_batch_create.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp, ctypes.POINTER(vp)]
        L.tm_batch_launch.argtypes = [vp, vp]
        L.tm_batch_destroy.argtypes = [vp]
        for fn in ("tm_batch_create", "tm_batch_launch", "tm_batch_destroy"):
            getattr(L, fn).restype = ctypes.c_int
        for fn in ("tm_server_create", "tm_server_submit", "tm_server_poll", "tm_server_wait",
                   "tm_server_get_stats", "tm_server_destroy", "tm_admit_batches"):
            getattr(L, fn).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(status: int):
    if status != TM_OK:
        raise TMError(status, lib().tm_last_error().decode())


# ------------------------------------------------------------------ dtypes

_NP_TO_TM = {np.dtype(np.int8): TM_I8, np.dtype(np.float32): TM_F32, np.dtype(np.float16): TM_F16}


_TORCH = None
_TORCH_TO_TM = None


def _torch():
    """torch, imported once (None where it is not installed)."""
    global _TORCH, _TORCH_TO_TM
    if _TORCH is None:
        try:
            import torch
        except ImportError:
            return None
        _TORCH_TO_TM = {torch.int8: TM_I8, torch.float32: TM_F32, torch.bfloat16: TM_BF16,
                        torch.float16: TM_F16}
        _TORCH = torch
    return _TORCH


def tm_dtype_of(arr) -> int:
    """tm_dtype of a numpy array or torch tensor."""
    torch = _torch()
    if torch is not None and isinstance(arr, torch.Tensor):
        return _TORCH_TO_TM[arr.dtype]
    return _NP_TO_TM[np.dtype(arr.dtype)]


def _desc(n, k, m1=0, m2=0, fold_mult=1, x_dtype=TM_I8, t_dtype=TM_I8, fold_store=TM_F32, flags=0, top_t=1,
          m3=0):
    return PlanDesc(n=int(n), k=int(k), m1=int(m1), m2=int(m2), fold_mult=int(fold_mult),
                    x_dtype=int(x_dtype), t_dtype=int(t_dtype), fold_store=int(fold_store),
                    flags=int(flags), top_t=int(top_t), m3=int(m3))


def _info_dict(info: PlanInfo) -> dict:
    return {f: getattr(info, f) for f, _ in PlanInfo._fields_}


def plan_params(n, k, m1=0, m2=0, fold_mult=1, x_dtype=TM_I8, t_dtype=TM_I8, fold_store=TM_F32,
                flags=0, top_t=1, m3=0) -> dict:
    """Host-only plan parameters (tm_plan_params)."""
    info = PlanInfo()
    _check(lib().tm_plan_params(ctypes.byref(_desc(n, k, m1, m2, fold_mult, x_dtype, t_dtype,
                                                   fold_store, flags, top_t, m3)), ctypes.byref(info)))
    return _info_dict(info)


def _stream_handle(stream) -> int:
    if stream is None:
        stream = _torch().cuda.current_stream()
    return int(stream.cuda_stream)


@dataclasses.dataclass
class MatchResult:
    shift: int
    m1_tilde: int
    m2_tilde: int
    n_candidates: int
    flags: int
    peak1: float
    peak2: float
    score: float
    err_bound: float = 0.0

    @property
    def nomatch(self) -> bool:
        return bool(self.flags & TM_R_NOMATCH)

    @property
    def exact(self) -> bool:
        return bool(self.flags & TM_R_EXACT)

    @property
    def near_tie(self) -> bool:
        return bool(self.flags & TM_R_NEAR_TIE)


def _row(r):
    if isinstance(r, np.void):
        return (int(r["shift"]), int(r["m1_tilde"]), int(r["m2_tilde"]), int(r["n_candidates"]),
                int(r["flags"]), float(r["peak1"]), float(r["peak2"]), float(r["score"]), float(r["err_bound"]))
    return (int(r.shift), int(r.m1_tilde), int(r.m2_tilde), int(r.n_candidates), int(r.flags),
            float(r.peak1), float(r.peak2), float(r.score), float(r.err_bound))


class Plan:
    """A template with its device state (tm_plan)."""

    def __init__(self, t, n: int, m1: int = 0, m2: int = 0, fold_mult: int = 1,
                 x_dtype: Optional[int] = None, fold_store: int = TM_F32, flags: int = 0,
                 stream=None, top_t: int = 1, m3: int = 0):
        if hasattr(t, "detach"):
            import torch
            tt = t.detach().cpu().contiguous()
            t_host = tt.view(torch.int16).numpy() if tt.dtype == torch.bfloat16 else tt.numpy()
        else:
            t_host = np.ascontiguousarray(t)
        t_dtype = tm_dtype_of(t)
        if x_dtype is None:
            x_dtype = t_dtype
        self.desc = _desc(n, t_host.shape[0], m1, m2, fold_mult, x_dtype, t_dtype, fold_store, flags, top_t, m3)
        self._t_host = np.ascontiguousarray(t_host)
        handle = ctypes.c_void_p()
        _check(lib().tm_plan_create(ctypes.byref(self.desc), self._t_host.ctypes.data, 0,
                                    _stream_handle(stream) if _torch_cuda() else None,
                                    ctypes.byref(handle)))
        self.handle = handle
        self._n = int(self.desc.n)              # plain ints for the per-call checks
        self._x_dtype = int(self.desc.x_dtype)
        info = PlanInfo()
        _check(lib().tm_plan_get_info(self.handle, ctypes.byref(info)))
        self.info = _info_dict(info)

    @property
    def n(self) -> int:
        return int(self.desc.n)

    @property
    def k(self) -> int:
        return int(self.desc.k)

    @property
    def m1(self) -> int:
        return int(self.info["m1"])

    @property
    def m2(self) -> int:
        return int(self.info["m2"])

    @property
    def m3(self) -> int:
        """Third modulus of a three-moduli plan, 0 otherwise."""
        return int(self.info["m3"])

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _check(lib().tm_plan_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _torch_cuda() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except ImportError:
        return False


def _check_signal(plan: Plan, x):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("x must be a CUDA (HIP) torch tensor")
    if x.numel() != plan._n or not x.is_contiguous():
        raise ValueError("x must be a contiguous tensor of N elements")
    if _TORCH_TO_TM.get(x.dtype) != plan._x_dtype:
        raise TypeError("x dtype does not match the plan")


def _check_out(out, count: int):
    """`out` must be a contiguous CUDA uint8 tensor with room for `count`
    results: the kernels write there without further checks."""
    torch = _torch()
    if not isinstance(out, torch.Tensor) or not out.is_cuda:
        raise TypeError("out must be a CUDA (HIP) torch tensor")
    if out.dtype != torch.uint8 or not out.is_contiguous():
        raise TypeError("out must be a contiguous uint8 tensor")
    if out.numel() < RESULT_BYTES * count:
        raise ValueError("out holds %d bytes; %d results need %d" % (out.numel(), count, RESULT_BYTES * count))


def match(plan: Plan, x, stream=None) -> MatchResult:
    """One match with a host result (waits for the stream)."""
    _check_signal(plan, x)
    res = Result()
    _check(lib().tm_match(plan.handle, x.data_ptr(), ctypes.addressof(res), _stream_handle(stream)))
    return MatchResult(*_row(res))


def match_into(plan: Plan, x, out, index: int = 0, stream=None):
    """One match writing a device result: `out` is a CUDA uint8 tensor of
    RESULT_BYTES*count bytes; nothing waits."""
    _check_signal(plan, x)
    if index < 0:
        raise ValueError("index must be >= 0")
    _check_out(out, index + 1)
    st = (_LIB or lib()).tm_match(plan.handle, x.data_ptr(), out.data_ptr() + RESULT_BYTES * index,
                                  _stream_handle(stream))
    if st != TM_OK:
        _check(st)


def match_noalloc(plan: Plan, x, out, index: int = 0, stream=None):
    """tm_match_noalloc: one match that allocates no device memory, writing
    its result into slot `index` of `out` (a CUDA uint8 tensor); nothing
    waits.  Calls that overlap on one GPU race (one scratch array per GPU)."""
    _check_signal(plan, x)
    if index < 0:
        raise ValueError("index must be >= 0")
    _check_out(out, index + 1)
    _check(lib().tm_match_noalloc(plan.handle, x.data_ptr(), out.data_ptr() + RESULT_BYTES * index,
                                  _stream_handle(stream)))


def results_from_device(out) -> List[MatchResult]:
    arr = out.cpu().numpy().view(RESULT_DTYPE)
    return [MatchResult(*_row(r)) for r in arr]


def match_batch(plans: Sequence[Plan], xs: Sequence, stream=None, out=None) -> Optional[List[MatchResult]]:
    """tm_match_batch.  With out=None the results come back to the host;
    with a CUDA uint8 tensor of RESULT_BYTES*count bytes they stay on the device."""
    count = len(plans)
    if count != len(xs):
        raise ValueError("plans and xs differ in length")
    for p, x in zip(plans, xs):
        _check_signal(p, x)
    parr = (ctypes.c_void_p * count)(*[p.handle.value for p in plans])
    xarr = (ctypes.c_void_p * count)(*[x.data_ptr() for x in xs])
    if out is not None:
        _check_out(out, count)
        _check(lib().tm_match_batch(count, parr, xarr, out.data_ptr(), _stream_handle(stream)))
        return None
    host = np.zeros(count, dtype=RESULT_DTYPE)
    _check(lib().tm_match_batch(count, parr, xarr, host.ctypes.data, _stream_handle(stream)))
    return [MatchResult(*_row(r)) for r in host]


class Batch:
    """A fixed list of (plan, signal) pairs whose pointer arrays are built once;
    run() enqueues tm_match_batch with results in a device buffer."""

    def __init__(self, plans: Sequence[Plan], xs: Sequence):
        if len(plans) != len(xs):
            raise ValueError("plans and xs differ in length")
        for p, x in zip(plans, xs):
            _check_signal(p, x)
        self.plans, self.xs = list(plans), list(xs)
        self.count = len(plans)
        self._p = (ctypes.c_void_p * self.count)(*[p.handle.value for p in plans])
        self._x = (ctypes.c_void_p * self.count)(*[x.data_ptr() for x in xs])

    def run(self, out, stream=None):
        """out: CUDA uint8 tensor of RESULT_BYTES*count bytes (device results, no wait)."""
        _check_out(out, self.count)
        _check(lib().tm_match_batch(self.count, self._p, self._x, out.data_ptr(),
                                    _stream_handle(stream)))


class BatchGraph:
    """tm_batch_*: a fixed list of (plan, signal) pairs whose launch sequence
    is captured once in a HIP graph; run() replays it, writing the results
    into the device buffer `out` given at creation."""

    def __init__(self, plans: Sequence[Plan], xs: Sequence, out, stream=None):
        if len(plans) != len(xs):
            raise ValueError("plans and xs differ in length")
        for p, x in zip(plans, xs):
            _check_signal(p, x)
        self.count = len(plans)
        _check_out(out, self.count)
        self.plans, self.xs, self.out = list(plans), list(xs), out     # kept alive with the graph
        parr = (ctypes.c_void_p * self.count)(*[p.handle.value for p in plans])
        xarr = (ctypes.c_void_p * self.count)(*[x.data_ptr() for x in xs])
        self.handle = ctypes.c_void_p()
        _check(lib().tm_batch_create(self.count, parr, xarr, out.data_ptr(), _stream_handle(stream),
                                     ctypes.byref(self.handle)))

    def run(self, stream=None):
        _check(lib().tm_batch_launch(self.handle, _stream_handle(stream)))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _check(lib().tm_batch_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def match_intermediates(plan: Plan, x, stream=None):
    """Match and return (result, y1, y2, r1, r2) with the intermediates as
    numpy float64 arrays."""
    import torch
    _check_signal(plan, x)
    m1, m2, k = plan.m1, plan.m2, plan.k
    dev = x.device
    y1 = torch.empty(m1 + k - 1, dtype=torch.float64, device=dev)
    y2 = torch.empty(m2 + k - 1, dtype=torch.float64, device=dev)
    r1 = torch.empty(m1, dtype=torch.float64, device=dev)
    r2 = torch.empty(m2, dtype=torch.float64, device=dev)
    res = Result()
    _check(lib().tm_match_intermediates(plan.handle, x.data_ptr(), ctypes.addressof(res),
                                        y1.data_ptr(), y2.data_ptr(), r1.data_ptr(),
                                        r2.data_ptr(), _stream_handle(stream)))
    return (MatchResult(*_row(res)), y1.cpu().numpy(), y2.cpu().numpy(), r1.cpu().numpy(),
            r2.cpu().numpy())


def profile_enable(on: bool = True):
    """Record HIP events around every fold kernel launch and every correlation
    kernel launch (tm_profile_enable)."""
    _check(lib().tm_profile_enable(1 if on else 0))


def profile_read(reset: bool = False):
    """(summed fold kernel milliseconds, fold launches) since the last reset."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().tm_profile_read(ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return ms.value, n.value


def profile_read_corr(reset: bool = False):
    """(summed correlation kernel milliseconds, launches) since the last reset:
    the int8 matrix-product kernel, or the in-LDS FFT finish kernel."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().tm_profile_read_corr(ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return ms.value, n.value


def admit_batches(footprints, budget_bytes: int, max_batch: int):
    """The server's first-in first-out admission rule on the host
    (tm_admit_batches): the batch index of every request."""
    fp = np.ascontiguousarray(np.asarray(footprints, dtype=np.int64))
    out = np.zeros(fp.shape[0], dtype=np.int32)
    _check(lib().tm_admit_batches(int(fp.shape[0]), fp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  int(budget_bytes), int(max_batch),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return out


class Server:
    """Continuous-batching request server (tm_server_*).  Keeps a reference to
    every submitted signal until its result has been taken."""

    def __init__(self, budget_bytes: int = 0, max_batch: int = 0, max_inflight: int = 0):
        d = ServerDesc(budget_bytes=int(budget_bytes), max_batch=int(max_batch),
                       max_inflight=int(max_inflight))
        self.handle = ctypes.c_void_p()
        _check(lib().tm_server_create(ctypes.byref(d), ctypes.byref(self.handle)))
        self._keep = {}

    def submit(self, plan: Plan, x) -> int:
        _check_signal(plan, x)
        t = ctypes.c_uint64()
        _check(lib().tm_server_submit(self.handle, plan.handle, x.data_ptr(), ctypes.byref(t)))
        self._keep[t.value] = (plan, x)
        return t.value

    def poll(self, ticket: int):
        """(done, MatchResult or None, latency in ns or None)."""
        res, lat, done = Result(), ctypes.c_int64(), ctypes.c_int()
        _check(lib().tm_server_poll(self.handle, ticket, ctypes.addressof(res), ctypes.byref(lat),
                                    ctypes.byref(done)))
        if not done.value:
            return False, None, None
        self._keep.pop(ticket, None)
        return True, MatchResult(*_row(res)), lat.value

    def wait(self, ticket: int):
        """(MatchResult, latency in ns)."""
        res, lat = Result(), ctypes.c_int64()
        st = lib().tm_server_wait(self.handle, ticket, ctypes.addressof(res), ctypes.byref(lat))
        self._keep.pop(ticket, None)
        _check(st)
        return MatchResult(*_row(res)), lat.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().tm_server_get_stats(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            _check(lib().tm_server_destroy(self.handle))
            self.handle = ctypes.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Many:
    """One plan, a fixed list of signals (tm_match_many); run() enqueues with
    results in a device buffer, match() returns host results."""

    def __init__(self, plan: Plan, xs: Sequence):
        for x in xs:
            _check_signal(plan, x)
        self.plan, self.xs = plan, list(xs)
        self.count = len(self.xs)
        self._x = (ctypes.c_void_p * self.count)(*[x.data_ptr() for x in self.xs])

    def run(self, out, stream=None):
        """out: CUDA uint8 tensor of RESULT_BYTES*count bytes (device results, no wait)."""
        _check_out(out, self.count)
        _check(lib().tm_match_many(self.plan.handle, self.count, self._x, out.data_ptr(),
                                   _stream_handle(stream)))

    def match(self, stream=None):
        res = (Result * self.count)()
        _check(lib().tm_match_many(self.plan.handle, self.count, self._x, ctypes.addressof(res),
                                   _stream_handle(stream)))
        return [MatchResult(*_row(r)) for r in res]

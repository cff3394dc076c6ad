"""Python binding of libtsqr.so (ctypes): argument marshalling only.

Every function of include/tsqr.h is exposed under the same name with the same
arguments (device pointers and streams passed as integers).  Convenience
wrappers that take PyTorch tensors -- :func:`geqr_r`, :func:`qr_uppers` --
only read ``data_ptr()``/strides and the current HIP stream, allocate the
output and the workspace with torch, and call the C entry points; every step of
the computation runs in the library's HIP kernels.  There is no fallback: if
the library is missing or no gfx950 device is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtsqr.so")

TSQR_MAX_N = 64
TSQR_F64 = 0
TSQR_F32 = 1
TSQR_ERR_HIP = 1
TSQR_ERR_UNSUPPORTED = 2
TSQR_ERR_NO_DEVICE = 3
TSQR_ERR_ALLOC = 4
TSQR_ERR_SCRATCH = 5
TSQR_NOALLOC_SCRATCH_BYTES = 32 << 20
TSQR_OPT_LEAF_ROWS = 1
TSQR_OPT_ROWS_PER_LANE = 2
TSQR_OPT_WAVES_PER_CU = 3

# (name, restype, argtypes) for every exported symbol of include/tsqr.h
_i, _i64, _p, _pi64 = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
SIGNATURES = [
    ("tsqr_create", _i, [ctypes.POINTER(_p), _i]),
    ("tsqr_create_planning", _i, [ctypes.POINTER(_p), _i]),
    ("tsqr_destroy", _i, [_p]),
    ("tsqr_last_hip_error", _i, [_p]),
    ("tsqr_status_string", ctypes.c_char_p, [_i]),
    ("tsqr_set_option", _i, [_p, _i, _i64]),
    ("tsqr_plan_info", _i, [_p, _i64, _i64, _i, _pi64, _pi64]),
    ("tsqr_tuning_add", _i, [_p, _i, _i64, _i64, _i64, _i64, _i64, _i]),
    ("tsqr_tuning_clear", _i, [_p]),
    ("tsqr_rows_per_lane_compiled", _i64, [_i, _i64, _pi64, _i64]),
    ("tsqr_workspace_bytes", _i64, [_p, _i64, _i64, _i]),
    ("tsqr_geqr_r_f64", _i, [_p, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p]),
    ("tsqr_geqr_r_f64_stamped", _i, [_p, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p, _p]),
    ("tsqr_geqr_r_f32", _i, [_p, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p]),
    ("tsqr_geqr_r_f64_noalloc", _i, [_p, _i64, _i64, _p, _i64, _p, _i64, _p]),
    ("tsqr_qr_uppers_f64", _i, [_p, _i64, _p, _p, _p, _p]),
    ("tsqr_qr_uppers_f32", _i, [_p, _i64, _p, _p, _p, _p]),
    ("tsqr_batch_plan_create", _i, [_p, _i64, _i64, _pi64, _pi64, _pi64, _i, ctypes.POINTER(_p)]),
    ("tsqr_batch_plan_destroy", _i, [_p]),
    ("tsqr_batch_workspace_bytes", _i64, [_p]),
    ("tsqr_batch_plan_info", _i, [_p, _pi64, _pi64, _pi64]),
    ("tsqr_batch_exec", _i, [_p, _p, _p, _i64, _p, _i64, _p]),
    ("tsqr_batch_exec_stamped", _i, [_p, _p, _p, _i64, _p, _i64, _p, _p]),
    ("tsqr_device_clock_khz", _i64, [_p]),
    ("tsqr_qr_workspace_bytes", _i64, [_p, _i64, _i64, _i]),
    ("tsqr_geqr_qr_f64", _i, [_p, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p, _i64, _p]),
    ("tsqr_geqr_qr_f32", _i, [_p, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p, _i64, _p]),
    ("tsqr_geqrf_f64", _i, [_p, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p]),
    ("tsqr_geqrf_f32", _i, [_p, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p]),
    ("tsqr_apply_qt_f64", _i, [_p, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p]),
    ("tsqr_apply_qt_f32", _i, [_p, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p]),
    ("tsqr_mixed_plan_create", _i, [_p, _i64, _i64, _i64, _i64, _i64, ctypes.POINTER(_p)]),
    ("tsqr_mixed_plan_destroy", _i, [_p]),
    ("tsqr_mixed_workspace_bytes", _i64, [_p]),
    ("tsqr_mixed_exec", _i, [_p, _p, _p, _i64, _p, _p, _i64, _p]),
    ("tsqr_batch_plan_schedule", _i, [_p, _p, _p]),
    ("tsqr_mixed_plan_create_sampled", _i, [_p, _i64, _i64, _i64, _i64, _i64, _i64, ctypes.c_uint64, ctypes.POINTER(_p)]),
    ("tsqr_mixed_rtilde_offset", _i64, [_p]),
    ("tsqr_mixed_exec_rtilde", _i, [_p, _p, _p, _p, _i64, _p, _p, _i64, _p]),
    ("tsqr_mixed_rtilde_exec", _i, [_p, _p, _p, _i64, _p]),
    ("tsqr_gemm_bf16", _i, [_p, _i, _i, _i64, _i64, _i64, ctypes.c_float, _p, _i64, _p, _i64, ctypes.c_float, _p,
                            _i64, _p]),
    ("tsqr_mlp_bias_act", _i, [_p, _p, _i64, _i64, _i64, _p, _i, _p]),
    ("tsqr_mlp_relu_grad", _i, [_p, _p, _p, _i64, _i64, _i64, _p]),
    ("tsqr_mlp_colsum", _i, [_p, _p, _i64, _i64, _i64, _p, _p]),
    ("tsqr_mlp_mse", _i, [_p, _p, _p, _p, _i64, _i64, _i64, _p, _p]),
    ("tsqr_mlp_adam", _i, [_p, _p, _p, _p, _p, _i64, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           _i64, _p]),
    ("tsqr_surrogate_features", _i, [_p, _p, _i64, _i64, _p, _p]),
    ("tsqr_surrogate_targets", _i, [_p, _p, _i64, _p, _i64, _i64, _p, _p]),
    ("tsqr_surrogate_apply", _i, [_p, _p, _p, _i64, _i64, _p, _p]),
]

_LOCK = threading.Lock()
_LIB = None


class TsqrError(RuntimeError):
    def __init__(self, fn: str, status: int, hip_error: int = 0):
        msg = f"{fn} returned {status}"
        if _LIB is not None:
            msg += " (" + _LIB.tsqr_status_string(status).decode() + ")"
        if hip_error:
            msg += f", hipError {hip_error}"
        super().__init__(msg)
        self.status = status


def load(path: str = LIB_PATH):
    """Load libtsqr.so and declare its signatures (raises if it is missing)."""
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(path):
                raise FileNotFoundError(
                    f"{path} is missing: build it with `python -m paper_1002_4250_amd.build`")
            lib = ctypes.CDLL(path)
            for name, res, args in SIGNATURES:
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _LIB = lib
        return _LIB


def lib():
    return load()


def _check(fn: str, status: int, handle=None):
    if status != 0:
        he = lib().tsqr_last_hip_error(handle) if handle else 0
        raise TsqrError(fn, status, he)


# ---- the C entry points under their own names -------------------------------

def tsqr_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check("tsqr_create", lib().tsqr_create(ctypes.byref(h), int(device)))
    return h.value


def tsqr_create_planning(cu_count: int = 256) -> int:
    h = ctypes.c_void_p()
    _check("tsqr_create_planning", lib().tsqr_create_planning(ctypes.byref(h), int(cu_count)))
    return h.value


def tsqr_destroy(handle: int) -> None:
    lib().tsqr_destroy(handle)


def tsqr_set_option(handle: int, option: int, value: int) -> None:
    _check("tsqr_set_option", lib().tsqr_set_option(handle, int(option), int(value)), handle)


def tsqr_plan_info(handle: int, m: int, n: int, dtype: int):
    lr, lv = ctypes.c_int64(), ctypes.c_int64()
    _check("tsqr_plan_info", lib().tsqr_plan_info(handle, m, n, dtype, ctypes.byref(lr), ctypes.byref(lv)), handle)
    return lr.value, lv.value


def tsqr_tuning_add(handle: int, dtype: int, n: int, m_max: int, rows_per_lane: int, waves_per_cu: int,
                    leaf_rows: int, batch: bool) -> None:
    _check("tsqr_tuning_add", lib().tsqr_tuning_add(handle, int(dtype), int(n), int(m_max), int(rows_per_lane),
                                                    int(waves_per_cu), int(leaf_rows), int(bool(batch))), handle)


def tsqr_tuning_clear(handle: int) -> None:
    _check("tsqr_tuning_clear", lib().tsqr_tuning_clear(handle), handle)


def tsqr_rows_per_lane_compiled(dtype: int, n: int) -> list:
    count = lib().tsqr_rows_per_lane_compiled(int(dtype), int(n), None, 0)
    if count < 0:
        raise TsqrError("tsqr_rows_per_lane_compiled", int(count))
    buf = (ctypes.c_int64 * max(int(count), 1))()
    got = lib().tsqr_rows_per_lane_compiled(int(dtype), int(n), buf, int(count))
    if got != count:
        raise TsqrError("tsqr_rows_per_lane_compiled", int(got))
    return [int(buf[i]) for i in range(count)]


def tsqr_workspace_bytes(handle: int, m: int, n: int, dtype: int) -> int:
    v = lib().tsqr_workspace_bytes(handle, int(m), int(n), int(dtype))
    if v < 0:
        raise TsqrError("tsqr_workspace_bytes", int(v))
    return int(v)


def tsqr_geqr_r_f64(handle, m, n, A, lda, R, ldr, ws, ws_bytes, stream) -> int:
    return lib().tsqr_geqr_r_f64(handle, m, n, A, lda, R, ldr, ws, ws_bytes, stream)


def tsqr_geqr_r_f32(handle, m, n, A, lda, R, ldr, ws, ws_bytes, stream) -> int:
    return lib().tsqr_geqr_r_f32(handle, m, n, A, lda, R, ldr, ws, ws_bytes, stream)


def tsqr_geqr_r_f64_noalloc(handle, m, n, A, lda, R, ldr, stream) -> int:
    return lib().tsqr_geqr_r_f64_noalloc(handle, m, n, A, lda, R, ldr, stream)


def tsqr_qr_uppers_f64(handle, n, R1, R2, tau, stream) -> int:
    return lib().tsqr_qr_uppers_f64(handle, n, R1, R2, tau, stream)


def tsqr_qr_uppers_f32(handle, n, R1, R2, tau, stream) -> int:
    return lib().tsqr_qr_uppers_f32(handle, n, R1, R2, tau, stream)


# ---- torch convenience layer ----------------------------------------------------

_HANDLES = {}


def handle(device: int = 0) -> int:
    """A process-wide handle per device (created on first use)."""
    with _LOCK:
        h = _HANDLES.get(device)
    if h is None:
        h = tsqr_create(device)
        with _LOCK:
            _HANDLES[device] = h
    return h


def _stream_ptr(torch, dev):
    return torch.cuda.current_stream(dev).cuda_stream


def _col_major(A):
    """(m, n, lda) of a column-major 2-D tensor (stride (1, lda))."""
    m, n = A.shape
    s0, s1 = A.stride()
    if s0 != 1 and m > 1:
        raise ValueError("A must be column-major: A.stride(0) == 1 (use A.t().contiguous().t())")
    if n > 1 and s1 < max(m, 1):
        # an expanded or overlapping view: the kernels read m*n distinct elements
        raise ValueError("A has a column stride below its row count (expanded or overlapping view); "
                         "pass A.contiguous() in column-major order")
    lda = s1 if n > 1 else max(m, 1)
    return m, n, lda


def _check_matrix(X, name, rows, cols, dtype, dev):
    """X must be a rows x cols column-major tensor of `dtype` on `dev` (the
    kernels take raw pointers, so a wrong output tensor is refused here);
    returns its leading dimension."""
    if X.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {X.dtype}")
    if X.device != dev:
        raise ValueError(f"{name} must be on {dev}, got {X.device}")
    if tuple(X.shape) != (rows, cols):
        raise ValueError(f"{name} must have shape ({rows}, {cols}), got {tuple(X.shape)}")
    if rows > 1 and X.stride(0) != 1:
        raise ValueError(f"{name} must be column-major (stride(0) == 1)")
    ld = X.stride(1) if cols > 1 else max(rows, 1)
    if ld < max(rows, 1):
        raise ValueError(f"{name} has a leading dimension below its row count")
    return ld


def _check_flat(X, name, numel, dtype, dev):
    """X must be a contiguous tensor of `dtype` on `dev` with at least `numel` elements."""
    if X.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {X.dtype}")
    if X.device != dev:
        raise ValueError(f"{name} must be on {dev}, got {X.device}")
    if not X.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if X.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, has {X.numel()}")


def _ws_bytes(ws, dev):
    if ws.device != dev or not ws.is_contiguous():
        raise ValueError("the workspace must be a contiguous tensor on the matrix's device")
    return ws.numel() * ws.element_size()


def workspace(m: int, n: int, dtype, device=None, h=None):
    """A uint8 workspace tensor large enough for geqr_r(m, n) with the
    handle's current options."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = h or handle(dev.index or 0)
    code = TSQR_F64 if dtype == torch.float64 else TSQR_F32
    nbytes = max(tsqr_workspace_bytes(h, m, n, code), 256)
    return torch.empty(nbytes, dtype=torch.uint8, device=dev)


def geqr_r(A, R=None, ws=None, h=None):
    """R factor (n-by-n, diag >= 0, column-major) of the column-major device
    matrix A (float64 or float32) by TSQR on the GPU."""
    import torch
    if A.dtype not in (torch.float64, torch.float32):
        raise TypeError("A must be float64 or float32")
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    m, n, lda = _col_major(A)
    dev = A.device
    h = h or handle(dev.index or 0)
    if R is None:
        R = torch.empty((n, n), dtype=A.dtype, device=dev).t()   # column-major n x n
    ldr = _check_matrix(R, "R", n, n, A.dtype, dev)
    if ws is None:
        ws = workspace(m, n, A.dtype, dev, h)
    fn = tsqr_geqr_r_f64 if A.dtype == torch.float64 else tsqr_geqr_r_f32
    st = fn(h, m, n, A.data_ptr(), lda, R.data_ptr(), ldr, ws.data_ptr(), _ws_bytes(ws, dev),
            _stream_ptr(torch, dev))
    _check(fn.__name__, st, h)
    return R


def geqr_r_stamped(A, R=None, ws=None, h=None, stamps=None):
    """``geqr_r`` for a float64 A that also measures where the time goes:
    returns (R, stamps), stamps an int64 device tensor (leaves, 4): per leaf
    its start, the end of its leaf phase and its exit on the device clock
    (``device_clock_khz`` kHz, arbitrary origin), and the tree level at
    which it stopped (plus 100 for the root)."""
    import torch
    if A.dtype != torch.float64 or not A.is_cuda:
        raise TypeError("A must be a float64 device tensor")
    m, n, lda = _col_major(A)
    dev = A.device
    h = h or handle(dev.index or 0)
    if R is None:
        R = torch.empty((n, n), dtype=A.dtype, device=dev).t()
    ldr = _check_matrix(R, "R", n, n, A.dtype, dev)
    if ws is None:
        ws = workspace(m, n, A.dtype, dev, h)
    leaves = tsqr_plan_info(h, m, n, TSQR_F64)[1] if n else 0
    if stamps is None:
        stamps = torch.zeros((max(leaves, 1), 4), dtype=torch.int64, device=dev)
    _check_flat(stamps, "stamps", 4 * leaves, torch.int64, dev)
    st = lib().tsqr_geqr_r_f64_stamped(h, m, n, A.data_ptr(), lda, R.data_ptr(), ldr, ws.data_ptr(),
                                       _ws_bytes(ws, dev), stamps.data_ptr(), _stream_ptr(torch, dev))
    _check("tsqr_geqr_r_f64_stamped", st, h)
    return R, stamps


def qr_uppers(R1, R2, tau=None, h=None):
    """The paper's operator in place on column-major n-by-n device tensors:
    R1 <- R, R2 <- V, tau <- reflector scalars.  Returns (R1, R2, tau)."""
    import torch
    n = R1.shape[0]
    if R1.dtype not in (torch.float64, torch.float32) or not R1.is_cuda:
        raise TypeError("R1 must be a float64 or float32 device tensor")
    for X in (R1, R2):
        if X.shape != (n, n) or (n > 1 and X.stride() != (1, n)):
            raise ValueError("R1 and R2 must be n-by-n column-major with leading dimension n")
        if X.dtype != R1.dtype or X.device != R1.device:
            raise TypeError("R1 and R2 must have the same dtype and device")
    h = h or handle(R1.device.index or 0)
    if tau is None:
        tau = torch.empty(max(n, 1), dtype=R1.dtype, device=R1.device)
    _check_flat(tau, "tau", n, R1.dtype, R1.device)
    fn = tsqr_qr_uppers_f64 if R1.dtype == torch.float64 else tsqr_qr_uppers_f32
    st = fn(h, n, R1.data_ptr(), R2.data_ptr(), tau.data_ptr(), _stream_ptr(torch, R1.device))
    _check(fn.__name__, st, h)
    return R1, R2, tau[:n]


# ---- batched ---------------------------------------------------------------

def _i64_array(values):
    import numpy as np
    a = np.ascontiguousarray(values, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def tsqr_batch_plan_create(handle, batch, n, m, a_offset, lda, dtype) -> int:
    """Plan for `batch` matrices; m, a_offset, lda are host integer sequences
    (lda may be None).  Returns the plan handle."""
    m_arr, m_p = _i64_array(m)
    o_arr, o_p = _i64_array(a_offset)
    if lda is None:
        l_p = ctypes.cast(None, ctypes.POINTER(ctypes.c_int64))
    else:
        l_arr, l_p = _i64_array(lda)
    plan = ctypes.c_void_p()
    st = lib().tsqr_batch_plan_create(handle, int(batch), int(n), m_p, o_p, l_p, int(dtype), ctypes.byref(plan))
    _check("tsqr_batch_plan_create", st, handle)
    return plan.value


def tsqr_batch_plan_destroy(plan) -> None:
    lib().tsqr_batch_plan_destroy(plan)


def tsqr_batch_workspace_bytes(plan) -> int:
    v = lib().tsqr_batch_workspace_bytes(plan)
    if v < 0:
        raise TsqrError("tsqr_batch_workspace_bytes", int(v))
    return int(v)


def tsqr_batch_plan_info(plan):
    t, l, r = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check("tsqr_batch_plan_info", lib().tsqr_batch_plan_info(plan, ctypes.byref(t), ctypes.byref(l), ctypes.byref(r)))
    return t.value, l.value, r.value


def tsqr_batch_plan_schedule(plan, batch):
    """(inst, tiles): int64 arrays of shape (batch, 7) and (tiles, 2), the
    schedule of a plan made for `batch` instances, as
    ``tsqr_batch_plan_schedule`` documents it."""
    import numpy as np
    t, _, _ = tsqr_batch_plan_info(plan)
    inst = np.zeros((int(batch), 7), dtype=np.int64)
    tiles = np.zeros((t, 2), dtype=np.int64)
    _check("tsqr_batch_plan_schedule",
           lib().tsqr_batch_plan_schedule(plan, inst.ctypes.data if inst.size else None,
                                          tiles.ctypes.data if tiles.size else None))
    return inst, tiles


def tsqr_batch_exec(plan, A, R, ldr, ws, ws_bytes, stream) -> int:
    return lib().tsqr_batch_exec(plan, A, R, ldr, ws, ws_bytes, stream)


def device_clock_khz(handle) -> int:
    """Rate of the device clock that ``BatchPlan.run_stamped`` reads, in kHz."""
    v = lib().tsqr_device_clock_khz(handle)
    if v <= 0:
        raise TsqrError("tsqr_device_clock_khz", int(v) if v > -1000 else int(-1000 - v))
    return int(v)


class BatchPlan:
    """Plan + workspace for a ragged batch held in one flat device tensor
    (instance b is the m[b]-by-n column-major block at element offset
    offsets[b]).  ``run(A_flat)`` returns a (batch, n, n) tensor whose [b] is
    instance b's R stored column-major (R[b].t() is the usual n x n view)."""

    def __init__(self, sizes, offsets, n, dtype, device=None, h=None):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.h = h or handle(self.dev.index or 0)
        self.n = int(n)
        self.batch = len(sizes)
        self.dtype = dtype
        code = TSQR_F64 if dtype == torch.float64 else TSQR_F32
        # elements of A the instances span (column-major, lda = m)
        self.a_elems = max([int(o) + int(m) * self.n for m, o in zip(sizes, offsets)] + [0])
        self.plan = tsqr_batch_plan_create(self.h, self.batch, self.n, sizes, offsets, None, code)
        nbytes = max(tsqr_batch_workspace_bytes(self.plan), 256)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)

    def info(self):
        return tsqr_batch_plan_info(self.plan)

    def run(self, A_flat, R=None):
        torch = self.torch
        _check_flat(A_flat, "A", self.a_elems, self.dtype, self.dev)
        if R is None:
            R = torch.empty((self.batch, self.n, self.n), dtype=self.dtype, device=self.dev)
        _check_flat(R, "R", self.batch * self.n * self.n, self.dtype, self.dev)
        st = tsqr_batch_exec(self.plan, A_flat.data_ptr(), R.data_ptr(), self.n, self.ws.data_ptr(),
                             self.ws.numel(), _stream_ptr(torch, self.dev))
        _check("tsqr_batch_exec", st, self.h)
        return R

    def run_stamped(self, A_flat, R=None, stamps=None):
        """``run`` that also measures the schedule: returns (R, stamps), stamps
        an int64 device tensor (tiles, 2) of each workgroup's start and end
        on the device clock (``device_clock_khz`` kHz, arbitrary origin), in
        the plan's tile order."""
        torch = self.torch
        _check_flat(A_flat, "A", self.a_elems, self.dtype, self.dev)
        if R is None:
            R = torch.empty((self.batch, self.n, self.n), dtype=self.dtype, device=self.dev)
        _check_flat(R, "R", self.batch * self.n * self.n, self.dtype, self.dev)
        tiles = self.info()[0]
        if stamps is None:
            stamps = torch.zeros((max(tiles, 1), 2), dtype=torch.int64, device=self.dev)
        _check_flat(stamps, "stamps", 2 * tiles, torch.int64, self.dev)
        st = lib().tsqr_batch_exec_stamped(self.plan, A_flat.data_ptr(), R.data_ptr(), self.n, self.ws.data_ptr(),
                                           self.ws.numel(), stamps.data_ptr(), _stream_ptr(torch, self.dev))
        _check("tsqr_batch_exec_stamped", st, self.h)
        return R, stamps

    def __del__(self):
        try:
            if getattr(self, "plan", None):
                tsqr_batch_plan_destroy(self.plan)
                self.plan = None
        except Exception:
            pass


# ---- mixed precision ------------------------------------------------------------

def tsqr_mixed_plan_create(handle, batch, m, n, lda, stride_a) -> int:
    plan = ctypes.c_void_p()
    st = lib().tsqr_mixed_plan_create(handle, int(batch), int(m), int(n), int(lda), int(stride_a), ctypes.byref(plan))
    _check("tsqr_mixed_plan_create", st, handle)
    return plan.value


def tsqr_mixed_plan_create_sampled(handle, batch, m, n, lda, stride_a, sample_rows, seed) -> int:
    plan = ctypes.c_void_p()
    st = lib().tsqr_mixed_plan_create_sampled(handle, int(batch), int(m), int(n), int(lda), int(stride_a),
                                              int(sample_rows), int(seed) & (2**64 - 1), ctypes.byref(plan))
    _check("tsqr_mixed_plan_create_sampled", st, handle)
    return plan.value


def tsqr_mixed_rtilde_offset(plan) -> int:
    v = lib().tsqr_mixed_rtilde_offset(plan)
    if v < 0:
        raise TsqrError("tsqr_mixed_rtilde_offset", int(v))
    return int(v)


def tsqr_mixed_plan_destroy(plan) -> None:
    lib().tsqr_mixed_plan_destroy(plan)


def tsqr_mixed_workspace_bytes(plan) -> int:
    v = lib().tsqr_mixed_workspace_bytes(plan)
    if v < 0:
        raise TsqrError("tsqr_mixed_workspace_bytes", int(v))
    return int(v)


def tsqr_mixed_exec(plan, A, R, ldr, fallback, ws, ws_bytes, stream) -> int:
    return lib().tsqr_mixed_exec(plan, A, R, ldr, fallback, ws, ws_bytes, stream)


class MixedPlan:
    """FP64-accurate R of `batch` FP32-stored m x n matrices held in one flat
    device tensor (instance b at element offset b * stride).  ``run(A)``
    returns (R, fallback): R a (batch, n, n) float64 tensor whose [b] is
    instance b's R stored column-major, fallback a list of 0/1 per instance
    (1: refactored by the FP64 path), which waits for the stream.
    ``launch(A, R, flags)`` only enqueues the work (no synchronization; the
    per-instance flags land in the int32 device tensor ``flags``), e.g. for
    capture in a HIP graph.  With ``sample_rows`` > 0 the FP32 factorization
    runs on a stratified row sample of that size (``seed`` picks it) instead
    of all of A; ``rtilde()`` returns the FP32 R~ of the last call."""

    def __init__(self, batch, m, n, stride=None, lda=None, device=None, h=None, sample_rows=0, seed=0):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.h = h or handle(self.dev.index or 0)
        self.batch, self.m, self.n = int(batch), int(m), int(n)
        lda = max(self.m, 1) if lda is None else int(lda)
        stride = lda * self.n if stride is None else int(stride)
        # elements of A the instances span
        self.a_elems = (self.batch - 1) * stride + (self.n - 1) * lda + self.m if self.batch and self.n and self.m else 0
        if sample_rows:
            self.plan = tsqr_mixed_plan_create_sampled(self.h, self.batch, self.m, self.n, lda, stride,
                                                       sample_rows, seed)
        else:
            self.plan = tsqr_mixed_plan_create(self.h, self.batch, self.m, self.n, lda, stride)
        nbytes = max(tsqr_mixed_workspace_bytes(self.plan), 256)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)

    def launch(self, A_flat, R, flags=None):
        torch = self.torch
        _check_flat(A_flat, "A", self.a_elems, torch.float32, self.dev)
        _check_flat(R, "R", self.batch * self.n * self.n, torch.float64, self.dev)
        if flags is not None:
            _check_flat(flags, "flags", self.batch, torch.int32, self.dev)
        st = tsqr_mixed_exec(self.plan, A_flat.data_ptr(), R.data_ptr(), self.n,
                             flags.data_ptr() if flags is not None else None, self.ws.data_ptr(),
                             self.ws.numel(), _stream_ptr(torch, self.dev))
        _check("tsqr_mixed_exec", st, self.h)

    def run(self, A_flat, R=None):
        torch = self.torch
        if R is None:
            R = torch.empty((self.batch, self.n, self.n), dtype=torch.float64, device=self.dev)
        flags = torch.zeros(max(self.batch, 1), dtype=torch.int32, device=self.dev)
        self.launch(A_flat, R, flags)
        return R, [int(v) for v in flags[:self.batch].cpu().tolist()]

    def launch_rtilde(self, A_flat, Rt, R, flags=None):
        """The correction with the caller's R~ (a (batch, n, n) float32 device
        tensor whose [b] is instance b's R~ stored column-major) instead of
        the plan's own FP32 factorization; otherwise as ``launch``."""
        torch = self.torch
        _check_flat(A_flat, "A", self.a_elems, torch.float32, self.dev)
        _check_flat(Rt, "Rt", self.batch * self.n * self.n, torch.float32, self.dev)
        _check_flat(R, "R", self.batch * self.n * self.n, torch.float64, self.dev)
        if flags is not None:
            _check_flat(flags, "flags", self.batch, torch.int32, self.dev)
        st = lib().tsqr_mixed_exec_rtilde(self.plan, A_flat.data_ptr(), Rt.data_ptr(), R.data_ptr(), self.n,
                                          flags.data_ptr() if flags is not None else None, self.ws.data_ptr(),
                                          self.ws.numel(), _stream_ptr(torch, self.dev))
        _check("tsqr_mixed_exec_rtilde", st, self.h)

    def launch_first_stage(self, A_flat):
        """Only the FP32 stage: R~ of A (or of the row sample) into the
        workspace, read with ``rtilde()``."""
        torch = self.torch
        _check_flat(A_flat, "A", self.a_elems, torch.float32, self.dev)
        st = lib().tsqr_mixed_rtilde_exec(self.plan, A_flat.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                                          _stream_ptr(torch, self.dev))
        _check("tsqr_mixed_rtilde_exec", st, self.h)

    def rtilde(self):
        """R~ of the last call, a (batch, n, n) float32 view of the workspace
        whose [b] is instance b's R~ stored column-major (read after the
        stream has finished the call)."""
        off = tsqr_mixed_rtilde_offset(self.plan)
        count = self.batch * self.n * self.n
        return self.ws[off:off + 4 * count].view(self.torch.float32).view(self.batch, self.n, self.n)

    def __del__(self):
        try:
            if getattr(self, "plan", None):
                tsqr_mixed_plan_destroy(self.plan)
                self.plan = None
        except Exception:
            pass


# ---- the Q factor -----------------------------------------------------------------

def tsqr_qr_workspace_bytes(handle, m, n, dtype=TSQR_F64) -> int:
    v = lib().tsqr_qr_workspace_bytes(handle, int(m), int(n), int(dtype))
    if v < 0:
        raise TsqrError("tsqr_qr_workspace_bytes", int(v) if v > -1000 else int(-1000 - v))
    return int(v)


def tsqr_geqr_qr_f64(handle, m, n, A, lda, Q, ldq, R, ldr, ws, ws_bytes, stream) -> int:
    return lib().tsqr_geqr_qr_f64(handle, m, n, A, lda, Q, ldq, R, ldr, ws, ws_bytes, stream)


def tsqr_geqr_qr_f32(handle, m, n, A, lda, Q, ldq, R, ldr, ws, ws_bytes, stream) -> int:
    return lib().tsqr_geqr_qr_f32(handle, m, n, A, lda, Q, ldq, R, ldr, ws, ws_bytes, stream)


class Factorization:
    """The factorization with its reflectors kept (``tsqr_geqrf_*``): ``R``,
    and ``apply_qt(B)`` = Q^T B for any device matrix B with m rows, without
    forming Q.  Holds the workspace the reflectors live in."""

    def __init__(self, A, h=None):
        import torch
        if A.dtype not in (torch.float64, torch.float32):
            raise TypeError("A must be float64 or float32")
        if not A.is_cuda:
            raise ValueError("A must be a device tensor")
        self.torch = torch
        self.m, self.n, lda = _col_major(A)
        self.dtype, self.dev = A.dtype, A.device
        self.h = h or handle(self.dev.index or 0)
        code = TSQR_F64 if A.dtype == torch.float64 else TSQR_F32
        self.ws = torch.empty(max(tsqr_qr_workspace_bytes(self.h, self.m, self.n, code), 256), dtype=torch.uint8,
                              device=self.dev)
        self.R = torch.empty((self.n, self.n), dtype=A.dtype, device=self.dev).t()
        fn = lib().tsqr_geqrf_f64 if A.dtype == torch.float64 else lib().tsqr_geqrf_f32
        st = fn(self.h, self.m, self.n, A.data_ptr(), lda, self.R.data_ptr(), max(self.n, 1), self.ws.data_ptr(),
                _ws_bytes(self.ws, self.dev), _stream_ptr(torch, self.dev))
        _check("tsqr_geqrf", st, self.h)

    def apply_qt(self, B, C=None):
        """C = Q^T B (n x k, column-major) for B (m x k, column-major) or a
        vector of length m (then C is a vector of length n)."""
        torch = self.torch
        vec = B.dim() == 1
        if vec:
            B = B.reshape(-1, 1)
        if B.dtype != self.dtype or B.device != self.dev:
            raise ValueError("B must match the factored matrix's dtype and device")
        mb, k, ldb = _col_major(B)
        if mb != self.m:
            raise ValueError(f"B has {mb} rows, the factored matrix {self.m}")
        if C is None:
            C = torch.empty((k, self.n), dtype=self.dtype, device=self.dev).t()
        ldc = _check_matrix(C, "C", self.n, k, self.dtype, self.dev)
        fn = lib().tsqr_apply_qt_f64 if self.dtype == torch.float64 else lib().tsqr_apply_qt_f32
        st = fn(self.h, self.m, self.n, k, B.data_ptr(), ldb, C.data_ptr(), ldc, self.ws.data_ptr(),
                _ws_bytes(self.ws, self.dev), _stream_ptr(torch, self.dev))
        _check("tsqr_apply_qt", st, self.h)
        return C.reshape(-1) if vec else C


def geqr_qr(A, Q=None, R=None, ws=None, h=None):
    """A = Q R for a column-major float64 or float32 device matrix A (m >= n):
    Q m x n with orthonormal columns, R n x n upper triangular with diag >= 0,
    both column-major.  Returns (Q, R)."""
    import torch
    if A.dtype not in (torch.float64, torch.float32):
        raise TypeError("A must be float64 or float32")
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    m, n, lda = _col_major(A)
    dev = A.device
    h = h or handle(dev.index or 0)
    if Q is None:
        Q = torch.empty((n, m), dtype=A.dtype, device=dev).t()
    if R is None:
        R = torch.empty((n, n), dtype=A.dtype, device=dev).t()
    ldq = _check_matrix(Q, "Q", m, n, A.dtype, dev)
    ldr = _check_matrix(R, "R", n, n, A.dtype, dev)
    code = TSQR_F64 if A.dtype == torch.float64 else TSQR_F32
    if ws is None:
        ws = torch.empty(max(tsqr_qr_workspace_bytes(h, m, n, code), 256), dtype=torch.uint8, device=dev)
    fn = tsqr_geqr_qr_f64 if A.dtype == torch.float64 else tsqr_geqr_qr_f32
    st = fn(h, m, n, A.data_ptr(), lda, Q.data_ptr(), ldq, R.data_ptr(), ldr, ws.data_ptr(),
            _ws_bytes(ws, dev), _stream_ptr(torch, dev))
    _check(fn.__name__, st, h)
    return Q, R

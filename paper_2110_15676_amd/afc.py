"""ctypes binding of libafc.so (C ABI in include/afc.h).

Argument marshalling only: every step of the AFC path runs in the HIP
library.  Entry points keep the C names.  Vectors passed to the step/solve
calls are torch float64 tensors on the GPU (device pointers); afc_create takes
numpy arrays (host memory) or torch GPU tensors (device memory).

The library is loaded on first use; if it has not been built this raises
instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libafc.so")

AFC_OK, AFC_WMAXIT = 0, 1
AFC_EINVAL, AFC_ENOMEM, AFC_ENOCONV, AFC_EBREAKDOWN, AFC_ENAN, AFC_EDEVICE, AFC_ECANCELED = -1, -2, -3, -4, -5, -6, -7
AFC_MEM_HOST, AFC_MEM_DEVICE = 0, 1
AFC_ALPHA_LIMITED, AFC_ALPHA_ONE, AFC_ALPHA_ZERO = 0, 1, 2
AFC_KRYLOV_BICGSTAB, AFC_KRYLOV_GMRES = 0, 1
AFC_PREC_FP64, AFC_PREC_MIXED = 0, 1
AFC_TOL_ABS_SQRTN, AFC_TOL_REL = 0, 1
AFC_LIMITER_MCL, AFC_LIMITER_MU = 0, 1
AFC_NOALLOC_SCRATCH_BYTES = 64 << 20  # include/afc.h


class afc_problem(ctypes.Structure):
    _fields_ = [
        ("n", c_int32), ("nnz", c_int64), ("mem_space", c_int32),
        ("row_ptr", c_void_p), ("col_idx", c_void_p), ("M", c_void_p), ("K", c_void_p),
        ("K_conv", c_void_p), ("ML", c_void_p), ("n_dir", c_int32), ("dir_idx", c_void_p), ("dir_val", c_void_p),
    ]


class afc_options(ctypes.Structure):
    _fields_ = [
        ("alpha_mode", c_int32), ("krylov", c_int32), ("restart", c_int32), ("precision", c_int32),
        ("lin_atol", c_double), ("lin_rtol", c_double), ("lin_maxit", c_int32),
        ("inner_rtol", c_double), ("inner_maxit", c_int32), ("refine_maxit", c_int32),
        ("fp_tol", c_double), ("fp_tol_mode", c_int32), ("fp_maxit", c_int32),
        ("prelimit", c_double), ("omega", c_double), ("dynamic_damping", c_int32),
        ("ssp_stages", c_int32), ("lanes_per_row", c_int32), ("profile", c_int32), ("limiter", c_int32),
        ("sstep", c_int32), ("sstep_shift", c_double), ("graphs", c_int32), ("lin_eta", c_double),
        ("stream", c_void_p),
    ]


class afc_request(ctypes.Structure):
    _fields_ = [
        ("kind", c_int32), ("problem", afc_problem), ("u0", c_void_p), ("F", c_void_p), ("dt", c_double),
        ("steps", c_int32), ("opt", afc_options),
    ]


class afc_server_config(ctypes.Structure):
    _fields_ = [
        ("slots", c_int32), ("hbm_budget_bytes", c_int64), ("fuse_max_nodes", c_int32), ("loop_threads", c_int32),
        ("loop_workgroups", c_int32), ("setup_threads", c_int32), ("max_active", c_int32), ("quantum_ms", c_double),
    ]


class afc_stats(ctypes.Structure):
    _fields_ = [
        ("status", c_int32), ("fp_iters", c_int32), ("krylov_iters", c_int64), ("inner_iters", c_int64),
        ("refine_sweeps", c_int32), ("res0", c_double), ("res", c_double), ("lin_res", c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = [
    "afc_default_options", "afc_create", "afc_set_options", "afc_step_ssprk3", "afc_step_cn",
    "afc_solve_stationary", "afc_destroy", "afc_status_str", "afc_last_error", "afc_kernel_time",
    "afc_batch_create", "afc_batch_offsets", "afc_batch_step_cn", "afc_batch_last_error", "afc_batch_destroy",
    "afc_footprint_bytes", "afc_server_create", "afc_server_submit", "afc_server_wait", "afc_server_poll", "afc_server_last_error",
    "afc_server_destroy", "afc_get_sell_info", "afc_get_krylov_sell_info", "afc_sell_layout", "afc_kernel_work", "afc_apply_operator",
    "afc_batch_set_schedule", "afc_batch_get_schedule", "afc_batch_autotune", "afc_step_cn_linear",
    "afc_step_mc_ssprk3", "afc_step_mc_cn", "afc_step_ssprk3_noalloc", "afc_residual_history",
    "afc_server_default_config", "afc_server_create_cfg", "afc_server_info",
]

AFC_REQ_CN, AFC_REQ_STATIONARY = 0, 1

AFC_KERNEL_SPMV32, AFC_KERNEL_SPMV64, AFC_KERNEL_DOTS, AFC_KERNEL_UPDATE = 0, 1, 2, 3
AFC_KERNEL_RESIDUAL, AFC_KERNEL_MCL, AFC_KERNEL_FINISH, AFC_KERNEL_COUNT = 4, 5, 6, 7

_lib = None


def lib():
    """Load libafc.so (once).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libafc.so is not built (run python -m paper_2110_15676_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        L.afc_default_options.argtypes = [POINTER(afc_options)]
        L.afc_default_options.restype = None
        L.afc_create.argtypes = [POINTER(afc_problem), POINTER(afc_options), POINTER(c_void_p)]
        L.afc_create.restype = c_int32
        L.afc_set_options.argtypes = [c_void_p, POINTER(afc_options)]
        L.afc_set_options.restype = c_int32
        L.afc_step_ssprk3.argtypes = [c_void_p, c_void_p, c_void_p, c_double, POINTER(afc_stats)]
        L.afc_step_ssprk3.restype = c_int32
        L.afc_step_ssprk3_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_double, POINTER(afc_stats)]
        L.afc_step_ssprk3_noalloc.restype = c_int32
        L.afc_step_cn.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_double, POINTER(afc_stats)]
        L.afc_step_cn.restype = c_int32
        L.afc_step_cn_linear.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_double, POINTER(afc_stats)]
        L.afc_step_cn_linear.restype = c_int32
        L.afc_step_mc_cn.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_double, POINTER(afc_stats)]
        L.afc_step_mc_cn.restype = c_int32
        L.afc_step_mc_ssprk3.argtypes = [c_void_p, c_void_p, c_void_p, c_double, POINTER(afc_stats)]
        L.afc_step_mc_ssprk3.restype = c_int32
        L.afc_solve_stationary.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, POINTER(afc_stats)]
        L.afc_solve_stationary.restype = c_int32
        L.afc_kernel_time.argtypes = [c_void_p, c_int32, POINTER(c_double), POINTER(c_int64), c_int32]
        L.afc_kernel_time.restype = c_int32
        L.afc_kernel_work.argtypes = [c_void_p, c_int32, POINTER(c_double), POINTER(c_int64)]
        L.afc_kernel_work.restype = c_int32
        L.afc_apply_operator.argtypes = [c_void_p, c_int32, c_void_p, c_void_p]
        L.afc_apply_operator.restype = c_int32
        L.afc_get_sell_info.argtypes = [c_void_p, POINTER(afc_sell_info)]
        L.afc_get_sell_info.restype = c_int32
        L.afc_get_krylov_sell_info.argtypes = [c_void_p, POINTER(afc_sell_info)]
        L.afc_get_krylov_sell_info.restype = c_int32
        L.afc_sell_layout.argtypes = [c_int32, c_void_p, c_void_p, POINTER(afc_sell_info)] + [c_void_p] * 5
        L.afc_sell_layout.restype = c_int32
        L.afc_batch_create.argtypes = [c_int32, POINTER(afc_problem), POINTER(afc_options), POINTER(c_void_p)]
        L.afc_batch_create.restype = c_int32
        L.afc_batch_offsets.argtypes = [c_void_p, POINTER(c_int64)]
        L.afc_batch_offsets.restype = c_int32
        L.afc_batch_step_cn.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(c_double), c_int32,
                                        POINTER(afc_stats)]
        L.afc_batch_step_cn.restype = c_int32
        L.afc_batch_set_schedule.argtypes = [c_void_p, POINTER(afc_batch_schedule)]
        L.afc_batch_set_schedule.restype = c_int32
        L.afc_batch_get_schedule.argtypes = [c_void_p, POINTER(afc_batch_schedule)]
        L.afc_batch_get_schedule.restype = c_int32
        L.afc_batch_autotune.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(c_double), c_int32,
                                         POINTER(afc_batch_schedule), POINTER(c_double), c_int32, POINTER(c_int32)]
        L.afc_batch_autotune.restype = c_int32
        L.afc_batch_last_error.argtypes = [c_void_p]
        L.afc_batch_last_error.restype = c_char_p
        L.afc_batch_destroy.argtypes = [c_void_p]
        L.afc_batch_destroy.restype = None
        L.afc_footprint_bytes.argtypes = [c_int32, c_int64, c_int32, POINTER(afc_options)]
        L.afc_footprint_bytes.restype = c_int64
        L.afc_server_create.argtypes = [c_int32, c_int64, POINTER(c_void_p)]
        L.afc_server_create.restype = c_int32
        L.afc_server_default_config.argtypes = [POINTER(afc_server_config)]
        L.afc_server_default_config.restype = None
        L.afc_server_create_cfg.argtypes = [POINTER(afc_server_config), POINTER(c_void_p)]
        L.afc_server_create_cfg.restype = c_int32
        L.afc_server_info.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)]
        L.afc_server_info.restype = c_int32
        L.afc_server_submit.argtypes = [c_void_p, POINTER(afc_request), POINTER(c_int64)]
        L.afc_server_submit.restype = c_int32
        L.afc_server_wait.argtypes = [c_void_p, c_int64, c_void_p, POINTER(afc_stats), POINTER(c_double)]
        L.afc_server_wait.restype = c_int32
        L.afc_server_poll.argtypes = [c_void_p, c_int64, POINTER(c_int32)]
        L.afc_server_poll.restype = c_int32
        L.afc_server_last_error.argtypes = [c_void_p]
        L.afc_server_last_error.restype = c_char_p
        L.afc_server_destroy.argtypes = [c_void_p]
        L.afc_server_destroy.restype = None
        L.afc_residual_history.argtypes = [c_void_p, POINTER(c_double), c_int32, POINTER(c_int32)]
        L.afc_residual_history.restype = c_int32
        L.afc_destroy.argtypes = [c_void_p]
        L.afc_destroy.restype = None
        L.afc_status_str.argtypes = [c_int32]
        L.afc_status_str.restype = c_char_p
        L.afc_last_error.argtypes = [c_void_p]
        L.afc_last_error.restype = c_char_p
        _lib = L
    return _lib


class afc_sell_info(ctypes.Structure):
    _fields_ = [("slices", c_int64), ("slots", c_int64), ("uniform_slices", c_int64),
                ("lane_delta_slots", c_int64), ("pattern_ints", c_int64), ("delta_bytes", c_int32),
                ("reserved", c_int32)]


class afc_batch_schedule(ctypes.Structure):
    _fields_ = [("threads", c_int32), ("workgroups", c_int32)]


class AFCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (afc_status_str(status), status, msg))
        self.status = status


def afc_status_str(status: int) -> str:
    return lib().afc_status_str(int(status)).decode()


def afc_last_error(h=None) -> str:
    return lib().afc_last_error(h).decode()


def afc_default_options(**overrides) -> afc_options:
    o = afc_options()
    lib().afc_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def _ptr(a):
    """(address, keepalive) of a contiguous numpy array or torch tensor."""
    if a is None:
        return None, None
    if isinstance(a, np.ndarray):
        a = np.ascontiguousarray(a)
        return a.ctypes.data, a
    if not a.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return a.data_ptr(), a


def _current_stream():
    import torch

    return torch.cuda.current_stream().cuda_stream


def afc_create(row_ptr, col_idx, M, K, K_conv=None, ML=None, dir_idx=None, dir_val=None, opts=None):
    """Create a handle from CSR arrays.  All arrays either numpy (host) or torch
    GPU tensors (device): int32 row_ptr/col_idx/dir_idx, float64 values."""
    is_np = isinstance(row_ptr, np.ndarray)
    if is_np:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        M = np.ascontiguousarray(M, dtype=np.float64)
        K = np.ascontiguousarray(K, dtype=np.float64)
        K_conv = None if K_conv is None else np.ascontiguousarray(K_conv, dtype=np.float64)
        ML = None if ML is None else np.ascontiguousarray(ML, dtype=np.float64)
        dir_idx = np.zeros(0, np.int32) if dir_idx is None else np.ascontiguousarray(dir_idx, dtype=np.int32)
        dir_val = np.zeros(0) if dir_val is None else np.ascontiguousarray(dir_val, dtype=np.float64)
    keep = []
    p = afc_problem()
    p.n = int(row_ptr.shape[0] - 1)
    p.nnz = int(col_idx.shape[0])
    p.mem_space = AFC_MEM_HOST if is_np else AFC_MEM_DEVICE
    for name, arr in (("row_ptr", row_ptr), ("col_idx", col_idx), ("M", M), ("K", K), ("K_conv", K_conv),
                      ("ML", ML), ("dir_idx", dir_idx), ("dir_val", dir_val)):
        addr, ka = _ptr(arr)
        keep.append(ka)
        setattr(p, name, addr)
    p.n_dir = 0 if dir_idx is None else int(dir_idx.shape[0])
    if opts is None:
        opts = afc_default_options()
    h = c_void_p()
    st = lib().afc_create(ctypes.byref(p), ctypes.byref(opts), ctypes.byref(h))
    if st != AFC_OK:
        raise AFCError(st, afc_last_error(None))
    return h


def afc_create_instance(inst, opts=None, conv=True):
    """afc_create from a paper_2110_15676_amd.inputs.Instance (host arrays)."""
    return afc_create(inst.row_ptr, inst.col, inst.M, inst.K, inst.K_conv if conv else None, None,
                      inst.dir_idx, inst.dir_val, opts)


def afc_set_options(h, opts):
    st = lib().afc_set_options(h, ctypes.byref(opts))
    if st != AFC_OK:
        raise AFCError(st, afc_last_error(h))


def _check_vec(t, n):
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            and t.numel() == n):
        raise ValueError("expected a contiguous float64 GPU tensor of %d elements" % n)


def _finish(h, st, stats, raise_on_error):
    if raise_on_error and st < 0:
        raise AFCError(st, afc_last_error(h))
    return st, stats.as_dict()


def afc_step_ssprk3(h, u, F, dt, raise_on_error=True):
    stats = afc_stats()
    st = lib().afc_step_ssprk3(h, u.data_ptr(), F.data_ptr(), float(dt), ctypes.byref(stats))
    return _finish(h, st, stats, raise_on_error)


def afc_step_ssprk3_noalloc(h, u, F, dt, raise_on_error=True):
    """afc_step_ssprk3 with its work vectors in the library's fixed per-GPU
    array (allocates nothing; see include/afc.h for the limits)."""
    stats = afc_stats()
    st = lib().afc_step_ssprk3_noalloc(h, u.data_ptr(), F.data_ptr(), float(dt), ctypes.byref(stats))
    return _finish(h, st, stats, raise_on_error)


def afc_step_cn(h, u, F_old, F_new, dt, raise_on_error=True):
    stats = afc_stats()
    st = lib().afc_step_cn(h, u.data_ptr(), F_old.data_ptr(), F_new.data_ptr(), float(dt), ctypes.byref(stats))
    return _finish(h, st, stats, raise_on_error)


def afc_step_cn_linear(h, u, F_old, F_new, dt, raise_on_error=True):
    """One linear Zal+CN step (fluxes at u* = 2 u~ - u^{n-1}, one linear solve)."""
    stats = afc_stats()
    st = lib().afc_step_cn_linear(h, u.data_ptr(), F_old.data_ptr(), F_new.data_ptr(), float(dt),
                                  ctypes.byref(stats))
    return _finish(h, st, stats, raise_on_error)


def afc_step_mc_ssprk3(h, u, F, dt, raise_on_error=True):
    """One SSP step (options.ssp_stages) with the time-dependent MC limiter."""
    stats = afc_stats()
    st = lib().afc_step_mc_ssprk3(h, u.data_ptr(), F.data_ptr(), float(dt), ctypes.byref(stats))
    return _finish(h, st, stats, raise_on_error)


def afc_step_mc_cn(h, u, F_old, F_new, dt, raise_on_error=True):
    """One MC+CN step (fixed point of Sec. 4)."""
    stats = afc_stats()
    st = lib().afc_step_mc_cn(h, u.data_ptr(), F_old.data_ptr(), F_new.data_ptr(), float(dt), ctypes.byref(stats))
    return _finish(h, st, stats, raise_on_error)


def afc_solve_stationary(h, u, F, init_low_order=False, raise_on_error=True):
    stats = afc_stats()
    st = lib().afc_solve_stationary(h, u.data_ptr(), F.data_ptr(), int(bool(init_low_order)), ctypes.byref(stats))
    return _finish(h, st, stats, raise_on_error)


def afc_residual_history(h):
    """Nonlinear residuals of the last fixed-point call on h (numpy array)."""
    n = c_int32()
    st = lib().afc_residual_history(h, None, 0, ctypes.byref(n))
    if st != AFC_OK:
        raise AFCError(st, "afc_residual_history")
    out = np.zeros(max(1, n.value))
    st = lib().afc_residual_history(h, out.ctypes.data_as(POINTER(c_double)), n.value, ctypes.byref(n))
    if st != AFC_OK:
        raise AFCError(st, "afc_residual_history")
    return out[:n.value]


def afc_kernel_time(h, kernel, reset=False):
    """(total milliseconds, launches) of one kernel class timed with HIP events."""
    ms = c_double()
    n = c_int64()
    st = lib().afc_kernel_time(h, int(kernel), ctypes.byref(ms), ctypes.byref(n), int(bool(reset)))
    if st != AFC_OK:
        raise AFCError(st, "afc_kernel_time")
    return ms.value, n.value


AFC_APPLY_RESIDUAL, AFC_APPLY_SCALED64, AFC_APPLY_SCALED32, AFC_APPLY_BICG = 0, 1, 2, 3


def afc_apply_operator(h, op, x, y):
    """y := y - A x (op 0) or y = A D^{-1} x (ops 1-3, FP64 / FP32 / BiCGStab
    SpMV) by the library's SELL kernels; x, y: device tensors of n doubles."""
    st = lib().afc_apply_operator(h, int(op), x.data_ptr(), y.data_ptr())
    if st != AFC_OK:
        raise AFCError(st, "afc_apply_operator")


def afc_kernel_work(h, kernel):
    """(algorithmic bytes, launches that did work) of one profiled kernel class."""
    b = c_double()
    n = c_int64()
    st = lib().afc_kernel_work(h, int(kernel), ctypes.byref(b), ctypes.byref(n))
    if st != AFC_OK:
        raise AFCError(st, "afc_kernel_work")
    return b.value, n.value


def afc_get_sell_info(h):
    """Sizes of the handle's SELL-64 matrix storage (dict)."""
    info = afc_sell_info()
    st = lib().afc_get_sell_info(h, ctypes.byref(info))
    if st != AFC_OK:
        raise AFCError(st, "afc_get_sell_info")
    return {name: getattr(info, name) for name, _ in afc_sell_info._fields_ if name != "reserved"}


def afc_get_krylov_sell_info(h):
    """Sizes of the SELL-64 storage of the handle's FP32 Krylov matrices (the
    pattern without its diagonal), as a dict."""
    info = afc_sell_info()
    st = lib().afc_get_krylov_sell_info(h, ctypes.byref(info))
    if st != AFC_OK:
        raise AFCError(st, "afc_get_krylov_sell_info")
    return {name: getattr(info, name) for name, _ in afc_sell_info._fields_ if name != "reserved"}


def afc_sell_layout(row_ptr, col):
    """Host SELL-64 layout of a CSR pattern (numpy int32 arrays): returns
    (info dict, slice_ptr, slice_delta, pattern, pos, lane_deltas)."""
    import numpy as np

    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    n = rp.shape[0] - 1
    info = afc_sell_info()
    ptr = lambda a: a.ctypes.data_as(c_void_p)  # noqa: E731
    st = lib().afc_sell_layout(n, ptr(rp), ptr(cl), ctypes.byref(info), None, None, None, None, None)
    if st != AFC_OK:
        raise AFCError(st, "afc_sell_layout")
    out = [np.zeros(max(1, m), dtype=np.int32) for m in (info.slices + 1, info.slices, info.pattern_ints,
                                                         rp[-1], info.lane_delta_slots)]
    st = lib().afc_sell_layout(n, ptr(rp), ptr(cl), ctypes.byref(info), *[ptr(a) for a in out])
    if st != AFC_OK:
        raise AFCError(st, "afc_sell_layout")
    sizes = (info.slices + 1, info.slices, info.pattern_ints, int(rp[-1]), info.lane_delta_slots)
    d = {name: getattr(info, name) for name, _ in afc_sell_info._fields_ if name != "reserved"}
    return (d, *[a[:m] for a, m in zip(out, sizes)])


def afc_destroy(h):
    if h is not None and h.value:
        lib().afc_destroy(h)


# ---------------------------------------------------------------------------
# batched CN-FCT
# ---------------------------------------------------------------------------


def _host_problem(row_ptr, col, M, K, dir_idx, dir_val, keep):
    arrs = [np.ascontiguousarray(row_ptr, dtype=np.int32), np.ascontiguousarray(col, dtype=np.int32),
            np.ascontiguousarray(M, dtype=np.float64), np.ascontiguousarray(K, dtype=np.float64),
            np.ascontiguousarray(dir_idx, dtype=np.int32), np.ascontiguousarray(dir_val, dtype=np.float64)]
    keep.extend(arrs)
    p = afc_problem()
    p.n = int(arrs[0].shape[0] - 1)
    p.nnz = int(arrs[1].shape[0])
    p.mem_space = AFC_MEM_HOST
    p.row_ptr, p.col_idx, p.M, p.K = (a.ctypes.data for a in arrs[:4])
    p.K_conv = None
    p.ML = None
    p.n_dir = int(arrs[4].shape[0])
    p.dir_idx = arrs[4].ctypes.data
    p.dir_val = arrs[5].ctypes.data
    return p


def afc_batch_create(instances, opts=None):
    """Batch handle from a list of inputs.Instance (host arrays)."""
    keep = []
    probs = (afc_problem * len(instances))()
    for q, inst in enumerate(instances):
        probs[q] = _host_problem(inst.row_ptr, inst.col, inst.M, inst.K, inst.dir_idx, inst.dir_val, keep)
    if opts is None:
        opts = afc_default_options(krylov=AFC_KRYLOV_BICGSTAB)
    b = c_void_p()
    st = lib().afc_batch_create(len(instances), probs, ctypes.byref(opts), ctypes.byref(b))
    if st != AFC_OK:
        raise AFCError(st, lib().afc_batch_last_error(None).decode())
    return b


def afc_batch_offsets(b, count):
    off = (c_int64 * (count + 1))()
    st = lib().afc_batch_offsets(b, off)
    if st != AFC_OK:
        raise AFCError(st, "afc_batch_offsets")
    return np.array(off[:], dtype=np.int64)


def afc_batch_step_cn(b, u, F, dt, steps, raise_on_error=True):
    """Advance every instance by `steps` CN-FCT steps; dt: one value per instance."""
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    stats = (afc_stats * dt.shape[0])()
    st = lib().afc_batch_step_cn(b, u.data_ptr(), F.data_ptr(), dt.ctypes.data_as(POINTER(c_double)), int(steps),
                                 stats)
    if raise_on_error and st < 0:
        raise AFCError(st, lib().afc_batch_last_error(b).decode())
    return st, [s.as_dict() for s in stats]


def afc_batch_set_schedule(b, threads, workgroups=0):
    """Workgroup size (256, 512, 1024) and workgroup count (0 = automatic) of
    the persistent launch; results do not depend on them."""
    sch = afc_batch_schedule(int(threads), int(workgroups))
    st = lib().afc_batch_set_schedule(b, ctypes.byref(sch))
    if st != AFC_OK:
        raise AFCError(st, lib().afc_batch_last_error(b).decode())


def afc_batch_get_schedule(b):
    sch = afc_batch_schedule()
    st = lib().afc_batch_get_schedule(b, ctypes.byref(sch))
    if st != AFC_OK:
        raise AFCError(st, "afc_batch_get_schedule")
    return sch.threads, sch.workgroups


def afc_batch_autotune(b, u, F, dt, trial_steps=1):
    """Time the candidate schedules on a scratch copy of u and keep the
    fastest; returns ((threads, workgroups), [trial ms ...])."""
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    chosen = afc_batch_schedule()
    times = (c_double * 16)()
    n = c_int32()
    st = lib().afc_batch_autotune(b, u.data_ptr(), F.data_ptr(), dt.ctypes.data_as(POINTER(c_double)),
                                  int(trial_steps), ctypes.byref(chosen), times, 16, ctypes.byref(n))
    if st != AFC_OK:
        raise AFCError(st, lib().afc_batch_last_error(b).decode())
    return (chosen.threads, chosen.workgroups), [times[i] for i in range(min(n.value, 16))]


def afc_batch_destroy(b):
    if b is not None and b.value:
        lib().afc_batch_destroy(b)


# ---------------------------------------------------------------------------
# request server
# ---------------------------------------------------------------------------


def afc_footprint_bytes(n, nnz, kind, opts=None):
    o = opts if opts is not None else afc_default_options()
    return int(lib().afc_footprint_bytes(int(n), int(nnz), int(kind), ctypes.byref(o)))


def afc_server_default_config(**overrides):
    c = afc_server_config()
    lib().afc_server_default_config(ctypes.byref(c))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def afc_server_create_cfg(cfg):
    s = c_void_p()
    st = lib().afc_server_create_cfg(ctypes.byref(cfg), ctypes.byref(s))
    if st != AFC_OK:
        raise AFCError(st, "afc_server_create_cfg")
    return s


def afc_server_info(s):
    """(rounds run by the fused lane, requests carried summed over rounds,
    admitted footprint in bytes)."""
    rounds = c_int64()
    carried = c_int64()
    used = c_int64()
    st = lib().afc_server_info(s, ctypes.byref(rounds), ctypes.byref(carried), ctypes.byref(used))
    if st != AFC_OK:
        raise AFCError(st, "afc_server_info")
    return rounds.value, carried.value, used.value


def afc_server_create(slots, hbm_budget_bytes):
    s = c_void_p()
    st = lib().afc_server_create(int(slots), int(hbm_budget_bytes), ctypes.byref(s))
    if st != AFC_OK:
        raise AFCError(st, "afc_server_create")
    return s


def afc_server_submit(s, kind, inst, opts, u0=None, dt=0.0, steps=0, conv=True):
    """Queue one request built from an inputs.Instance; returns its id."""
    keep = []
    req = afc_request()
    req.kind = int(kind)
    req.problem = _host_problem(inst.row_ptr, inst.col, inst.M, inst.K, inst.dir_idx, inst.dir_val, keep)
    if conv:
        kc = np.ascontiguousarray(inst.K_conv, dtype=np.float64)
        keep.append(kc)
        req.problem.K_conv = kc.ctypes.data
    F = np.ascontiguousarray(inst.F, dtype=np.float64)
    keep.append(F)
    req.F = F.ctypes.data
    if u0 is not None:
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        keep.append(u0)
        req.u0 = u0.ctypes.data
    req.dt = float(dt)
    req.steps = int(steps)
    req.opt = opts
    rid = c_int64()
    st = lib().afc_server_submit(s, ctypes.byref(req), ctypes.byref(rid))
    if st != AFC_OK:
        raise AFCError(st, lib().afc_server_last_error(s).decode())
    return rid.value


def afc_server_wait(s, rid, n):
    """(status, u (numpy), stats dict, (queued s, service s, latency s))."""
    u = np.zeros(n)
    stats = afc_stats()
    times = (c_double * 3)()
    st = lib().afc_server_wait(s, int(rid), u.ctypes.data, ctypes.byref(stats), times)
    return st, u, stats.as_dict(), tuple(times)


def afc_server_poll(s, rid):
    """True once request rid has finished (non-blocking)."""
    done = c_int32()
    st = lib().afc_server_poll(s, int(rid), ctypes.byref(done))
    if st != AFC_OK:
        raise AFCError(st, "unknown request id %d" % int(rid))
    return bool(done.value)


def afc_server_destroy(s):
    if s is not None and s.value:
        lib().afc_server_destroy(s)

"""Python binding of the kdcd C-ABI (include/kdcd.h).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the solvers runs in the HIP library
``libkdcd.so`` built in this package directory.  Importing this module on a
machine without the built library raises immediately -- there is no CPU
fallback.

The binding checks what the C-ABI cannot see through plain pointers
(device, dtype, contiguity and lengths of every buffer), so that a wrong
tensor becomes a Python error rather than an out-of-bounds device access.
"""
from __future__ import annotations

import ctypes
import os
from typing import NamedTuple, Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("KDCD_LIBRARY") or os.path.join(_HERE, "libkdcd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"kdcd HIP library not built: {LIB_PATH} is missing "
                      "(run __graft_entry__.build())")
_lib = ctypes.CDLL(LIB_PATH)

KERNEL_LINEAR, KERNEL_POLY, KERNEL_RBF = 0, 1, 2
DENSE, CSR_FORMAT = 0, 1
COMPUTE = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "bf16x3": 4}
FLAG_GRAPH = 1
FLAG_TIME_PRODUCT = 4
FLAG_TIME_SAMPLE = 8
FLAG_LOOKAHEAD = 16
FLAG_SERIAL = 32

STATUS = {0: "KDCD_OK", -1: "KDCD_ERR_INVALID_ARG", -2: "KDCD_ERR_UNSUPPORTED",
          -3: "KDCD_ERR_INDEX_RANGE", -4: "KDCD_ERR_INDEX_DUPLICATE", -5: "KDCD_ERR_NOT_SPD",
          -6: "KDCD_ERR_NONFINITE", -7: "KDCD_ERR_HIP", -8: "KDCD_ERR_ALLOC",
          -9: "KDCD_ERR_WORKSPACE"}


class Kernel(NamedTuple):
    """Table 1 kernel: kind 0 linear, 1 polynomial (c + x.z)^degree, 2 RBF exp(-sigma |x-z|^2)."""
    kind: int
    sigma: float = 0.0
    c: float = 0.0
    degree: int = 1


class CSR(NamedTuple):
    """CSR matrix on the device: row_ptr int64 (m+1), col_idx int32 (nnz), values float64 (nnz)."""
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    values: torch.Tensor
    m: int
    n: int


class KdcdError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({kdcd_status_string(status)})")


class _Matrix(ctypes.Structure):
    _fields_ = [("format", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("values", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class _Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("c", ctypes.c_double)]


class _Profile(ctypes.Structure):
    _fields_ = [("kblock_ms", ctypes.c_double), ("kblock_launches", ctypes.c_int64),
                ("finish_ms", ctypes.c_double), ("finish_launches", ctypes.c_int64),
                ("recur_ms", ctypes.c_double), ("recur_launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class _BatchProblem(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int32), ("loss", ctypes.c_int32),
                ("param", ctypes.c_double), ("sigma", ctypes.c_double),
                ("y", ctypes.c_void_p), ("alpha", ctypes.c_void_p), ("trace", ctypes.c_void_p)]


class _Sampling(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("epsilon", ctypes.c_double),
                ("tau", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("idx_out", ctypes.c_void_p), ("features_out", ctypes.c_void_p),
                ("grad_out", ctypes.c_void_p), ("pool", ctypes.c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("compute", ctypes.c_int32), ("loss", ctypes.c_int32),
                ("snapshot_every", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("snapshots", ctypes.c_void_p), ("trace", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("profile", ctypes.c_void_p), ("monitor_every", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tol", ctypes.c_double),
                ("outer_done", ctypes.c_void_p), ("rel_err", ctypes.c_void_p),
                ("monitor_log", ctypes.c_void_p), ("monitor_log_len", ctypes.c_int64)]


_P = ctypes.c_void_p
_lib.kdcd_ksvm_solve.restype = ctypes.c_int
_lib.kdcd_ksvm_solve.argtypes = [_P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int64, _P, _P, _P, _P]
_lib.kdcd_krr_solve.restype = ctypes.c_int
_lib.kdcd_krr_solve.argtypes = _lib.kdcd_ksvm_solve.argtypes
_lib.kdcd_krr_solve_noalloc.restype = ctypes.c_int
_lib.kdcd_krr_solve_noalloc.argtypes = _lib.kdcd_ksvm_solve.argtypes
_lib.kdcd_batch_solve.restype = ctypes.c_int
_lib.kdcd_batch_solve.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P, _P,
                                  ctypes.c_int32, _P, _P]
_lib.kdcd_sampler_create.restype = ctypes.c_int
_lib.kdcd_sampler_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint64]
_lib.kdcd_sampler_destroy.restype = None
_lib.kdcd_sampler_destroy.argtypes = [_P]
_lib.kdcd_sampler_get_params.restype = ctypes.c_int
_lib.kdcd_sampler_get_params.argtypes = [_P, _P, _P]
_lib.kdcd_sampler_set_params.restype = ctypes.c_int
_lib.kdcd_sampler_set_params.argtypes = [_P, _P, _P]
_lib.kdcd_sampler_forward.restype = ctypes.c_int
_lib.kdcd_sampler_forward.argtypes = [_P, _P, ctypes.c_int64, _P, _P]
_lib.kdcd_sampler_grad.restype = ctypes.c_int
_lib.kdcd_sampler_grad.argtypes = [_P, _P, _P, ctypes.c_int64, _P, _P, _P]
_lib.kdcd_sampler_train.restype = ctypes.c_int
_lib.kdcd_sampler_train.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_float, _P, _P]
_lib.kdcd_sampler_keys.restype = ctypes.c_int
_lib.kdcd_sampler_keys.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                   ctypes.c_int64, _P, _P]
_lib.kdcd_sampler_select.restype = ctypes.c_int
_lib.kdcd_sampler_select.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_uint64, ctypes.c_int64, _P, _P]
_lib.kdcd_ksvm_solve_sampled.restype = ctypes.c_int
_lib.kdcd_ksvm_solve_sampled.argtypes = [_P, _P, _P, ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_int64, _P, _P, _P, _P]
_lib.kdcd_graph_cache_clear.restype = None
_lib.kdcd_graph_cache_clear.argtypes = []
_lib.kdcd_tune_configs.restype = ctypes.c_int32
_lib.kdcd_tune_configs.argtypes = [ctypes.c_int32, _P, _P, _P, ctypes.c_int32]
_lib.kdcd_tune_set.restype = ctypes.c_int
_lib.kdcd_tune_set.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
_lib.kdcd_tune_get.restype = ctypes.c_int32
_lib.kdcd_tune_get.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
_lib.kdcd_autotune.restype = ctypes.c_int
_lib.kdcd_autotune.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]
_lib.kdcd_batch_eval.restype = ctypes.c_int
_lib.kdcd_batch_eval.argtypes = [_P, _P, _P, ctypes.c_int32, _P, _P]
_lib.kdcd_autotune_batch.restype = ctypes.c_int
_lib.kdcd_autotune_batch.argtypes = [_P, _P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, _P, _P, _P]
_lib.kdcd_tune_save.restype = ctypes.c_int
_lib.kdcd_tune_save.argtypes = [ctypes.c_char_p]
_lib.kdcd_tune_load.restype = ctypes.c_int
_lib.kdcd_tune_load.argtypes = [ctypes.c_char_p]
_lib.kdcd_kernel_rhs.restype = ctypes.c_int
_lib.kdcd_kernel_rhs.argtypes = [_P, _P, _P, ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int32, _P]
_lib.kdcd_ksvm_eval.restype = ctypes.c_int
_lib.kdcd_ksvm_eval.argtypes = [_P, _P, _P, ctypes.c_double, ctypes.c_int32, _P, _P, _P]
_lib.kdcd_krr_eval.restype = ctypes.c_int
_lib.kdcd_krr_eval.argtypes = [_P, _P, _P, ctypes.c_double, _P, _P, _P]
_lib.kdcd_workspace_bytes.restype = ctypes.c_size_t
_lib.kdcd_workspace_bytes.argtypes = [ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32]
_lib.kdcd_nystrom_features.restype = ctypes.c_int
_lib.kdcd_nystrom_features.argtypes = [_P, _P, _P, ctypes.c_int32, ctypes.c_double, _P, _P,
                                       ctypes.c_int64, _P]
_lib.kdcd_lowrank_solve.restype = ctypes.c_int
_lib.kdcd_lowrank_solve.argtypes = [ctypes.c_int32, _P, _P, ctypes.c_double, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int64, _P, _P, _P, _P, _P]
_lib.kdcd_status_string.restype = ctypes.c_char_p
_lib.kdcd_status_string.argtypes = [ctypes.c_int]
_lib.kdcd_version.restype = ctypes.c_char_p
_lib.kdcd_version.argtypes = []


def kdcd_status_string(status: int) -> str:
    return _lib.kdcd_status_string(int(status)).decode()


def kdcd_version() -> str:
    return _lib.kdcd_version().decode()


# ------------------------------------------------------------- marshalling

def _dev(t: torch.Tensor, dtype: torch.dtype, n: Optional[int], name: str) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {n}")
    return t.data_ptr()


def _matrix(A) -> tuple[_Matrix, int, int]:
    mat = _Matrix()
    if isinstance(A, CSR):
        m, n = int(A.m), int(A.n)
        _dev(A.row_ptr, torch.int64, m + 1, "A.row_ptr")
        nnz = int(A.values.numel())
        mat.format, mat.m, mat.n, mat.ld, mat.nnz = CSR_FORMAT, m, n, n, nnz
        mat.values = _dev(A.values, torch.float64, nnz, "A.values")
        mat.row_ptr = A.row_ptr.data_ptr()
        mat.col_idx = _dev(A.col_idx, torch.int32, nnz, "A.col_idx")
    else:
        if A.dim() != 2:
            raise ValueError("dense A must be 2-D (m x n)")
        m, n = A.shape
        if A.stride(1) != 1:
            raise ValueError("dense A must be row-major with unit column stride")
        mat.format, mat.m, mat.n, mat.ld, mat.nnz = DENSE, m, n, A.stride(0), 0
        if A.device.type != "cuda" or A.dtype != torch.float64:
            raise TypeError("dense A must be a float64 GPU tensor")
        mat.values = A.data_ptr()
        mat.row_ptr = mat.col_idx = None
    return mat, int(mat.m), int(mat.n)


def _kernel(k) -> _Kernel:
    k = k if isinstance(k, Kernel) else Kernel(*k)
    return _Kernel(int(k.kind), int(k.degree), float(k.sigma), float(k.c))


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class _MonitorOut:
    def __init__(self, n_outer=0, every=0, log=False):
        self.outer = ctypes.c_int64(-1)
        self.rel = ctypes.c_double(float("nan"))
        # one record per evaluation: every `every` outer iterations and after the last
        # (log may also be the caller's (records, 4) float64 device tensor)
        if isinstance(log, torch.Tensor):
            _dev(log, torch.float64, None, "monitor_log")
            if log.dim() != 2 or log.shape[1] != 4:
                raise ValueError("monitor_log must be a (records, 4) tensor")
            self.log = log
        else:
            self.log = (torch.full((n_outer // max(every, 1) + 2, 4), float("nan"),
                                   dtype=torch.float64, device="cuda") if log else None)


def _options(compute, loss, snapshot_every, snapshots, trace, workspace, profile, flags,
             m, n_outer, n_updates, monitor_every=0, tol=0.0, mon=None):
    o = _Options()
    o.monitor_every = int(monitor_every)
    o.tol = float(tol)
    if mon is not None:
        o.outer_done = ctypes.cast(ctypes.pointer(mon.outer), ctypes.c_void_p)
        o.rel_err = ctypes.cast(ctypes.pointer(mon.rel), ctypes.c_void_p)
        if mon.log is not None:
            o.monitor_log = mon.log.data_ptr()
            o.monitor_log_len = mon.log.shape[0]
    o.compute = COMPUTE[compute] if isinstance(compute, str) else int(compute)
    o.loss = int(loss)
    o.snapshot_every = int(snapshot_every)
    o.flags = int(flags)
    if snapshot_every:
        rows = -(-n_outer // int(snapshot_every))
        o.snapshots = _dev(snapshots, torch.float64, rows * m, "snapshots")
    if trace is not None:
        o.trace = _dev(trace, torch.float64, n_updates, "trace")
    if workspace is not None:
        o.workspace = _dev(workspace, torch.uint8, None, "workspace")
        o.workspace_bytes = workspace.numel()
    prof = None
    if profile:
        prof = _Profile()
        o.profile = ctypes.cast(ctypes.pointer(prof), ctypes.c_void_p)
    return o, prof


def _result(prof, mon):
    """Profile fields and / or the monitor's outcome as one dict, or None."""
    if prof is None and mon is None:
        return None
    out = {f: getattr(prof, f) for f, _ in _Profile._fields_} if prof is not None else {}
    if mon is not None:
        out["outer_done"] = mon.outer.value
        out["rel_err"] = mon.rel.value
        if mon.log is not None:
            # (outer iterations done, certified relative error, objective, seconds)
            out["log"] = [tuple(r) for r in mon.log.cpu().tolist() if r[0] == r[0]]
    return out


def _solve(fn, name, A, y, kernel, param, b, s, H, idx, alpha, compute, loss, snapshot_every,
           snapshots, trace, workspace, profile, flags, stream, monitor_every=0, tol=0.0,
           monitor_log=False):
    mat, m, _ = _matrix(A)
    _dev(y, torch.float64, m, "y")
    _dev(alpha, torch.float64, m, "alpha")
    _dev(idx, torch.int32, int(H) * int(b), "idx")
    n_outer = -(-int(H) // max(int(s), 1))
    mon = _MonitorOut(n_outer, int(monitor_every), monitor_log) if monitor_every else None
    opt, prof = _options(compute, loss, snapshot_every, snapshots, trace, workspace, profile,
                         flags, m, n_outer, int(H) * int(b), monitor_every, tol, mon)
    kern = _kernel(kernel)
    st = fn(ctypes.byref(mat), y.data_ptr(), ctypes.byref(kern), float(param), int(b), int(s),
            int(H), idx.data_ptr(), alpha.data_ptr(), ctypes.byref(opt), _stream(stream))
    if st != 0:
        raise KdcdError(st, name)
    return _result(prof, mon)


def kdcd_ksvm_solve(A, y, kernel, C, b, s, H, idx, alpha, *, compute="f64", loss=1,
                    snapshot_every=0, snapshots=None, trace=None, workspace=None, profile=False,
                    flags=0, stream=None, monitor_every=0, tol=0.0, monitor_log=False):
    """s-step DCD for K-SVM (Algorithm 2); alpha is updated in place.
    Returns a dict with the stage timings (profile=True) and the monitor's
    outer_done / rel_err (monitor_every > 0; with monitor_log=True also its
    records as "log"), else None."""
    return _solve(_lib.kdcd_ksvm_solve, "kdcd_ksvm_solve", A, y, kernel, C, b, s, H, idx, alpha,
                  compute, loss, snapshot_every, snapshots, trace, workspace, profile, flags,
                  stream, monitor_every, tol, monitor_log)


def kdcd_krr_solve(A, y, kernel, lam, b, s, H, idx, alpha, *, compute="f64", snapshot_every=0,
                   snapshots=None, trace=None, workspace=None, profile=False, flags=0,
                   stream=None, monitor_every=0, tol=0.0, monitor_log=False):
    """s-step BDCD for K-RR (Algorithm 4); alpha is updated in place."""
    return _solve(_lib.kdcd_krr_solve, "kdcd_krr_solve", A, y, kernel, lam, b, s, H, idx, alpha,
                  compute, 1, snapshot_every, snapshots, trace, workspace, profile, flags, stream,
                  monitor_every, tol, monitor_log)


def kdcd_krr_solve_noalloc(A, y, kernel, lam, b, s, H, idx, alpha, *, compute="f64",
                           snapshot_every=0, snapshots=None, trace=None, stream=None):
    """kdcd_krr_solve with the library's fixed device workspace (no allocation)."""
    return _solve(_lib.kdcd_krr_solve_noalloc, "kdcd_krr_solve_noalloc", A, y, kernel, lam, b, s,
                  H, idx, alpha, compute, 1, snapshot_every, snapshots, trace, None, False, 0,
                  stream)


NOALLOC_SCRATCH_BYTES = 32 << 20


def kdcd_nystrom_features(A, kernel, L, jitter, Phi, X=None, stream=None):
    """Nystrom factor of K from the landmark rows L of A into Phi (rows of X,
    or of A when X is None): Phi Phi'^T = K(X, A_L) (K_LL + jitter I)^{-1} K(A_L, X')."""
    mat, m, n = _matrix(A)
    r = int(L.numel())
    _dev(L, torch.int32, r, "L")
    xm = None
    rows = m
    if X is not None:
        xm, rows, _ = _matrix(X)
    if Phi.dim() != 2 or Phi.shape[0] < rows or Phi.stride(1) != 1 or Phi.shape[1] < r:
        raise ValueError("Phi must be a row-major (rows x >= r) float64 GPU tensor")
    if Phi.device.type != "cuda" or Phi.dtype != torch.float64:
        raise TypeError("Phi must be a float64 GPU tensor")
    kern = _kernel(kernel)
    st = _lib.kdcd_nystrom_features(ctypes.byref(mat), ctypes.byref(kern), L.data_ptr(), r,
                                    float(jitter), ctypes.byref(xm) if xm is not None else None,
                                    Phi.data_ptr(), Phi.stride(0), _stream(stream))
    if st != 0:
        raise KdcdError(st, "kdcd_nystrom_features")


def kdcd_lowrank_solve(problem, Phi, y, param, b, s, H, idx, alpha, *, z=None, loss=1,
                       snapshot_every=0, snapshots=None, trace=None, profile=False, stream=None):
    """Algorithm 2 ("ksvm") or 4 ("krr") with K replaced by Phi Phi^T; alpha
    is updated in place, z (r doubles, optional) receives Phi^T beta."""
    pid = {"ksvm": 0, "krr": 1}[problem] if isinstance(problem, str) else int(problem)
    mat, m, r = _matrix(Phi)
    _dev(y, torch.float64, m, "y")
    _dev(alpha, torch.float64, m, "alpha")
    _dev(idx, torch.int32, int(H) * int(b), "idx")
    zp = _dev(z, torch.float64, r, "z") if z is not None else None
    n_outer = -(-int(H) // max(int(s), 1))
    opt, prof = _options("f64", loss, snapshot_every, snapshots, trace, None, profile, 0, m,
                         n_outer, int(H) * int(b))
    st = _lib.kdcd_lowrank_solve(pid, ctypes.byref(mat), y.data_ptr(), float(param), int(b),
                                 int(s), int(H), idx.data_ptr(), alpha.data_ptr(), zp,
                                 ctypes.byref(opt), _stream(stream))
    if st != 0:
        raise KdcdError(st, "kdcd_lowrank_solve")
    return _result(prof, None)


class BatchProblem(NamedTuple):
    """One problem of kdcd_batch_solve.  problem: "ksvm" or "krr"; param: C or
    lambda; sigma: the RBF width of this problem (ignored by other kernels);
    y, alpha (updated in place) and the optional trace (H*b entries) are
    float64 GPU tensors."""
    problem: str
    param: float
    sigma: float
    y: torch.Tensor
    alpha: torch.Tensor
    loss: int = 1
    trace: Optional[torch.Tensor] = None


def kdcd_batch_solve(A, kernel, b, s, H, idx, problems, *, compute="f64", workspace=None,
                     profile=False, flags=0, stream=None, monitor_every=0, tol=0.0,
                     monitor_log=False):
    """Batched s-step solves sharing every kernel-block product: K-RR problem p
    equals kdcd_krr_solve(..., b, s, H, ...) and K-SVM problem q equals
    kdcd_ksvm_solve(..., 1, s*b, H*b, ...) over the same idx.  With the monitor
    (FP64) the batch stops once every problem's certified bound is <= tol; the
    result's rel_err is the largest bound."""
    mat, m, _ = _matrix(A)
    _dev(idx, torch.int32, int(H) * int(b), "idx")
    arr = _batch_array(problems, m, H, b)
    n_outer = -(-int(H) // max(int(s), 1))
    mon = _MonitorOut(n_outer, int(monitor_every), monitor_log) if monitor_every else None
    opt, prof = _options(compute, 1, 0, None, None, workspace, profile, flags, m, n_outer, 0,
                         monitor_every, tol, mon)
    kern = _kernel(kernel)
    st = _lib.kdcd_batch_solve(ctypes.byref(mat), ctypes.byref(kern), int(b), int(s), int(H),
                               idx.data_ptr(), arr, len(problems), ctypes.byref(opt),
                               _stream(stream))
    if st != 0:
        raise KdcdError(st, "kdcd_batch_solve")
    return _result(prof, mon)


def _batch_array(problems, m, H, b):
    arr = (_BatchProblem * max(len(problems), 1))()
    for i, q in enumerate(problems):
        q = q if isinstance(q, BatchProblem) else BatchProblem(**q)
        if q.problem not in ("ksvm", "krr"):
            raise ValueError(f"problem {i}: kind must be 'ksvm' or 'krr'")
        arr[i].problem = 0 if q.problem == "ksvm" else 1
        arr[i].loss = int(q.loss)
        arr[i].param = float(q.param)
        arr[i].sigma = float(q.sigma)
        arr[i].y = _dev(q.y, torch.float64, m, f"problems[{i}].y")
        arr[i].alpha = _dev(q.alpha, torch.float64, m, f"problems[{i}].alpha")
        arr[i].trace = (None if q.trace is None else
                        _dev(q.trace, torch.float64, int(H) * int(b), f"problems[{i}].trace"))
    return arr


def kdcd_kernel_rhs(A, kernel, S, beta, beta_scale=None, *, want_W=False, compute="f64",
                    stream=None):
    """r[j] = sum_p K(a_p, a_{S_j}) beta_p (beta_scale_p); W = K(A_S, A_S) if want_W."""
    mat, m, _ = _matrix(A)
    sb = int(S.numel())
    _dev(S, torch.int32, sb, "S")
    _dev(beta, torch.float64, m, "beta")
    bs = _dev(beta_scale, torch.float64, m, "beta_scale") if beta_scale is not None else None
    r = torch.empty(sb, dtype=torch.float64, device=beta.device)
    W = torch.empty(sb * sb, dtype=torch.float64, device=beta.device) if want_W else None
    kern = _kernel(kernel)
    cmp = COMPUTE[compute] if isinstance(compute, str) else int(compute)
    st = _lib.kdcd_kernel_rhs(ctypes.byref(mat), ctypes.byref(kern), S.data_ptr(), sb,
                              beta.data_ptr(), bs, r.data_ptr(),
                              W.data_ptr() if W is not None else None, cmp, _stream(stream))
    if st != 0:
        raise KdcdError(st, "kdcd_kernel_rhs")
    return (r, W.view(sb, sb)) if want_W else r


def kdcd_ksvm_eval(A, y, kernel, C, alpha, loss=1, stream=None) -> dict:
    mat, m, _ = _matrix(A)
    _dev(y, torch.float64, m, "y")
    _dev(alpha, torch.float64, m, "alpha")
    out = (ctypes.c_double * 4)()
    st = _lib.kdcd_ksvm_eval(ctypes.byref(mat), y.data_ptr(), ctypes.byref(_kernel(kernel)),
                             float(C), int(loss), alpha.data_ptr(), out, _stream(stream))
    if st != 0:
        raise KdcdError(st, "kdcd_ksvm_eval")
    return {"dual": out[0], "primal": out[1], "gap": out[2], "kkt": out[3]}


def kdcd_krr_eval(A, y, kernel, lam, alpha, stream=None) -> dict:
    mat, m, _ = _matrix(A)
    _dev(y, torch.float64, m, "y")
    _dev(alpha, torch.float64, m, "alpha")
    out = (ctypes.c_double * 2)()
    st = _lib.kdcd_krr_eval(ctypes.byref(mat), y.data_ptr(), ctypes.byref(_kernel(kernel)),
                            float(lam), alpha.data_ptr(), out, _stream(stream))
    if st != 0:
        raise KdcdError(st, "kdcd_krr_eval")
    return {"objective": out[0], "residual_norm": out[1]}


def kdcd_workspace_bytes(problem, A, kernel, b, s, compute="f64") -> int:
    mat, _, _ = _matrix(A)
    cmp = COMPUTE[compute] if isinstance(compute, str) else int(compute)
    return int(_lib.kdcd_workspace_bytes(int(problem), ctypes.byref(mat),
                                         ctypes.byref(_kernel(kernel)), int(b), int(s), cmp))


# ------------------------------------------------------------ learned sampler

SAMPLER_NPARAMS = 4545


def _check(st, name):
    if st != 0:
        raise KdcdError(st, name)


class Sampler:
    """A learned coordinate sampler (MLP 4 -> 64 -> 64 -> 1) living on the
    current GPU: thin owner of the kdcd_sampler handle."""

    def __init__(self, seed: int = 0):
        h = ctypes.c_void_p()
        _check(_lib.kdcd_sampler_create(ctypes.byref(h), int(seed)), "kdcd_sampler_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.kdcd_sampler_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self, stream=None) -> torch.Tensor:
        out = torch.empty(SAMPLER_NPARAMS, dtype=torch.float32, device="cuda")
        _check(_lib.kdcd_sampler_get_params(self.handle, out.data_ptr(), _stream(stream)),
               "kdcd_sampler_get_params")
        return out

    def set_params(self, params: torch.Tensor, stream=None):
        _dev(params, torch.float32, SAMPLER_NPARAMS, "params")
        _check(_lib.kdcd_sampler_set_params(self.handle, params.data_ptr(), _stream(stream)),
               "kdcd_sampler_set_params")

    def forward(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        n = x.shape[0]
        _dev(x, torch.float32, 4 * n, "x")
        out = torch.empty(n, dtype=torch.float32, device="cuda")
        _check(_lib.kdcd_sampler_forward(self.handle, x.data_ptr(), n, out.data_ptr(),
                                         _stream(stream)), "kdcd_sampler_forward")
        return out

    def grad(self, x: torch.Tensor, t: torch.Tensor, stream=None):
        n = x.shape[0]
        _dev(x, torch.float32, 4 * n, "x")
        _dev(t, torch.float32, n, "t")
        g = torch.empty(SAMPLER_NPARAMS, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(_lib.kdcd_sampler_grad(self.handle, x.data_ptr(), t.data_ptr(), n, g.data_ptr(),
                                      loss.data_ptr(), _stream(stream)), "kdcd_sampler_grad")
        return g, loss

    def train(self, x: torch.Tensor, t: torch.Tensor, batch: int, epochs: int, lr: float,
              stream=None) -> torch.Tensor:
        n = x.shape[0]
        _dev(x, torch.float32, 4 * n, "x")
        _dev(t, torch.float32, n, "t")
        losses = torch.zeros(max(int(epochs), 1), dtype=torch.float32, device="cuda")
        _check(_lib.kdcd_sampler_train(self.handle, x.data_ptr(), t.data_ptr(), n, int(batch),
                                       int(epochs), float(lr), losses.data_ptr(),
                                       _stream(stream)), "kdcd_sampler_train")
        return losses[:int(epochs)]

    def keys(self, x: torch.Tensor, tau: float, seed: int, outer: int, stream=None):
        n = x.shape[0]
        _dev(x, torch.float32, 4 * n, "x")
        out = torch.empty(n, dtype=torch.float32, device="cuda")
        _check(_lib.kdcd_sampler_keys(self.handle, x.data_ptr(), n, float(tau), int(seed),
                                      int(outer), out.data_ptr(), _stream(stream)),
               "kdcd_sampler_keys")
        return out


def kdcd_sampler_select(keys: torch.Tensor, s: int, epsilon: float, seed: int, outer: int,
                        stream=None) -> torch.Tensor:
    """The s coordinates of outer iteration `outer` from float32 keys."""
    m = keys.numel()
    _dev(keys, torch.float32, m, "keys")
    S = torch.empty(int(s), dtype=torch.int32, device="cuda")
    _check(_lib.kdcd_sampler_select(keys.data_ptr(), m, int(s), float(epsilon), int(seed),
                                    int(outer), S.data_ptr(), _stream(stream)),
           "kdcd_sampler_select")
    return S


def kdcd_ksvm_solve_sampled(A, y, kernel, C, s, H, alpha, *, model=None, epsilon=0.0, tau=1.0,
                            seed=0, pool=0, idx_out=None, features_out=None, grad_out=None, loss=1,
                            trace=None, snapshot_every=0, snapshots=None, workspace=None,
                            profile=False, flags=0, stream=None, monitor_every=0, tol=0.0,
                            monitor_log=False):
    """Algorithm 2 (b = 1) with the coordinates drawn on the device by
    `model` (a Sampler; None draws uniformly).  Returns (idx_out, profile or
    None); alpha is updated in place."""
    mat, m, _ = _matrix(A)
    _dev(y, torch.float64, m, "y")
    _dev(alpha, torch.float64, m, "alpha")
    H = int(H)
    if idx_out is None:
        idx_out = torch.empty(H, dtype=torch.int32, device="cuda")
    smp = _Sampling()
    smp.model = model.handle if model is not None else None
    smp.epsilon = float(epsilon)
    smp.tau = float(tau)
    smp.seed = int(seed)
    smp.pool = int(pool)
    smp.idx_out = _dev(idx_out, torch.int32, H, "idx_out")
    if features_out is not None:
        smp.features_out = _dev(features_out, torch.float32, 4 * H, "features_out")
    if grad_out is not None:
        smp.grad_out = _dev(grad_out, torch.float64, m, "grad_out")
    n_outer = -(-H // max(int(s), 1))
    mon = _MonitorOut(n_outer, int(monitor_every), monitor_log) if monitor_every else None
    opt, prof = _options("f64", loss, snapshot_every, snapshots, trace, workspace, profile, flags,
                         m, n_outer, H, monitor_every, tol, mon)
    kern = _kernel(kernel)
    st = _lib.kdcd_ksvm_solve_sampled(ctypes.byref(mat), y.data_ptr(), ctypes.byref(kern),
                                      float(C), int(s), H, ctypes.byref(smp), alpha.data_ptr(),
                                      ctypes.byref(opt), _stream(stream))
    _check(st, "kdcd_ksvm_solve_sampled")
    return idx_out, _result(prof, mon)


# ------------------------------------------------------------------ tuning

def _compute_id(compute):
    return COMPUTE[compute] if isinstance(compute, str) else int(compute)


def kdcd_tune_configs(compute="f64") -> list:
    """[(bm, bn, waves)] of the tile configurations, indexed by id."""
    n = _lib.kdcd_tune_configs(_compute_id(compute), None, None, None, 0)
    bm, bn, w = (ctypes.c_int32 * max(n, 1))(), (ctypes.c_int32 * max(n, 1))(), (ctypes.c_int32 * max(n, 1))()
    _lib.kdcd_tune_configs(_compute_id(compute), bm, bn, w, n)
    return [(bm[i], bn[i], w[i]) for i in range(n)]


def kdcd_tune_set(compute, n, sb, config_id):
    _check(_lib.kdcd_tune_set(_compute_id(compute), int(n), int(sb), int(config_id)),
           "kdcd_tune_set")


def kdcd_tune_get(compute, n, sb) -> int:
    return int(_lib.kdcd_tune_get(_compute_id(compute), int(n), int(sb)))


def kdcd_autotune(A, kernel, sb, compute="f64", reps=10, stream=None):
    """Time every configuration on A; returns (best id, mean launch us)."""
    mat, _, _ = _matrix(A)
    kern = _kernel(kernel)
    best = ctypes.c_int32(-1)
    us = ctypes.c_double(0.0)
    _check(_lib.kdcd_autotune(ctypes.byref(mat), ctypes.byref(kern), int(sb), _compute_id(compute),
                              int(reps), ctypes.byref(best), ctypes.byref(us), _stream(stream)),
           "kdcd_autotune")
    return best.value, us.value


def kdcd_autotune_batch(A, kernel, sb, problems, compute="f64", reps=5, stream=None):
    """Time every batched-product configuration on these problems; returns
    (best id, mean launch us), recorded under compute + TUNE_BATCH."""
    mat, m, _ = _matrix(A)
    arr = _batch_array(problems, m, 0, 1)
    best = ctypes.c_int32(-1)
    us = ctypes.c_double(0.0)
    _check(_lib.kdcd_autotune_batch(ctypes.byref(mat), ctypes.byref(_kernel(kernel)), int(sb), arr,
                                    len(problems), _compute_id(compute), int(reps),
                                    ctypes.byref(best), ctypes.byref(us), _stream(stream)),
           "kdcd_autotune_batch")
    return best.value, us.value


TUNE_BATCH = 16


def kdcd_batch_eval(A, kernel, problems, stream=None) -> list:
    """FP64 objectives of every problem of a batch in one shared kernel pass:
    K-RR {objective, residual_norm}, K-SVM {dual, primal, gap, kkt}."""
    mat, m, _ = _matrix(A)
    arr = _batch_array(problems, m, 0, 1)
    out = (ctypes.c_double * (4 * len(problems)))()
    _check(_lib.kdcd_batch_eval(ctypes.byref(mat), ctypes.byref(_kernel(kernel)), arr,
                                len(problems), out, _stream(stream)), "kdcd_batch_eval")
    res = []
    for i, q in enumerate(problems):
        kind = q.problem if isinstance(q, BatchProblem) else q["problem"]
        o = out[4 * i:4 * i + 4]
        if kind == "krr":
            res.append({"objective": o[0], "residual_norm": o[1]})
        else:
            res.append({"dual": o[0], "primal": o[1], "gap": o[2], "kkt": o[3]})
    return res


def kdcd_tune_save(path):
    _check(_lib.kdcd_tune_save(str(path).encode()), "kdcd_tune_save")


def kdcd_tune_load(path):
    _check(_lib.kdcd_tune_load(str(path).encode()), "kdcd_tune_load")


def kdcd_graph_cache_clear():
    """Destroy the graphs cached by calls with flags=FLAG_GRAPH."""
    _lib.kdcd_graph_cache_clear()

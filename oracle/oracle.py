"""ctypes wrapper around the plain FP64 CPU oracle (kdcd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.  It shares no code
with the HIP library; the two only see the same seeded inputs.

Matrices are passed either as a dense float64 numpy array (row-major) or as a
CSR tuple ``(row_ptr int64, col_idx int32, val float64, m, n)`` with sorted
column indices in every row.  Kernels are ``(kind, sigma, c, degree)`` with
kind 0 = linear, 1 = polynomial (c + x.y)^degree, 2 = RBF exp(-sigma ||x-y||^2)
(the paper's Table 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kdcd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

LINEAR, POLY, RBF = 0, 1, 2


class Kernel(NamedTuple):
    kind: int
    sigma: float = 0.0
    c: float = 0.0
    degree: int = 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: -O2, no FP contraction, OpenMP over rows."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Matrix(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("dense", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("c", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # KDCD_ORACLE_LIBRARY: a prebuilt variant of the same source (for
        # example the AddressSanitizer build), loaded as is
        path = os.environ.get("KDCD_ORACLE_LIBRARY")
        if not path:
            build()
            path = LIB
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_kernel_eval.restype = dbl
        L.orc_kernel_eval.argtypes = [P, P, i64, i64]
        L.orc_kernel_block.argtypes = [P, P, P, i64, P, i64, P]
        L.orc_kernel_rhs.argtypes = [P, P, P, i64, P, P]
        L.orc_kernel_matvec.argtypes = [P, P, P, P]
        L.orc_dcd_ksvm.argtypes = [P, P, P, dbl, ctypes.c_int, i64, P, P, P]
        L.orc_sstep_dcd_ksvm.argtypes = [P, P, P, dbl, ctypes.c_int, i64, i64, P, P, P]
        L.orc_bdcd_krr.argtypes = [P, P, P, dbl, i64, i64, P, P, P]
        L.orc_sstep_bdcd_krr.argtypes = [P, P, P, dbl, i64, i64, i64, P, P, P]
        L.orc_ksvm_eval.argtypes = [P, P, P, dbl, ctypes.c_int, P, P, P]
        L.orc_krr_eval.argtypes = [P, P, P, dbl, P, P, P]
        for f in ("orc_dcd_ksvm", "orc_sstep_dcd_ksvm", "orc_bdcd_krr", "orc_sstep_bdcd_krr"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Threads of later oracle calls (for timing; results do not depend on it)."""
    lib().orc_set_threads(int(n))


class _Args:
    """Keeps numpy buffers alive while a call runs."""

    def __init__(self, A, kernel):
        self.keep = []
        mat = _Matrix()
        if isinstance(A, tuple):
            row_ptr, col_idx, val, m, n = A
            row_ptr = self._arr(row_ptr, np.int64)
            col_idx = self._arr(col_idx, np.int32)
            val = self._arr(val, np.float64)
            mat.m, mat.n, mat.ld = m, n, n
            mat.dense = None
            mat.row_ptr, mat.col_idx, mat.val = row_ptr.ctypes.data, col_idx.ctypes.data, val.ctypes.data
        else:
            A = self._arr(A, np.float64)
            mat.m, mat.n = A.shape
            mat.ld = A.shape[1]
            mat.dense = A.ctypes.data
            mat.row_ptr = mat.col_idx = mat.val = None
        self.m = int(mat.m)
        self.mat = mat
        k = Kernel(*kernel) if not isinstance(kernel, Kernel) else kernel
        self.kern = _Kernel(int(k.kind), int(k.degree), float(k.sigma), float(k.c))

    def _arr(self, x, dtype):
        x = np.ascontiguousarray(x, dtype=dtype)
        self.keep.append(x)
        return x

    def ptr(self, x, dtype):
        return self._arr(x, dtype).ctypes.data

    @property
    def A(self):
        return ctypes.byref(self.mat)

    @property
    def K(self):
        return ctypes.byref(self.kern)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def kernel_eval(A, kernel, p, q) -> float:
    a = _Args(A, kernel)
    return float(lib().orc_kernel_eval(a.A, a.K, int(p), int(q)))


def kernel_block(A, kernel, rows, cols) -> np.ndarray:
    a = _Args(A, kernel)
    rows = a._arr(rows, np.int32)
    cols = a._arr(cols, np.int32)
    out = np.empty((rows.size, cols.size))
    lib().orc_kernel_block(a.A, a.K, rows.ctypes.data, rows.size, cols.ctypes.data, cols.size,
                           out.ctypes.data)
    return out


def kernel_matrix(A, kernel) -> np.ndarray:
    m = A[3] if isinstance(A, tuple) else A.shape[0]
    r = np.arange(m, dtype=np.int32)
    return kernel_block(A, kernel, r, r)


def kernel_rhs(A, kernel, S, beta) -> np.ndarray:
    """r_j = sum_p K(a_p, a_{S_j}) beta_p."""
    a = _Args(A, kernel)
    S = a._arr(S, np.int32)
    beta = a._arr(beta, np.float64)
    r = np.empty(S.size)
    lib().orc_kernel_rhs(a.A, a.K, S.ctypes.data, S.size, beta.ctypes.data, r.ctypes.data)
    return r


def kernel_matvec(A, kernel, beta) -> np.ndarray:
    a = _Args(A, kernel)
    beta = a._arr(beta, np.float64)
    out = np.empty(a.m)
    lib().orc_kernel_matvec(a.A, a.K, beta.ctypes.data, out.ctypes.data)
    return out


def dcd_ksvm(A, y, kernel, C, H, idx, alpha0=None, loss=1, s=None):
    """Algorithm 1 (s is None) or Algorithm 2 (s-step).  Returns (alpha_H, theta[H])."""
    a = _Args(A, kernel)
    alpha = np.zeros(a.m) if alpha0 is None else np.array(alpha0, dtype=np.float64, copy=True)
    theta = np.empty(int(H))
    yp = a.ptr(y, np.float64)
    ip = a.ptr(np.asarray(idx)[:H], np.int32)
    if s is None:
        rc = lib().orc_dcd_ksvm(a.A, yp, a.K, float(C), int(loss), int(H), ip,
                                alpha.ctypes.data, theta.ctypes.data)
    else:
        rc = lib().orc_sstep_dcd_ksvm(a.A, yp, a.K, float(C), int(loss), int(s), int(H), ip,
                                      alpha.ctypes.data, theta.ctypes.data)
    _check(rc, "dcd_ksvm")
    return alpha, theta


def bdcd_krr(A, y, kernel, lam, b, H, idx, alpha0=None, s=None):
    """Algorithm 3 (s is None) or Algorithm 4 (s-step).  Returns (alpha_H, delta[H*b])."""
    a = _Args(A, kernel)
    alpha = np.zeros(a.m) if alpha0 is None else np.array(alpha0, dtype=np.float64, copy=True)
    delta = np.empty(int(H) * int(b))
    yp = a.ptr(y, np.float64)
    ip = a.ptr(np.asarray(idx)[: H * b], np.int32)
    if s is None:
        rc = lib().orc_bdcd_krr(a.A, yp, a.K, float(lam), int(b), int(H), ip,
                                alpha.ctypes.data, delta.ctypes.data)
    else:
        rc = lib().orc_sstep_bdcd_krr(a.A, yp, a.K, float(lam), int(b), int(s), int(H), ip,
                                      alpha.ctypes.data, delta.ctypes.data)
    _check(rc, "bdcd_krr")
    return alpha, delta


def ksvm_eval(A, y, kernel, C, alpha, loss=1) -> dict:
    a = _Args(A, kernel)
    out = np.empty(4)
    Qa = np.empty(a.m)
    lib().orc_ksvm_eval(a.A, a.ptr(y, np.float64), a.K, float(C), int(loss),
                        a.ptr(alpha, np.float64), out.ctypes.data, Qa.ctypes.data)
    return {"dual": out[0], "primal": out[1], "gap": out[2], "kkt": out[3], "Qa": Qa}


def krr_eval(A, y, kernel, lam, alpha) -> dict:
    a = _Args(A, kernel)
    out = np.empty(2)
    res = np.empty(a.m)
    lib().orc_krr_eval(a.A, a.ptr(y, np.float64), a.K, float(lam), a.ptr(alpha, np.float64),
                       out.ctypes.data, res.ctypes.data)
    return {"objective": out[0], "residual_norm": out[1], "residual": res}


def nystrom_features(A, kernel, landmarks, jitter) -> np.ndarray:
    """Nystrom features Phi = K(A, A_L) L^{-T} with L L^T = K(A_L, A_L) + jitter I
    (Cholesky), so that Phi Phi^T = K_AL (K_LL + jitter I)^{-1} K_LA: the
    approximation of the kernel matrix from the landmark rows L that the
    paper's conclusion proposes for the sampled kernel block.  Solving with
    Phi and the linear kernel solves the approximated problem."""
    L = np.asarray(landmarks)
    m = A[3] if isinstance(A, tuple) else A.shape[0]
    K_AL = kernel_block(A, kernel, np.arange(m), L)
    K_LL = kernel_block(A, kernel, L, L) + jitter * np.eye(L.size)
    C = np.linalg.cholesky(K_LL)                  # lower triangular
    return np.linalg.solve(C, K_AL.T).T           # rows phi_i = C^{-1} k_i

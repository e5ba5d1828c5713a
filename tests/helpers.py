"""Shared helpers of the GPU tests: device upload and the parity measure."""
import numpy as np
import torch


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def idx_dev(idx):
    return torch.as_tensor(np.ascontiguousarray(idx, dtype=np.int32)).to("cuda")


def max_rel(x, ref):
    """max_i |x_i - ref_i| / max_i |ref_i| -- the element-wise parity measure."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(float(np.abs(ref).max()) if ref.size else 0.0, 1e-300)
    return float(np.abs(x - ref).max()) / scale if ref.size else 0.0


def assert_parity(x, ref, tol, what=""):
    err = max_rel(x, ref)
    assert err <= tol, f"{what}: max element error {err:.3e} relative to max|ref| exceeds {tol:.1e}"
    return err

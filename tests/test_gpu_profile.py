"""Stage timings of a profiled solve: every stage is timed once per outer
iteration, the durations are positive and fit inside the solve's span, and
profiling does not change the result."""
import numpy as np
import pytest
import torch

from paper_2406_18001_amd import inputs
from tests.helpers import dev, idx_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("s", [4, 64])          # s*b = 32 (W tiles) and 512 (gathered Gram)
@pytest.mark.parametrize("compute", ["f64", "bf16x3"])
def test_profile_stages(s, compute):
    from paper_2406_18001_amd import kdcd as K
    d = inputs.dense_krr_c2(m=3000, n=64, seed=5)
    m, b, H = 3000, 8, 5 * s + 3
    A, y = dev(d["A"]), dev(d["y"])
    idx = idx_dev(inputs.krr_indices(m, b, H, seed=1))
    kern = (2, 1.0, 0.0, 1)
    a0 = torch.zeros(m, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(A, y, kern, 1e-3, b, s, H, idx, a0, compute=compute)
    a1 = torch.zeros(m, dtype=torch.float64, device="cuda")
    p = K.kdcd_krr_solve(A, y, kern, 1e-3, b, s, H, idx, a1, compute=compute, profile=True)
    assert torch.equal(a0, a1)
    n_outer = -(-H // s)
    for st in ("kblock", "finish", "recur"):
        assert p[f"{st}_launches"] == n_outer, st
        assert p[f"{st}_ms"] > 0.0, st
    assert p["total_ms"] > 0.0
    assert p["kblock_ms"] + p["finish_ms"] + p["recur_ms"] <= p["total_ms"] * 1.001 + 1e-3


def test_profile_product_only():
    from paper_2406_18001_amd import kdcd as K
    d = inputs.dense_krr_c2(m=3000, n=64, seed=5)
    m, b, s, H = 3000, 8, 64, 200
    A, y = dev(d["A"]), dev(d["y"])
    idx = idx_dev(inputs.krr_indices(m, b, H, seed=1))
    a0 = torch.zeros(m, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(A, y, (2, 1.0, 0.0, 1), 1e-3, b, s, H, idx, a0)
    a1 = torch.zeros(m, dtype=torch.float64, device="cuda")
    p = K.kdcd_krr_solve(A, y, (2, 1.0, 0.0, 1), 1e-3, b, s, H, idx, a1, profile=True,
                         flags=K.FLAG_TIME_PRODUCT)
    assert torch.equal(a0, a1)
    assert p["kblock_launches"] == -(-H // s) and p["kblock_ms"] > 0.0
    assert p["finish_launches"] == 0 and p["recur_launches"] == 0
    assert p["kblock_ms"] <= p["total_ms"] * 1.001 + 1e-3
    # one product launch in eight (outer iterations 0, 8, 16, ...)
    a2 = torch.zeros(m, dtype=torch.float64, device="cuda")
    q = K.kdcd_krr_solve(A, y, (2, 1.0, 0.0, 1), 1e-3, b, s, H, idx, a2, profile=True,
                         flags=K.FLAG_TIME_PRODUCT | K.FLAG_TIME_SAMPLE)
    assert torch.equal(a0, a2)
    n_outer = -(-H // s)
    assert q["kblock_launches"] == -(-n_outer // 8) and q["kblock_ms"] > 0.0
    assert q["finish_launches"] == 0 and q["recur_launches"] == 0

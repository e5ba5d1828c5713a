"""kdcd_krr_solve_noalloc (workspace in the library's fixed device array)
against kdcd_krr_solve (workspace allocated per call): two calls in a row,
the second on a smaller input, each equal to the allocating solve bit for bit
(the same kernels run in the same order on the same data)."""
import numpy as np
import pytest
import torch

from paper_2406_18001_amd import inputs
from tests.helpers import dev, idx_dev

pytestmark = pytest.mark.gpu

RBF1 = (2, 1.0, 0.0, 1)


@pytest.fixture(scope="module")
def K():
    from paper_2406_18001_amd import kdcd
    return kdcd


def _pair(K, A, y, lam, b, s, H, idx, alpha0, compute="f64"):
    a_ref = dev(alpha0)
    t_ref = torch.zeros(H * b, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(A, y, RBF1, lam, b, s, H, idx, a_ref, trace=t_ref, compute=compute)
    a = dev(alpha0)
    t = torch.zeros(H * b, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve_noalloc(A, y, RBF1, lam, b, s, H, idx, a, trace=t, compute=compute)
    torch.cuda.synchronize()
    assert torch.equal(a, a_ref), float((a - a_ref).abs().max())
    assert torch.equal(t, t_ref), float((t - t_ref).abs().max())
    return a


def test_noalloc_equals_allocating_solve_twice(K):
    # first call: C2 at full size in the benchmark's configuration (b = 8, s = 64),
    # two outer iterations from a warm start
    d = inputs.dense_krr_c2()
    m = d["A"].shape[0]
    rng = np.random.default_rng(3)
    idx = idx_dev(inputs.krr_indices(m, 8, 128, seed=0))
    a = _pair(K, dev(d["A"]), dev(d["y"]), 1e-3, 8, 64, 128, idx, rng.standard_normal(m) * 1e-4)
    assert float(a.abs().max()) > 0.0
    # second call: a smaller problem (other m, n, b, s, ragged last outer iteration);
    # the array keeps the first call's contents, which the solve must not read
    d2 = inputs.dense_krr_c2(m=3000, n=100, seed=9)
    idx2 = idx_dev(inputs.krr_indices(3000, 4, 37, seed=2))
    _pair(K, dev(d2["A"]), dev(d2["y"]), 1e-2, 4, 8, 37, idx2, np.zeros(3000))
    # and a mixed-precision solve, whose low-precision copy of A also lives there
    _pair(K, dev(d2["A"]), dev(d2["y"]), 1e-2, 4, 8, 37, idx2, np.zeros(3000), compute="bf16x3")


def test_noalloc_refuses_what_does_not_fit(K):
    m = 5_000_000                    # norms and row table alone exceed 32 MiB
    A = torch.zeros((m, 1), dtype=torch.float64, device="cuda")
    y = torch.zeros(m, dtype=torch.float64, device="cuda")
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    idx = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_krr_solve_noalloc(A, y, RBF1, 1.0, 1, 1, 1, idx, a)
    assert e.value.status == -9
    assert float(a.abs().max()) == 0.0

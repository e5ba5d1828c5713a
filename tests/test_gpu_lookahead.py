"""The overlapped outer loop (KDCD_FLAG_OVERLAP: recurrence of iteration k
on a second stream while the product of k+1 runs, with the rows of S_k
corrected afterwards) against the serial loop and the oracle.  Only the order of the sums of r
differs from the serial loop, so the two agree to a few ulps; both meet the
oracle at the FP64 bound; repeated runs are bit for bit identical."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2406_18001_amd import inputs
from tests.helpers import assert_parity, dev, idx_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2406_18001_amd import kdcd
    return kdcd


@pytest.mark.parametrize("b,s,H", [(8, 16, 200), (1, 64, 300), (4, 5, 23), (16, 2, 40), (32, 8, 50)])
def test_krr_lookahead_matches_serial_and_oracle(K, b, s, H):
    d = inputs.dense_krr_c2(m=1500, n=80, seed=b + s)
    A, y = dev(d["A"]), dev(d["y"])
    idx_h = inputs.krr_indices(1500, b, H, seed=1)
    idx = idx_dev(idx_h)
    kern = (2, 1.0, 0.0, 1)
    out = {}
    for name, flags in (("la", K.FLAG_OVERLAP), ("la2", K.FLAG_OVERLAP), ("serial", 0)):
        a = torch.zeros(1500, dtype=torch.float64, device="cuda")
        tr = torch.zeros(H * b, dtype=torch.float64, device="cuda")
        K.kdcd_krr_solve(A, y, kern, 1e-3, b, s, H, idx, a, trace=tr, flags=flags)
        out[name] = (a.cpu().numpy(), tr.cpu().numpy())
    assert np.array_equal(out["la"][0], out["la2"][0]) and np.array_equal(out["la"][1], out["la2"][1])
    assert_parity(out["la"][0], out["serial"][0], 1e-12, "alpha vs serial")
    assert_parity(out["la"][1], out["serial"][1], 1e-11, "trace vs serial")
    ref, dref = O.bdcd_krr(d["A"], d["y"], O.Kernel(O.RBF, sigma=1.0), 1e-3, b, H, idx_h, s=s)
    assert_parity(out["la"][0], ref, 1e-9, "alpha vs oracle")
    assert_parity(out["la"][1], dref, 1e-9, "trace vs oracle")


@pytest.mark.parametrize("loss", [1, 2])
def test_ksvm_lookahead_heavy_repeats(K, loss):
    """m = 300 with 64 steps per outer iteration: consecutive blocks share many
    coordinates, and a block repeats coordinates within itself."""
    d = inputs.dense_ksvm_c1(m=300, n=24, seed=3)
    A, y = dev(d["A"]), dev(d["y"])
    H, s = 64 * 30 + 17, 64
    idx_h = inputs.ksvm_indices(300, H, seed=2)
    kern = (2, 1.0 / 24, 0.0, 1)
    res = []
    for flags in (K.FLAG_OVERLAP, 0):
        a = torch.zeros(300, dtype=torch.float64, device="cuda")
        tr = torch.zeros(H, dtype=torch.float64, device="cuda")
        K.kdcd_ksvm_solve(A, y, kern, 0.5, 1, s, H, idx_dev(idx_h), a, loss=loss, trace=tr,
                          flags=flags)
        res.append((a.cpu().numpy(), tr.cpu().numpy()))
    assert_parity(res[0][0], res[1][0], 1e-12, "alpha vs serial")
    ref, th = O.dcd_ksvm(d["A"], d["y"], O.Kernel(O.RBF, sigma=1.0 / 24), 0.5, H, idx_h, loss=loss, s=s)
    assert_parity(res[0][0], ref, 1e-9, "alpha")
    assert_parity(res[0][1], th, 1e-9, "theta")


def test_lookahead_snapshots_warm_start_and_poly(K):
    d = inputs.dense_krr_c2(m=1000, n=40, seed=6)
    A, y = dev(d["A"]), dev(d["y"])
    b, s, H = 4, 8, 77
    idx_h = inputs.krr_indices(1000, b, H, seed=3)
    a0 = np.random.default_rng(5).standard_normal(1000) * 0.01
    kern = (1, 0.0, 1.0, 2)
    rows = -(-(-(-H // s)) // 3)
    snaps = {}
    for flags in (K.FLAG_OVERLAP, 0):
        a = dev(a0)
        sn = torch.zeros(rows * 1000, dtype=torch.float64, device="cuda")
        K.kdcd_krr_solve(A, y, kern, 1e-2, b, s, H, idx_dev(idx_h), a, snapshot_every=3,
                         snapshots=sn, flags=flags)
        snaps[flags] = (a.cpu().numpy(), sn.cpu().numpy())
    assert_parity(snaps[K.FLAG_OVERLAP][1], snaps[0][1], 1e-12, "snapshots")
    ref, _ = O.bdcd_krr(d["A"], d["y"], O.Kernel(O.POLY, c=1.0, degree=2), 1e-2, b, H, idx_h,
                        alpha0=a0, s=s)
    assert_parity(snaps[K.FLAG_OVERLAP][0], ref, 1e-9, "alpha")

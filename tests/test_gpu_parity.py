"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Bar: the plain FP64 path matches the oracle to 1e-9 relative error, measured
element by element as max_i |x_i - ref_i| / max_i |ref_i|, on the same seeded
inputs.  Cases span several tiles with ragged tails in m, n and s*b, the
paper's degenerate cases (duplicate coordinates inside a block, overlapping
K-RR blocks, s not dividing H, the last partial outer iteration) and the
full-size workloads the benchmark times.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2406_18001_amd import inputs
from tests.helpers import assert_parity, dev, idx_dev, max_rel

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def K():
    from paper_2406_18001_amd import kdcd
    return kdcd


def kern(kind, sigma=0.0, c=0.0, degree=1):
    return (kind, sigma, c, degree)


RBF1 = kern(2, sigma=1.0)
POLY13 = kern(1, c=1.0, degree=3)
LIN = kern(0)


# --------------------------------------------------------- kernel block pass

@pytest.mark.parametrize("m,n,sb", [(700, 100, 1), (700, 100, 5), (1001, 77, 33), (333, 512, 64),
                                    (2000, 64, 100), (517, 130, 512), (64, 16, 1024)])
@pytest.mark.parametrize("kk", [RBF1, POLY13, LIN, kern(2, sigma=0.05)])
def test_kernel_rhs_and_gram_match_oracle(K, m, n, sb, kk):
    A = inputs.dense_krr_c2(m=m, n=n, seed=m + n)["A"]
    rng = np.random.default_rng(sb)
    S = rng.integers(0, m, size=sb).astype(np.int32)
    beta = rng.standard_normal(m)
    okern = O.Kernel(kk[0], sigma=kk[1], c=kk[2], degree=kk[3])
    r_ref = O.kernel_rhs(A, okern, S, beta)
    W_ref = O.kernel_block(A, okern, S, S)
    r, W = K.kdcd_kernel_rhs(dev(A), kk, idx_dev(S), dev(beta), want_W=True)
    assert_parity(r.cpu().numpy(), r_ref, 1e-11, "r")
    assert_parity(W.cpu().numpy(), W_ref, 1e-12, "W")


def test_kernel_rhs_beta_scale_and_leading_dimension(K):
    m, n, ld = 300, 40, 48
    base = inputs.dense_krr_c2(m=m, n=ld, seed=5)["A"]
    A_pad = dev(base)
    A_view = A_pad[:, :n]                      # ld = 48 > n = 40
    rng = np.random.default_rng(0)
    S = rng.integers(0, m, size=20).astype(np.int32)
    beta, scale = rng.standard_normal(m), np.where(rng.random(m) < 0.5, -1.0, 1.0)
    ref = O.kernel_rhs(base[:, :n].copy(), O.Kernel(2, sigma=0.7), S, beta * scale)
    r = K.kdcd_kernel_rhs(A_view, kern(2, sigma=0.7), idx_dev(S), dev(beta), dev(scale))
    assert_parity(r.cpu().numpy(), ref, 1e-11, "r")


# --------------------------------------------------------------- K-SVM solve

def _ksvm_case(K, A, y, kk, C, s, H, idx, loss=1, alpha0=None):
    okern = O.Kernel(kk[0], sigma=kk[1], c=kk[2], degree=kk[3])
    a_ref, th_ref = O.dcd_ksvm(A, y, okern, C, H, idx, alpha0=alpha0, loss=loss, s=s)
    alpha = dev(np.zeros(A.shape[0]) if alpha0 is None else alpha0)
    trace = torch.zeros(H, dtype=torch.float64, device="cuda")
    K.kdcd_ksvm_solve(dev(A), dev(y), kk, C, 1, s, H, idx_dev(idx), alpha, loss=loss, trace=trace)
    err = assert_parity(alpha.cpu().numpy(), a_ref, TOL, f"alpha s={s}")
    assert_parity(trace.cpu().numpy(), th_ref, TOL, f"theta s={s}")
    return err


@pytest.mark.parametrize("s", [1, 8])
@pytest.mark.parametrize("sigma", [1.0, 1.0 / 64])
def test_ksvm_c1_config(K, s, sigma):
    """C1 as configured (2000 x 64, RBF sigma=1, C=1, H=500) and its coupled
    variant sigma = 1/64, at s in {1, 8}."""
    d = inputs.dense_ksvm_c1()
    idx = inputs.ksvm_indices(2000, 500, seed=0)
    _ksvm_case(K, d["A"], d["y"], kern(2, sigma=sigma), 1.0, s, 500, idx)


@pytest.mark.parametrize("s,H", [(1, 37), (3, 100), (16, 100), (64, 190), (100, 300), (512, 600),
                                 (1024, 1024)])
def test_ksvm_duplicates_and_ragged(K, s, H):
    """m = 90 with long blocks: most blocks repeat coordinates; s does not divide H."""
    d = inputs.dense_ksvm_c1(m=90, n=37, seed=3)
    idx = inputs.ksvm_indices(90, H, seed=1)
    _ksvm_case(K, d["A"], d["y"], kern(2, sigma=0.1), 0.8, s, H, idx)


@pytest.mark.parametrize("kk", [POLY13, LIN, kern(1, c=0.5, degree=2)])
@pytest.mark.parametrize("loss", [1, 2])
def test_ksvm_kernels_and_losses(K, kk, loss):
    d = inputs.dense_ksvm_c1(m=257, n=20, seed=8)
    A = d["A"] / np.sqrt(20.0)
    idx = inputs.ksvm_indices(257, 400, seed=2)
    _ksvm_case(K, A, d["y"], kk, 0.5, 32, 400, idx, loss=loss)


def test_ksvm_warm_start(K):
    d = inputs.dense_ksvm_c1(m=150, n=16, seed=4)
    a0 = np.random.default_rng(0).uniform(0, 1.0, 150)
    idx = inputs.ksvm_indices(150, 200, seed=9)
    _ksvm_case(K, d["A"], d["y"], kern(2, sigma=0.2), 1.0, 8, 200, idx, alpha0=a0)


# ---------------------------------------------------------------- K-RR solve

def _krr_case(K, A, y, kk, lam, b, s, H, idx, alpha0=None, tol=TOL):
    okern = O.Kernel(kk[0], sigma=kk[1], c=kk[2], degree=kk[3])
    a_ref, d_ref = O.bdcd_krr(A, y, okern, lam, b, H, idx, alpha0=alpha0, s=s)
    alpha = dev(np.zeros(A.shape[0]) if alpha0 is None else alpha0)
    trace = torch.zeros(H * b, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(dev(A), dev(y), kk, lam, b, s, H, idx_dev(idx), alpha, trace=trace)
    err = assert_parity(alpha.cpu().numpy(), a_ref, tol, f"alpha b={b} s={s}")
    assert_parity(trace.cpu().numpy(), d_ref, tol, f"delta b={b} s={s}")
    return err


@pytest.mark.parametrize("s", [1, 4, 16, 64])
def test_krr_c2_recipe_small(K, s):
    """C2's recipe (rows N(0,I)/sqrt(512), RBF sigma=1, lambda=1e-3, b=8) at m = 2000."""
    d = inputs.dense_krr_c2(m=2000)
    idx = inputs.krr_indices(2000, 8, 200, seed=0)
    _krr_case(K, d["A"], d["y"], RBF1, 1e-3, 8, s, 200, idx)


@pytest.mark.parametrize("b,s,H", [(1, 7, 50), (3, 5, 23), (5, 7, 50), (8, 128, 128), (16, 32, 70),
                                   (16, 64, 64), (32, 16, 40), (32, 8, 33), (1, 200, 430),
                                   (2, 100, 250), (4, 64, 150), (8, 40, 90)])
def test_krr_blocks_overlap_and_ragged(K, b, s, H):
    """m = 97: blocks overlap heavily; b, s and H are ragged against every tile
    (s*b up to 1024, several 64-element panels, a ragged last panel)."""
    d = inputs.dense_krr_c2(m=97, n=45, seed=6)
    idx = inputs.krr_indices(97, b, H, seed=4)
    _krr_case(K, d["A"], d["y"], kern(2, sigma=0.5), 1e-2, b, s, H, idx)


@pytest.mark.parametrize("kk", [POLY13, LIN])
def test_krr_other_kernels(K, kk):
    d = inputs.dense_krr_c2(m=300, n=24, seed=2)
    idx = inputs.krr_indices(300, 4, 120, seed=3)
    _krr_case(K, d["A"], d["y"], kk, 1e-1, 4, 10, 120, idx)


@pytest.mark.parametrize("b,s", [(1, 300), (2, 160), (4, 100), (8, 50)])
def test_krr_panels_few_repeats(K, b, s):
    """m = 5000: several 64-element panels, a few repeated coordinates per outer iteration."""
    d = inputs.dense_krr_c2(m=5000, n=40, seed=8)
    idx = inputs.krr_indices(5000, b, 2 * s, seed=5)
    _krr_case(K, d["A"], d["y"], RBF1, 1e-3, b, s, 2 * s, idx)


def test_krr_c2_full_size_first_outer_iteration(K):
    """C2 at full size (20000 x 512, b = 8, s = 64): the launch configuration the
    benchmark times, checked over one outer iteration on every coordinate."""
    d = inputs.dense_krr_c2()
    idx = inputs.krr_indices(20000, 8, 64, seed=0)
    _krr_case(K, d["A"], d["y"], RBF1, 1e-3, 8, 64, 64, idx)


# ------------------------------------------------------ properties and errors

def test_unsupported_shapes_are_refused(K):
    """Blocks wider than 16 keep the recurrence at <= 512 threads; s*b <= 1024."""
    d = inputs.dense_krr_c2(m=3000, n=8, seed=1)
    idx = idx_dev(inputs.krr_indices(3000, 32, 32, seed=0))
    a = torch.zeros(3000, dtype=torch.float64, device="cuda")
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_krr_solve(dev(d["A"]), dev(d["y"]), RBF1, 1e-2, 32, 32, 32, idx, a)
    assert e.value.status == -2


def test_determinism_and_resume(K):
    d = inputs.dense_krr_c2(m=1500, n=96, seed=9)
    A, y = dev(d["A"]), dev(d["y"])
    idx = inputs.krr_indices(1500, 8, 96, seed=7)
    I = idx_dev(idx)
    runs = []
    for _ in range(2):
        a = torch.zeros(1500, dtype=torch.float64, device="cuda")
        K.kdcd_krr_solve(A, y, RBF1, 1e-3, 8, 16, 96, I, a)
        runs.append(a.cpu().numpy())
    assert np.array_equal(runs[0], runs[1])
    # resuming: two calls equal one call bit for bit (the overlapped loop sums
    # r in another order across the split: equal to rounding)
    one = torch.zeros(1500, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(A, y, RBF1, 1e-3, 8, 16, 96, I, one)
    a = torch.zeros(1500, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(A, y, RBF1, 1e-3, 8, 16, 48, I, a)
    K.kdcd_krr_solve(A, y, RBF1, 1e-3, 8, 16, 48, idx_dev(idx[48 * 8:]), a)
    assert torch.equal(a, one)
    with pytest.raises(K.KdcdError):         # an unknown flag bit is refused
        K.kdcd_krr_solve(A, y, RBF1, 1e-3, 8, 16, 48, I, a, flags=2)


def test_snapshots(K):
    d = inputs.dense_ksvm_c1(m=400, n=10, seed=1)
    idx = inputs.ksvm_indices(400, 100, seed=0)
    A, y, I = dev(d["A"]), dev(d["y"]), idx_dev(idx)
    snaps = torch.zeros(4 * 400, dtype=torch.float64, device="cuda")   # ceil(ceil(100/8)/4) = 4
    a = torch.zeros(400, dtype=torch.float64, device="cuda")
    K.kdcd_ksvm_solve(A, y, RBF1, 1.0, 1, 8, 100, I, a, snapshot_every=4, snapshots=snaps)
    snaps = snaps.view(4, 400).cpu().numpy()
    for row, H in enumerate((32, 64, 96, 100)):
        ref, _ = O.dcd_ksvm(d["A"], d["y"], O.Kernel(2, sigma=1.0), 1.0, H, idx, s=8)
        assert_parity(snaps[row], ref, TOL, f"snapshot {row}")


def test_device_errors(K):
    d = inputs.dense_krr_c2(m=50, n=8, seed=1)
    A, y = dev(d["A"]), dev(d["y"])
    a = torch.zeros(50, dtype=torch.float64, device="cuda")
    bad = idx_dev(np.array([1, 2, 50, 3], dtype=np.int32))
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_krr_solve(A, y, RBF1, 1e-2, 2, 1, 2, bad, a)
    assert e.value.status == -3
    dup = idx_dev(np.array([4, 4, 1, 2], dtype=np.int32))
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_krr_solve(A, y, RBF1, 1e-2, 2, 2, 2, dup, a)
    assert e.value.status == -4
    ys = dev(np.where(np.arange(50) % 2 == 0, 1.0, -1.0))
    with pytest.raises(K.KdcdError) as e:           # labels must be +-1
        K.kdcd_ksvm_solve(A, y, RBF1, 1.0, 1, 1, 2, idx_dev([0, 1]), a)
    assert e.value.status == -1
    with pytest.raises(K.KdcdError) as e:           # alpha_0 outside [0, C]
        K.kdcd_ksvm_solve(A, ys, RBF1, 1.0, 1, 1, 2, idx_dev([0, 1]), a + 2.0)
    assert e.value.status == -1
    nan_y = y.clone()
    nan_y[3] = float("nan")
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_krr_solve(A, nan_y, RBF1, 1e-2, 2, 1, 1, idx_dev([0, 1]), a)
    assert e.value.status == -6
    with pytest.raises(ValueError):                 # too short an index buffer never reaches HIP
        K.kdcd_krr_solve(A, y, RBF1, 1e-2, 2, 1, 3, idx_dev([0, 1]), a)


def test_eval_matches_oracle(K):
    d = inputs.dense_ksvm_c1(m=600, n=12, seed=2)
    a = np.random.default_rng(1).uniform(0, 1, 600)
    ok = O.Kernel(2, sigma=0.3)
    ref = O.ksvm_eval(d["A"], d["y"], ok, 1.0, a)
    got = K.kdcd_ksvm_eval(dev(d["A"]), dev(d["y"]), kern(2, sigma=0.3), 1.0, dev(a))
    for key in ("dual", "primal", "gap", "kkt"):
        assert abs(got[key] - ref[key]) <= 1e-10 * max(1.0, abs(ref[key])), key
    c = inputs.dense_krr_c2(m=600, n=12, seed=2)
    refk = O.krr_eval(c["A"], c["y"], ok, 1e-2, a)
    gotk = K.kdcd_krr_eval(dev(c["A"]), dev(c["y"]), kern(2, sigma=0.3), 1e-2, dev(a))
    assert abs(gotk["objective"] - refk["objective"]) <= 1e-10 * abs(refk["objective"])
    assert abs(gotk["residual_norm"] - refk["residual_norm"]) <= 1e-9 * refk["residual_norm"]

"""Parity at the configurations' own sizes, where a launch's grid no longer
holds one workgroup per row tile and every workgroup walks several row tiles
(carrying its column sums across them): C4 (200000 x 1024, s*b = 512), C5
(500000 x 256, s = 64) and m = 140000 matrices with few columns that drive the
same walk cheaply.

Where the oracle cannot finish a whole outer iteration in seconds the checks
use outputs it computes one by one (sampled columns of r, the whole Gram W) or
an identity of the method that holds at any size:

  K-RR (reading R6) minimises 1/2 a^T (K/lambda + m I) a - y^T a.  When alpha
  vanishes outside a row set R that holds every sampled row, a block step only
  sees the rows of R, and the problem on R alone with m' = |R|,
  lambda' = lambda m / m' and y' = y m' / m has the same steps: its block
  matrix and right-hand side are the full problem's times m'/m.  K-SVM steps
  on such an alpha are those of the problem on R with no change at all.

The warm starts are dense wherever the oracle runs at full size, so that every
row group contributes to r.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2406_18001_amd import inputs
from tests.helpers import assert_parity, dev, idx_dev, max_rel

pytestmark = pytest.mark.gpu

RBF1 = (2, 1.0, 0.0, 1)
TOL_R = {"f64": 1e-11, "f32": 1e-5, "bf16x3": 1e-5, "f16": 2e-3, "bf16": 1.5e-2}


@pytest.fixture(scope="module")
def K():
    from paper_2406_18001_amd import kdcd
    return kdcd


@pytest.fixture(scope="module")
def c4():
    d = inputs.dense_c4()
    d["A_dev"] = dev(d["A"])
    return d


@pytest.fixture(scope="module")
def walk():
    """m = 140000, n = 32: beyond 1024 row tiles of 128 rows."""
    d = inputs.dense_c4(m=140000, n=32, n_classes=4, seed=21)
    d["A_dev"] = dev(d["A"])
    return d


@pytest.mark.parametrize("sb", [16, 64, 512])
def test_rhs_row_group_walk(K, walk, sb):
    A = walk["A"]
    m = A.shape[0]
    rng = np.random.default_rng(sb)
    S = rng.integers(0, m, size=sb).astype(np.int32)
    beta = rng.standard_normal(m)
    ok = O.Kernel(O.RBF, sigma=1.0)
    r_ref = O.kernel_rhs(A, ok, S, beta)
    W_ref = O.kernel_block(A, ok, S, S)
    for compute in ("f64", "f32", "bf16x3", "f16", "bf16"):
        r, W = K.kdcd_kernel_rhs(walk["A_dev"], RBF1, idx_dev(S), dev(beta), want_W=True,
                                 compute=compute)
        err = assert_parity(r.cpu().numpy(), r_ref, TOL_R[compute], f"r {compute} sb={sb}")
        print(f"m={m} n=32 sb={sb} {compute}: r error {err:.2e}")
        assert_parity(W.cpu().numpy(), W_ref, 1e-12, f"W {compute} sb={sb}")


@pytest.mark.parametrize("compute", ["f64", "bf16x3", "f32", "f16", "bf16"])
def test_rhs_c4_full_size(K, c4, compute):
    """C4's kernel block (200000 x 1024, s*b = 512): W whole, r on 16 columns."""
    A = c4["A"]
    m = A.shape[0]
    rng = np.random.default_rng(4)
    S = inputs.krr_indices(m, 16, 32, seed=0)
    beta = rng.standard_normal(m)
    r, W = K.kdcd_kernel_rhs(c4["A_dev"], RBF1, idx_dev(S), dev(beta), want_W=True,
                             compute=compute)
    ok = O.Kernel(O.RBF, sigma=1.0)
    cols = np.linspace(0, 511, 16).astype(int)
    r_ref = O.kernel_rhs(A, ok, S[cols], beta)
    err = assert_parity(r.cpu().numpy()[cols], r_ref, TOL_R[compute], f"r {compute}")
    print(f"C4 {compute}: r error on 16 columns {err:.2e}")
    if compute == "f64":
        assert_parity(W.cpu().numpy(), O.kernel_block(A, ok, S, S), 1e-12, "W")


def _restricted(m, support, idx):
    """Rows R = support U idx (sorted) and idx renumbered into R."""
    R = np.union1d(support, idx).astype(np.int64)
    pos = np.full(m, -1, dtype=np.int64)
    pos[R] = np.arange(R.size)
    return R, pos[idx].astype(np.int32)


def test_krr_c4_one_outer_iteration(K, c4):
    """C4 K-RR (b = 16, s = 32, lambda = 1e-3, sigma = 1) for one outer iteration
    from a warm start on 20000 rows, against the oracle on the restricted problem."""
    A, y = c4["A"], c4["y"]
    m, b, s, lam = A.shape[0], 16, 32, 1e-3
    rng = np.random.default_rng(5)
    T = rng.choice(m, 20000, replace=False)
    alpha0 = np.zeros(m)
    alpha0[T] = rng.standard_normal(T.size) * 1e-4
    idx = inputs.krr_indices(m, b, s, seed=0)
    a = dev(alpha0)
    tr = torch.zeros(s * b, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(c4["A_dev"], dev(y), RBF1, lam, b, s, s, idx_dev(idx), a, trace=tr)
    R, idx_r = _restricted(m, T, idx)
    mr = R.size
    ref, th = O.bdcd_krr(A[R], y[R] * (mr / m), O.Kernel(O.RBF, sigma=1.0), lam * m / mr, b, s,
                         idx_r, alpha0=alpha0[R], s=s)
    got = a.cpu().numpy()
    assert_parity(got[R], ref, 1e-9, "alpha on R")
    assert np.array_equal(np.delete(got, R), np.delete(alpha0, R))
    assert_parity(tr.cpu().numpy(), th, 1e-9, "Delta alpha")


@pytest.mark.parametrize("sigma", [2.0 / 256, 2.0])
def test_ksvm_c5_one_outer_iteration(K, sigma):
    """C5 K-SVM-L1 (500000 x 256, C = 10, s = 64) for one outer iteration from a
    dense warm start, against the oracle at full size.  sigma = 2 is C5 as
    written (off-diagonal kernel values underflow to 0, reading R11); 2/256 is
    the coupled variant C5s."""
    d = inputs.dense_ksvm_c5()
    A, y = d["A"], d["y"]
    m, s, C = A.shape[0], 64, 10.0
    rng = np.random.default_rng(6)
    alpha0 = rng.uniform(0.0, C, m)
    idx = inputs.ksvm_indices(m, s, seed=0)
    a = dev(alpha0)
    tr = torch.zeros(s, dtype=torch.float64, device="cuda")
    K.kdcd_ksvm_solve(dev(A), dev(y), (2, sigma, 0.0, 1), C, 1, s, s, idx_dev(idx), a, trace=tr)
    ref, th = O.dcd_ksvm(A, y, O.Kernel(O.RBF, sigma=sigma), C, s, idx, alpha0=alpha0, s=s)
    assert_parity(a.cpu().numpy(), ref, 1e-9, "alpha")
    assert_parity(tr.cpu().numpy(), th, 1e-9, "theta")


def test_batch_row_group_walk(K, walk):
    """The C4 batch (8-point K-RR sweep + one-vs-rest K-SVMs, b = 16, s = 32) at
    m = 140000: one outer iteration from dense warm starts; every problem against
    its single solve and one problem per sigma group plus two K-SVMs against the
    oracle at full size."""
    A, y, Y = walk["A"], walk["y"], walk["Y_ovr"]
    m, b, s = A.shape[0], 16, 32
    rng = np.random.default_rng(7)
    idx = inputs.krr_indices(m, b, s, seed=1)
    I = idx_dev(idx)
    a_krr = rng.standard_normal(m) * 1e-4
    a_svm = rng.uniform(0.0, 1.0, m)
    probs = [K.BatchProblem("krr", lam, sig, dev(y), dev(a_krr),
                            trace=torch.zeros(s * b, dtype=torch.float64, device="cuda"))
             for lam, sig in inputs.KRR_SWEEP_C4]
    probs += [K.BatchProblem("ksvm", 1.0, 1.0, dev(Y[c]), dev(a_svm),
                             trace=torch.zeros(s * b, dtype=torch.float64, device="cuda"))
              for c in range(Y.shape[0])]
    K.kdcd_batch_solve(walk["A_dev"], RBF1, b, s, s, I, probs)
    checked = set()
    for i, (lam, sig) in enumerate(inputs.KRR_SWEEP_C4):
        a1 = dev(a_krr)
        K.kdcd_krr_solve(walk["A_dev"], dev(y), (2, sig, 0.0, 1), lam, b, s, s, I, a1)
        assert_parity(probs[i].alpha.cpu().numpy(), a1.cpu().numpy(), 1e-11, f"krr {i}")
        if sig not in checked:
            checked.add(sig)
            ref, _ = O.bdcd_krr(A, y, O.Kernel(O.RBF, sigma=sig), lam, b, s, idx,
                                alpha0=a_krr, s=s)
            assert_parity(probs[i].alpha.cpu().numpy(), ref, 1e-9, f"krr {i} oracle")
    nk = len(inputs.KRR_SWEEP_C4)
    for c in range(Y.shape[0]):
        a1 = dev(a_svm)
        K.kdcd_ksvm_solve(walk["A_dev"], dev(Y[c]), RBF1, 1.0, 1, s * b, s * b, I, a1)
        assert_parity(probs[nk + c].alpha.cpu().numpy(), a1.cpu().numpy(), 1e-11, f"svm {c}")
        if c < 2:
            ref, th = O.dcd_ksvm(A, Y[c], O.Kernel(O.RBF, sigma=1.0), 1.0, s * b, idx,
                                 alpha0=a_svm, s=s * b)
            assert_parity(probs[nk + c].alpha.cpu().numpy(), ref, 1e-9, f"svm {c} oracle")
            assert_parity(probs[nk + c].trace.cpu().numpy(), th, 1e-9, f"svm {c} theta")


def test_batch_c4_full_size_matches_single(K, c4):
    """The C4 batch at its own size for one outer iteration: every problem equals
    its single solve (whose kernel block the tests above check against the
    oracle), FP64 and bf16x3."""
    A, y, Y = c4["A_dev"], dev(c4["y"]), c4["Y_ovr"]
    m, b, s = c4["A"].shape[0], 16, 32
    idx = idx_dev(inputs.krr_indices(m, b, s, seed=2))
    rng = np.random.default_rng(8)
    a_krr = rng.standard_normal(m) * 1e-4
    a_svm = rng.uniform(0.0, 1.0, m)
    # bf16x3: the batched and single products use different MFMA shapes, whose
    # FP32 sums round differently (a few ulps of each kernel value)
    for compute, tol in (("f64", 1e-11), ("bf16x3", 5e-5)):
        probs = [K.BatchProblem("krr", lam, sig, y, dev(a_krr)) for lam, sig in inputs.KRR_SWEEP_C4]
        probs += [K.BatchProblem("ksvm", 1.0, 1.0, dev(Y[c]), dev(a_svm)) for c in range(10)]
        K.kdcd_batch_solve(A, RBF1, b, s, s, idx, probs, compute=compute)
        for i, (lam, sig) in enumerate(inputs.KRR_SWEEP_C4):
            a1 = dev(a_krr)
            K.kdcd_krr_solve(A, y, (2, sig, 0.0, 1), lam, b, s, s, idx, a1, compute=compute)
            assert_parity(probs[i].alpha.cpu().numpy(), a1.cpu().numpy(), tol, f"{compute} krr {i}")
        for c in range(10):
            a1 = dev(a_svm)
            K.kdcd_ksvm_solve(A, dev(Y[c]), RBF1, 1.0, 1, s * b, s * b, idx, a1, compute=compute)
            assert_parity(probs[8 + c].alpha.cpu().numpy(), a1.cpu().numpy(), tol,
                          f"{compute} svm {c}")

"""Sparse K-RR with the RBF kernel on news20-shaped rows (long, heavy-tailed
rows over a million columns; the Table 4 workload) through the CSR path,
against the FP64 oracle: a reduced matrix with every block size of Table 4
and several s, and the full-size matrix for its first outer iterations in
the configuration the benchmark times."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2406_18001_amd import inputs
from tests.helpers import assert_parity, dev, idx_dev

pytestmark = pytest.mark.gpu

TOL = 1e-9
RBF1 = (2, 1.0, 0.0, 1)


@pytest.fixture(scope="module")
def K():
    from paper_2406_18001_amd import kdcd
    return kdcd


def to_gpu(K, c):
    return K.CSR(torch.as_tensor(c["row_ptr"]).cuda(), torch.as_tensor(c["col_idx"]).cuda(),
                 torch.as_tensor(c["val"]).cuda(), c["m"], c["n"])


def as_oracle(c):
    return (c["row_ptr"], c["col_idx"], c["val"], c["m"], c["n"])


@pytest.fixture(scope="module")
def small():
    return inputs.csr_news20(m=1500, n=80000, seed=7)


@pytest.mark.parametrize("b", [1, 2, 4])
@pytest.mark.parametrize("s", [1, 5, 16])
def test_news20_krr_small(K, small, b, s):
    c = small
    H = 48
    idx = inputs.krr_indices(c["m"], b, H, seed=b)
    ref, ref_tr = O.bdcd_krr(as_oracle(c), c["y"], O.Kernel(O.RBF, sigma=1.0), 1e-3, b, H, idx,
                             s=s)
    alpha = torch.zeros(c["m"], dtype=torch.float64, device="cuda")
    tr = torch.zeros(H * b, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(to_gpu(K, c), dev(c["y"]), RBF1, 1e-3, b, s, H, idx_dev(idx), alpha, trace=tr)
    assert_parity(alpha.cpu().numpy(), ref, TOL, "alpha")
    assert_parity(tr.cpu().numpy(), ref_tr, TOL, "trace")


@pytest.mark.parametrize("kk", [RBF1, (1, 0.0, 1.0, 3), (0, 0.0, 0.0, 1)])
@pytest.mark.parametrize("sb", [1, 5, 8, 13, 40])
def test_news20_kernel_rhs(K, small, kk, sb):
    """r and W of one block for every kernel, with the longest rows (several
    chunks of the sampled-row panel) and short ones in the block."""
    c = small
    lens = np.diff(c["row_ptr"])
    order = np.argsort(lens)
    S = np.concatenate([order[-(sb // 2):] if sb > 1 else order[-1:], order[:sb - max(sb // 2, 1)]])
    S = S.astype(np.int32)
    beta = np.random.default_rng(sb).standard_normal(c["m"])
    ok = O.Kernel(kk[0], sigma=kk[1], c=kk[2], degree=kk[3])
    r, W = K.kdcd_kernel_rhs(to_gpu(K, c), kk, idx_dev(S), dev(beta), want_W=True)
    assert_parity(r.cpu().numpy(), O.kernel_rhs(as_oracle(c), ok, S, beta), 1e-11, "r")
    assert_parity(W.cpu().numpy().reshape(S.size, S.size), O.kernel_block(as_oracle(c), ok, S, S),
                  1e-12, "W")


def test_news20_full_size_first_outer_iterations(K):
    """19996 x 1355191, 9.2e6 stored entries, b = 4, s = 16: the first two
    outer iterations, every coordinate, against the oracle."""
    c = inputs.csr_news20()
    b, s, H = 4, 16, 32
    idx = inputs.krr_indices(c["m"], b, H, seed=0)
    ref, _ = O.bdcd_krr(as_oracle(c), c["y"], O.Kernel(O.RBF, sigma=1.0), 1e-3, b, H, idx, s=s)
    alpha = torch.zeros(c["m"], dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(to_gpu(K, c), dev(c["y"]), RBF1, 1e-3, b, s, H, idx_dev(idx), alpha)
    assert_parity(alpha.cpu().numpy(), ref, TOL, "alpha")


@pytest.fixture(scope="module")
def longrows():
    # news20-shaped rows without the clip at the panel size: many rows longer
    # than 3072 stored entries, summed over pieces
    return inputs.csr_news20(m=700, n=60000, mean_nnz=1200.0, max_nnz=9000, seed=11)


def test_news20_rows_longer_than_panel_rhs(K, longrows):
    c = longrows
    lens = np.diff(c["row_ptr"])
    assert (lens > 3072).sum() >= 20
    ok = O.Kernel(O.RBF, sigma=1.0)
    beta = np.random.default_rng(1).standard_normal(c["m"])
    order = np.argsort(lens)
    for S in (order[-1:], order[-3:], np.concatenate([order[-4:], order[:6]]), order[::35]):
        S = np.asarray(S, dtype=np.int32)
        r, W = K.kdcd_kernel_rhs(to_gpu(K, c), RBF1, idx_dev(S), dev(beta), want_W=True)
        assert_parity(r.cpu().numpy(), O.kernel_rhs(as_oracle(c), ok, S, beta), 1e-11, "r")
        assert_parity(W.cpu().numpy(), O.kernel_block(as_oracle(c), ok, S, S), 1e-12, "W")


@pytest.mark.parametrize("b,s", [(1, 8), (2, 4), (4, 1)])
def test_news20_rows_longer_than_panel_krr(K, longrows, b, s):
    c = longrows
    H = 24
    idx = inputs.krr_indices(c["m"], b, H, seed=3)
    ref, _ = O.bdcd_krr(as_oracle(c), c["y"], O.Kernel(O.RBF, sigma=1.0), 1e-3, b, H, idx, s=s)
    alpha = torch.zeros(c["m"], dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(to_gpu(K, c), dev(c["y"]), RBF1, 1e-3, b, s, H, idx_dev(idx), alpha)
    assert_parity(alpha.cpu().numpy(), ref, TOL, "alpha")

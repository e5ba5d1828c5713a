"""On-device convergence monitor: the maintained dual vector, the certified
bound it reports, early stopping, and the error paths.

The monitor's quantities have closed forms in the oracle's objective
evaluators: K-RR rel = (||y - M a||^2 / 2m) / (|f| - that) from
(objective, residual norm); K-SVM rel = gap / |dual| from (dual, gap).
Both are compared with the oracle at the final iterate; an early stop is
checked against a plain solve of exactly the reported number of outer
iterations (bit for bit: the monitor does not change the iteration)."""
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


def krr_rel(ev, m):
    bound = 0.5 * ev["residual_norm"] ** 2 / m
    return bound / (abs(ev["objective"]) - bound)


@pytest.mark.parametrize("warm", [False, True])
def test_krr_monitor_value_and_iterates(K, warm):
    d = inputs.dense_krr_c2(m=2000, n=64, seed=8)
    m, b, s, H = 2000, 8, 16, 16 * 12 + 5
    idx = inputs.krr_indices(m, b, H, seed=3)
    kern = (2, 1.0, 0.0, 1)
    a0 = np.zeros(m)
    if warm:     # start from a partly converged iterate: the initial residual needs K a0
        w = torch.zeros(m, dtype=torch.float64, device="cuda")
        K.kdcd_krr_solve(dev(d["A"]), dev(d["y"]), kern, 1e-3, b, s, 40 * s,
                         idx_dev(inputs.krr_indices(m, b, 40 * s, seed=9)), w)
        a0 = w.cpu().numpy()
    a = dev(a0)
    info = K.kdcd_krr_solve(dev(d["A"]), dev(d["y"]), kern, 1e-3, b, s, H, idx_dev(idx), a,
                            monitor_every=4, tol=0.0)
    plain = dev(a0)
    K.kdcd_krr_solve(dev(d["A"]), dev(d["y"]), kern, 1e-3, b, s, H, idx_dev(idx), plain)
    assert torch.equal(a, plain)
    assert info["outer_done"] == -(-H // s)
    ev = O.krr_eval(d["A"], d["y"], O.Kernel(O.RBF, sigma=1.0), 1e-3, a.cpu().numpy())
    ref = krr_rel(ev, m)
    assert ref > 0
    assert abs(info["rel_err"] - ref) <= 1e-7 * ref


@pytest.mark.parametrize("loss", [1, 2])
def test_ksvm_monitor_value_and_early_stop(K, loss):
    d = inputs.dense_ksvm_c1(m=1500, n=16, seed=9)
    m, s, C = 1500, 32, 1.0
    H = 40 * m
    idx = inputs.ksvm_indices(m, H, seed=4)
    kern = (2, 1.0 / 16, 0.0, 1)
    okern = O.Kernel(O.RBF, sigma=1.0 / 16)
    # no stop: the reported gap matches the oracle's at the end of 3 epochs
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    H3 = 3 * m
    info = K.kdcd_ksvm_solve(dev(d["A"]), dev(d["y"]), kern, C, 1, s, H3, idx_dev(idx[:H3]), a,
                             loss=loss, monitor_every=5, tol=0.0)
    ev = O.ksvm_eval(d["A"], d["y"], okern, C, a.cpu().numpy(), loss=loss)
    ref = ev["gap"] / abs(ev["dual"])
    assert abs(info["rel_err"] - ref) <= 1e-7 * ref + 1e-12, (info["rel_err"], ref)
    # stop at 1e-4: the result equals a plain solve of the reported outer iterations
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    info = K.kdcd_ksvm_solve(dev(d["A"]), dev(d["y"]), kern, C, 1, s, H, idx_dev(idx), a,
                             loss=loss, monitor_every=10, tol=1e-4)
    k = info["outer_done"]
    assert 0 < k < H // s and k % 10 == 0 and info["rel_err"] <= 1e-4
    plain = torch.zeros(m, dtype=torch.float64, device="cuda")
    K.kdcd_ksvm_solve(dev(d["A"]), dev(d["y"]), kern, C, 1, s, k * s, idx_dev(idx[:k * s]), plain,
                      loss=loss)
    assert torch.equal(a, plain)
    ev = O.ksvm_eval(d["A"], d["y"], okern, C, a.cpu().numpy(), loss=loss)
    assert ev["gap"] / abs(ev["dual"]) <= 1e-4 * (1 + 1e-6)


def test_krr_early_stop_and_snapshots(K):
    d = inputs.dense_krr_c2(m=3000, n=64, seed=10)
    m, b, s = 3000, 8, 32
    H = 400 * s
    idx = inputs.krr_indices(m, b, H, seed=5)
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    rows = -(-(H // s) // 50)
    snaps = torch.full((rows * m,), 7.0, dtype=torch.float64, device="cuda")
    info = K.kdcd_krr_solve(dev(d["A"]), dev(d["y"]), (2, 1.0, 0.0, 1), 1e-3, b, s, H,
                            idx_dev(idx), a, monitor_every=8, tol=1e-6, snapshot_every=50,
                            snapshots=snaps)
    k = info["outer_done"]
    assert k < H // s and info["rel_err"] <= 1e-6
    ev = O.krr_eval(d["A"], d["y"], O.Kernel(O.RBF, sigma=1.0), 1e-3, a.cpu().numpy())
    assert krr_rel(ev, m) <= 1e-6 * (1 + 1e-6)
    # every snapshot taken after the stop holds the final iterate
    sn = snaps.view(rows, m)
    for r in range(rows):
        if (r + 1) * 50 >= k:
            assert torch.equal(sn[r], a)


def test_sampled_solve_with_monitor(K):
    d = inputs.dense_ksvm_c5(m=3000, n=32, seed=25)
    m, C, s = 3000, 10.0, 64
    kern = (2, 2.0 / 32, 0.0, 1)
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    idx, info = K.kdcd_ksvm_solve_sampled(dev(d["A"]), dev(d["y"]), kern, C, s, 60 * m, a,
                                          seed=3, monitor_every=16, tol=1e-3)
    k = info["outer_done"]
    assert 0 < k < -(-60 * m // s) and info["rel_err"] <= 1e-3
    a_ref, _ = O.dcd_ksvm(d["A"], d["y"], O.Kernel(O.RBF, sigma=2.0 / 32), C, k * s,
                          idx.cpu().numpy()[:k * s], s=s)
    assert_parity(a.cpu().numpy(), a_ref, 1e-9, "alpha")


def test_monitor_errors(K):
    d = inputs.dense_krr_c2(m=300, n=8, seed=1)
    idx = idx_dev(inputs.krr_indices(300, 2, 20, seed=0))
    a = torch.zeros(300, dtype=torch.float64, device="cuda")
    args = (dev(d["A"]), dev(d["y"]), (2, 1.0, 0.0, 1), 1e-3, 2, 5, 20, idx, a)
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_krr_solve(*args, monitor_every=2, tol=-1.0)
    assert e.value.status == -1
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_krr_solve(*args, monitor_every=2, tol=1e-6, compute="f32")
    assert e.value.status == -2
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_krr_solve(*args, monitor_every=2, tol=1e-6, flags=K.FLAG_GRAPH)
    assert e.value.status == -2


def csr_of(K, c):
    return K.CSR(torch.as_tensor(c["row_ptr"]).cuda(), torch.as_tensor(c["col_idx"]).cuda(),
                 torch.as_tensor(c["val"]).cuda(), c["m"], c["n"])


@pytest.mark.parametrize("s", [8, 32])
def test_csr_ksvm_monitor_value_and_early_stop(K, s):
    """CSR K-SVM (C3 recipe, small): s = 8 runs the broadcast product, s = 32
    the dense-head product; the certified gap against the oracle's at the
    final iterate, and an early stop against a plain solve."""
    c = inputs.csr_ksvm_c3(m=2000, n=1500, nnz_per_row=20, seed=41)
    m, C = c["m"], 1.0
    kern, okern = (1, 0.0, 1.0, 3), O.Kernel(O.POLY, c=1.0, degree=3)
    A, oA = csr_of(K, c), (c["row_ptr"], c["col_idx"], c["val"], c["m"], c["n"])
    H = 4 * m
    idx = inputs.ksvm_indices(m, H, seed=6)
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    H2 = 2 * m
    info = K.kdcd_ksvm_solve(A, dev(c["y"]), kern, C, 1, s, H2, idx_dev(idx[:H2]), a,
                             monitor_every=5, tol=0.0, monitor_log=True)
    ev = O.ksvm_eval(oA, c["y"], okern, C, a.cpu().numpy())
    ref = ev["gap"] / abs(ev["dual"])
    assert abs(info["rel_err"] - ref) <= 1e-7 * ref + 1e-12, (info["rel_err"], ref)
    log = info["log"]
    n_outer = -(-H2 // s)
    assert [int(r[0]) for r in log] == list(range(5, n_outer + 1, 5)) + (
        [n_outer] if n_outer % 5 else [])
    assert log[-1][1] == info["rel_err"]
    assert all(t1 > t0 for (_, _, _, t0), (_, _, _, t1) in zip(log, log[1:]))
    # stop at the bound the logged run certified half-way (same iterates)
    j = len(log) // 2
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    info = K.kdcd_ksvm_solve(A, dev(c["y"]), kern, C, 1, s, H, idx_dev(idx), a,
                             monitor_every=5, tol=log[j][1])
    k = info["outer_done"]
    assert 0 < k <= int(log[j][0]) and k % 5 == 0 and info["rel_err"] <= log[j][1]
    plain = torch.zeros(m, dtype=torch.float64, device="cuda")
    K.kdcd_ksvm_solve(A, dev(c["y"]), kern, C, 1, s, k * s, idx_dev(idx[:k * s]), plain)
    assert torch.equal(a, plain)


def test_csr_krr_monitor_value(K):
    """CSR K-RR with the RBF kernel (b = 4, s = 8: the dense-head product):
    the certified bound against the oracle's residual at the final iterate."""
    c = inputs.csr_ksvm_c3(m=1500, n=1200, nnz_per_row=15, seed=43)
    m, b, s, lam = c["m"], 4, 8, 1e-2
    y = np.random.default_rng(2).standard_normal(m)
    A, oA = csr_of(K, c), (c["row_ptr"], c["col_idx"], c["val"], c["m"], c["n"])
    H = 40 * s + 3
    idx = inputs.krr_indices(m, b, H, seed=8)
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    info = K.kdcd_krr_solve(A, dev(y), (2, 0.5, 0.0, 1), lam, b, s, H, idx_dev(idx), a,
                            monitor_every=7, tol=0.0)
    ev = O.krr_eval(oA, y, O.Kernel(O.RBF, sigma=0.5), lam, a.cpu().numpy())
    ref = krr_rel(ev, m)
    assert abs(info["rel_err"] - ref) <= 1e-7 * ref


@pytest.mark.parametrize("compute,tol", [("bf16x3", 1e-4), ("bf16", 5e-2), ("f16", 5e-2)])
def test_lowp_monitor(K, compute, tol):
    """Low-precision K-RR products store their kernel block for the monitor:
    the certified bound follows the exact problem's (oracle) within the
    kernel's rounding, and an early stop matches a plain solve."""
    d = inputs.dense_krr_c2(m=2000, n=64, seed=8)
    m, b, s, H = 2000, 8, 16, 16 * 20
    idx = inputs.krr_indices(m, b, H, seed=3)
    kern = (2, 1.0, 0.0, 1)
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    info = K.kdcd_krr_solve(dev(d["A"]), dev(d["y"]), kern, 1e-3, b, s, H, idx_dev(idx), a,
                            compute=compute, monitor_every=4, tol=0.0, monitor_log=True)
    ev = O.krr_eval(d["A"], d["y"], O.Kernel(O.RBF, sigma=1.0), 1e-3, a.cpu().numpy())
    ref = krr_rel(ev, m)
    assert abs(info["rel_err"] - ref) <= tol * ref, (info["rel_err"], ref)
    assert len(info["log"]) == H // s // 4 and info["log"][-1][1] == info["rel_err"]
    stop_at = info["log"][2][1] * 1.0000001      # reached at the third evaluation
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    info = K.kdcd_krr_solve(dev(d["A"]), dev(d["y"]), kern, 1e-3, b, s, H, idx_dev(idx), a,
                            compute=compute, monitor_every=4, tol=stop_at)
    k = info["outer_done"]
    assert k <= 12 and k % 4 == 0 and info["rel_err"] <= stop_at, k
    plain = torch.zeros(m, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(dev(d["A"]), dev(d["y"]), kern, 1e-3, b, s, k * s, idx_dev(idx[:k * s * b]),
                     plain, compute=compute)
    assert torch.equal(a, plain)


def test_batch_monitor_value_and_early_stop(K):
    """Batched solves (two K-RR and two K-SVM problems over two sigma groups,
    FP64): the batch's bound is the largest of the problems' certified bounds
    (each against the oracle), the log follows it, and a stop at a logged
    bound equals a plain batched solve of the reported outer iterations, every
    problem bit for bit."""
    d = inputs.dense_ksvm_c1(m=1500, n=32, seed=12)
    m, b, s = 1500, 4, 8
    A = dev(d["A"])
    ys = dev(d["y"])
    yr = dev(np.random.default_rng(5).standard_normal(m))
    kern = (2, 1.0 / 32, 0.0, 1)
    spec = [("krr", 1.0, 1.0 / 32, yr, 1), ("krr", 0.1, 0.5 / 32, yr, 1),
            ("ksvm", 1.0, 1.0 / 32, ys, 1), ("ksvm", 0.5, 0.5 / 32, ys, 2)]
    H = 40 * s + 3
    idx = idx_dev(inputs.krr_indices(m, b, H, seed=4))

    def problems():
        return [K.BatchProblem(kind, par, sg, y, torch.zeros(m, dtype=torch.float64, device="cuda"),
                               loss=loss) for kind, par, sg, y, loss in spec]

    ps = problems()
    info = K.kdcd_batch_solve(A, kern, b, s, H, idx, ps, monitor_every=3, tol=0.0,
                              monitor_log=True)
    refs = []
    for (kind, par, sg, y, loss), q in zip(spec, ps):
        ok = O.Kernel(O.RBF, sigma=sg)
        a = q.alpha.cpu().numpy()
        if kind == "krr":
            refs.append(krr_rel(O.krr_eval(d["A"], y.cpu().numpy(), ok, par, a), m))
        else:
            ev = O.ksvm_eval(d["A"], y.cpu().numpy(), ok, par, a, loss=loss)
            refs.append(ev["gap"] / abs(ev["dual"]))
    assert all(0 < r < 1e3 for r in refs), refs      # every bound certifiable here
    ref = max(refs)
    assert abs(info["rel_err"] - ref) <= 1e-7 * ref, (info["rel_err"], refs)
    log = info["log"]
    n_outer = -(-H // s)
    assert [int(r[0]) for r in log] == list(range(3, n_outer + 1, 3)) + (
        [n_outer] if n_outer % 3 else [])
    assert log[-1][1] == info["rel_err"]
    fin = [i for i, r in enumerate(log) if np.isfinite(r[1])]   # early bounds may be infinite
    j = fin[len(fin) // 2]
    ps = problems()
    info = K.kdcd_batch_solve(A, kern, b, s, H, idx, ps, monitor_every=3, tol=log[j][1])
    k = info["outer_done"]
    assert 0 < k <= int(log[j][0]) and k % 3 == 0 and info["rel_err"] <= log[j][1]
    plain = problems()
    K.kdcd_batch_solve(A, kern, b, s, k * s, idx[:k * s * b], plain)
    for q1, q2 in zip(ps, plain):
        assert torch.equal(q1.alpha, q2.alpha)
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_batch_solve(A, kern, b, s, H, idx, problems(), compute="bf16x3", monitor_every=3,
                           tol=1e-6)
    assert e.value.status == -2

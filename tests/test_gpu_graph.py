"""KDCD_FLAG_GRAPH: the captured launch sequence, replayed, gives the eager
result of the same (serial) outer loop bit for bit.  Every replay is checked, with the program's own eager
work (resets, in-place changes of the inputs, other solves) and
synchronisations between the replays, so that a replay reading stale or
wrongly cleared memory shows up."""
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
    yield kdcd
    kdcd.kdcd_graph_cache_clear()


def test_krr_graph_replays_equal_eager(K):
    d = inputs.dense_krr_c2(m=3000, n=96, seed=3)
    A, y = dev(d["A"]), dev(d["y"])
    idx = idx_dev(inputs.krr_indices(3000, 8, 203, seed=1))
    kern = (2, 1.0, 0.0, 1)
    eager = torch.zeros(3000, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(A, y, kern, 1e-3, 8, 16, 203, idx, eager)
    alpha = torch.zeros(3000, dtype=torch.float64, device="cuda")
    for rep in range(4):
        alpha.zero_()
        K.kdcd_krr_solve(A, y, kern, 1e-3, 8, 16, 203, idx, alpha, flags=K.FLAG_GRAPH)
        torch.cuda.synchronize()
        assert torch.equal(alpha, eager), f"replay {rep}"
        tmp = torch.zeros_like(alpha)                 # unrelated eager work in between
        K.kdcd_krr_solve(A, y, kern, 1e-2, 8, 4, 40, idx, tmp)
    # the graph reads the current contents of its inputs
    y.mul_(2.0)
    eager2 = torch.zeros_like(alpha)
    K.kdcd_krr_solve(A, y, kern, 1e-3, 8, 16, 203, idx, eager2)
    alpha.zero_()
    K.kdcd_krr_solve(A, y, kern, 1e-3, 8, 16, 203, idx, alpha, flags=K.FLAG_GRAPH)
    assert torch.equal(alpha, eager2)
    assert_parity(alpha.cpu().numpy(), 2.0 * eager.cpu().numpy(), 1e-12, "linear in y")


def test_ksvm_graph_with_trace_snapshots_and_warm_start(K):
    d = inputs.dense_ksvm_c1(m=1200, n=32, seed=4)
    A, y = dev(d["A"]), dev(d["y"])
    H, s = 300, 32
    idx = inputs.ksvm_indices(1200, H, seed=2)
    kern = (2, 1.0 / 32, 0.0, 1)
    a0 = np.random.default_rng(1).uniform(0, 1.0, 1200)
    rows = -(-(-(-H // s)) // 3)
    outs = []
    for flags in (0, K.FLAG_GRAPH, K.FLAG_GRAPH, K.FLAG_GRAPH):
        a = dev(a0)
        tr = torch.zeros(H, dtype=torch.float64, device="cuda")
        sn = torch.zeros(rows * 1200, dtype=torch.float64, device="cuda")
        K.kdcd_ksvm_solve(A, y, kern, 1.0, 1, s, H, idx_dev(idx), a, loss=2, trace=tr,
                          snapshot_every=3, snapshots=sn, flags=flags)
        outs.append((a.cpu(), tr.cpu(), sn.cpu()))
    for o in outs[1:]:
        for x, ref in zip(o, outs[0]):
            assert torch.equal(x, ref)
    a_ref, _ = O.dcd_ksvm(d["A"], d["y"], O.Kernel(O.RBF, sigma=1 / 32), 1.0, H, idx,
                          alpha0=a0, loss=2, s=s)
    assert_parity(outs[1][0].numpy(), a_ref, 1e-9, "alpha")


@pytest.mark.parametrize("compute", ["f64", "bf16x3"])
def test_batch_graph_replays_equal_eager(K, compute):
    d = inputs.dense_c4(m=2000, n=64, n_classes=3, seed=5)
    A, y = dev(d["A"]), dev(d["y"])
    Y = [dev(d["Y_ovr"][c]) for c in range(3)]
    b, s, H = 4, 8, 50
    idx = idx_dev(inputs.krr_indices(2000, b, H, seed=0))

    def run(flags):
        probs = [K.BatchProblem("krr", 1e-3, sg, y, torch.zeros(2000, dtype=torch.float64, device="cuda"))
                 for sg in (0.5, 1.0)]
        probs += [K.BatchProblem("ksvm", 1.0, 1.0, yc, torch.zeros(2000, dtype=torch.float64, device="cuda"),
                                 trace=torch.zeros(H * b, dtype=torch.float64, device="cuda"))
                  for yc in Y]
        return probs

    eager = run(0)
    K.kdcd_batch_solve(A, (2, 1.0, 0.0, 1), b, s, H, idx, eager, compute=compute)
    g = run(K.FLAG_GRAPH)
    for rep in range(3):
        for p in g:
            p.alpha.zero_()
            if p.trace is not None:
                p.trace.fill_(7.0)
        K.kdcd_batch_solve(A, (2, 1.0, 0.0, 1), b, s, H, idx, g, compute=compute,
                           flags=K.FLAG_GRAPH)
        torch.cuda.synchronize()
        for pe, pg in zip(eager, g):
            assert torch.equal(pe.alpha, pg.alpha), f"replay {rep}"
            if pe.trace is not None:
                assert torch.equal(pe.trace, pg.trace)


def test_graph_reports_device_errors_on_every_replay(K):
    d = inputs.dense_krr_c2(m=500, n=16, seed=1)
    A, y = dev(d["A"]), dev(d["y"])
    idx = idx_dev(inputs.krr_indices(500, 4, 20, seed=0))
    a = torch.zeros(500, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(A, y, (2, 1.0, 0.0, 1), 1e-3, 4, 5, 20, idx, a, flags=K.FLAG_GRAPH)
    idx[7] = 500                                     # out of range, read at replay time
    for _ in range(2):
        with pytest.raises(K.KdcdError) as e:
            K.kdcd_krr_solve(A, y, (2, 1.0, 0.0, 1), 1e-3, 4, 5, 20, idx, a, flags=K.FLAG_GRAPH)
        assert e.value.status == -3
    idx[7] = idx[6]                                  # a duplicate inside one block
    a.zero_()
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_krr_solve(A, y, (2, 1.0, 0.0, 1), 1e-3, 4, 5, 20, idx, a, flags=K.FLAG_GRAPH)
    assert e.value.status == -4


def test_graph_cache_eviction_keeps_results(K):
    d = inputs.dense_krr_c2(m=800, n=16, seed=2)
    A, y = dev(d["A"]), dev(d["y"])
    idx = idx_dev(inputs.krr_indices(800, 2, 60, seed=0))
    for lam in [10.0 ** (-k) for k in range(1, 12)]:      # 11 keys > 8 cache entries
        a = torch.zeros(800, dtype=torch.float64, device="cuda")
        e = torch.zeros(800, dtype=torch.float64, device="cuda")
        K.kdcd_krr_solve(A, y, (2, 1.0, 0.0, 1), lam, 2, 6, 60, idx, a, flags=K.FLAG_GRAPH)
        K.kdcd_krr_solve(A, y, (2, 1.0, 0.0, 1), lam, 2, 6, 60, idx, e)
        assert torch.equal(a, e)
    K.kdcd_graph_cache_clear()
    a = torch.zeros(800, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(A, y, (2, 1.0, 0.0, 1), 1e-3, 2, 6, 60, idx, a, flags=K.FLAG_GRAPH)
    e = torch.zeros(800, dtype=torch.float64, device="cuda")
    K.kdcd_krr_solve(A, y, (2, 1.0, 0.0, 1), 1e-3, 2, 6, 60, idx, e)
    assert torch.equal(a, e)


def test_sampled_solve_refuses_graph(K):
    m = 200
    A = torch.randn(m, 8, dtype=torch.float64, device="cuda")
    y = torch.ones(m, dtype=torch.float64, device="cuda")
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_ksvm_solve_sampled(A, y, (2, 1.0, 0.0, 1), 1.0, 8, 16, a, flags=K.FLAG_GRAPH)
    assert e.value.status == -2


def _csr(K, c):
    return K.CSR(torch.as_tensor(c["row_ptr"]).cuda(), torch.as_tensor(c["col_idx"]).cuda(),
                 torch.as_tensor(c["val"]).cuda(), c["m"], c["n"])


@pytest.mark.parametrize("case", ["krr_f64", "krr_bf16x3", "ksvm_f64", "ksvm_csr"])
def test_windowed_graph_equals_eager(K, case):
    """Solves with at least 18 whole blocks replay a graph of 16 outer
    iterations window after window (the index blocks copied on the device from
    a counter): every result equals the eager solve bit for bit, also for a
    later call with another H and other index values in the same buffer (the
    same graph), with eager work and synchronisations in between."""
    if case.startswith("krr"):
        d = inputs.dense_krr_c2(m=2500, n=64, seed=5)
        A, y, m = dev(d["A"]), dev(d["y"]), 2500
        b, s, kern, par = 8, 16, (2, 1.0, 0.0, 1), 1e-3
        comp = "bf16x3" if case.endswith("bf16x3") else "f64"
        solve = lambda H, idx, a, **kw: K.kdcd_krr_solve(A, y, kern, par, b, s, H, idx, a,
                                                         compute=comp, **kw)
        draw = lambda H, seed: inputs.krr_indices(m, b, H, seed=seed)
    else:
        if case == "ksvm_csr":
            c = inputs.csr_ksvm_c3(m=3000, n=2000, nnz_per_row=20, seed=31)
            A, y, m, kern, s = _csr(K, c), dev(c["y"]), 3000, (1, 0.0, 1.0, 3), 32
        else:
            d = inputs.dense_ksvm_c1(m=2000, n=64, seed=5)
            A, y, m, kern, s = dev(d["A"]), dev(d["y"]), 2000, (2, 1.0, 0.0, 1), 8
        b, par = 1, 1.0
        solve = lambda H, idx, a, **kw: K.kdcd_ksvm_solve(A, y, kern, par, b, s, H, idx, a, **kw)
        draw = lambda H, seed: inputs.ksvm_indices(m, H, seed=seed)
    Hmax = s * 60
    buf = idx_dev(draw(Hmax, 1))
    g = torch.zeros(m, dtype=torch.float64, device="cuda")
    for H, seed in ((s * 40 + 3, 1), (s * 57, 2), (s * 18, 3), (s * 40 + 3, 1)):
        buf.copy_(idx_dev(draw(Hmax, seed)))
        eager = torch.zeros(m, dtype=torch.float64, device="cuda")
        solve(H, buf, eager)
        g.zero_()
        solve(H, buf, g, flags=K.FLAG_GRAPH)
        torch.cuda.synchronize()
        assert torch.equal(g, eager), (case, H, seed)


def test_batch_graph_and_eager_call_share_a_workspace(K):
    """A graph call and an eager call on one caller workspace: every replay runs
    with the graph's own problems (its batch descriptor is rewritten by a
    kernel inside the graph, not left in the workspace from the capture)."""
    m = 1500
    d = inputs.dense_c4(m=m, n=64, n_classes=3, seed=6)
    A, y = dev(d["A"]), dev(d["y"])
    b, s, H = 4, 8, 40
    idx = idx_dev(inputs.krr_indices(m, b, H, seed=1))
    ws = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")
    kern = (2, 1.0, 0.0, 1)

    def probs(lam):
        return [K.BatchProblem("krr", lam, sg, y, torch.zeros(m, dtype=torch.float64, device="cuda"))
                for sg in (0.5, 1.0)]

    ref = probs(1e-3)
    K.kdcd_batch_solve(A, kern, b, s, H, idx, ref)
    g, other = probs(1e-3), probs(1e-2)
    for rep in range(3):
        for p in g:
            p.alpha.zero_()
        K.kdcd_batch_solve(A, kern, b, s, H, idx, g, flags=K.FLAG_GRAPH, workspace=ws)
        torch.cuda.synchronize()
        for pr, pg in zip(ref, g):
            assert torch.equal(pr.alpha, pg.alpha), f"replay {rep}"
        for p in other:
            p.alpha.zero_()
        K.kdcd_batch_solve(A, kern, b, s, H, idx, other, workspace=ws)   # same workspace
        torch.cuda.synchronize()
        assert all(float(p.alpha.abs().max()) > 0 for p in other)

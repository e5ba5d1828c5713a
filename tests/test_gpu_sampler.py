"""The learned sampler on the GPU against the sampler oracle (oracle/sampler.py)
and the FP64 solve oracle.

* initial weights: bit-exact (both sides evaluate the same Philox outputs and
  round the same FP64 products to float32);
* MLP forward, loss gradient and Adam steps: FP32 device arithmetic against
  the FP64 oracle, to tolerances derived from float32 rounding over sums of a
  few hundred terms;
* selection: given the device's float32 keys, the chosen coordinates are
  bit-exact against the oracle's ranking and slot draws;
* the sampled K-SVM solve: alpha against the FP64 oracle replaying the
  realised coordinates (1e-9), the maintained gradient against
  Q alpha - 1 + omega alpha from the oracle (1e-9), the recorded features
  against the oracle state, and the selection of a later outer iteration
  recomputed from the device's own state;
* a trained sampler reaches a lower dual objective than uniform sampling
  after the same number of coordinate updates.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import sampler as SO
from paper_2406_18001_amd import inputs
from tests.helpers import assert_parity, dev, idx_dev, max_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2406_18001_amd import kdcd
    return kdcd


def f32(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def test_initial_weights_bit_exact(K):
    for seed in (0, 1, 2 ** 40 + 7):
        smp = K.Sampler(seed)
        np.testing.assert_array_equal(smp.get_params().cpu().numpy(), SO.init_params(seed))


def test_forward_matches_oracle(K):
    smp = K.Sampler(3)
    p = SO.init_params(3).astype(np.float64)
    rng = np.random.default_rng(0)
    p32 = (p + 0.2 * rng.standard_normal(p.size)).astype(np.float32)
    smp.set_params(f32(p32))
    X = rng.standard_normal((3000, 4)).astype(np.float32)
    out = smp.forward(f32(X)).cpu().numpy()
    ref, _, _ = SO.forward(p32.astype(np.float64), X.astype(np.float64))
    assert_parity(out, ref, 2e-5, "f(x)")


@pytest.mark.parametrize("n", [1, 100, 128, 1000, 4097])
def test_gradient_matches_oracle(K, n):
    smp = K.Sampler(4)
    p32 = SO.init_params(4)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 4)).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    g, loss = smp.grad(f32(X), f32(t))
    L, gref = SO.loss_and_grad(p32.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    assert_parity(g.cpu().numpy(), gref, 1e-4, "gradient")
    assert abs(loss.item() - L) <= 1e-5 * abs(L)


def test_adam_steps_match_oracle(K):
    smp = K.Sampler(5)
    p0 = SO.init_params(5)
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (600, 4)).astype(np.float32)
    t = (np.abs(X[:, 0] - X[:, 1]) + 0.5 * X[:, 3]).astype(np.float32)
    lr = 1e-3
    # one step: the Adam direction is +-lr for every clearly nonzero gradient
    smp.train(f32(X), f32(t), batch=600, epochs=1, lr=lr)
    p1 = smp.get_params().cpu().numpy().astype(np.float64)
    _, g = SO.loss_and_grad(p0.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    ref, _, _ = SO.adam_step(p0.astype(np.float64), g, 0.0, 0.0, 1, lr)
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.max(np.abs(p1 - ref)[big]) <= 1e-3 * lr + 1e-7
    assert np.max(np.abs(p1 - ref)) <= 2 * lr + 1e-7
    # many steps: same loss curve to FP32 accuracy
    smp.set_params(f32(p0))
    losses = smp.train(f32(X), f32(t), batch=64, epochs=25, lr=3e-3).cpu().numpy()
    _, ref_losses = SO.train(p0, X.astype(np.float64), t.astype(np.float64), 64, 25, 3e-3)
    assert losses[-1] < 0.3 * losses[0]
    np.testing.assert_allclose(losses, ref_losses, rtol=0.05)


def test_keys_and_selection_match_oracle(K):
    smp = K.Sampler(6)
    p32 = SO.init_params(6)
    rng = np.random.default_rng(2)
    for m, s, eps, tau, k in [(1024, 1, 0.0, 1.0, 0), (5000, 7, 0.3, 0.5, 3),
                              (70000, 64, 0.1, 0.2, 11), (3000, 1024, 0.0, 2.0, 5),
                              (1000, 1000, 0.5, 1.0, 2), (20000, 512, 1.0, 1.0, 9),
                              (100000, 1024, 0.2, 1.0, 4), (300000, 64, 0.0, 0.7, 1)]:
        X = rng.standard_normal((m, 4)).astype(np.float32)
        keys = smp.keys(f32(X), tau, seed=77, outer=k)
        kk = keys.cpu().numpy()
        scores, _, _ = SO.forward(p32.astype(np.float64), X.astype(np.float64))
        ref = SO.gumbel_keys(scores, tau, k, 77)
        assert np.max(np.abs(kk - ref) / (1.0 + np.abs(ref))) < 2e-5
        S = K.kdcd_sampler_select(keys, s, eps, seed=77, outer=k).cpu().numpy()
        np.testing.assert_array_equal(S, SO.select(kk, s, eps, k, 77))


def test_selection_with_heavy_ties(K):
    rng = np.random.default_rng(3)
    # chunked path (few candidates) and radix path (chunks x s above 8192)
    for m, s in [(5000, 100), (3000, 1024), (50000, 33), (100000, 700), (100000, 1024)]:
        keys = (np.round(rng.standard_normal(m) * 8) / 8).astype(np.float32)
        keys[:7] = keys.max()
        S = K.kdcd_sampler_select(f32(keys), s, 0.0, seed=1, outer=0).cpu().numpy()
        np.testing.assert_array_equal(S, SO.select(keys, s, 0.0, 0, 1))


def test_selection_errors(K):
    # up to 2048 coordinates are ranked by one sort (any number of ties); above
    # that the radix path holds at most 2048 keys tied at the threshold
    S = K.kdcd_sampler_select(f32(np.zeros(2000)), 10, 0.0, seed=0, outer=0).cpu().numpy()
    np.testing.assert_array_equal(S, np.arange(10))
    for m in (5000, 100000):
        with pytest.raises(K.KdcdError) as e:
            K.kdcd_sampler_select(f32(np.zeros(m)), 10, 0.0, seed=0, outer=0)
        assert e.value.status == -2
    bad = np.zeros(100, dtype=np.float32)
    bad[3] = np.nan
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_sampler_select(f32(bad), 10, 0.0, seed=0, outer=0)
    assert e.value.status == -6
    with pytest.raises(K.KdcdError) as e:
        K.kdcd_sampler_select(f32(np.ones(10)), 11, 0.0, seed=0, outer=0)
    assert e.value.status == -1


def oracle_grad(A, y, kern, C, alpha, loss):
    om = 1.0 / (2.0 * C) if loss == 2 else 0.0
    Kb = O.kernel_matvec(A, kern, y * alpha)
    return y * Kb - 1.0 + om * alpha


@pytest.mark.parametrize("loss", [1, 2])
@pytest.mark.parametrize("warm", [False, True])
def test_uniform_sampled_solve(K, loss, warm):
    d = inputs.dense_ksvm_c5(m=1500, n=48, seed=21)
    A, y = d["A"], d["y"]
    m, C, s, H = 1500, 2.0, 16, 403
    sig = 2.0 / 48
    kern = O.Kernel(O.RBF, sigma=sig)
    a0 = np.random.default_rng(0).uniform(0, C, m) * (np.arange(m) % 3 == 0) if warm else np.zeros(m)
    alpha = dev(a0)
    g = torch.zeros(m, dtype=torch.float64, device="cuda")
    feats = torch.zeros(4 * H, dtype=torch.float32, device="cuda")
    trace = torch.zeros(H, dtype=torch.float64, device="cuda")
    idx, _ = K.kdcd_ksvm_solve_sampled(dev(A), dev(y), (2, sig, 0.0, 1), C, s, H, alpha,
                                       seed=5, features_out=feats, grad_out=g, loss=loss,
                                       trace=trace)
    idx = idx.cpu().numpy()
    n_outer = -(-H // s)
    ref_idx = np.concatenate([SO.select(np.zeros(m, np.float32), min(s, H - k * s), 1.0, k, 5)
                              for k in range(n_outer)])
    np.testing.assert_array_equal(idx, ref_idx)
    a_ref, th_ref = O.dcd_ksvm(A, y, kern, C, H, idx, alpha0=a0, loss=loss, s=s)
    assert_parity(alpha.cpu().numpy(), a_ref, 1e-9, "alpha")
    assert_parity(trace.cpu().numpy(), th_ref, 1e-9, "theta")
    assert_parity(g.cpu().numpy(), oracle_grad(A, y, kern, C, a_ref, loss), 1e-9, "gradient")
    # features of outer iteration 0 and 7 against the oracle state
    F = feats.cpu().numpy().reshape(H, 4)
    for k in (0, 7):
        ak = a0 if k == 0 else O.dcd_ksvm(A, y, kern, C, k * s, idx, alpha0=a0, loss=loss, s=s)[0]
        gk = oracle_grad(A, y, kern, C, ak, loss)
        S = idx[k * s:(k + 1) * s]
        ref = SO.ksvm_features(ak[S], gk[S], np.ones(s), y[S], C)
        np.testing.assert_allclose(F[k * s:(k + 1) * s], ref, rtol=1e-6, atol=1e-6)


def test_learned_sampled_solve_replays_and_selects_exactly(K):
    d = inputs.dense_ksvm_c5(m=2000, n=32, seed=22)
    A, y = d["A"], d["y"]
    m, C, s = 2000, 10.0, 32
    sig = 2.0 / 32
    smp = K.Sampler(9)
    eps, tau, seed = 0.2, 0.5, 13
    kk = 5
    H = (kk + 1) * s + 7
    runs = {}
    for HH in (kk * s, H):
        alpha = torch.zeros(m, dtype=torch.float64, device="cuda")
        g = torch.zeros(m, dtype=torch.float64, device="cuda")
        idx, _ = K.kdcd_ksvm_solve_sampled(dev(A), dev(y), (2, sig, 0.0, 1), C, s, HH, alpha,
                                           model=smp, epsilon=eps, tau=tau, seed=seed, grad_out=g)
        runs[HH] = (idx.cpu().numpy(), alpha.cpu().numpy(), g.cpu().numpy())
    idx, a_gpu, _ = runs[H]
    np.testing.assert_array_equal(idx[:kk * s], runs[kk * s][0])
    a_ref, _ = O.dcd_ksvm(A, y, O.Kernel(O.RBF, sigma=sig), C, H, idx, s=s)
    assert_parity(a_gpu, a_ref, 1e-9, "alpha")
    # outer iteration kk from the device's own state after kk iterations
    _, ak, gk = runs[kk * s]
    X = SO.ksvm_features(ak, gk, np.ones(m), y, C)       # the device's float32 features
    keys = smp.keys(f32(X), tau, seed, kk).cpu().numpy()
    np.testing.assert_array_equal(idx[kk * s:(kk + 1) * s], SO.select(keys, s, eps, kk, seed))
    # the first outer iteration from alpha = 0: features are exact in float32
    X0 = SO.ksvm_features(np.zeros(m), -np.ones(m), np.ones(m), y, C)
    keys0 = smp.keys(f32(X0), tau, seed, 0).cpu().numpy()
    np.testing.assert_array_equal(idx[:s], SO.select(keys0, s, eps, 0, seed))


def test_trained_sampler_beats_uniform(K):
    """Train on the features and realised |theta| of a uniform run on one
    instance of the C5 recipe (reduced size, sigma = 2/n), then run the learned
    draw on another instance for as many updates as the uniform draw: its dual
    objective is lower."""
    m, n, C, s = 4000, 64, 10.0, 64
    d = inputs.dense_ksvm_c5(m=m, n=n, seed=23)
    A, y = dev(d["A"]), dev(d["y"])
    kern = (2, 2.0 / n, 0.0, 1)
    mt, nt = 3000, 128                                  # the training instance
    dt = inputs.dense_ksvm_c5(m=mt, n=nt, seed=24)
    H = 3 * mt
    alpha = torch.zeros(mt, dtype=torch.float64, device="cuda")
    feats = torch.zeros(4 * H, dtype=torch.float32, device="cuda")
    trace = torch.zeros(H, dtype=torch.float64, device="cuda")
    K.kdcd_ksvm_solve_sampled(dev(dt["A"]), dev(dt["y"]), (2, 2.0 / nt, 0.0, 1), C, s, H, alpha,
                              seed=100, features_out=feats, trace=trace)
    x = feats.view(H, 4)
    t = torch.log(1e-7 + trace.abs() / C).float()
    smp = K.Sampler(1)
    losses = smp.train(x.contiguous(), t.contiguous(), batch=512, epochs=15, lr=3e-3)
    assert losses[-1].item() < 0.7 * losses[0].item()
    results = {}
    for name, model, eps, tau, pool in (("uniform", None, 1.0, 1.0, 0),
                                        ("learned", smp, 0.3, 1.0, 0),
                                        ("pool", smp, 0.5, 1.0, 256)):
        a = torch.zeros(m, dtype=torch.float64, device="cuda")
        K.kdcd_ksvm_solve_sampled(A, y, kern, C, s, m, a, model=model, epsilon=eps, tau=tau,
                                  pool=pool, seed=200)
        results[name] = K.kdcd_ksvm_eval(A, y, kern, C, a)
    print({k: (v["dual"], v["gap"]) for k, v in results.items()})
    for name in ("learned", "pool"):
        assert results[name]["dual"] < results["uniform"]["dual"]
        assert results[name]["gap"] < 0.7 * results["uniform"]["gap"]


@pytest.mark.parametrize("pool,s", [(256, 32), (64, 64), (2048, 100)])
def test_pool_sampled_solve_replays_and_selects_exactly(K, pool, s):
    d = inputs.dense_ksvm_c5(m=3000, n=32, seed=24)
    A, y = d["A"], d["y"]
    m, C = 3000, 5.0
    sig = 2.0 / 32
    smp = K.Sampler(10)
    eps, tau, seed = 0.25, 0.7, 17
    kk = 4
    H = (kk + 1) * s + 3
    runs = {}
    for HH in (kk * s, H):
        alpha = torch.zeros(m, dtype=torch.float64, device="cuda")
        g = torch.zeros(m, dtype=torch.float64, device="cuda")
        idx, _ = K.kdcd_ksvm_solve_sampled(dev(A), dev(y), (2, sig, 0.0, 1), C, s, HH, alpha,
                                           model=smp, epsilon=eps, tau=tau, seed=seed, pool=pool,
                                           grad_out=g)
        runs[HH] = (idx.cpu().numpy(), alpha.cpu().numpy(), g.cpu().numpy())
    idx, a_gpu, g_gpu = runs[H]
    np.testing.assert_array_equal(idx[:kk * s], runs[kk * s][0])
    a_ref, _ = O.dcd_ksvm(A, y, O.Kernel(O.RBF, sigma=sig), C, H, idx, s=s)
    assert_parity(a_gpu, a_ref, 1e-9, "alpha")
    assert_parity(g_gpu, oracle_grad(A, y, O.Kernel(O.RBF, sigma=sig), C, a_ref, 1), 1e-9, "g")
    for k, (ak, gk) in ((0, (np.zeros(m), -np.ones(m))), (kk, runs[kk * s][1:])):
        X = SO.ksvm_features(ak, gk, np.ones(m), y, C)
        keys = smp.keys(f32(X), tau, seed, k).cpu().numpy()      # noise of coordinate i
        cand = SO.pool_candidates(m, pool, k, seed)
        ref = SO.select_pool(keys[cand], cand, m, s, eps, k, seed)
        np.testing.assert_array_equal(idx[k * s:(k + 1) * s], ref)


def test_pool_argument_errors(K):
    m = 500
    A = torch.randn(m, 8, dtype=torch.float64, device="cuda")
    y = torch.ones(m, dtype=torch.float64, device="cuda")
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    smp = K.Sampler(0)
    for pool, s in ((16, 32), (4096, 32)):
        with pytest.raises(K.KdcdError) as e:
            K.kdcd_ksvm_solve_sampled(A, y, (2, 1.0, 0.0, 1), 1.0, s, 64, a, model=smp, pool=pool)
        assert e.value.status == -1

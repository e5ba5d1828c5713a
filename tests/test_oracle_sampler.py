"""Pins of the learned-sampler oracle (oracle/sampler.py) against values and
properties fixed outside it: Philox's published known-answer vectors, the
Gumbel-max property (the argmax of score/tau + Gumbel noise is distributed as
softmax(score/tau)), brute-force ranking, hand-evaluated networks, central
finite differences of the loss, and Adam's closed forms under constant
gradients."""
import json
import math
import os

import numpy as np
import pytest

from oracle import sampler as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.json")


def test_philox_known_answers():
    cases = json.load(open(GOLD))["cases"]
    for c in cases:
        ctr = [int(x, 16) for x in c["ctr"]]
        key = [int(x, 16) for x in c["key"]]
        out = S.philox4x32_10([ctr], key)[0]
        assert [int(v) for v in out] == [int(x, 16) for x in c["out"]]


def test_philox_counters_are_independent_streams():
    x = S.philox4x32_10([[i, 7, 0, 0] for i in range(20000)], S.seed_key(3))
    u = S.to_unit(x[:, 0])
    assert np.all((u > 0) & (u < 1))
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1 / 12) < 0.005
    assert len(np.unique(x[:, 0])) == 20000
    y = S.philox4x32_10([[i, 8, 0, 0] for i in range(20000)], S.seed_key(3))
    assert np.corrcoef(S.to_unit(y[:, 0]), u)[0, 1] < 0.03


def test_gumbel_max_samples_softmax():
    scores = np.array([0.0, 1.0, -0.5, 2.0, 0.3], dtype=np.float32)
    tau = 0.7
    trials = 20000
    counts = np.zeros(5)
    for k in range(trials):
        counts[np.argmax(S.gumbel_keys(scores, tau, k, seed=11))] += 1
    p = np.exp(scores / tau)
    p /= p.sum()
    assert np.max(np.abs(counts / trials - p)) < 0.012, (counts / trials, p)


def test_select_top_keys_ties_and_uniform_slots():
    rng = np.random.default_rng(0)
    keys = rng.standard_normal(300).astype(np.float32)
    keys[[10, 20, 30]] = 5.0                     # a tie at the top: smaller index first
    top = S.select(keys, 12, 0.0, k=0, seed=1)
    ranked = sorted(range(300), key=lambda i: (-float(keys[i]), i))
    assert list(top) == ranked[:12]
    assert list(top[:3]) == [10, 20, 30]
    uni = np.concatenate([S.select(keys, 64, 1.0, k=k, seed=2) for k in range(200)])
    assert uni.min() >= 0 and uni.max() < 300
    hist = np.bincount(uni, minlength=300)
    assert hist.min() > 10 and hist.max() < 80      # 42.7 expected per coordinate
    mix = S.select(keys, 64, 0.25, k=3, seed=4)
    ctr = [[j, 3, S.TAG_SLOT, 0] for j in range(64)]
    x = S.philox4x32_10(ctr, S.seed_key(4))
    is_uni = S.to_unit(x[:, 0]) < 0.25
    assert 5 <= is_uni.sum() <= 30
    assert list(mix[~is_uni]) == ranked[:int((~is_uni).sum())]


def test_forward_of_hand_built_network():
    p = np.zeros(S.NPARAMS)
    w = S.unpack(np.arange(S.NPARAMS, dtype=np.float64))   # offsets of each block
    o_W1, o_W2, o_w3, o_b3 = int(w["W1"][0, 0]), int(w["W2"][0, 0]), int(w["w3"][0]), int(w["b3"])
    p[o_W1 + 0] = 1.0          # h1_0 = tanh(x_0)
    p[o_W1 + 4 + 3] = -2.0     # h1_1 = tanh(-2 x_3)
    p[o_W2 + 0] = 1.0          # h2_0 = tanh(h1_0)
    p[o_W2 + 64 + 1] = 0.5     # h2_1 = tanh(0.5 h1_1)
    p[o_w3 + 0] = 2.0
    p[o_w3 + 1] = -1.0
    p[o_b3] = 0.25
    X = np.array([[0.3, 9.0, -4.0, 1.0], [-1.2, 0.0, 0.0, -0.5]])
    f, _, _ = S.forward(p, X)
    for r in range(2):
        x0, x3 = X[r, 0], X[r, 3]
        ref = 2.0 * math.tanh(math.tanh(x0)) - math.tanh(0.5 * math.tanh(-2.0 * x3)) + 0.25
        assert abs(f[r] - ref) < 1e-15


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    p = S.init_params(9).astype(np.float64) + 0.05 * rng.standard_normal(S.NPARAMS)
    X = rng.standard_normal((37, 4))
    t = rng.standard_normal(37)
    L, g = S.loss_and_grad(p, X, t)
    h = 1e-6
    picks = np.concatenate([rng.choice(S.NPARAMS, 200, replace=False), [S.NPARAMS - 1, 0, 300]])
    for q in picks:
        e = np.zeros(S.NPARAMS)
        e[q] = h
        fd = (S.loss_and_grad(p + e, X, t)[0] - S.loss_and_grad(p - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-7 * max(1.0, abs(g[q])) + 1e-9, (q, fd, g[q])
    assert abs(L - 0.5 * np.mean((S.forward(p, X)[0] - t) ** 2)) < 1e-15


def test_gradient_of_constant_network():
    p = np.zeros(S.NPARAMS)
    p[-1] = 0.75                                   # f(x) = b3 for every x
    X = np.random.default_rng(1).standard_normal((10, 4))
    t = np.linspace(-1, 1, 10)
    L, g = S.loss_and_grad(p, X, t)
    assert abs(L - 0.5 * np.mean((0.75 - t) ** 2)) < 1e-15
    assert abs(g[-1] - np.mean(0.75 - t)) < 1e-15
    assert np.all(g[:-1] == 0.0)


def test_adam_closed_forms():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 4.0])
    m = v = np.zeros(3)
    for step in range(1, 6):                       # constant gradient: bias correction is exact
        p_new, m, v = S.adam_step(p, g, m, v, step, lr=0.01)
        np.testing.assert_allclose(p_new - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)
        p = p_new
    p2, _, _ = S.adam_step(p, np.zeros(3), np.zeros(3), np.zeros(3), 1, lr=0.1)
    assert np.all(p2 == p)


def test_init_is_glorot_and_seeded():
    a = S.init_params(1)
    b = S.init_params(1)
    c = S.init_params(2)
    assert a.dtype == np.float32 and np.array_equal(a, b) and not np.array_equal(a, c)
    w = S.unpack(a.astype(np.float64))
    for name, bound in (("W1", math.sqrt(6 / 68)), ("W2", math.sqrt(6 / 128)), ("w3", math.sqrt(6 / 65))):
        x = np.abs(w[name])
        assert x.max() <= bound * (1 + 1e-7) and x.max() > 0.8 * bound
    assert np.all(w["b1"] == 0) and np.all(w["b2"] == 0) and w["b3"] == 0


def test_train_reduces_loss_and_single_batch_is_one_adam_step():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (400, 4))
    t = np.abs(X[:, 0] - X[:, 1]) + 0.5 * X[:, 3]
    p0 = S.init_params(3)
    p, losses = S.train(p0, X, t, batch=64, epochs=30, lr=3e-3)
    assert losses[-1] < 0.25 * losses[0]
    p1, _ = S.train(p0, X, t, batch=400, epochs=1, lr=1e-3)
    _, g = S.loss_and_grad(p0, X, t)
    ref, _, _ = S.adam_step(p0.astype(np.float64), g, 0, 0, 1, 1e-3)
    np.testing.assert_allclose(p1, ref, rtol=0, atol=1e-15)


def test_slog_feature_values():
    g = np.array([0.0, 1.0, -1.0, 2.0 ** -20, -(2.0 ** -21), 3.0 * 2 ** -20, 0.75, 1e6, -5e-7])
    x = S.slog(g)
    # |g| 2^20 = v: v < 1 kept, else 1 + log2 at powers of two, linear between them
    expect = np.array([0.0, 21.0, -21.0, 1.0, -0.5, 1 + 1 + 0.5, 1 + 19 + 0.5,
                       1 + 39 + (1e6 * 2 ** 20 / 2 ** 39 - 1), -(5e-7 * 2 ** 20)]) / 8
    np.testing.assert_allclose(x, expect, rtol=1e-6, atol=0)
    gg = np.sort(np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).uniform(-8, 2, 10000))
    xs = S.slog(gg)
    assert np.all(np.diff(xs) >= 0)                          # monotone
    assert np.all(np.sign(xs) == np.sign(gg))


def test_ksvm_features_hand_rows():
    """Feature map (alpha_i / C, slog g_i, K_ii, y_i) on rows worked out by hand:
    a swapped column, alpha * C instead of alpha / C, or a missing 1/8 fails."""
    C = 10.0
    alpha = [2.5, 0.0, 10.0, 5.0]
    g = [2.0 ** -20, 0.5 * 2.0 ** -20, 2.0 ** -10, -3.0 * 2.0 ** -20]
    kdiag = [1.0, 8.0, 1.0, 0.25]
    y = [1.0, 1.0, -1.0, -1.0]
    # slog: v = |g| 2^20; v = 1 -> 1; v = 0.5 -> 0.5; v = 2^10 = 0.5 * 2^11 -> 1 + 10 + 0 = 11;
    # v = 3 = 0.75 * 2^2 -> 1 + 1 + 0.5 = 2.5; then sign(g) and a factor 1/8
    expect = np.array([[0.25, 0.125, 1.0, 1.0],
                       [0.0, 0.0625, 8.0, 1.0],
                       [1.0, 1.375, 1.0, -1.0],
                       [0.5, -0.3125, 0.25, -1.0]], dtype=np.float32)
    x = S.ksvm_features(alpha, g, kdiag, y, C)
    assert x.dtype == np.float32 and x.shape == (4, 4)
    np.testing.assert_array_equal(x, expect)


def test_pool_candidates_and_pool_selection():
    c = np.concatenate([S.pool_candidates(50, 512, k, seed=3) for k in range(100)])
    assert c.min() >= 0 and c.max() < 50
    h = np.bincount(c, minlength=50)
    assert h.min() > 850 and h.max() < 1200          # 1024 expected per coordinate
    cand = S.pool_candidates(1000, 64, 7, seed=2)
    keys = np.random.default_rng(0).standard_normal(64).astype(np.float32)
    out = S.select_pool(keys, cand, 1000, 16, 0.0, 7, 2)
    ranked = sorted(range(64), key=lambda j: (-float(keys[j]), j))
    assert list(out) == [int(cand[j]) for j in ranked[:16]]

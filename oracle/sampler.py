"""Plain FP64 reference of the learned coordinate sampler (numpy).

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's baseline
leg, never by the product path; it shares no code with the HIP library.

The paper draws the coordinates of Algorithms 1-4 uniformly at random (or
cyclically); the index sequence is an input of every step.  The learned
sampler replaces that draw: a small MLP scores every coordinate from its
current state, and s coordinates are drawn by Gumbel-top-k over the scores,
with a share epsilon of the slots drawn uniformly.  Everything the draw
needs is defined here:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC 2011): ten rounds of two 32x32->64 multiplies with the
  Weyl-sequence key schedule; it is the one counter-based generator both the
  oracle and the device code implement from its definition.
* Counter layout: coordinate noise of outer iteration k uses counter
  (i, k, 0, 0); slot j of outer iteration k uses (j, k, 1, 0); parameter p of
  the initial weights uses (p, 0, 2, 0).  The key is (seed mod 2^32,
  seed >> 32).  A 32-bit output x maps to u = (x + 0.5) / 2^32 in (0, 1).
* Gumbel noise G = -log(-log u); the key of coordinate i is the float32
  rounding of score_i / tau + G_i (computed in FP64).  Keys are ranked by
  value, ties by the smaller index.
* Slot j is uniform when u(x0) < epsilon, and then takes coordinate
  floor(x1 * m / 2^32); otherwise it takes the next best key.
* Pool variant: only P candidates floor(x0 * m / 2^32), counters (j, k, 3, 0),
  are scored; each keeps the noise of its coordinate and they are ranked by
  key, ties by pool position.
* MLP 4 -> 64 -> 64 -> 1 with tanh hidden units; flat parameter layout
  W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3 (4545 floats);
  Glorot-uniform weights (bound sqrt(6/(fan_in+fan_out))), zero biases.
* Loss 1/(2n) sum (f(x_i) - t_i)^2; Adam (Kingma and Ba, ICLR 2015,
  Algorithm 1) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
* K-SVM features of coordinate i: (alpha_i / C, slog(g_i), K_ii, y_i) with the
  full dual gradient g = Q alpha - 1 + omega alpha, Q = diag(y) K diag(y), and
  slog the signed pseudo-logarithm below (float32 throughout: alpha_i / C is
  the float32 rounding of alpha_i * (1/C)).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = 0xFFFFFFFF

NIN, NH = 4, 64
SIZES = [("W1", NH * NIN), ("b1", NH), ("W2", NH * NH), ("b2", NH), ("w3", NH), ("b3", 1)]
NPARAMS = sum(n for _, n in SIZES)

TAG_NOISE, TAG_SLOT, TAG_INIT, TAG_POOL = 0, 1, 2, 3


# ------------------------------------------------------------------ Philox

def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32 with 10 rounds.  ctr: (N, 4) integers < 2^32; key: 2 ints.
    Returns (N, 4) uint64 holding 32-bit outputs."""
    c = np.array(ctr, dtype=np.uint64).reshape(-1, 4) & np.uint64(MASK32)
    c0, c1, c2, c3 = (c[:, j].copy() for j in range(4))
    k0, k1 = int(key[0]) & MASK32, int(key[1]) & MASK32
    m0, m1, msk = np.uint64(M0), np.uint64(M1), np.uint64(MASK32)
    for _ in range(10):
        p0 = c0 * m0                      # < 2^64: exact in uint64
        p1 = c2 * m1
        hi0, lo0 = p0 >> np.uint64(32), p0 & msk
        hi1, lo1 = p1 >> np.uint64(32), p1 & msk
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + W0) & MASK32
        k1 = (k1 + W1) & MASK32
    return np.stack([c0, c1, c2, c3], axis=1)


def seed_key(seed: int):
    return (seed & MASK32, (seed >> 32) & MASK32)


def to_unit(x) -> np.ndarray:
    """32-bit integer -> u in (0, 1), exactly representable in FP64."""
    return (np.asarray(x, dtype=np.float64) + 0.5) / 4294967296.0


def gumbel(u) -> np.ndarray:
    return -np.log(-np.log(u))


def coordinate_noise(m: int, k: int, seed: int) -> np.ndarray:
    """Gumbel noise of coordinates 0..m-1 in outer iteration k."""
    i = np.arange(m, dtype=np.uint64)
    ctr = np.stack([i, np.full(m, k), np.full(m, TAG_NOISE), np.zeros(m)], axis=1)
    return gumbel(to_unit(philox4x32_10(ctr, seed_key(seed))[:, 0]))


def gumbel_keys(scores, tau: float, k: int, seed: int) -> np.ndarray:
    """float32 key of every coordinate: rounding of score/tau + Gumbel noise."""
    s = np.asarray(scores, dtype=np.float32).astype(np.float64)
    return (s / tau + coordinate_noise(s.shape[0], k, seed)).astype(np.float32)


def select(keys, s: int, epsilon: float, k: int, seed: int) -> np.ndarray:
    """The s coordinates of outer iteration k from float32 keys."""
    keys = np.asarray(keys, dtype=np.float32)
    m = keys.shape[0]
    order = np.lexsort((np.arange(m), -keys.astype(np.float64)))   # key desc, index asc
    j = np.arange(s, dtype=np.uint64)
    ctr = np.stack([j, np.full(s, k), np.full(s, TAG_SLOT), np.zeros(s)], axis=1)
    x = philox4x32_10(ctr, seed_key(seed))
    out = np.empty(s, dtype=np.int32)
    nxt = 0
    for t in range(s):
        if to_unit(x[t, 0]) < epsilon:
            out[t] = int((int(x[t, 1]) * m) >> 32)
        else:
            out[t] = order[nxt]
            nxt += 1
    return out


def pool_candidates(m: int, P: int, k: int, seed: int) -> np.ndarray:
    """The P candidates of outer iteration k: floor(x0 m / 2^32) from counters
    (j, k, 3, 0); drawn with replacement."""
    j = np.arange(P, dtype=np.uint64)
    ctr = np.stack([j, np.full(P, k), np.full(P, TAG_POOL), np.zeros(P)], axis=1)
    x = philox4x32_10(ctr, seed_key(seed))[:, 0]
    return ((x * np.uint64(m)) >> np.uint64(32)).astype(np.int32)


def select_pool(keys_pool, cand, m: int, s: int, epsilon: float, k: int, seed: int) -> np.ndarray:
    """Slots of outer iteration k when only the pool `cand` is scored: the pool
    is ranked by key (ties by pool position); uniform slots as in select."""
    keys_pool = np.asarray(keys_pool, dtype=np.float32)
    P = keys_pool.shape[0]
    order = np.lexsort((np.arange(P), -keys_pool.astype(np.float64)))
    j = np.arange(s, dtype=np.uint64)
    ctr = np.stack([j, np.full(s, k), np.full(s, TAG_SLOT), np.zeros(s)], axis=1)
    x = philox4x32_10(ctr, seed_key(seed))
    out = np.empty(s, dtype=np.int32)
    nxt = 0
    for t in range(s):
        if to_unit(x[t, 0]) < epsilon:
            out[t] = int((int(x[t, 1]) * m) >> 32)
        else:
            out[t] = cand[order[nxt]]
            nxt += 1
    return out


# --------------------------------------------------------------------- MLP

def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, n in SIZES:
        out[name] = p[o:o + n]
        o += n
    out["W1"] = out["W1"].reshape(NH, NIN)
    out["W2"] = out["W2"].reshape(NH, NH)
    out["b3"] = out["b3"][0]
    return out


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights from Philox, zero biases, rounded to float32."""
    fan = {"W1": (NIN, NH), "W2": (NH, NH), "w3": (NH, 1)}
    idx = np.arange(NPARAMS, dtype=np.uint64)
    ctr = np.stack([idx, np.zeros(NPARAMS), np.full(NPARAMS, TAG_INIT), np.zeros(NPARAMS)], axis=1)
    u = to_unit(philox4x32_10(ctr, seed_key(seed))[:, 0])
    p = np.zeros(NPARAMS)
    o = 0
    for name, n in SIZES:
        if name in fan:
            a = np.sqrt(6.0 / (fan[name][0] + fan[name][1]))
            p[o:o + n] = a * (2.0 * u[o:o + n] - 1.0)
        o += n
    return p.astype(np.float32)


def forward(p, X):
    """Scores f(x) of the rows of X (n x 4), plus the hidden activations."""
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ w["W1"].T + w["b1"])
    h2 = np.tanh(h1 @ w["W2"].T + w["b2"])
    return h2 @ w["w3"] + w["b3"], h1, h2


def loss_and_grad(p, X, t):
    """L = 1/(2n) sum (f(x_i) - t_i)^2 and dL/dp by backpropagation."""
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = X.shape[0]
    f, h1, h2 = forward(p, X)
    e = f - t
    loss = 0.5 * np.sum(e * e) / n
    d_out = e / n                              # dL/df
    g_w3 = h2.T @ d_out
    g_b3 = np.sum(d_out)
    dz2 = np.outer(d_out, w["w3"]) * (1.0 - h2 * h2)
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ w["W2"]) * (1.0 - h1 * h1)
    g_W1 = dz1.T @ X
    g_b1 = dz1.sum(axis=0)
    grad = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
    return loss, grad


def adam_step(p, g, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def train(p, X, t, batch: int, epochs: int, lr: float):
    """Minibatches in data order (the last one may be short), one Adam step
    each.  Returns (params, loss of every epoch before its updates' end: the
    mean of the minibatch losses weighted by their sizes)."""
    p = np.asarray(p, dtype=np.float64).copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    n = X.shape[0]
    step = 0
    losses = []
    for _ in range(epochs):
        tot = 0.0
        for o in range(0, n, batch):
            L, g = loss_and_grad(p, X[o:o + batch], t[o:o + batch])
            tot += L * min(batch, n - o)
            step += 1
            p, m, v = adam_step(p, g, m, v, step, lr)
        losses.append(tot / n)
    return p, np.array(losses)


# ------------------------------------------------------------ K-SVM state

def slog(g) -> np.ndarray:
    """Signed pseudo-logarithm of g in float32: v = float32(|g| 2^20); for
    v < 1 the value is v, otherwise 1 + (e - 1) + (2 mant - 1) with
    v = mant 2^e, mant in [0.5, 1) (a piecewise-linear log2 that is exact
    at powers of two); the sign of g is restored and the result divided by 8."""
    g = np.asarray(g, dtype=np.float64)
    v = (np.abs(g) * 1048576.0).astype(np.float32)
    mant, e = np.frexp(v)
    frac = (np.float32(2.0) * mant.astype(np.float32)) - np.float32(1.0)
    big = np.float32(1.0) + ((e - 1).astype(np.float32) + frac)
    L = np.where(v < np.float32(1.0), v, big).astype(np.float32)
    return (np.sign(g).astype(np.float32) * L * np.float32(0.125)).astype(np.float32)


def ksvm_features(alpha, g, kdiag, y, C) -> np.ndarray:
    """float32 features (n x 4) of the coordinates given by the arrays."""
    a = (np.asarray(alpha, dtype=np.float64) * (1.0 / C)).astype(np.float32)
    return np.stack([a, slog(g), np.asarray(kdiag, dtype=np.float32),
                     np.asarray(y, dtype=np.float32)], axis=1)

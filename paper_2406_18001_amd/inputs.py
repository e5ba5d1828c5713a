"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the HIP path, the CPU oracle and the benchmark.  It
holds only random draws and data shaping (labels, CSR structure, index
sequences); none of the method's arithmetic (kernel maps, coordinate updates,
objectives) lives here.

The paper's datasets (LIBSVM sets in its Table 2 and Table 3) are not
available; the generators below stand in for them with the shapes, value
distributions and structure of five workloads:

  C1  dense K-SVM, 2000 x 64, N(0,1) entries, labels from a random hyperplane
  C2  dense K-RR, 20000 x 512, rows N(0,I)/sqrt(n), targets sin(A u) + noise
  C3  sparse K-SVM, CSR 100000 x 50000, 50 distinct columns per row drawn with
      Zipf(1.1) column frequencies, U(0,1) values, rows L2-normalised
  C4  dense mixed-precision / batched, 200000 x 1024, N(0,1)/sqrt(n)
  C5  dense K-SVM for the learned sampler, 500000 x 256, N(0,1), labels from a
      random two-layer tanh network

Every generator takes ``m``/``n`` overrides so that tests can build the same
recipe at sizes the oracle finishes in seconds.  Data seeds are 100 + config
number; coordinate index sequences use seed 0.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "sign_pm1", "flip_labels", "ksvm_indices", "krr_indices",
    "dense_ksvm_c1", "dense_krr_c2", "csr_ksvm_c3", "dense_c4", "dense_ksvm_c5",
    "csr_to_dense", "KRR_SWEEP_C4",
]

# (lambda, sigma) grid of the batched K-RR sweep on C4.
KRR_SWEEP_C4 = [(lam, sig) for lam in (1e-4, 1e-3) for sig in (0.5, 1.0, 2.0, 4.0)]


def sign_pm1(z: np.ndarray) -> np.ndarray:
    """sign with sign(0) := +1, as float64 labels in {-1, +1}."""
    return np.where(z >= 0.0, 1.0, -1.0)


def flip_labels(y: np.ndarray, frac: float, rng: np.random.Generator) -> np.ndarray:
    """Flip exactly round(frac * m) distinct labels."""
    y = y.copy()
    k = int(round(frac * y.shape[0]))
    if k > 0:
        pos = rng.choice(y.shape[0], size=k, replace=False)
        y[pos] = -y[pos]
    return y


def ksvm_indices(m: int, H: int, seed: int = 0) -> np.ndarray:
    """H coordinates drawn uniformly with replacement (duplicates are legal)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, m, size=H, dtype=np.int64).astype(np.int32)


def krr_indices(m: int, b: int, H: int, seed: int = 0) -> np.ndarray:
    """H blocks of b coordinates; each block is drawn without replacement
    (Floyd's algorithm, vectorised over blocks), blocks are independent so two
    blocks may share coordinates.  Returned flat, length H*b, block-major."""
    if b > m:
        raise ValueError("block size b must not exceed m")
    rng = np.random.default_rng(seed)
    out = np.empty((H, b), dtype=np.int64)
    for pos, jj in enumerate(range(m - b, m)):
        t = rng.integers(0, jj + 1, size=H, dtype=np.int64)
        if pos:
            dup = (out[:, :pos] == t[:, None]).any(axis=1)
            t = np.where(dup, jj, t)
        out[:, pos] = t
    return out.reshape(-1).astype(np.int32)


def landmarks(m: int, r: int, seed: int = 0) -> np.ndarray:
    """r distinct rows of [0, m), uniformly without replacement (Nystrom
    landmarks), in draw order."""
    if r > m:
        raise ValueError("cannot draw more landmarks than rows")
    rng = np.random.default_rng(seed)
    return rng.choice(m, size=r, replace=False).astype(np.int32)


def dense_ksvm_c1(m: int = 2000, n: int = 64, flip: float = 0.05, seed: int = 101) -> dict:
    """C1: A ~ N(0,1); y = sign(A w), w ~ N(0, I); `flip` of the labels flipped."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    w = rng.standard_normal(n)
    y = flip_labels(sign_pm1(A @ w), flip, rng)
    return {"A": A, "y": y}


def dense_krr_c2(m: int = 20000, n: int = 512, seed: int = 102) -> dict:
    """C2: rows N(0, I)/sqrt(n); y = sin(A u) + 0.01 N(0,1), u ~ N(0, I)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    u = rng.standard_normal(n)
    y = np.sin(A @ u) + 0.01 * rng.standard_normal(m)
    return {"A": A, "y": y}


def _zipf_cdf(n: int, a: float) -> np.ndarray:
    p = np.arange(1, n + 1, dtype=np.float64) ** (-a)
    c = np.cumsum(p)
    return c / c[-1]


def csr_ksvm_c3(m: int = 100000, n: int = 50000, nnz_per_row: int = 50,
                zipf_a: float = 1.1, flip: float = 0.05, seed: int = 103) -> dict:
    """C3: CSR with exactly `nnz_per_row` distinct columns per row.

    Column ranks follow a Zipf(zipf_a) law truncated to [1, n] and are mapped
    to column ids through a seeded random permutation.  Values are U(0,1) and
    every row is L2-normalised.  Labels: y = sign(A w) with w ~ N(0,1) on a
    random 10% of the columns (zero elsewhere), then `flip` of them flipped.
    Columns are sorted within each row; row_ptr is int64, col_idx int32.
    """
    if nnz_per_row > n:
        raise ValueError("nnz_per_row must not exceed n")
    rng = np.random.default_rng(seed)
    cdf = _zipf_cdf(n, zipf_a)
    perm = rng.permutation(n)
    cols = np.empty((m, nnz_per_row), dtype=np.int64)
    draw = max(2 * nnz_per_row + 20, 64)
    todo = np.arange(m)
    while todo.size:
        u = rng.random((todo.size, draw))
        ranks = np.minimum(np.searchsorted(cdf, u, side="right"), n - 1)
        # first occurrences, in draw order
        order = np.argsort(ranks, axis=1, kind="stable")
        srt = np.take_along_axis(ranks, order, axis=1)
        first_sorted = np.ones_like(srt, dtype=bool)
        first_sorted[:, 1:] = srt[:, 1:] != srt[:, :-1]
        first = np.zeros_like(first_sorted)
        np.put_along_axis(first, order, first_sorted, axis=1)
        cnt = first.sum(axis=1)
        ok = cnt >= nnz_per_row
        rows_ok = todo[ok]
        if rows_ok.size:
            f = first[ok]
            r = ranks[ok]
            # position of each first occurrence; keep the first nnz_per_row
            csum = np.cumsum(f, axis=1)
            keep = f & (csum <= nnz_per_row)
            cols[rows_ok] = r[keep].reshape(rows_ok.size, nnz_per_row)
        todo = todo[~ok]
    cols = np.sort(perm[cols], axis=1)
    vals = rng.random((m, nnz_per_row))
    vals /= np.sqrt((vals * vals).sum(axis=1, keepdims=True))
    w = np.zeros(n)
    support = rng.choice(n, size=max(1, n // 10), replace=False)
    w[support] = rng.standard_normal(support.size)
    margin = (vals * w[cols]).sum(axis=1)
    y = flip_labels(sign_pm1(margin), flip, rng)
    row_ptr = np.arange(0, (m + 1) * nnz_per_row, nnz_per_row, dtype=np.int64)
    return {"row_ptr": row_ptr, "col_idx": cols.reshape(-1).astype(np.int32),
            "val": vals.reshape(-1).copy(), "m": m, "n": n, "y": y}


def csr_news20(m: int = 19996, n: int = 1355191, mean_nnz: float = 455.0,
               sigma_len: float = 0.8, max_nnz: int = 16384, zipf_a: float = 1.1,
               flip: float = 0.05, seed: int = 106) -> dict:
    """Sparse rows shaped like news20.binary (19996 x 1355191, about 9.1e6
    stored entries, Table 3): row lengths lognormal with mean `mean_nnz` and
    log-spread `sigma_len`, clipped to [1, max_nnz]; distinct columns per row
    drawn from a Zipf(zipf_a) law over a seeded permutation of the columns;
    values (0.1 + U(0,1)) * log(1 + n / rank), rows L2-normalised; labels
    sign(A w) for w ~ N(0,1) on a random 10% of the columns, `flip` of them
    flipped (the targets of K-RR as well).  Columns sorted within each row."""
    rng = np.random.default_rng(seed)
    mu = np.log(mean_nnz) - 0.5 * sigma_len ** 2
    lens = np.clip(np.rint(np.exp(rng.normal(mu, sigma_len, m))), 1, min(max_nnz, n))
    lens = lens.astype(np.int64)
    cdf = _zipf_cdf(n, zipf_a)
    perm = rng.permutation(n)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(lens)
    col_idx = np.empty(row_ptr[-1], dtype=np.int32)
    val = np.empty(row_ptr[-1], dtype=np.float64)
    for i in range(m):
        L = int(lens[i])
        draws = np.empty(0, dtype=np.int64)
        while True:
            r = np.minimum(np.searchsorted(cdf, rng.random(2 * L + 32), side="right"), n - 1)
            draws = np.concatenate([draws, r])
            uniq, first = np.unique(draws, return_index=True)
            if uniq.size >= L:
                break
        ranks = draws[np.sort(first)[:L]]          # the first L distinct ranks, in draw order
        c = perm[ranks]
        order = np.argsort(c)
        v = (0.1 + rng.random(L)) * np.log1p(n / (ranks + 1.0))
        v = v[order]
        col_idx[row_ptr[i]:row_ptr[i + 1]] = c[order]
        val[row_ptr[i]:row_ptr[i + 1]] = v / np.sqrt(np.dot(v, v))
    w = np.zeros(n)
    support = rng.choice(n, size=max(1, n // 10), replace=False)
    w[support] = rng.standard_normal(support.size)
    margin = np.add.reduceat(val * w[col_idx], row_ptr[:-1])
    y = flip_labels(sign_pm1(margin), flip, rng)
    return {"row_ptr": row_ptr, "col_idx": col_idx, "val": val, "m": m, "n": n, "y": y}


def csr_to_dense(row_ptr: np.ndarray, col_idx: np.ndarray, val: np.ndarray,
                 m: int, n: int) -> np.ndarray:
    """Densify a CSR matrix (small cases only)."""
    A = np.zeros((m, n))
    for i in range(m):
        s, e = row_ptr[i], row_ptr[i + 1]
        A[i, col_idx[s:e]] = val[s:e]
    return A


def dense_c4(m: int = 200000, n: int = 1024, n_classes: int = 10, seed: int = 104) -> dict:
    """C4: rows N(0,1)/sqrt(n); K-RR targets as in C2; one-vs-rest labels from
    class = argmax(A Z), Z ~ N(0, I) of size n x n_classes (no flips)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    u = rng.standard_normal(n)
    y = np.sin(A @ u) + 0.01 * rng.standard_normal(m)
    Z = rng.standard_normal((n, n_classes))
    cls = np.argmax(A @ Z, axis=1)
    Y = np.where(cls[None, :] == np.arange(n_classes)[:, None], 1.0, -1.0)
    return {"A": A, "y": y, "Y_ovr": Y, "classes": cls}


def dense_ksvm_c5(m: int = 500000, n: int = 256, hidden: int = 64, flip: float = 0.03,
                  seed: int = 105) -> dict:
    """C5: A ~ N(0,1); y = sign(v . tanh(W1 a / sqrt(n))), W1 ~ N(0,1) of size
    hidden x n, v ~ N(0,1); `flip` of the labels flipped."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    W1 = rng.standard_normal((hidden, n))
    v = rng.standard_normal(hidden)
    y = flip_labels(sign_pm1(np.tanh(A @ W1.T / np.sqrt(n)) @ v), flip, rng)
    return {"A": A, "y": y}

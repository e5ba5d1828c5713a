"""The K-RR lookahead loop against the FP64 oracle and against the serial loop.

In the lookahead loop the recurrence of index block k (Algorithm 4's inner
loop) runs in workgroup 0 of the launch that computes block k+1's kernel
block; that product reduces r_{k+1} against the iterate before block k's
updates and stores the kernel rows of block k's coordinates, and the finish
pass of block k+1 adds those rows times the updates to r_{k+1} and the
updates to alpha.  That is r_{k+1} = U_{k+1}^T alpha_{k+1} of Algorithm 4 up
to rounding, so the bar is the plain FP64 path's: 1e-9 relative error against
the oracle, element by element, on alpha and on every update.  Cases cover
one and two recurrence elements per thread, b from 1 to 8, ragged last outer
iterations, coordinates repeated across the blocks of one outer iteration
(the canonical-element sums and the m term of the Gram), a warm start, and
C2 at full size in the benchmark's configuration (where the loop is the
default).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2406_18001_amd import inputs
from tests.helpers import assert_parity, dev, idx_dev, max_rel

pytestmark = pytest.mark.gpu

TOL = 1e-9
RBF1 = (2, 1.0, 0.0, 1)
POLY13 = (1, 0.0, 1.0, 3)


@pytest.fixture(scope="module")
def K():
    from paper_2406_18001_amd import kdcd
    return kdcd


def _solve(K, A, y, kk, lam, b, s, H, idx, flags, alpha0=None, profile=False):
    alpha = dev(np.zeros(A.shape[0]) if alpha0 is None else alpha0)
    trace = torch.zeros(H * b, dtype=torch.float64, device="cuda")
    res = K.kdcd_krr_solve(dev(A), dev(y), kk, lam, b, s, H, idx_dev(idx), alpha, trace=trace,
                           flags=flags, profile=profile)
    return alpha.cpu().numpy(), trace.cpu().numpy(), res


def _oracle(A, y, kk, lam, b, s, H, idx, alpha0=None):
    okern = O.Kernel(kk[0], sigma=kk[1], c=kk[2], degree=kk[3])
    return O.bdcd_krr(A, y, okern, lam, b, H, idx, alpha0=alpha0, s=s)


@pytest.mark.parametrize("m,n,b,s,H", [
    (3000, 64, 8, 32, 167),     # s*b = 256, six outer iterations, the last of 7 blocks
    (2000, 128, 4, 64, 256),    # s*b = 256, four whole outer iterations
    (1500, 48, 1, 256, 700),    # b = 1, the last outer iteration of 188 blocks
    (2500, 32, 8, 64, 300),     # s*b = 512: two recurrence elements per thread
    (4000, 96, 2, 200, 1000),   # s*b = 400, ragged against the 64-row tiles
    (1200, 16, 8, 40, 90),      # s*b = 320, n = 16 (one K chunk)
])
def test_lookahead_matches_oracle(K, m, n, b, s, H):
    d = inputs.dense_krr_c2(m=m, n=n, seed=m + b)
    idx = inputs.krr_indices(m, b, H, seed=s)
    a_ref, d_ref = _oracle(d["A"], d["y"], RBF1, 1e-3, b, s, H, idx)
    a, t, res = _solve(K, d["A"], d["y"], RBF1, 1e-3, b, s, H, idx, K.FLAG_LOOKAHEAD,
                       profile=True)
    assert_parity(a, a_ref, TOL, f"alpha b={b} s={s}")
    assert_parity(t, d_ref, TOL, f"delta b={b} s={s}")
    # only the last block's recurrence is a launch of its own
    assert res["recur_launches"] == 1


def test_lookahead_repeated_coordinates(K):
    """m = 300 against s*b = 256: most coordinates come back within one outer
    iteration and across consecutive ones."""
    d = inputs.dense_krr_c2(m=300, n=32, seed=3)
    idx = inputs.krr_indices(300, 8, 200, seed=1)
    kern = (2, 0.5, 0.0, 1)
    a_ref, d_ref = _oracle(d["A"], d["y"], kern, 1e-2, 8, 32, 200, idx)
    a, t, _ = _solve(K, d["A"], d["y"], kern, 1e-2, 8, 32, 200, idx, K.FLAG_LOOKAHEAD)
    assert_parity(a, a_ref, TOL, "alpha")
    assert_parity(t, d_ref, TOL, "delta")
    # the sums over repeated coordinates have one order: runs agree bit for bit
    a2, t2, _ = _solve(K, d["A"], d["y"], kern, 1e-2, 8, 32, 200, idx, K.FLAG_LOOKAHEAD)
    assert np.array_equal(a, a2) and np.array_equal(t, t2)


def test_lookahead_warm_start_poly(K):
    d = inputs.dense_krr_c2(m=1000, n=48, seed=4)
    a0 = np.random.default_rng(2).standard_normal(1000) * 0.1
    idx = inputs.krr_indices(1000, 4, 256, seed=6)
    a_ref, d_ref = _oracle(d["A"], d["y"], POLY13, 1e-1, 4, 64, 256, idx, alpha0=a0)
    a, t, _ = _solve(K, d["A"], d["y"], POLY13, 1e-1, 4, 64, 256, idx, K.FLAG_LOOKAHEAD,
                     alpha0=a0)
    assert_parity(a, a_ref, TOL, "alpha")
    assert_parity(t, d_ref, TOL, "delta")


def test_lookahead_refused_shapes_run_serially(K):
    """b = 16 and s*b = 1024 are outside the lookahead recurrence; the flag then
    leaves the serial loop in place (one recurrence launch per outer iteration)."""
    d = inputs.dense_krr_c2(m=1500, n=32, seed=5)
    for b, s, H in [(16, 16, 64), (8, 128, 256)]:
        idx = inputs.krr_indices(1500, b, H, seed=b)
        a_ref, d_ref = _oracle(d["A"], d["y"], RBF1, 1e-3, b, s, H, idx)
        a, t, res = _solve(K, d["A"], d["y"], RBF1, 1e-3, b, s, H, idx, K.FLAG_LOOKAHEAD,
                           profile=True)
        assert_parity(a, a_ref, TOL, f"alpha b={b}")
        assert_parity(t, d_ref, TOL, f"delta b={b}")
        assert res["recur_launches"] == (H + s - 1) // s


def test_lookahead_fp64_needs_whole_k_chunks(K):
    """The FP64 lookahead product takes n in whole 16-column chunks: n = 40 with
    the flag runs the serial loop, to the same bar."""
    d = inputs.dense_krr_c2(m=1500, n=40, seed=9)
    b, s, H = 8, 32, 200
    idx = inputs.krr_indices(1500, b, H, seed=3)
    a_ref, d_ref = _oracle(d["A"], d["y"], RBF1, 1e-3, b, s, H, idx)
    a, t, res = _solve(K, d["A"], d["y"], RBF1, 1e-3, b, s, H, idx, K.FLAG_LOOKAHEAD,
                       profile=True)
    assert_parity(a, a_ref, TOL, "alpha n=40")
    assert_parity(t, d_ref, TOL, "delta n=40")
    assert res["recur_launches"] == (H + s - 1) // s


def test_lookahead_duplicate_in_block_is_refused(K):
    d = inputs.dense_krr_c2(m=1000, n=32, seed=7)
    idx = inputs.krr_indices(1000, 8, 96, seed=2)
    idx[40 * 8 + 3] = idx[40 * 8 + 5]          # block 40 (outer iteration 1) repeats a coordinate
    with pytest.raises(K.KdcdError) as e:
        _solve(K, d["A"], d["y"], RBF1, 1e-3, 8, 32, 96, idx, K.FLAG_LOOKAHEAD)
    assert e.value.status == -4                 # KDCD_ERR_INDEX_DUPLICATE


def test_c2_default_is_lookahead_and_matches_serial(K):
    """C2 at full size (20000 x 512, b = 8, s = 64, H = 2000): the default takes
    the lookahead loop; it agrees with the serial loop, and the first outer
    iterations with the oracle."""
    d = inputs.dense_krr_c2()
    idx = inputs.krr_indices(20000, 8, 2000, seed=0)
    a_la, t_la, res = _solve(K, d["A"], d["y"], RBF1, 1e-3, 8, 64, 2000, idx, 0, profile=True)
    assert res["recur_launches"] == 1
    a_se, t_se, res = _solve(K, d["A"], d["y"], RBF1, 1e-3, 8, 64, 2000, idx, K.FLAG_SERIAL,
                             profile=True)
    assert res["recur_launches"] == 32
    assert max_rel(a_la, a_se) <= TOL
    assert max_rel(t_la, t_se) <= TOL
    # three outer iterations against the oracle
    a_ref, d_ref = _oracle(d["A"], d["y"], RBF1, 1e-3, 8, 64, 192, idx[:192 * 8])
    a3, t3, _ = _solve(K, d["A"], d["y"], RBF1, 1e-3, 8, 64, 192, idx[:192 * 8],
                       K.FLAG_LOOKAHEAD)
    assert_parity(a3, a_ref, TOL, "alpha")
    assert_parity(t3, d_ref, TOL, "delta")


def _krr_rel(ev, m):
    bound = 0.5 * ev["residual_norm"] ** 2 / m
    return bound / (abs(ev["objective"]) - bound)


@pytest.mark.parametrize("H_outer,every", [(13, 4), (12, 16)])
def test_lookahead_monitor_value(K, H_outer, every):
    """The monitor inside the lookahead loop: the iterate is the unmonitored
    lookahead solve's bit for bit, and the reported bound matches the oracle's
    at the end (also when the only evaluation is the final one)."""
    m, n, b, s = 2000, 64, 8, 32
    H = H_outer * s - 3
    d = inputs.dense_krr_c2(m=m, n=n, seed=12)
    idx = inputs.krr_indices(m, b, H, seed=2)
    a = dev(np.zeros(m))
    info = K.kdcd_krr_solve(dev(d["A"]), dev(d["y"]), RBF1, 1e-3, b, s, H, idx_dev(idx), a,
                            monitor_every=every, tol=0.0, flags=K.FLAG_LOOKAHEAD)
    plain, _, _ = _solve(K, d["A"], d["y"], RBF1, 1e-3, b, s, H, idx, K.FLAG_LOOKAHEAD)
    assert np.array_equal(a.cpu().numpy(), plain)
    assert info["outer_done"] == H_outer
    ev = O.krr_eval(d["A"], d["y"], O.Kernel(O.RBF, sigma=1.0), 1e-3, plain)
    ref = _krr_rel(ev, m)
    assert ref > 0 and abs(info["rel_err"] - ref) <= 1e-7 * ref


def test_lookahead_monitor_early_stop(K):
    """Stop at 1e-6: the result equals a lookahead solve of exactly the reported
    outer iterations (to rounding: there the last block's recurrence is a launch
    of its own), and the oracle's bound at it is within the target."""
    m, n, b, s = 3000, 64, 8, 32
    H = 400 * s
    d = inputs.dense_krr_c2(m=m, n=n, seed=10)
    idx = inputs.krr_indices(m, b, H, seed=5)
    a = dev(np.zeros(m))
    info = K.kdcd_krr_solve(dev(d["A"]), dev(d["y"]), RBF1, 1e-3, b, s, H, idx_dev(idx), a,
                            monitor_every=8, tol=1e-6, flags=K.FLAG_LOOKAHEAD)
    k = info["outer_done"]
    assert 0 < k < H // s and k % 8 == 0 and info["rel_err"] <= 1e-6
    plain, _, _ = _solve(K, d["A"], d["y"], RBF1, 1e-3, b, s, k * s, idx[:k * s * b],
                         K.FLAG_LOOKAHEAD)
    assert max_rel(a.cpu().numpy(), plain) <= 1e-12
    ev = O.krr_eval(d["A"], d["y"], O.Kernel(O.RBF, sigma=1.0), 1e-3, plain)
    assert _krr_rel(ev, m) <= 1e-6 * (1 + 1e-6)


def test_lookahead_in_a_captured_graph(K):
    """A whole-call graph of the lookahead loop (fewer than 18 whole blocks, so
    the call is captured, not windowed): every replay equals the eager solve."""
    m, n, b, s, H = 2000, 64, 8, 32, 5 * 32 - 3
    d = inputs.dense_krr_c2(m=m, n=n, seed=13)
    idx = inputs.krr_indices(m, b, H, seed=4)
    ref, _, _ = _solve(K, d["A"], d["y"], RBF1, 1e-3, b, s, H, idx, K.FLAG_LOOKAHEAD)
    A, y, I = dev(d["A"]), dev(d["y"]), idx_dev(idx)
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    for rep in range(3):
        a.zero_()
        K.kdcd_krr_solve(A, y, RBF1, 1e-3, b, s, H, I, a,
                         flags=K.FLAG_GRAPH | K.FLAG_LOOKAHEAD)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), ref), f"replay {rep}"


@pytest.mark.parametrize("case", range(8))
def test_lookahead_equals_serial_on_seeded_shapes(K, case):
    """Seeded shapes across the lookahead's range (b in 1..8, 256 <= s*b <= 512,
    ragged H, n a multiple of 16, m from below s*b to well above): the
    lookahead loop and the serial loop agree to the parity bar."""
    rng = np.random.default_rng(100 + case)
    b = int(rng.choice([1, 2, 4, 8]))
    s = int(rng.integers(256 // b, 512 // b + 1))
    n = 16 * int(rng.integers(1, 9))
    m = int(rng.integers(200, 6000))
    H = int(rng.integers(2 * s, 6 * s))
    d = inputs.dense_krr_c2(m=m, n=n, seed=200 + case)
    idx = inputs.krr_indices(m, b, H, seed=300 + case)
    kern = (2, float(rng.choice([0.25, 1.0])), 0.0, 1)
    lam = float(rng.choice([1e-3, 1e-2]))
    a_la, t_la, res = _solve(K, d["A"], d["y"], kern, lam, b, s, H, idx, K.FLAG_LOOKAHEAD,
                             profile=True)
    assert res["recur_launches"] == 1
    a_se, t_se, _ = _solve(K, d["A"], d["y"], kern, lam, b, s, H, idx, K.FLAG_SERIAL)
    assert max_rel(a_la, a_se) <= TOL, (m, n, b, s, H)
    assert max_rel(t_la, t_se) <= TOL, (m, n, b, s, H)


@pytest.mark.parametrize("compute", ["bf16x3", "f16", "bf16", "f32"])
def test_lookahead_low_precision(K, compute):
    """The lookahead loop with a low-precision product (the kernel rows of the
    previous block's coordinates then come from the FP64 Gram launch): the
    updates follow the serial low-precision loop's within the precision's own
    error, and for bf16x3 the objective matches the FP64 solve's to 1e-6 as the
    serial loop's does."""
    m, n, b, s = 3000, 512, 8, 32
    H = 12 * s - 5
    d = inputs.dense_c4(m=m, n=n, seed=7)
    idx = inputs.krr_indices(m, b, H, seed=1)
    kern = RBF1
    A, y, I = dev(d["A"]), dev(d["y"]), idx_dev(idx)

    def run(flags, comp):
        a = torch.zeros(m, dtype=torch.float64, device="cuda")
        t = torch.zeros(H * b, dtype=torch.float64, device="cuda")
        res = K.kdcd_krr_solve(A, y, kern, 1e-3, b, s, H, I, a, trace=t, compute=comp,
                               flags=flags, profile=True)
        return a, t, res

    a_la, t_la, res = run(K.FLAG_LOOKAHEAD, compute)
    assert res["recur_launches"] == 1
    a_se, t_se, res = run(K.FLAG_SERIAL, compute)
    assert res["recur_launches"] == -(-H // s)
    # the two loops take the product's rounding at different places (the
    # lookahead adds block k's updates through FP64 kernel rows), so their
    # updates differ at the level of the precision's kernel-value error
    bound = {"bf16x3": 5e-6, "f32": 5e-6, "f16": 1e-2, "bf16": 5e-2}[compute]
    assert max_rel(t_la.cpu().numpy(), t_se.cpu().numpy()) <= bound
    a64, _, _ = run(K.FLAG_SERIAL, "f64")
    f_la = K.kdcd_krr_eval(A, y, kern, 1e-3, a_la)["objective"]
    f_se = K.kdcd_krr_eval(A, y, kern, 1e-3, a_se)["objective"]
    f64 = K.kdcd_krr_eval(A, y, kern, 1e-3, a64)["objective"]
    assert abs(f_la - f64) <= max(2 * abs(f_se - f64), 1e-6 * abs(f64)), (f_la, f_se, f64)
    if compute in ("bf16x3", "f32"):
        assert abs(f_la - f64) <= 1e-6 * abs(f64)


@pytest.mark.parametrize("compute", ["bf16x3", "f32"])
def test_lookahead_low_precision_ragged(K, compute):
    """The low-precision lookahead at n = 40 and m = 1037 (partial K chunks and
    row tiles; the FP64 Gram launch over two index blocks then has ragged rows
    too): it runs, and its updates follow the serial loop's within the
    precision's error."""
    m, n, b, s = 1037, 40, 8, 40
    H = 6 * s - 3
    d = inputs.dense_c4(m=m, n=n, seed=11)
    idx = inputs.krr_indices(m, b, H, seed=5)
    A, y, I = dev(d["A"]), dev(d["y"]), idx_dev(idx)

    def run(flags):
        a = torch.zeros(m, dtype=torch.float64, device="cuda")
        t = torch.zeros(H * b, dtype=torch.float64, device="cuda")
        res = K.kdcd_krr_solve(A, y, RBF1, 1e-3, b, s, H, I, a, trace=t, compute=compute,
                               flags=flags, profile=True)
        return a.cpu().numpy(), t.cpu().numpy(), res

    a_la, t_la, res = run(K.FLAG_LOOKAHEAD)
    assert res["recur_launches"] == 1
    a_se, t_se, _ = run(K.FLAG_SERIAL)
    assert max_rel(t_la, t_se) <= 5e-6
    assert max_rel(a_la, a_se) <= 5e-6

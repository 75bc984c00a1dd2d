"""Pins that tie the FP64 oracle to what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form from Theorem 1's proof, a library solve, a hand-derived value, an
independent solver or an invariant.  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(n=6, n_ang=12, bins=9, seed=11, noise=0.01, M=1, N=1):
    p = synth.make_problem(n=n, n_ang=n_ang, bins=bins, seed=seed, noise=noise, M=M, N=N)
    A = oracle.as_matrix(p.row_ptr, p.col, p.val, p.ncols)
    return p, A


def _diff_matrix(H, W):
    """Backward-difference operator of Eq. 2 as an explicit sparse matrix.

    Built entry by entry from the definition (independent of the oracle's
    array slicing): rows 0..HW-1 are vertical differences, HW..2HW-1
    horizontal ones; differences reaching outside the image are zero rows.
    """
    rows, cols, vals = [], [], []
    for s in range(H):
        for t in range(W):
            k = s * W + t
            if s >= 1:
                rows += [k, k]
                cols += [k, (s - 1) * W + t]
                vals += [1.0, -1.0]
            if t >= 1:
                rows += [H * W + k, H * W + k]
                cols += [k, s * W + t - 1]
                vals += [1.0, -1.0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * H * W, H * W))


def _tv_from_matrix(K, x, H, W):
    g = K @ x.ravel()
    return float(np.sum(np.hypot(g[:H * W], g[H * W:])))


# --------------------------------------------------------------------------
# Products (both block products of Alg. 1)
# --------------------------------------------------------------------------

def test_adjoint_identity_and_dense_products():
    p, A = _tiny(n=9, n_ang=14, bins=15)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(p.ncols)
    r = rng.standard_normal(p.nrows)
    lhs = float(oracle.forward(A, x) @ r)
    rhs = 0.5 * float(x @ oracle.backproject(A, r))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)
    D = np.zeros((p.nrows, p.ncols))
    for i in range(p.nrows):
        D[i, p.col[p.row_ptr[i]:p.row_ptr[i + 1]]] = p.val[p.row_ptr[i]:p.row_ptr[i + 1]]
    assert np.allclose(oracle.forward(A, x), D @ x, rtol=0, atol=1e-12)
    assert np.allclose(oracle.backproject(A, r), 2.0 * D.T @ r, rtol=0, atol=1e-12)


def test_tiles_reassemble_and_transpose():
    p, _ = _tiny(n=10, n_ang=9, bins=15, M=3, N=4)
    ro, co = synth.block_offsets(9, 15, 100, 3, 4)
    blocks = oracle.tiles(p.row_ptr, p.col, p.val, ro, co)
    full = oracle.as_matrix(p.row_ptr, p.col, p.val, p.ncols).toarray()
    for i in range(3):
        for j in range(4):
            ptr, lc, lv = blocks[(i, j)]
            sub = sp.csr_matrix((lv, lc, ptr), shape=(ro[i + 1] - ro[i], co[j + 1] - co[j])).toarray()
            assert np.array_equal(sub, full[ro[i]:ro[i + 1], co[j]:co[j + 1]])
            tp, tc, tv = blocks[("T", i, j)]
            subT = sp.csr_matrix((tv, tc, tp), shape=(co[j + 1] - co[j], ro[i + 1] - ro[i])).toarray()
            assert np.array_equal(subT, sub.T)
            for k in range(len(tp) - 1):
                assert np.all(np.diff(tc[tp[k]:tp[k + 1]]) > 0)


# --------------------------------------------------------------------------
# lambda = 0 dynamics: Eq. 3, Theorem 1 and its proof (Eq. 4-7)
# --------------------------------------------------------------------------

def test_power_iteration_matches_eigensolver():
    p, A = _tiny()
    ev = np.linalg.eigvalsh((A.T @ A).toarray())
    assert abs(oracle.power_umax(A) - ev[-1]) <= 1e-10 * ev[-1]


@pytest.mark.parametrize("factor", [0.9, 0.2])
def test_modal_closed_form_of_delayed_iteration(factor):
    """Each eigenmode of A^T A follows c_{k+1} = c_k - 2 mu u c_{k-1}.

    Its roots are v = (1 +- sqrt(1 - 8 mu u)) / 2 (Eq. 7), so with
    x_{-1} = x_0 = 0 the error coefficient after epoch k is
    alpha v1^{k+1} + beta v2^{k+1}, alpha + beta = alpha v1 + beta v2 = c_0.
    """
    p, A = _tiny()
    AtA = (A.T @ A).toarray()
    u, V = np.linalg.eigh(AtA)
    xstar = np.linalg.solve(AtA, A.T @ p.y)
    mu = factor / (2.0 * u[-1])
    E = 60
    _, _, hist = oracle.bsgd_tv(A, p.y, mu, 0.0, E, 0, (p.H, p.W), record=True)
    c0 = V.T @ (-xstar)
    sq = np.sqrt((1.0 - 8.0 * mu * u).astype(complex))
    v1, v2 = (1.0 + sq) / 2.0, (1.0 - sq) / 2.0
    alpha = c0 * (1.0 - v2) / (v1 - v2)
    beta = c0 * (v1 - 1.0) / (v1 - v2)
    scale = np.linalg.norm(xstar)
    for k in range(1, E + 1):
        pred = (alpha * v1 ** (k + 1) + beta * v2 ** (k + 1)).real
        got = V.T @ (hist[k - 1] - xstar)
        assert np.max(np.abs(got - pred)) <= 1e-9 * scale, k


def test_converges_to_least_squares_full_rank():
    p, A = _tiny(n=5, n_ang=8, bins=9)
    Ad = A.toarray()
    assert np.linalg.matrix_rank(Ad) == p.ncols
    xls = np.linalg.lstsq(Ad, p.y, rcond=None)[0]
    mu = oracle.step_size(oracle.power_umax(A), 0.9)
    x, _ = oracle.bsgd_tv(A, p.y, mu, 0.0, 15000, 0, (p.H, p.W))
    assert np.linalg.norm(x - xls) <= 1e-8 * np.linalg.norm(xls)


def test_converges_to_min_norm_solution_rank_deficient():
    p, A = _tiny(n=4, n_ang=3, bins=7)
    Ad = A.toarray()
    assert np.linalg.matrix_rank(Ad) < p.ncols
    xmn = np.linalg.pinv(Ad) @ p.y
    mu = oracle.step_size(oracle.power_umax(A), 0.9)
    x, _ = oracle.bsgd_tv(A, p.y, mu, 0.0, 12000, 0, (p.H, p.W))
    assert np.linalg.norm(x - xmn) <= 1e-7 * np.linalg.norm(xmn)


def test_step_threshold_diverges_at_predicted_rate():
    """Above 1/(2 u_max) the top mode grows by |v| = sqrt(2 mu u_max) per epoch."""
    p, A = _tiny()
    umax = np.linalg.eigvalsh((A.T @ A).toarray())[-1]
    xstar = np.linalg.lstsq(A.toarray(), p.y, rcond=None)[0]
    mu = 1.05 / (2.0 * umax)
    _, _, hist = oracle.bsgd_tv(A, p.y, mu, 0.0, 1200, 0, (p.H, p.W), record=True)
    e = np.array([np.linalg.norm(h - xstar) for h in hist])
    assert e[-1] > 1e3 * e[0]
    # the growing mode pair is complex (8 mu u > 1), so compare envelopes over
    # windows longer than its oscillation period
    rate = (e[-30:].max() / e[-430:-400].max()) ** (1.0 / 400.0)
    assert abs(rate - math.sqrt(2.0 * mu * umax)) < 1e-3
    # just below the threshold the same problem converges, at the spectral
    # radius of the companion matrix (Eq. 4): max over modes of |v1|, |v2|
    mu = 0.95 / (2.0 * umax)
    u = np.linalg.eigvalsh((A.T @ A).toarray())
    sq = np.sqrt((1.0 - 8.0 * mu * u).astype(complex))
    radius = max(np.abs((1.0 + sq) / 2.0).max(), np.abs((1.0 - sq) / 2.0).max())
    _, _, hist = oracle.bsgd_tv(A, p.y, mu, 0.0, 4000, 0, (p.H, p.W), record=True)
    e = np.array([np.linalg.norm(h - xstar) for h in hist])
    assert e[-1] < 1e-2 * e[0]
    rate = (e[-1] / e[-1001]) ** (1.0 / 1000.0)
    assert abs(rate - radius) < 1e-4


# --------------------------------------------------------------------------
# TV (Eq. 2)
# --------------------------------------------------------------------------

def test_tv_hand_values():
    g = json.load(open(os.path.join(GOLDEN, "tv_hand.json")))
    for case in g["cases"]:
        assert abs(oracle.tv2(np.array(case["image"])) - case["tv"]) < 1e-14
    for case in g["cases_3d"]:
        assert abs(oracle.tv3(np.array(case["volume"])) - case["tv"]) < 1e-14


def test_tv_closed_forms():
    H, W, h, k = 7, 5, 0.3, 3
    assert oracle.tv2(np.full((H, W), 2.5)) == 0.0
    step_rows = np.zeros((H, W))
    step_rows[k:, :] = h
    assert abs(oracle.tv2(step_rows) - W * h) < 1e-14
    step_cols = np.zeros((H, W))
    step_cols[:, k:] = h
    assert abs(oracle.tv2(step_cols) - H * h) < 1e-14
    x = np.random.default_rng(1).standard_normal((H, W))
    assert abs(oracle.tv2(-3.0 * x) - 3.0 * oracle.tv2(x)) < 1e-12
    assert abs(oracle.tv2(x + 7.0) - oracle.tv2(x)) < 1e-12
    assert abs(oracle.tv3(x[None]) - oracle.tv2(x)) < 1e-12
    K = _diff_matrix(H, W)
    assert abs(_tv_from_matrix(K, x, H, W) - oracle.tv2(x)) < 1e-12


def test_difference_operator_and_adjoint():
    H, W = 6, 9
    K = _diff_matrix(H, W)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((H, W))
    dv, dh = oracle.grad2(x)
    g = K @ x.ravel()
    assert np.allclose(dv.ravel(), g[:H * W], atol=1e-14)
    assert np.allclose(dh.ravel(), g[H * W:], atol=1e-14)
    pv, ph = rng.standard_normal((H, W)), rng.standard_normal((H, W))
    pv[0, :] = 0.0
    ph[:, 0] = 0.0
    adj = K.T @ np.concatenate([pv.ravel(), ph.ravel()])
    assert np.allclose(oracle.grad2_adj(pv, ph).ravel(), adj, atol=1e-14)


# --------------------------------------------------------------------------
# TV prox step of Alg. 1 by FGP
# --------------------------------------------------------------------------

def test_fgp_hand_values():
    g = json.load(open(os.path.join(GOLDEN, "fgp_hand.json")))
    c0 = g["cases"][0]
    out = oracle.fgp_prox2(np.array(c0["b"]), c0["theta"], c0["iters"])
    assert np.max(np.abs(out - np.array(c0["expected"]))) < 1e-15
    c1 = g["cases"][1]
    for k, exp in c1["expected_by_iters"].items():
        out = oracle.fgp_prox2(np.array(c1["b"]), c1["theta"], int(k))
        assert np.max(np.abs(out - np.array(exp))) < 1e-15, k


def test_fista_sequence_invariant():
    tau = oracle.fista_tau(50)
    assert tau[0] == 1.0
    assert np.allclose(tau[1:] ** 2 - tau[1:], tau[:-1] ** 2, rtol=1e-14)
    assert np.all(tau >= (np.arange(51) + 2) / 2.0 - 1e-12)


def _pdhg_tv(b, theta, iters):
    """Independent solver: accelerated primal-dual (Chambolle-Pock) for
    min_x 1/2||x-b||^2 + theta ||K x||_{2,1} with K the explicit difference matrix."""
    H, W = b.shape
    K = _diff_matrix(H, W)
    n = H * W
    x = b.ravel().copy()
    xbar = x.copy()
    y = np.zeros(2 * n)
    tau = sigma = 0.99 / math.sqrt(8.0)
    for _ in range(iters):
        y = y + sigma * (K @ xbar)
        nrm = np.maximum(1.0, np.hypot(y[:n], y[n:]) / theta)
        y[:n] /= nrm
        y[n:] /= nrm
        x_old = x
        x = (x - tau * (K.T @ y) + tau * b.ravel()) / (1.0 + tau)
        th = 1.0 / math.sqrt(1.0 + 2.0 * tau)
        tau *= th
        sigma /= th
        xbar = x + th * (x - x_old)
    return x.reshape(H, W), y


@pytest.mark.parametrize("theta", [0.05, 0.3])
def test_prox_converged_duality_gap_and_independent_solver(theta):
    H = W = 8
    b = np.random.default_rng(3).random((H, W))
    x, (pv, ph) = oracle.fgp_prox2(b, theta, 20000, return_dual=True)
    K = _diff_matrix(H, W)
    assert np.all(np.hypot(pv, ph) <= 1.0 + 1e-12)
    pvec = np.concatenate([pv.ravel(), ph.ravel()])
    xd = b.ravel() - theta * (K.T @ pvec)
    assert np.allclose(x.ravel(), xd, atol=1e-13)
    primal = 0.5 * np.sum((xd - b.ravel()) ** 2) + theta * _tv_from_matrix(K, xd, H, W)
    dual = 0.5 * np.sum(b ** 2) - 0.5 * np.sum(xd ** 2)
    assert 0.0 <= primal - dual + 1e-14
    assert primal - dual < 1e-10
    # independent solver; strong convexity bounds the distance of each
    # solution to the minimiser by sqrt(2 * its duality gap)
    xi, yi = _pdhg_tv(b, theta, 40000)
    gap_i = 0.5 * np.sum((xi - b) ** 2) + theta * _tv_from_matrix(K, xi, H, W) \
        - (0.5 * np.sum(b ** 2) - 0.5 * np.sum((b.ravel() - K.T @ yi) ** 2))
    assert gap_i >= -1e-14
    bound = math.sqrt(2 * max(primal - dual, 0)) + math.sqrt(2 * gap_i)
    assert bound < 1e-3
    assert np.linalg.norm(xi - x) <= bound + 1e-12


def test_prox_row_step_closed_form():
    """b = h [s >= k]: the prox is theta/k above row k and h - theta/(H-k) from row k on."""
    H, W, k, h, theta = 9, 6, 4, 1.0, 0.4
    b = np.zeros((H, W))
    b[k:, :] = h
    x = oracle.fgp_prox2(b, theta, 30000)
    want = np.zeros((H, W))
    want[:k, :] = theta / k
    want[k:, :] = h - theta / (H - k)
    assert np.max(np.abs(x - want)) < 1e-9


def test_prox_invariants():
    rng = np.random.default_rng(4)
    b = rng.random((12, 10))
    for iters in (1, 5, 20, 200):
        x = oracle.fgp_prox2(b, 0.1, iters)
        assert abs(x.mean() - b.mean()) < 1e-14
    c = np.full((5, 7), 0.37)
    assert np.max(np.abs(oracle.fgp_prox2(c, 0.2, 20) - c)) < 1e-15
    assert np.array_equal(oracle.fgp_prox2(b, 0.0, 20), b)
    b2 = b + 0.05 * rng.standard_normal(b.shape)
    pa = oracle.fgp_prox2(b, 0.2, 5000)
    pb = oracle.fgp_prox2(b2, 0.2, 5000)
    assert np.linalg.norm(pa - pb) <= np.linalg.norm(b - b2) + 1e-9
    # 3-D prox of a volume that does not vary across slices equals the 2-D prox
    vol = np.repeat(b[None], 3, axis=0)
    x3 = oracle.fgp_prox3(vol, 0.1, 3000)
    x2 = oracle.fgp_prox2(b, 0.1, 3000)
    assert np.max(np.abs(x3 - x2[None])) < 1e-6


def test_prox3_duality_gap():
    D, H, W = 3, 5, 4
    b = np.random.default_rng(5).random((D, H, W))
    theta = 0.1
    x, p = oracle.fgp_prox3(b, theta, 30000, return_dual=True)
    assert np.all(np.sqrt(p[0] ** 2 + p[1] ** 2 + p[2] ** 2) <= 1.0 + 1e-12)
    primal = 0.5 * np.sum((x - b) ** 2) + theta * oracle.tv3(x)
    dual = 0.5 * np.sum(b ** 2) - 0.5 * np.sum(x ** 2)
    assert -1e-14 <= primal - dual < 1e-9


def test_fgp3_hand_values():
    """Finite-K iterates of the 3-D FGP against hand-derived values: the dual
    step 1/(12 theta) and the momentum (two voxels along each axis, K = 1..3)
    and the R^3 ball projection with the adjoint stencil (2 x 2 x 2, K = 1, 2)."""
    g = json.load(open(os.path.join(GOLDEN, "fgp3_hand.json")))
    c0 = g["cases"][0]
    for axis, b in c0["b_by_axis"].items():
        b = np.array(b)
        for k, exp in c0["expected_by_iters"].items():
            out = oracle.fgp_prox3(b, c0["theta"], int(k))
            assert np.max(np.abs(out.ravel() - np.array(exp))) < 1e-15, (axis, k)
    c1 = g["cases"][1]
    for k, exp in c1["expected_by_iters"].items():
        out = oracle.fgp_prox3(np.array(c1["b"]), c1["theta"], int(k))
        assert np.max(np.abs(out - np.array(exp))) < 1e-15, k


# --------------------------------------------------------------------------
# Blocking (Section 2.1): changes rounding only
# --------------------------------------------------------------------------

@pytest.mark.parametrize("M,N", [(1, 1), (2, 2), (4, 3), (3, 5)])
def test_blocked_epoch_matches_unblocked(M, N):
    p, A = _tiny(n=12, n_ang=12, bins=19, M=M, N=N)
    ro, co = synth.block_offsets(12, 19, p.ncols, M, N)
    blocks = oracle.tiles(p.row_ptr, p.col, p.val, ro, co)
    mu = oracle.step_size(oracle.power_umax(A))
    lam = 50.0
    xa, ra = oracle.initial_state(A, p.y)
    xb, rb = xa.copy(), ra.copy()
    for _ in range(5):
        xa, ra = oracle.bsgd_epoch(A, p.y, xa, ra, mu, lam, 10, (p.H, p.W))
        xb, rb = oracle.bsgd_epoch_blocked(blocks, ro, co, p.y, xb, rb, mu, lam, 10, (p.H, p.W))
    assert np.max(np.abs(xa - xb)) <= 1e-12 * np.max(np.abs(xa))
    assert np.max(np.abs(ra - rb)) <= 1e-12 * np.max(np.abs(ra))


def test_block_products_sum_to_whole():
    p, A = _tiny(n=10, n_ang=8, bins=15, M=2, N=3)
    ro, co = synth.block_offsets(8, 15, p.ncols, 2, 3)
    blocks = oracle.tiles(p.row_ptr, p.col, p.val, ro, co)
    rng = np.random.default_rng(6)
    x, r = rng.random(p.ncols), rng.random(p.nrows)
    z = np.concatenate([sum(oracle.block_forward(blocks, ro, co, i, j, x[co[j]:co[j + 1]])
                            for j in range(3)) for i in range(2)])
    g = np.concatenate([sum(oracle.block_backproject(blocks, ro, co, i, j, r[ro[i]:ro[i + 1]])
                            for i in range(2)) for j in range(3)])
    assert np.allclose(z, oracle.forward(A, x), atol=1e-12)
    assert np.allclose(g, oracle.backproject(A, r), atol=1e-12)


# --------------------------------------------------------------------------
# Whole method on the small workload
# --------------------------------------------------------------------------

def test_resume_from_state_is_exact():
    p, A = _tiny(n=8, n_ang=10, bins=13)
    mu = oracle.step_size(oracle.power_umax(A))
    x1, r1 = oracle.bsgd_tv(A, p.y, mu, 30.0, 12, 20, (p.H, p.W))
    xa, ra = oracle.bsgd_tv(A, p.y, mu, 30.0, 5, 20, (p.H, p.W))
    x2, r2 = oracle.bsgd_tv(A, p.y, mu, 30.0, 7, 20, (p.H, p.W), state=(xa, ra))
    assert np.array_equal(x1, x2) and np.array_equal(r1, r2)


def test_theorem2_margin_diagnostic_runs():
    """Diagnostic only (the truncated prox is inexact): the Eq. 8 margin is finite."""
    p, A = _tiny(n=8, n_ang=10, bins=13)
    mu = oracle.step_size(oracle.power_umax(A))
    _, _, hist = oracle.bsgd_tv(A, p.y, mu, 30.0, 6, 20, (p.H, p.W), record=True)
    m = [oracle.thm2_margin(A, p.y, hist[k - 1], hist[k], hist[k + 1], mu) for k in range(1, 5)]
    assert all(np.isfinite(m))


def test_theorem2_margin_hand_value_and_quadratic_identity():
    """Eq. 8's margin f(x^k) + <d, grad f(x^{k-1})> + ||d||^2/(2 mu) - f(x^{k+1}).

    Hand value: A = [1], y = 0, so f(v) = v^2 and grad f(v) = 2v; with
    x^{k-1} = 0, x^k = 1, x^{k+1} = 2, mu = 1/4: 1 + 0 + 2 - 4 = -1.
    Identity: f is quadratic, so f(x^{k+1}) = f(x^k) + <d, grad f(x^k)> + ||A d||^2
    and grad f(u) - grad f(v) = 2 A^T A (u - v); the margin is therefore
    2 <A d, A (x^{k-1} - x^k)> + ||d||^2/(2 mu) - ||A d||^2 for any vectors.
    """
    A1 = sp.csr_matrix(np.array([[1.0]]))
    m = oracle.thm2_margin(A1, np.zeros(1), np.zeros(1), np.ones(1), np.full(1, 2.0), 0.25)
    assert abs(m + 1.0) < 1e-15
    p, A = _tiny(n=6, n_ang=8, bins=9)
    rng = np.random.default_rng(21)
    Ad = A.toarray()
    for _ in range(3):
        xp, xc, xn = (rng.standard_normal(A.shape[1]) for _ in range(3))
        mu = 10.0 ** rng.uniform(-3, -1)
        d = xn - xc
        want = 2.0 * (Ad @ d) @ (Ad @ (xp - xc)) + d @ d / (2.0 * mu) - (Ad @ d) @ (Ad @ d)
        got = oracle.thm2_margin(A, p.y, xp, xc, xn, mu)
        assert abs(got - want) <= 1e-10 * (abs(want) + d @ d / mu)


def test_c1_reconstruction_improves():
    p = synth.make_problem("c1_64", with_transpose=False)
    A = oracle.as_matrix(p.row_ptr, p.col, p.val, p.ncols)
    mu = oracle.step_size(oracle.power_umax(A))
    x, _ = oracle.bsgd_tv(A, p.y, mu, p.lam, p.epochs, p.prox_iters, (p.H, p.W))
    xt = p.x_true.ravel()
    assert np.linalg.norm(x - xt) / np.linalg.norm(xt) < 0.2


def test_epoch_is_line8_then_line9():
    """One epoch equals argmin_t ||t - x^||^2 + 2 mu lam TV(t) with x^ = x + 2 mu A^T r.

    x^ is formed here with dense products and the minimiser by the
    independent primal-dual solver (its 1/2-scaled weight is mu lam).
    """
    p, A = _tiny(n=6, n_ang=8, bins=9)
    Ad = A.toarray()
    mu = 0.9 / (2.0 * np.linalg.eigvalsh(Ad.T @ Ad)[-1])
    lam = 0.1 / mu
    rng = np.random.default_rng(8)
    x = rng.random(p.ncols)
    r = p.y - Ad @ rng.random(p.ncols)
    x_new, r_new = oracle.bsgd_epoch(A, p.y, x, r, mu, lam, 20000, (p.H, p.W))
    assert np.allclose(r_new, p.y - Ad @ x, atol=1e-12)
    xhat = (x + 2.0 * mu * Ad.T @ r).reshape(p.H, p.W)
    ref, _ = _pdhg_tv(xhat, mu * lam, 40000)
    assert np.max(np.abs(x_new.reshape(p.H, p.W) - ref)) < 1e-4
    far, _ = _pdhg_tv(xhat, 2.0 * mu * lam, 40000)
    assert np.max(np.abs(far - ref)) > 1e-2


def test_multi_rhs_batch_equals_independent_runs():
    """A batch of S right-hand sides with per-RHS lambdas decouples into S single runs."""
    p, A = _tiny(n=8, n_ang=10, bins=13)
    mu = oracle.step_size(oracle.power_umax(A))
    rng = np.random.default_rng(12)
    Y = np.stack([p.y, A @ rng.random(p.ncols), p.y * 0.5, np.zeros(p.nrows)])
    lam = np.array([30.0, 0.0, 5.0, 12.0])
    X, R = oracle.bsgd_tv_multi(A, Y, mu, lam, 6, 20, (p.H, p.W), volume=False)
    for j in range(4):
        xj, rj = oracle.bsgd_tv(A, Y[j], mu, lam[j], 6, 20, (p.H, p.W))
        assert np.allclose(X[j], xj, rtol=0, atol=1e-13) and np.allclose(R[j], rj, rtol=0, atol=1e-12)


def test_multi_rhs_volume_of_identical_slices_is_2d():
    """Identical slices: the 3-D TV across them adds nothing; the converged prox is the 2-D one."""
    p, A = _tiny(n=8, n_ang=10, bins=13)
    mu = oracle.step_size(oracle.power_umax(A))
    Y = np.stack([p.y] * 3)
    lam = 3000.0
    X3, _ = oracle.bsgd_tv_multi(A, Y, mu, lam, 3, 4000, (p.H, p.W), volume=True)
    x2, _ = oracle.bsgd_tv(A, p.y, mu, lam, 3, 4000, (p.H, p.W))
    for j in range(3):
        assert np.max(np.abs(X3[j] - x2)) < 1e-6 * np.max(np.abs(x2))


# --------------------------------------------------------------------------
# Comparison methods (Simulations section, Fig. 2): ISTA and GD
# --------------------------------------------------------------------------

def test_gd_modal_closed_form():
    """GD on f: each eigenmode of A^T A decays by (1 - 2 mu u) per iteration.

    With x_0 = 0, V^T (x_k - x*) = (1 - 2 mu u)^k V^T (-x*), x* the
    normal-equations solution (eigh and solve, not the oracle's products).
    """
    p, A = _tiny()
    AtA = (A.T @ A).toarray()
    u, V = np.linalg.eigh(AtA)
    xstar = np.linalg.solve(AtA, A.T @ p.y)
    mu = 0.9 / (2.0 * u[-1])
    _, _, hist = oracle.gd(A, p.y, mu, 50, record=True)
    c0 = V.T @ (-xstar)
    for k in range(1, 51):
        pred = (1.0 - 2.0 * mu * u) ** k * c0
        assert np.max(np.abs(V.T @ (hist[k - 1] - xstar) - pred)) <= 1e-10 * np.linalg.norm(xstar)


def test_ista_with_zero_lambda_is_gd_and_first_iterate_matches_bsgd():
    p, A = _tiny()
    mu = oracle.step_size(oracle.power_umax(A))
    xa, _ = oracle.ista_tv(A, p.y, mu, 0.0, 7, 0, (p.H, p.W))
    xb, _ = oracle.gd(A, p.y, mu, 7)
    assert np.array_equal(xa, xb)
    # from x = 0 both methods use r = y in their first step
    x1, _ = oracle.ista_tv(A, p.y, mu, 40.0, 1, 20, (p.H, p.W))
    x2, _ = oracle.bsgd_tv(A, p.y, mu, 40.0, 1, 20, (p.H, p.W))
    assert np.array_equal(x1, x2)


def test_ista_objective_decreases_with_converged_prox():
    """With mu <= 1/L (L = 2 u_max) and an exact prox, F decreases at every ISTA step.

    This is the sufficient-decrease property of the proximal gradient method
    (Beck & Teboulle, SIAM J. Imaging Sci. 2(1), 2009, Lemma 2.3), which the
    delayed method does not have.
    """
    p, A = _tiny(n=6, n_ang=10, bins=9)
    mu = oracle.step_size(oracle.power_umax(A), 0.9)
    lam = 2.0
    _, _, hist = oracle.ista_tv(A, p.y, mu, lam, 25, 3000, (p.H, p.W), record=True)
    F = [oracle.objective(A, p.y, np.zeros(p.ncols), lam, (p.H, p.W))]
    F += [oracle.objective(A, p.y, h, lam, (p.H, p.W)) for h in hist]
    assert all(F[k + 1] <= F[k] * (1 + 1e-12) for k in range(len(F) - 1))
    assert F[-1] < 0.5 * F[0]


def test_ista_and_bsgd_reach_the_same_minimiser():
    """Both methods converge to the unique minimiser of F (Theorem 2 for BSGD).

    Checked with a converged prox: the two limits agree, and the limit is a
    fixed point of the proximal gradient map (the optimality condition of F).
    """
    p, A = _tiny(n=5, n_ang=8, bins=9)
    mu = oracle.step_size(oracle.power_umax(A), 0.9)
    lam, K, E = 1.0, 400, 300
    xi, _ = oracle.ista_tv(A, p.y, mu, lam, E, K, (p.H, p.W))
    xb, _ = oracle.bsgd_tv(A, p.y, mu, lam, E, K, (p.H, p.W))
    scale = np.linalg.norm(xi)
    assert np.linalg.norm(xi - xb) <= 1e-7 * scale
    step = oracle.prox(xi + mu * oracle.backproject(A, p.y - oracle.forward(A, xi)),
                       mu * lam, 20000, (p.H, p.W))
    assert np.linalg.norm(step - xi) <= 1e-7 * scale


# --------------------------------------------------------------------------
# Algorithm 1 on drawn block subsets (Simulations section, alpha and gamma)
# --------------------------------------------------------------------------

def test_block_subset_draws():
    rm, cm = synth.block_subsets(400, 5, 8, 0.5, 0.4, seed=3)
    assert all(bin(int(m)).count("1") == 2 for m in rm)
    assert all(bin(int(m)).count("1") == 4 for m in cm)
    assert all(int(m) < (1 << 5) for m in rm) and all(int(m) < (1 << 8) for m in cm)
    hits = np.array([[(int(m) >> j) & 1 for j in range(8)] for m in cm]).mean(axis=0)
    assert np.all(np.abs(hits - 0.5) < 0.1)       # uniform over the blocks
    rm2, cm2 = synth.block_subsets(400, 5, 8, 0.5, 0.4, seed=3)
    assert np.array_equal(rm, rm2) and np.array_equal(cm, cm2)
    assert np.allclose(oracle.selected_epochs(rm, cm, 5, 8), np.arange(1, 401) * 8 / 40)
    full_r, full_c = synth.block_subsets(3, 64, 64, 1.0, 1.0, seed=0)
    assert all(int(m) == (1 << 64) - 1 for m in full_r) and all(int(m) == (1 << 64) - 1
                                                                 for m in full_c)


@pytest.mark.parametrize("M,N", [(1, 1), (2, 3)])
def test_selected_with_every_block_is_algorithm1(M, N):
    p, A = _tiny(n=8, n_ang=10, bins=13, M=M, N=N)
    ro, co = synth.block_offsets(10, 13, p.ncols, M, N)
    blocks = oracle.tiles(p.row_ptr, p.col, p.val, ro, co)
    mu = oracle.step_size(oracle.power_umax(A))
    x0 = synth.seeded_vector(p.ncols, 4)
    all_r, all_c = [(1 << M) - 1] * 6, [(1 << N) - 1] * 6
    x, r, _, hist = oracle.bsgd_selected(blocks, ro, co, p.y, mu, 30.0, 20, (p.H, p.W), all_r,
                                         all_c, x0=x0, record=True)
    _, _, ref = oracle.bsgd_tv(A, p.y, mu, 30.0, 6, 20, (p.H, p.W), x0=x0, record=True)
    for a, b in zip(hist, ref):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_selected_column_subsets_converge_to_least_squares():
    """All row blocks, half the column blocks per iteration, lam = 0.

    A fixed point must zero A_{J_j}^T (y - A x) for every column block, so
    the only limit is the least-squares solution (a library solve).
    """
    p, A = _tiny(n=5, n_ang=8, bins=9, M=2, N=2)
    assert np.linalg.matrix_rank(A.toarray()) == p.ncols
    xls = np.linalg.lstsq(A.toarray(), p.y, rcond=None)[0]
    ro, co = synth.block_offsets(8, 9, p.ncols, 2, 2)
    blocks = oracle.tiles(p.row_ptr, p.col, p.val, ro, co)
    mu = oracle.step_size(oracle.power_umax(A))
    rm, cm = synth.block_subsets(24000, 2, 2, 0.5, 1.0, seed=5)
    x, _, _ = oracle.bsgd_selected(blocks, ro, co, p.y, mu, 0.0, 0, (p.H, p.W), rm, cm)
    assert np.linalg.norm(x - xls) <= 1e-8 * np.linalg.norm(xls)


def test_selected_row_subsets_converge_on_consistent_data():
    """Half the row blocks per iteration, lam = 0, y = A x_true exactly.

    With row subsets a fixed point must zero every (A_{I_i}^{J_j})^T r_{I_i}
    separately, which only a consistent system allows; then the limit is
    x_true (full column rank).  With noisy y the iterates stay in a
    neighbourhood of the least-squares solution instead.
    """
    p, A = _tiny(n=5, n_ang=8, bins=9, M=2, N=2, noise=0.0)
    assert np.linalg.matrix_rank(A.toarray()) == p.ncols
    xt = p.x_true.ravel()
    ro, co = synth.block_offsets(8, 9, p.ncols, 2, 2)
    blocks = oracle.tiles(p.row_ptr, p.col, p.val, ro, co)
    mu = oracle.step_size(oracle.power_umax(A))
    rm, cm = synth.block_subsets(20000, 2, 2, 1.0, 0.5, seed=5)
    x, _, _ = oracle.bsgd_selected(blocks, ro, co, p.y, mu, 0.0, 0, (p.H, p.W), rm, cm)
    assert np.linalg.norm(x - xt) <= 1e-8 * np.linalg.norm(xt)
    pn, An = _tiny(n=5, n_ang=8, bins=9, M=2, N=2, noise=0.05)
    bn = oracle.tiles(pn.row_ptr, pn.col, pn.val, ro, co)
    xls = np.linalg.lstsq(An.toarray(), pn.y, rcond=None)[0]
    xn, _, _ = oracle.bsgd_selected(bn, ro, co, pn.y, mu, 0.0, 0, (pn.H, pn.W), rm[:6000],
                                    cm[:6000])
    err = np.linalg.norm(xn - xls) / np.linalg.norm(xls)
    assert 1e-6 < err < 0.05


def test_selected_leaves_unselected_blocks_and_rows():
    """lam = 0: x outside the drawn column blocks and r outside the drawn row blocks stay put;
    the kept products of the drawn pairs equal dense block products of the old x."""
    p, A = _tiny(n=8, n_ang=12, bins=11, M=3, N=4)
    ro, co = synth.block_offsets(12, 11, p.ncols, 3, 4)
    blocks = oracle.tiles(p.row_ptr, p.col, p.val, ro, co)
    D = A.toarray()
    mu = oracle.step_size(oracle.power_umax(A))
    x, r, Z = oracle.selected_initial_state(blocks, ro, co, p.y, synth.seeded_vector(p.ncols, 9))
    rm, cm = synth.block_subsets(5, 3, 4, 0.5, 0.34, seed=8)
    for t in range(5):
        xn, rn, Zn = oracle.selected_iteration(blocks, ro, co, p.y, x, r, Z, mu, 0.0, 0,
                                               (p.H, p.W), int(rm[t]), int(cm[t]))
        I = oracle.mask_members(int(rm[t]), 3)
        J = oracle.mask_members(int(cm[t]), 4)
        for j in range(4):
            sl = slice(int(co[j]), int(co[j + 1]))
            if j in J:
                g = sum(2.0 * D[int(ro[i]):int(ro[i + 1]), sl].T @ r[int(ro[i]):int(ro[i + 1])]
                        for i in I)
                assert np.allclose(xn[sl], x[sl] + mu * g, rtol=0, atol=1e-12)
            else:
                assert np.array_equal(xn[sl], x[sl])
        for i in range(3):
            rs = slice(int(ro[i]), int(ro[i + 1]))
            if i in I:
                for j in J:
                    sl = slice(int(co[j]), int(co[j + 1]))
                    assert np.allclose(Zn[j, rs], D[rs, sl] @ x[sl], rtol=0, atol=1e-12)
                assert np.allclose(rn[rs], p.y[rs] - Zn[:, rs].sum(axis=0), rtol=0, atol=1e-12)
            else:
                assert np.array_equal(rn[rs], r[rs]) and np.array_equal(Zn[:, rs], Z[:, rs])
        x, r, Z = xn, rn, Zn

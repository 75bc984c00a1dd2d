"""ISTA / GD epochs and iterations over drawn block subsets against the FP64 oracle (GPU)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import (ITERATE_REL, PRODUCT_REL, f32, matrix, mu_for, plan_for, problem,
                         ragged_problem, rel_l2)

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _cases():
    return {
        "c1": lambda: problem("c1_64"),
        "medium": lambda: problem(None, H=192, W=192, n_ang=180, bins=273, M=4, N=4, seed=7),
        # non-square image, 3 x 5 uneven blocks, ragged tiles and view groups
        "ragged": ragged_problem,
    }


def _y(p):
    return f32(p.y).astype(np.float64)


# --------------------------------------------------------------------------
# ISTA and GD (bsgd_state_set_method)
# --------------------------------------------------------------------------

def _run_method(p, plan, method, mu, lam, epochs, K, fused=False, x0=None):
    import paper_1812_01307_amd as bsgd
    st = bsgd.bsgd_state_create(plan, 1)
    if fused:
        bsgd.bsgd_state_attach_fused(st, bsgd.bsgd_fused_create(plan))
    bsgd.bsgd_state_set_method(st, method)
    bsgd.bsgd_state_init(st, _dev(f32(p.y)), None if x0 is None else _dev(f32(x0)))
    xs = []
    for _ in range(epochs):
        bsgd.bsgd_run_epochs(st, mu, lam, 1, K)
        xs.append(_host(bsgd.bsgd_get_x(st)))
    return xs, st


@pytest.mark.parametrize("name", ["c1", "medium", "ragged"])
@pytest.mark.parametrize("form", ["rows", "staged", "fused"])
def test_ista_trajectory_matches_oracle(name, form):
    import paper_1812_01307_amd as bsgd
    p = _cases()[name]()
    plan = plan_for(p, staged=form == "staged")
    mu = float(np.float32(mu_for(p)))
    lam, E = 5.0, 12
    _, _, ref = oracle.ista_tv(matrix(p), _y(p), mu, lam, E, 20, (p.H, p.W), record=True)
    xs, st = _run_method(p, plan, bsgd.BSGD_METHOD_ISTA, mu, lam, E, 20, fused=form == "fused")
    errs = [rel_l2(a, b) for a, b in zip(xs, ref)]
    assert max(errs) <= ITERATE_REL, (max(errs), int(np.argmax(errs)))
    # the state keeps r = y - A x of the iterate before the last one
    r = _host(bsgd.bsgd_get_r(st))
    assert rel_l2(r, _y(p) - oracle.forward(matrix(p), ref[-2])) <= ITERATE_REL


@pytest.mark.parametrize("fused", [False, True])
def test_ista_and_gd_on_c1_whole_runs(fused):
    """100 epochs of ISTA at the workload's lambda and a lambda the prox moves, and of GD."""
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    A, y = matrix(p), _y(p)
    for lam in (p.lam, 200.0):
        _, _, ref = oracle.ista_tv(A, y, mu, lam, p.epochs, p.prox_iters, (p.H, p.W), record=True)
        xs, _ = _run_method(p, plan, bsgd.BSGD_METHOD_ISTA, mu, lam, p.epochs, p.prox_iters,
                            fused=fused)
        assert max(rel_l2(a, b) for a, b in zip(xs, ref)) <= ITERATE_REL, lam
    _, _, ref = oracle.gd(A, y, mu, p.epochs, record=True)
    xs, _ = _run_method(p, plan, bsgd.BSGD_METHOD_ISTA, mu, 0.0, p.epochs, 0, fused=fused)
    assert max(rel_l2(a, b) for a, b in zip(xs, ref)) <= ITERATE_REL


def test_methods_alternate_on_one_state():
    """BSGD epochs, then ISTA epochs from the reached iterate, on the block store and on the
    single-pass store (two single-direction passes per ISTA epoch); the two forms agree to
    FP32 rounding."""
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    lam = 20.0
    A, y = matrix(p), _y(p)
    xb, _, refb = oracle.bsgd_tv(A, y, mu, lam, 6, 20, (p.H, p.W), record=True)
    _, _, refi = oracle.ista_tv(A, y, mu, lam, 6, 20, (p.H, p.W), x0=xb, record=True)
    for fused in (False, True):
        st = bsgd.bsgd_state_create(plan, 1)
        if fused:
            F = bsgd.bsgd_fused_create(plan)
            bsgd.bsgd_state_attach_fused(st, F)
        bsgd.bsgd_state_init(st, _dev(f32(p.y)))
        bsgd.bsgd_run_epochs(st, mu, lam, 6, 20)
        assert rel_l2(_host(bsgd.bsgd_get_x(st)), refb[-1]) <= ITERATE_REL
        bsgd.bsgd_state_set_method(st, bsgd.BSGD_METHOD_ISTA)
        xs = []
        for _ in range(6):
            bsgd.bsgd_run_epochs(st, mu, lam, 1, 20)
            xs.append(_host(bsgd.bsgd_get_x(st)))
        assert max(rel_l2(a, b) for a, b in zip(xs, refi)) <= ITERATE_REL, fused
        _, n, _ = bsgd.bsgd_get_stats(st)
        assert n == 12
    xa, _ = _run_method(p, plan, bsgd.BSGD_METHOD_ISTA, mu, lam, 5, 20, fused=False)
    xf, _ = _run_method(p, plan, bsgd.BSGD_METHOD_ISTA, mu, lam, 5, 20, fused=True)
    assert max(rel_l2(a, b) for a, b in zip(xf, xa)) <= 1e-6


def test_ista_batch_state_matches_oracle_per_rhs():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    S, lam, E = 4, 20.0, 8
    rng = np.random.default_rng(31)
    Y = f32(p.y[:, None] * (1.0 + 0.1 * rng.standard_normal((1, S))))
    st = bsgd.bsgd_state_create(plan, S)
    bsgd.bsgd_state_set_method(st, bsgd.BSGD_METHOD_ISTA)
    bsgd.bsgd_state_init(st, _dev(Y))
    bsgd.bsgd_run_epochs(st, mu, lam, E, 20)
    X = _host(bsgd.bsgd_get_x(st)).reshape(p.ncols, S)
    A = matrix(p)
    for j in range(S):
        xr, _ = oracle.ista_tv(A, Y[:, j].astype(np.float64), mu, lam, E, 20, (p.H, p.W))
        assert rel_l2(X[:, j], xr) <= ITERATE_REL, j


def test_set_method_validation():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    st = bsgd.bsgd_state_create(plan_for(p), 1)
    with pytest.raises(bsgd.BsgdError):
        bsgd.bsgd_state_set_method(st, 2)


@pytest.mark.parametrize("fused", [False, True])
def test_ista_full_size_sampled(fused):
    """512 x 512, 720 x 729 rays (the bench's launch: single-pass store or row kernels): one
    GD epoch from a seeded x0, sampled rays of the residual and pixels of the new iterate
    against one-by-one FP64 sums (the residual is recomputed in FP64)."""
    import paper_1812_01307_amd as bsgd
    p = problem("c2_512")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    rng = np.random.default_rng(41)
    x0 = f32(rng.random(p.ncols))
    st = bsgd.bsgd_state_create(plan, 1)
    if fused:
        F = bsgd.bsgd_fused_create(plan)
        bsgd.bsgd_state_attach_fused(st, F)
    bsgd.bsgd_state_set_method(st, bsgd.BSGD_METHOD_ISTA)
    bsgd.bsgd_state_init(st, _dev(f32(p.y)), _dev(x0))
    bsgd.bsgd_run_epochs(st, mu, 0.0, 1, 0)
    x1 = _host(bsgd.bsgd_get_x(st))
    r_gpu = _host(bsgd.bsgd_get_r(st))
    A = oracle.as_matrix(p.row_ptr, p.col, f32(p.val).astype(np.float64), p.ncols)
    r = _y(p) - A @ x0.astype(np.float64)
    absr = np.abs(A) @ np.abs(x0.astype(np.float64)) + np.abs(_y(p))
    rows = rng.choice(p.nrows, 4000, replace=False)
    assert np.all(np.abs(r_gpu[rows] - r[rows]) <= PRODUCT_REL * absr[rows] + 1e-30)
    tp, tc, tv = p.ensure_transpose()
    for j in rng.choice(p.ncols, 2000, replace=False):
        a, b = tp[j], tp[j + 1]
        v = np.asarray(tv[a:b], np.float32).astype(np.float64)
        c = tc[a:b]
        g = 2.0 * float(np.dot(v, r[c]))
        bound = 2.0 * float(np.dot(np.abs(v), absr[c]))
        # the device residual and the sum over it each contribute up to PRODUCT_REL
        tol = 2 * PRODUCT_REL * mu * bound + 1e-6 * (abs(x0[j]) + abs(x1[j]))
        assert abs(x1[j] - (x0[j] + mu * g)) <= tol


# --------------------------------------------------------------------------
# Drawn block subsets (bsgd_run_selected)
# --------------------------------------------------------------------------

def _blocks(p):
    """The M x N blocks of A with the FP32-rounded values the device holds."""
    return oracle.tiles(p.row_ptr, p.col, f32(p.val).astype(np.float64), p.row_off, p.col_off)


def _selected_state(p, plan, x0=None):
    import paper_1812_01307_amd as bsgd
    st = bsgd.bsgd_state_create(plan, 1, flags=bsgd.BSGD_STATE_BLOCK_SELECT)
    bsgd.bsgd_state_init(st, _dev(f32(p.y)), None if x0 is None else _dev(f32(x0)))
    return st


def _run_selected(st, mu, lam, rm, cm, K):
    import paper_1812_01307_amd as bsgd
    xs = []
    for t in range(len(rm)):
        bsgd.bsgd_run_selected(st, mu, lam, rm[t:t + 1], cm[t:t + 1], K)
        xs.append(_host(bsgd.bsgd_get_x(st)))
    return xs


@pytest.mark.parametrize("name,alpha,gamma", [("c1", 0.5, 0.5), ("medium", 0.5, 0.5),
                                              ("ragged", 0.4, 0.67), ("ragged", 1.0, 0.34)])
@pytest.mark.parametrize("lam", [0.0, 5.0])
def test_selected_trajectory_matches_oracle(name, alpha, gamma, lam):
    import paper_1812_01307_amd as bsgd
    p = _cases()[name]()
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    T = 24
    rm, cm = synth.block_subsets(T, p.M, p.N, alpha, gamma, seed=17)
    x0 = f32(synth.seeded_vector(p.ncols, 5, 0.1))
    _, _, _, ref = oracle.bsgd_selected(_blocks(p), p.row_off, p.col_off, _y(p), mu, lam, 20,
                                        (p.H, p.W), rm, cm, x0=x0.astype(np.float64),
                                        record=True)
    st = _selected_state(p, plan, x0)
    xs = _run_selected(st, mu, lam, rm, cm, 20)
    errs = [rel_l2(a, b) for a, b in zip(xs, ref)]
    assert max(errs) <= ITERATE_REL, (max(errs), int(np.argmax(errs)))
    _, n, _ = bsgd.bsgd_get_stats(st)
    assert n == T


def test_selected_c1_visible_tv_and_all_blocks():
    """Every block drawn: an iteration is an epoch of Algorithm 1 (oracle bsgd_tv); and a
    whole run at a lambda the prox moves with half the blocks drawn."""
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    A, y = matrix(p), _y(p)
    full = np.full(30, 3, np.uint64)
    _, _, ref = oracle.bsgd_tv(A, y, mu, 200.0, 30, 20, (p.H, p.W), record=True)
    xs = _run_selected(_selected_state(p, plan), mu, 200.0, full, full, 20)
    assert max(rel_l2(a, b) for a, b in zip(xs, ref)) <= ITERATE_REL
    rm, cm = synth.block_subsets(100, 2, 2, 0.5, 0.5, seed=23)
    _, _, _, ref = oracle.bsgd_selected(_blocks(p), p.row_off, p.col_off, y, mu, 200.0, 20,
                                        (p.H, p.W), rm, cm, record=True)
    st = _selected_state(p, plan)
    bsgd.bsgd_run_selected(st, mu, 200.0, rm, cm, 20)
    assert rel_l2(_host(bsgd.bsgd_get_x(st)), ref[-1]) <= ITERATE_REL


def test_selected_load_recomputes_kept_products():
    """bsgd_state_load sets the kept products from the loaded x: a resumed run equals the
    oracle started from (x, r, Z = block products of x)."""
    import paper_1812_01307_amd as bsgd
    p = ragged_problem()
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    rng = np.random.default_rng(3)
    x = f32(rng.random(p.ncols))
    r = f32(rng.standard_normal(p.nrows))
    rm, cm = synth.block_subsets(10, p.M, p.N, 0.6, 0.67, seed=29)
    blocks = _blocks(p)
    _, _, Z = oracle.selected_initial_state(blocks, p.row_off, p.col_off, _y(p),
                                            x.astype(np.float64))
    _, _, _, ref = oracle.bsgd_selected(blocks, p.row_off, p.col_off, _y(p), mu, 5.0, 20,
                                        (p.H, p.W), rm, cm,
                                        state=(x.astype(np.float64), r.astype(np.float64), Z),
                                        record=True)
    st = _selected_state(p, plan)
    bsgd.bsgd_state_load(st, _dev(x), _dev(r), 0)
    xs = _run_selected(st, mu, 5.0, rm, cm, 20)
    assert max(rel_l2(a, b) for a, b in zip(xs, ref)) <= ITERATE_REL


def test_selected_validation():
    import paper_1812_01307_amd as bsgd
    p = ragged_problem()
    plan = plan_for(p)
    st = bsgd.bsgd_state_create(plan, 1)
    bsgd.bsgd_state_init(st, _dev(f32(p.y)))
    with pytest.raises(bsgd.BsgdError):          # no kept products in this state
        bsgd.bsgd_run_selected(st, 1e-4, 0.0, [1], [1], 0)
    st = _selected_state(p, plan)
    for rows, cols in (([0], [1]), ([1], [0]), ([1 << 3], [1]), ([1], [1 << 5])):
        with pytest.raises(bsgd.BsgdError):
            bsgd.bsgd_run_selected(st, 1e-4, 0.0, rows, cols, 0)
    with pytest.raises(bsgd.BsgdError):
        bsgd.bsgd_run_selected(st, 1e-4, 1.0, [1], [1], 0)   # lam > 0 needs prox iterations
    with pytest.raises(bsgd.BsgdError):
        bsgd.bsgd_state_workspace_size(plan, 4, bsgd.BSGD_STATE_BLOCK_SELECT)
    _, n, _ = bsgd.bsgd_get_stats(st)
    assert n == 0

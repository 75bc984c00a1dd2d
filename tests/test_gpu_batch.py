"""Several right-hand sides (batches and volumes), slot restarts and HIP graphs (GPU)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import ITERATE_REL, f32, matrix, mu_for, plan_for, problem, rel_l2

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _batch_inputs(p, S):
    """S sinograms on p's geometry: the problem's y, other seeded phantoms, a zero slot."""
    ys = [p.y]
    for j in range(1, S - 1):
        x = synth.ellipse_phantom(p.H, p.W, 10, 500 + j).ravel()
        ys.append(matrix(p) @ x)
    ys.append(np.zeros(p.nrows))
    return np.stack(ys)  # (S, r)


def _to_rows(M):
    """(S, n) per-RHS arrays -> the [n][S] row-major device layout."""
    return np.ascontiguousarray(np.asarray(M).T)


@pytest.mark.parametrize("schedule", [0, 1])
def test_batch_state_matches_oracle_per_slot(schedule):
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    S = 4
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    Y = f32(_batch_inputs(p, S)).astype(np.float64)
    lam = np.array([p.lam, 20.0, 0.0, 200.0])
    st = bsgd.bsgd_state_create(plan, S)
    bsgd.bsgd_state_set_prox_schedule(st, schedule)
    bsgd.bsgd_state_init(st, _dev(f32(_to_rows(Y)).ravel()))
    bsgd.bsgd_state_set_lambda(st, lam)
    _, _, ref = oracle.bsgd_tv_multi(matrix(p), Y, mu, lam, 25, p.prox_iters, (p.H, p.W),
                                     volume=False, record=True)
    for k in range(25):
        bsgd.bsgd_run_epochs(st, mu, -1.0, 1, p.prox_iters)
        X = _host(bsgd.bsgd_get_x(st)).reshape(p.ncols, S).T
        for j in range(S - 1):
            assert rel_l2(X[j], ref[k][j]) <= ITERATE_REL, (k, j)
        assert np.max(np.abs(X[S - 1])) == 0.0
    rn = bsgd.bsgd_get_stats_rhs(st)
    R = _host(bsgd.bsgd_get_r(st)).reshape(p.nrows, S).T
    for j in range(S):
        assert abs(rn[j] - float(np.sum(R[j] ** 2))) <= 1e-9 * max(rn[j], 1e-30)


def test_volume_state_matches_oracle():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    S = 8
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    A = matrix(p)
    X_true = np.stack([synth.ellipse_phantom(p.H, p.W, 10, 1000 + s).ravel() for s in range(S)])
    Y = f32(np.asarray(A @ X_true.T).T).astype(np.float64)
    lam, K, E = 20.0, 20, 15
    st = bsgd.bsgd_state_create(plan, S, flags=bsgd.BSGD_STATE_VOLUME)
    bsgd.bsgd_state_init(st, _dev(f32(_to_rows(Y)).ravel()))
    _, _, ref = oracle.bsgd_tv_multi(A, Y, mu, lam, E, K, (p.H, p.W), volume=True, record=True)
    for k in range(E):
        bsgd.bsgd_run_epochs(st, mu, lam, 1, K)
        X = _host(bsgd.bsgd_get_x(st)).reshape(p.ncols, S).T
        assert rel_l2(X, ref[k]) <= ITERATE_REL, k


@pytest.mark.parametrize("name,S", [("ragged", 64), ("c1", 128), ("c1", 4), ("ragged", 32)])
def test_volume_prox_chunks_match_oracle(name, S):
    """Slice counts below, at and above the 32-slice chunks of the 3-D prox; ragged pixel tiles."""
    import paper_1812_01307_amd as bsgd
    from gpu_helpers import ragged_problem
    p = ragged_problem() if name == "ragged" else problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    A = matrix(p)
    X_true = np.stack([synth.ellipse_phantom(p.H, p.W, 6, 2000 + s).ravel() for s in range(S)])
    Y = f32(np.asarray(A @ X_true.T).T).astype(np.float64)
    lam, K, E = 30.0, 12, 3
    st = bsgd.bsgd_state_create(plan, S, flags=bsgd.BSGD_STATE_VOLUME)
    bsgd.bsgd_state_init(st, _dev(f32(_to_rows(Y)).ravel()))
    _, _, ref = oracle.bsgd_tv_multi(A, Y, mu, lam, E, K, (p.H, p.W), volume=True, record=True)
    for k in range(E):
        bsgd.bsgd_run_epochs(st, mu, lam, 1, K)
        X = _host(bsgd.bsgd_get_x(st)).reshape(p.ncols, S).T
        assert rel_l2(X, ref[k]) <= ITERATE_REL, k


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 7, 20])
def test_volume_prox_schedules_agree_bitwise(K):
    """The temporally blocked 3-D prox (launches of up to three iterations on
    recomputed halos, row segments of 64) against the per-iteration kernel:
    same per-voxel arithmetic, so bitwise equal; on a ragged image taller than
    one row segment, with slice and column counts that are not multiples of
    the block's owned cells; and against the oracle."""
    import paper_1812_01307_amd as bsgd
    p = problem(None, H=150, W=70, n_ang=30, bins=121, M=2, N=3, seed=31, lam=0.0)
    S = 32
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    A = matrix(p)
    X_true = np.stack([synth.ellipse_phantom(p.H, p.W, 6, 3000 + s).ravel() for s in range(S)])
    Y = f32(np.asarray(A @ X_true.T).T).astype(np.float64)
    lam, E = 40.0, 3
    xs = []
    for schedule in (1, 0):
        st = bsgd.bsgd_state_create(plan, S, flags=bsgd.BSGD_STATE_VOLUME)
        bsgd.bsgd_state_set_prox_schedule(st, schedule)
        bsgd.bsgd_state_init(st, _dev(f32(_to_rows(Y)).ravel()))
        bsgd.bsgd_run_epochs(st, mu, lam, E, K)
        xs.append(_host(bsgd.bsgd_get_x(st)))
    assert np.array_equal(xs[0], xs[1])
    if K in (3, 20):
        _, _, ref = oracle.bsgd_tv_multi(A, Y, mu, lam, E, K, (p.H, p.W), volume=True,
                                         record=True)
        X = xs[1].reshape(p.ncols, S).T
        assert rel_l2(X, ref[-1]) <= ITERATE_REL


def test_slot_restart_leaves_other_slots_bitwise_unchanged():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    S = 4
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    Y = f32(_batch_inputs(p, S))
    lam = [20.0, 20.0, 5.0, 0.0]
    y_new = f32(matrix(p) @ synth.ellipse_phantom(p.H, p.W, 10, 77).ravel())
    x0 = f32(np.random.default_rng(3).random(p.ncols))

    def run(restart):
        st = bsgd.bsgd_state_create(plan, S)
        bsgd.bsgd_state_init(st, _dev(_to_rows(Y).ravel()))
        bsgd.bsgd_state_set_lambda(st, lam)
        bsgd.bsgd_run_epochs(st, mu, -1.0, 5, 20)
        if restart:
            bsgd.bsgd_state_set_rhs(st, 2, _dev(y_new), _dev(x0))
        bsgd.bsgd_run_epochs(st, mu, -1.0, 5, 20)
        return _host(bsgd.bsgd_get_x(st)).reshape(p.ncols, S).T

    a, b = run(False), run(True)
    for j in (0, 1, 3):
        assert np.array_equal(a[j], b[j]), j
    # the restarted slot matches a fresh 5-epoch run of the same data and start
    st = bsgd.bsgd_state_create(plan, S)
    Y2 = np.zeros_like(Y)
    Y2[2] = y_new
    X0 = np.zeros((S, p.ncols), np.float32)
    X0[2] = x0
    bsgd.bsgd_state_init(st, _dev(_to_rows(Y2).ravel()), _dev(_to_rows(X0).ravel()))
    bsgd.bsgd_state_set_lambda(st, lam)
    bsgd.bsgd_run_epochs(st, mu, -1.0, 5, 20)
    fresh = _host(bsgd.bsgd_get_x_rhs(st, 2))
    # same data and start; the restart's initial residual is summed by the
    # one-RHS kernel, so agreement is to rounding, not bitwise
    assert rel_l2(b[2], fresh) <= 1e-6
    # ... and it agrees with the oracle
    A = matrix(p)
    x, r = oracle.initial_state(A, y_new.astype(np.float64), x0.astype(np.float64))
    x, _ = oracle.bsgd_tv(A, y_new.astype(np.float64), mu, 5.0, 5, 20, (p.H, p.W), state=(x, r))
    assert rel_l2(fresh, x) <= ITERATE_REL


@pytest.mark.parametrize("S,flags", [(1, 0), (4, 0), (8, 1)])
def test_graph_replay_is_bitwise_equal(S, flags):
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    Y = f32(_batch_inputs(p, S)) if S > 1 else f32(p.y[None])
    y = _dev(_to_rows(Y).ravel())
    lam = 20.0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        st = bsgd.bsgd_state_create(plan, S, flags=flags)
        bsgd.bsgd_state_init(st, y)
        bsgd.bsgd_run_epochs(st, mu, lam, 10, 20)
        ref = _host(bsgd.bsgd_get_x(st))
        st2 = bsgd.bsgd_state_create(plan, S, flags=flags)
        bsgd.bsgd_state_init(st2, y)
        g = bsgd.bsgd_graph_create(st2, mu, lam, 2, 20)
        for k in range(5):
            bsgd.bsgd_graph_launch(g)
            s.synchronize()
            # eager work between replays
            torch.zeros(1000, device="cuda").add_(1.0)
        out = _host(bsgd.bsgd_get_x(st2))
        _, ep, _ = bsgd.bsgd_get_stats(st2)
    assert ep == 10
    assert np.array_equal(out, ref)
    with pytest.raises(bsgd.BsgdError, match="even"):
        bsgd.bsgd_graph_create(st2, mu, lam, 3, 20, stream=s)


@pytest.mark.parametrize("S", [4, 8, 16, 64, 256, 512])
def test_batch_widths_match_oracle(S):
    """Every lane split of the several-RHS products (entry groups, RHS chunks)."""
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    Y = f32(_batch_inputs(p, S)).astype(np.float64)
    lam = np.random.default_rng(S).uniform(0.0, 40.0, S)
    lam[S // 2] = 0.0
    st = bsgd.bsgd_state_create(plan, S)
    bsgd.bsgd_state_init(st, _dev(f32(_to_rows(Y)).ravel()))
    bsgd.bsgd_state_set_lambda(st, lam)
    lam32 = lam.astype(np.float32).astype(np.float64)
    _, _, ref = oracle.bsgd_tv_multi(matrix(p), Y, mu, lam32, 3, 10, (p.H, p.W), volume=False,
                                     record=True)
    for k in range(3):
        bsgd.bsgd_run_epochs(st, mu, -1.0, 1, 10)
        X = _host(bsgd.bsgd_get_x(st)).reshape(p.ncols, S).T
        errs = [rel_l2(X[j], ref[k][j]) for j in range(S - 1)]
        assert max(errs) <= ITERATE_REL, (k, int(np.argmax(errs)), max(errs))
        assert np.max(np.abs(X[S - 1])) == 0.0

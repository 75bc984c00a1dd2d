"""Single-pass epochs (tile-sliced store) against the FP64 oracle (GPU, through the C ABI)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import (ITERATE_REL, PRODUCT_REL, abs_matrix, f32, matrix, mu_for, plan_for,
                         problem, ragged_problem, rel_l2)

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _cases():
    return {
        "c1": lambda: problem("c1_64"),
        # many slices per (tile, chunk) unit, full and partial 64 x 64 tiles
        "medium": lambda: problem(None, H=176, W=176, n_ang=180, bins=273, M=4, N=4, seed=7),
        # most rays miss the image (empty rows and empty chunks)
        "wide": lambda: problem(None, H=64, W=64, n_ang=16, bins=2500, M=2, N=2, seed=8),
        # non-square, ragged 8 x 8 and 64 x 64 tiles, ragged view groups
        "ragged": ragged_problem,
        # a single pixel row and a single tile column
        "strip": lambda: problem(None, H=1, W=40, n_ang=12, bins=45, M=2, N=2, seed=9, lam=0.0),
    }


def _segments(p, view_len):
    """Independent count of (ray, 64 x 64 tile) pairs with an entry, from the host CSR."""
    rows = np.repeat(np.arange(p.nrows, dtype=np.int64), np.diff(p.row_ptr))
    col = np.asarray(p.col, np.int64)
    s, t = col // p.W, col % p.W
    ftw = (p.W + 63) // 64
    key = rows * (((p.H + 63) // 64) * ftw) + (s // 64) * ftw + t // 64
    return len(np.unique(key))


def _fused(plan, chunks=0, waves=None, flags=0):
    import paper_1812_01307_amd as bsgd
    F = bsgd.bsgd_fused_create(plan, chunks, flags)
    if waves:
        bsgd.bsgd_fused_set_waves(F, waves)
    return F


@pytest.mark.parametrize("name", ["c1", "medium", "wide", "ragged", "strip"])
@pytest.mark.parametrize("view_len", [None, 0])
def test_fused_products_match_oracle(name, view_len):
    import paper_1812_01307_amd as bsgd
    p = _cases()[name]()
    plan = plan_for(p, view_len=view_len)
    F = _fused(plan)
    tiles, chunks, segs, slices, entries, cbytes = bsgd.bsgd_fused_shape(F)
    assert cbytes == 1  # rays: steps between successive pixels of a tile are below 256
    assert tiles == ((p.H + 63) // 64) * ((p.W + 63) // 64)
    assert segs == _segments(p, view_len)
    assert slices * 64 >= segs and entries >= p.nnz and entries % 256 == 0
    A, Aabs = matrix(p), abs_matrix(p)
    rng = np.random.default_rng(11)
    x = f32(rng.random(p.ncols))
    xa = f32(rng.standard_normal(p.ncols))
    r = f32(rng.standard_normal(p.nrows))
    y = f32(rng.standard_normal(p.nrows))
    mu = 1.3e-3
    ax, g = bsgd.bsgd_fused_apply(F, _dev(x), _dev(r))
    res, step = bsgd.bsgd_fused_apply(F, _dev(x), _dev(r), y=_dev(y), xadd=_dev(xa), mu=mu)
    ax, g, res, step = map(_host, (ax, g, res, step))
    bound_f = PRODUCT_REL * (Aabs @ np.abs(x)) + 1e-30
    bound_b = PRODUCT_REL * 2 * (Aabs.T @ np.abs(r)) + 1e-30
    ref_ax = oracle.forward(A, x)
    ref_g = oracle.backproject(A, r)
    assert np.all(np.abs(ax - ref_ax) <= bound_f)
    assert np.all(np.abs(g - ref_g) <= bound_b)
    assert np.all(np.abs(res - (y - ref_ax)) <= bound_f + 1e-7 * np.abs(y))
    assert np.all(np.abs(step - (xa + mu * ref_g)) <= mu * bound_b + 1e-7 * np.abs(xa))
    # every chunk count and wave count gives the same sums up to rounding
    groups = -(-p.nrows // (8 * p.bins)) if view_len is None else -(-p.nrows // 64)
    for q, w in ((1, 2), (groups, 8), (max(1, groups // 2), 4)):
        F2 = _fused(plan, q, w)
        ax2, g2 = bsgd.bsgd_fused_apply(F2, _dev(x), _dev(r))
        assert np.all(np.abs(_host(ax2) - ref_ax) <= bound_f)
        assert np.all(np.abs(_host(g2) - ref_g) <= bound_b)
    # 16-bit addresses give the same addresses, so the same sums bitwise
    Fw = _fused(plan, flags=bsgd.BSGD_FUSED_WIDE)
    assert bsgd.bsgd_fused_shape(Fw)[5] == 2
    axw, gw = bsgd.bsgd_fused_apply(Fw, _dev(x), _dev(r))
    ax0, g0 = bsgd.bsgd_fused_apply(F, _dev(x), _dev(r))
    assert np.array_equal(_host(axw), _host(ax0)) and np.array_equal(_host(gw), _host(g0))


def _run(p, plan, F, mu, lam, epochs, K, vt=0):
    import paper_1812_01307_amd as bsgd
    st = bsgd.bsgd_state_create(plan, 1, vt)
    if F is not None:
        bsgd.bsgd_state_attach_fused(st, F)
    bsgd.bsgd_state_init(st, _dev(f32(p.y)))
    xs = []
    for _ in range(epochs):
        bsgd.bsgd_run_epochs(st, mu, lam, 1, K)
        xs.append(_host(bsgd.bsgd_get_x(st)))
    return xs, st


@pytest.mark.parametrize("name", ["c1", "medium", "wide", "ragged"])
@pytest.mark.parametrize("view_len", [None, 0])
def test_fused_trajectory_matches_oracle(name, view_len):
    import paper_1812_01307_amd as bsgd
    p = _cases()[name]()
    plan = plan_for(p, view_len=view_len)
    F = _fused(plan)
    mu = float(np.float32(mu_for(p)))
    lam, E = 5.0, 12
    _, _, ref = oracle.bsgd_tv(matrix(p), f32(p.y).astype(np.float64), mu, lam, E, 20,
                               (p.H, p.W), record=True)
    xs, st = _run(p, plan, F, mu, lam, E, 20)
    errs = [rel_l2(a, b) for a, b in zip(xs, ref)]
    assert max(errs) <= ITERATE_REL, (max(errs), int(np.argmax(errs)))
    # the residual carried to the next epoch is y - A x_{E-1}
    r = _host(bsgd.bsgd_get_r(st))
    x_prev = ref[-2]
    r_ref = f32(p.y).astype(np.float64) - oracle.forward(matrix(p), x_prev)
    assert rel_l2(r, r_ref) <= ITERATE_REL
    # detached, the same state runs the row kernels again
    xr, _ = _run(p, plan, None, mu, lam, E, 20)
    assert max(rel_l2(a, b) for a, b in zip(xs, xr)) <= 1e-6


def test_fused_c1_lambda_zero_and_visible_tv():
    """Whole c1 runs (100 epochs) at the workload's lambda, lambda = 0 and a lambda the prox moves."""
    p = problem("c1_64")
    plan = plan_for(p)
    F = _fused(plan)
    mu = float(np.float32(mu_for(p)))
    for lam in (p.lam, 0.0, 200.0):
        _, _, ref = oracle.bsgd_tv(matrix(p), f32(p.y).astype(np.float64), mu, lam, p.epochs,
                                   p.prox_iters, (p.H, p.W), record=True)
        xs, _ = _run(p, plan, F, mu, lam, p.epochs, p.prox_iters)
        assert max(rel_l2(a, b) for a, b in zip(xs, ref)) <= ITERATE_REL, lam


def test_fused_fp16_values():
    import paper_1812_01307_amd as bsgd
    p = _cases()["medium"]()
    plan = plan_for(p, f16=True)
    F = _fused(plan)
    mu = float(np.float32(mu_for(p)))
    E = 10
    xs, _ = _run(p, plan, F, mu, 5.0, E, 20, vt=bsgd.BSGD_VAL_F16)
    vals = p.val.astype(np.float32).astype(np.float16).astype(np.float64)
    A16 = oracle.as_matrix(p.row_ptr, p.col, vals, p.ncols)
    _, _, ref = oracle.bsgd_tv(A16, f32(p.y).astype(np.float64), mu, 5.0, E, 20, (p.H, p.W),
                               record=True)
    assert max(rel_l2(a, b) for a, b in zip(xs, ref)) <= ITERATE_REL
    # products in FP16 values against the FP16-rounded matrix
    rng = np.random.default_rng(3)
    x = f32(rng.random(p.ncols))
    r = f32(rng.standard_normal(p.nrows))
    ax, g = bsgd.bsgd_fused_apply(F, _dev(x), _dev(r), vt=bsgd.BSGD_VAL_F16)
    Aabs = abs_matrix(p)
    assert np.all(np.abs(_host(ax) - A16 @ x) <= PRODUCT_REL * (Aabs @ np.abs(x)) + 1e-30)
    assert np.all(np.abs(_host(g) - 2 * (A16.T @ r))
                  <= PRODUCT_REL * 2 * (Aabs.T @ np.abs(r)) + 1e-30)


def test_fused_runs_are_bitwise_reproducible_and_graphs_replay_exactly():
    import paper_1812_01307_amd as bsgd
    p = _cases()["medium"]()
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    F = _fused(plan)
    a, _ = _run(p, plan, F, mu, 20.0, 6, 20)
    b, _ = _run(p, plan, F, mu, 20.0, 6, 20)
    assert all(np.array_equal(u, v) for u, v in zip(a, b))
    # a second store built from the same plan is identical, so are its results
    c, _ = _run(p, plan, _fused(plan), mu, 20.0, 6, 20)
    assert all(np.array_equal(u, v) for u, v in zip(a, c))
    # 6 epochs as 3 replays of a 2-epoch graph, with eager work between replays
    s = torch.cuda.Stream()
    st = bsgd.bsgd_state_create(plan)
    bsgd.bsgd_state_attach_fused(st, F)
    with torch.cuda.stream(s):
        bsgd.bsgd_state_init(st, _dev(f32(p.y)), stream=s)
        gr = bsgd.bsgd_graph_create(st, mu, 20.0, 2, 20, stream=s)
        for k in range(3):
            bsgd.bsgd_graph_launch(gr, stream=s)
            s.synchronize()
            x = _host(bsgd.bsgd_get_x(st, stream=s))
            assert np.array_equal(x, a[2 * k + 1]), k
            _ = torch.ones(1000, device="cuda").sum().item()


def test_graph_refuses_replay_after_state_changes():
    """A graph bakes in the iterate parity and the attached store: a replay after
    an odd eager epoch, or after the store was detached or swapped, is refused,
    and an even eager run in between keeps replays exact."""
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    F = _fused(plan)
    ref, _ = _run(p, plan, F, mu, 20.0, 8, 20)
    s = torch.cuda.Stream()
    st = bsgd.bsgd_state_create(plan)
    bsgd.bsgd_state_attach_fused(st, F)
    with torch.cuda.stream(s):
        bsgd.bsgd_state_init(st, _dev(f32(p.y)), stream=s)
        gr = bsgd.bsgd_graph_create(st, mu, 20.0, 2, 20, stream=s)
        bsgd.bsgd_graph_launch(gr, stream=s)
        bsgd.bsgd_run_epochs(st, mu, 20.0, 1, 20, stream=s)  # odd: buffers change parity
        with pytest.raises(bsgd.BsgdError, match="parity"):
            bsgd.bsgd_graph_launch(gr, stream=s)
        bsgd.bsgd_run_epochs(st, mu, 20.0, 1, 20, stream=s)  # parity restored
        bsgd.bsgd_graph_launch(gr, stream=s)  # epochs 5, 6
        s.synchronize()
        assert np.array_equal(_host(bsgd.bsgd_get_x(st, stream=s)), ref[5])
        # the graph keeps the store it captured alive
        assert gr.fused is F
        bsgd.bsgd_state_attach_fused(st, None)
        with pytest.raises(bsgd.BsgdError, match="configuration"):
            bsgd.bsgd_graph_launch(gr, stream=s)
        bsgd.bsgd_state_attach_fused(st, F)  # new partials buffer: still refused
        with pytest.raises(bsgd.BsgdError, match="configuration"):
            bsgd.bsgd_graph_launch(gr, stream=s)
        bsgd.bsgd_state_set_overlap(st, 2)
        gr2 = bsgd.bsgd_graph_create(st, mu, 20.0, 2, 20, stream=s)
        bsgd.bsgd_graph_launch(gr2, stream=s)  # epochs 7, 8
        s.synchronize()
        assert np.array_equal(_host(bsgd.bsgd_get_x(st, stream=s)), ref[7])


def test_fused_validation():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p)
    F = _fused(plan)
    other = plan_for(p)
    st = bsgd.bsgd_state_create(other)
    with pytest.raises(bsgd.BsgdError, match="another plan"):
        bsgd.bsgd_state_attach_fused(st, F)
    groups = -(-p.nrows // (8 * p.bins))
    with pytest.raises(bsgd.BsgdError, match="chunks"):
        bsgd.bsgd_fused_workspace_size(plan, groups + 1)
    with pytest.raises(bsgd.BsgdError, match="waves"):
        bsgd.bsgd_fused_set_waves(F, 3)
    st = bsgd.bsgd_state_create(plan)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(bsgd.BsgdError) as e:
        bsgd.bsgd_state_attach_fused(st, F, small)
    assert e.value.status == bsgd.BSGD_ERR_WORKSPACE
    bsgd.bsgd_state_attach_fused(st, F)
    bsgd.bsgd_state_attach_fused(st, None)


def test_fused_f16_state_needs_f16_store():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p, f16=True)
    F = _fused(plan)
    st16 = bsgd.bsgd_state_create(plan, 1, bsgd.BSGD_VAL_F16)
    bsgd.bsgd_state_attach_fused(st16, F)
    plain = plan_for(p)
    F32 = _fused(plain)
    st = bsgd.bsgd_state_create(plain, 1, bsgd.BSGD_VAL_F32)
    bsgd.bsgd_state_attach_fused(st, F32)


def test_fused_full_size_sampled():
    """512 x 512, 720 x 729 rays: the bench's store and launch, sampled rows and pixels."""
    import paper_1812_01307_amd as bsgd
    p = problem("c2_512")
    plan = plan_for(p)
    F = _fused(plan)
    tiles, chunks, segs, slices, entries, cbytes = bsgd.bsgd_fused_shape(F)
    assert tiles == 64 and segs > p.nrows and entries >= p.nnz and cbytes == 1
    rng = np.random.default_rng(12)
    x = f32(rng.random(p.ncols))
    r = f32(rng.standard_normal(p.nrows))
    ax, g = bsgd.bsgd_fused_apply(F, _dev(x), _dev(r))
    ax, g = _host(ax), _host(g)
    rows = rng.choice(p.nrows, 4000, replace=False)
    for k in rows:
        a, b = p.row_ptr[k], p.row_ptr[k + 1]
        v = p.val[a:b].astype(np.float32).astype(np.float64)
        c = p.col[a:b]
        ref = float(np.dot(v, x[c].astype(np.float64)))
        assert abs(ax[k] - ref) <= PRODUCT_REL * float(np.dot(np.abs(v), np.abs(x[c]))) + 1e-30
    tp, tc, tv = p.ensure_transpose()
    for j in rng.choice(p.ncols, 2000, replace=False):
        a, b = tp[j], tp[j + 1]
        v = np.asarray(tv[a:b], np.float32).astype(np.float64)
        c = tc[a:b]
        ref = 2.0 * float(np.dot(v, r[c].astype(np.float64)))
        assert abs(g[j] - ref) <= PRODUCT_REL * 2 * float(np.dot(np.abs(v), np.abs(r[c]))) + 1e-30


def test_fused_general_matrix_uses_wide_columns():
    """Rows that are not rays (random ascending columns): steps exceed 255, 16-bit columns."""
    import paper_1812_01307_amd as bsgd
    import synth
    rng = np.random.default_rng(17)
    H, W, nrows = 70, 45, 900
    ncols = H * W
    lens = rng.integers(0, 120, nrows)
    lens[::50] = 0  # some empty rows
    cols = [np.sort(rng.choice(ncols, n, replace=False)).astype(np.int32) for n in lens]
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate(cols).astype(np.int32)
    val = rng.random(len(col)) * 1.5
    tp, tc, tv = synth.transpose_csr(nrows, ncols, row_ptr, col, val)
    plan = bsgd.plan_from_host(nrows, ncols, row_ptr, col, val, tp, tc, tv, 3, 2,
                               [0, 300, 600, 900], [0, 1500, ncols], H, W, 1, view_len=0)
    F = _fused(plan)
    assert bsgd.bsgd_fused_shape(F)[5] == 2
    A = oracle.as_matrix(row_ptr, col, f32(val).astype(np.float64), ncols)
    Aabs = oracle.as_matrix(row_ptr, col, np.abs(f32(val).astype(np.float64)), ncols)
    x = f32(rng.random(ncols))
    r = f32(rng.standard_normal(nrows))
    ax, g = bsgd.bsgd_fused_apply(F, _dev(x), _dev(r))
    assert np.all(np.abs(_host(ax) - A @ x) <= PRODUCT_REL * (Aabs @ np.abs(x)) + 1e-30)
    assert np.all(np.abs(_host(g) - 2 * (A.T @ r)) <= PRODUCT_REL * 2 * (Aabs.T @ np.abs(r)) + 1e-30)
    # a few epochs against the oracle
    y = f32(A @ rng.random(ncols))
    mu = float(np.float32(oracle.step_size(oracle.power_umax(A))))
    _, _, ref = oracle.bsgd_tv(A, y.astype(np.float64), mu, 3.0, 8, 20, (H, W), record=True)
    st = bsgd.bsgd_state_create(plan)
    bsgd.bsgd_state_attach_fused(st, F)
    bsgd.bsgd_state_init(st, _dev(y))
    for k in range(8):
        bsgd.bsgd_run_epochs(st, mu, 3.0, 1, 20)
        assert rel_l2(_host(bsgd.bsgd_get_x(st)), ref[k]) <= ITERATE_REL, k


@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_fused_overlap_modes_agree_bitwise(name):
    """The ray half of the reduce on the second stream (modes 0, 1) or in order (mode 2)."""
    import paper_1812_01307_amd as bsgd
    p = _cases()[name]()
    plan = plan_for(p)
    F = _fused(plan)
    mu = float(np.float32(mu_for(p)))
    outs = []
    for mode in (0, 1, 2):
        st = bsgd.bsgd_state_create(plan, 1)
        bsgd.bsgd_state_attach_fused(st, F)
        bsgd.bsgd_state_set_overlap(st, mode)
        bsgd.bsgd_state_init(st, _dev(f32(p.y)))
        bsgd.bsgd_run_epochs(st, mu, 5.0, 9, 20)
        outs.append((_host(bsgd.bsgd_get_x(st)), _host(bsgd.bsgd_get_r(st))))
    for x, r in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and np.array_equal(r, outs[0][1])


def test_count_reuse_and_invalidation_give_identical_stores():
    """bsgd_fused_create reuses the segment count of bsgd_fused_workspace_size;
    a block export in between (which overwrites the plan's scratch) and a
    different chunk count force a recount.  Every store must be the same."""
    import ctypes
    import paper_1812_01307_amd as bsgd
    from paper_1812_01307_amd import capi
    p = _cases()["medium"]()
    plan = plan_for(p)
    rng = np.random.default_rng(5)
    x = f32(rng.random(p.ncols))
    r = f32(rng.standard_normal(p.nrows))

    def raw_create(chunks, between=None):
        n = bsgd.bsgd_fused_workspace_size(plan, chunks)
        if between:
            between()
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        h = capi._vp()
        capi._check("bsgd_fused_create", capi._lib.bsgd_fused_create(
            plan.handle, chunks, 0, capi._ptr(ws), n, capi._stream(), ctypes.byref(h)))
        return capi.Fused(h, ws, plan)

    def products(F):
        ax, g = bsgd.bsgd_fused_apply(F, _dev(x), _dev(r))
        return _host(ax), _host(g), bsgd.bsgd_fused_shape(F)

    ref = products(bsgd.bsgd_fused_create(plan, 0))
    for F in (raw_create(0), raw_create(0, lambda: bsgd.bsgd_tile_export(plan, 1, 1)),
              raw_create(2), raw_create(0)):
        got = products(F)
        if got[2][1] == ref[2][1]:  # same chunk count: bitwise the same store
            assert got[2] == ref[2]
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        else:
            assert np.allclose(got[0], ref[0], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_fwd_only_plan_gives_the_same_single_pass_results(name):
    """A plan without the A^T block store builds the same tile-sliced store: the
    column-sum bounds come from At's rows either way, so one-RHS, batch and
    ISTA epochs and the Lanczos estimate equal the full plan's bitwise."""
    import paper_1812_01307_amd as bsgd
    p = _cases()[name]()
    full, lean = plan_for(p), plan_for(p, fwd_only=True)
    F_full, F_lean = _fused(full), _fused(lean)
    assert bsgd.bsgd_fused_shape(F_full) == bsgd.bsgd_fused_shape(F_lean)
    u_full = bsgd.bsgd_lanczos_umax_fused(F_full, 6)
    assert bsgd.bsgd_lanczos_umax_fused(F_lean, 6) == u_full
    mu = float(np.float32(mu_for(p)))
    y4 = np.stack([f32(p.y) * s for s in (1.0, 0.5, 2.0, 0.0)])

    def run(plan, F, S, ista=False):
        st = bsgd.bsgd_state_create(plan, S)
        bsgd.bsgd_state_attach_fused(st, F)
        if ista:
            bsgd.bsgd_state_set_method(st, bsgd.BSGD_METHOD_ISTA)
        y = f32(p.y) if S == 1 else np.ascontiguousarray(y4[:S].T).ravel()
        bsgd.bsgd_state_init(st, _dev(f32(y)))
        bsgd.bsgd_run_epochs(st, mu, 20.0, 5, 20)
        return _host(bsgd.bsgd_get_x(st))

    for S, ista in ((1, False), (4, False), (1, True)):
        assert np.array_equal(run(full, F_full, S, ista), run(lean, F_lean, S, ista)), (S, ista)


def test_fwd_only_plan_refuses_calls_that_need_the_transpose():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p, fwd_only=True)
    r = _dev(f32(p.y))

    def unsupported(fn, *a, **k):
        with pytest.raises(bsgd.BsgdError) as e:
            fn(*a, **k)
        assert e.value.status == bsgd.BSGD_ERR_UNSUPPORTED, fn

    unsupported(bsgd.bsgd_backproject, plan, r)
    unsupported(bsgd.bsgd_backproject_block, plan, 0, 0,
                _dev(f32(p.y[p.row_off[0]:p.row_off[1]])))
    unsupported(bsgd.bsgd_tile_export, plan, 0, 0, transposed=True)
    unsupported(bsgd.bsgd_power_umax, plan, 3)
    unsupported(bsgd.bsgd_lanczos_umax, plan, 3)
    unsupported(bsgd.bsgd_state_create, plan, 1, flags=bsgd.BSGD_STATE_BLOCK_SELECT)
    mu = float(np.float32(mu_for(p)))
    st = bsgd.bsgd_state_create(plan, 1)   # no tile-sliced store attached
    bsgd.bsgd_state_init(st, r)
    unsupported(bsgd.bsgd_run_epochs, st, mu, 20.0, 1, 20)
    F = _fused(plan)
    st4 = bsgd.bsgd_state_create(plan, 4)
    bsgd.bsgd_state_attach_fused(st4, F)
    bsgd.bsgd_state_set_method(st4, bsgd.BSGD_METHOD_ISTA)
    bsgd.bsgd_state_init(st4, _dev(np.zeros(p.nrows * 4, np.float32)))
    unsupported(bsgd.bsgd_run_epochs, st4, mu, 20.0, 1, 20)
    # the forward direction and the single pass stay available
    x = _dev(f32(np.ones(p.ncols)))
    ref = oracle.forward(matrix(p), np.ones(p.ncols))
    assert rel_l2(_host(bsgd.bsgd_forward(plan, x)), ref) <= 1e-6
    bsgd.bsgd_state_attach_fused(st, F)
    bsgd.bsgd_run_epochs(st, mu, 20.0, 1, 20)
    with pytest.raises(bsgd.BsgdError) as e:
        bsgd.plan_from_host(p.nrows, p.ncols, p.row_ptr, p.col, p.val, *p.ensure_transpose(),
                            p.M, p.N, p.row_off, p.col_off, p.H, p.W, 1, view_len=p.bins,
                            staged="bwd", fwd_only=True)
    assert e.value.status == bsgd.BSGD_ERR_INVALID


@pytest.mark.parametrize("name,f16", [("c1", False), ("medium", False), ("ragged", False),
                                      ("strip", False), ("medium", True)])
def test_single_pass_only_plan_builds_the_same_store_from_a(name, f16):
    """A plan without block stores builds the tile-sliced store from A's CSR:
    the block store keeps A's entries in row order, so both builds walk the
    same entries in the same order and give the same store; the Lanczos
    estimate and one-RHS, batch and ISTA epochs equal the full plan's bitwise."""
    import paper_1812_01307_amd as bsgd
    p = _cases()[name]()
    full, bare = plan_for(p, f16=f16), plan_for(p, f16=f16, single_pass=True)
    F_full, F_bare = _fused(full), _fused(bare)
    assert bsgd.bsgd_fused_shape(F_full) == bsgd.bsgd_fused_shape(F_bare)
    vt = bsgd.BSGD_VAL_F16 if f16 else bsgd.BSGD_VAL_F32
    assert (bsgd.bsgd_lanczos_umax_fused(F_bare, 6, vt=vt)
            == bsgd.bsgd_lanczos_umax_fused(F_full, 6, vt=vt))
    rng = np.random.default_rng(11)
    x = _dev(f32(rng.random(p.ncols)))
    r = _dev(f32(rng.standard_normal(p.nrows)))
    for a, b in zip(bsgd.bsgd_fused_apply(F_full, x, r, vt=vt),
                    bsgd.bsgd_fused_apply(F_bare, x, r, vt=vt)):
        assert np.array_equal(_host(a), _host(b))
    mu = float(np.float32(mu_for(p)))
    y4 = np.stack([f32(p.y) * s for s in (1.0, 0.5, 2.0, 0.0)])

    def run(plan, F, S, ista=False):
        st = bsgd.bsgd_state_create(plan, S, vt)
        bsgd.bsgd_state_attach_fused(st, F)
        if ista:
            bsgd.bsgd_state_set_method(st, bsgd.BSGD_METHOD_ISTA)
        y = f32(p.y) if S == 1 else np.ascontiguousarray(y4[:S].T).ravel()
        bsgd.bsgd_state_init(st, _dev(f32(y)))
        bsgd.bsgd_run_epochs(st, mu, 20.0, 5, 20)
        return _host(bsgd.bsgd_get_x(st))

    for S, ista in ((1, False), (4, False), (1, True)):
        assert np.array_equal(run(full, F_full, S, ista), run(bare, F_bare, S, ista)), (S, ista)


def test_single_pass_only_plan_matches_oracle():
    """The store built from A's CSR against the FP64 oracle directly (products
    and a 12-epoch trajectory on the ragged geometry)."""
    import paper_1812_01307_amd as bsgd
    p = _cases()["ragged"]()
    plan = plan_for(p, single_pass=True)
    F = _fused(plan)
    rng = np.random.default_rng(5)
    x = f32(rng.random(p.ncols))
    r = f32(rng.standard_normal(p.nrows))
    ax, g = bsgd.bsgd_fused_apply(F, _dev(x), _dev(r))
    A, Aabs = matrix(p), abs_matrix(p)
    assert np.all(np.abs(_host(ax) - A @ x) <= PRODUCT_REL * (Aabs @ np.abs(x)) + 1e-30)
    assert np.all(np.abs(_host(g) - 2 * (A.T @ r)) <= PRODUCT_REL * 2 * (Aabs.T @ np.abs(r))
                  + 1e-30)
    mu = float(np.float32(mu_for(p)))
    _, _, ref = oracle.bsgd_tv(A, f32(p.y).astype(np.float64), mu, 5.0, 12, 20, (p.H, p.W),
                               record=True)
    xs, _ = _run(p, plan, F, mu, 5.0, 12, 20)
    assert max(rel_l2(a, b) for a, b in zip(xs, ref)) <= ITERATE_REL


def test_single_pass_only_plan_refuses_calls_that_need_a_block_store():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p, single_pass=True)
    assert plan.source is not None  # the plan holds A's device arrays
    y = _dev(f32(p.y))
    x = _dev(f32(np.ones(p.ncols)))

    def unsupported(fn, *a, **k):
        with pytest.raises(bsgd.BsgdError) as e:
            fn(*a, **k)
        assert e.value.status == bsgd.BSGD_ERR_UNSUPPORTED, fn

    unsupported(bsgd.bsgd_forward, plan, x)
    unsupported(bsgd.bsgd_forward_block, plan, 0, 0,
                _dev(f32(np.ones(p.col_off[1] - p.col_off[0]))))
    unsupported(bsgd.bsgd_tile_nnz, plan, 0, 0)
    unsupported(bsgd.bsgd_tile_export, plan, 0, 0)
    unsupported(bsgd.bsgd_backproject, plan, y)
    unsupported(bsgd.bsgd_power_umax, plan, 3)
    unsupported(bsgd.bsgd_state_create, plan, 1, flags=bsgd.BSGD_STATE_BLOCK_SELECT)
    st = bsgd.bsgd_state_create(plan, 1)
    unsupported(bsgd.bsgd_state_init, st, y, x)
    st4 = bsgd.bsgd_state_create(plan, 4)
    bsgd.bsgd_state_init(st4, _dev(np.zeros(p.nrows * 4, np.float32)))
    unsupported(bsgd.bsgd_state_set_rhs, st4, 0, y, x)
    # without x0 the states start (r = y) and run on the tile-sliced store
    F = _fused(plan)
    mu = float(np.float32(mu_for(p)))
    bsgd.bsgd_state_init(st, y)
    bsgd.bsgd_state_attach_fused(st, F)
    bsgd.bsgd_run_epochs(st, mu, 20.0, 1, 20)
    bsgd.bsgd_state_set_rhs(st4, 0, y)
    bsgd.bsgd_state_attach_fused(st4, F)
    bsgd.bsgd_run_epochs(st4, mu, 20.0, 1, 20)
    for staged in (True, "fwd"):
        with pytest.raises(bsgd.BsgdError) as e:
            plan_for(p, single_pass=True, staged=staged)
        assert e.value.status == bsgd.BSGD_ERR_INVALID
    with pytest.raises(bsgd.BsgdError) as e:
        plan_for(p, single_pass=True, autotune=True)
    assert e.value.status == bsgd.BSGD_ERR_INVALID


@pytest.mark.parametrize("fault", ["order", "duplicate", "range"])
def test_single_pass_only_plan_checks_a_columns_at_store_build(fault):
    """Without a block store, A's columns are first read by the store build's
    count pass, which rejects a column out of range or out of order (the
    count pass only compares columns; nothing is addressed with them)."""
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    col = p.col.copy()
    k = int(np.argmax(np.diff(p.row_ptr) >= 3))  # a row with 3 entries or more
    a = int(p.row_ptr[k])
    if fault == "order":
        col[a], col[a + 1] = col[a + 1], col[a]
    elif fault == "duplicate":
        col[a + 1] = col[a]
    else:
        col[int(p.row_ptr[k + 1]) - 1] = p.ncols
    plan = bsgd.plan_from_host(p.nrows, p.ncols, p.row_ptr, col, p.val, *p.ensure_transpose(),
                               p.M, p.N, p.row_off, p.col_off, p.H, p.W, 1, view_len=p.bins,
                               single_pass=True)
    for fn in (bsgd.bsgd_fused_workspace_size, bsgd.bsgd_fused_create):
        with pytest.raises(bsgd.BsgdError, match="column") as e:
            fn(plan, 0)
        assert e.value.status == bsgd.BSGD_ERR_INVALID


def _fixed_point_step(A, r):
    """Absolute rounding of one term of the single pass's fixed-point A^T r: the
    exponent e is the largest with every column sum of |A| times max |r| below
    2^30 and every |a| max |r| below 2^21 (the FP32 rounding of a term is exact
    below 2^22); a term is rounded to a multiple of 2^-e, off by 2^-(e+1) at
    most."""
    Aabs = abs(A)
    rmax = float(np.max(np.abs(np.asarray(r, np.float32))))
    smax = float(np.max(np.asarray(Aabs.sum(axis=0)).ravel()))
    amax = float(Aabs.max())
    es = np.frexp(smax * rmax)[1]
    et = np.frexp(amax * rmax)[1]
    e = min(max(min(30 - es, 21 - et), -200), 200)
    return 2.0 ** -(e + 1)


def _volume_stack(D, H, W, n_ang, bins):
    """D slices of one 2-D parallel-beam matrix, block-diagonal: rows of slice d
    (angle-major within the slice) see only the pixels of slice d."""
    import synth
    rp, col, val = synth.projection_matrix(H, W, n_ang, bins)
    nr, npx = n_ang * bins, H * W
    row_ptr = np.concatenate([[0]] + [rp[1:] + d * rp[-1] for d in range(D)]).astype(np.int64)
    cols = np.concatenate([col.astype(np.int64) + d * npx for d in range(D)]).astype(np.int32)
    vals = np.tile(val, D)
    return D * nr, D * npx, row_ptr, cols, vals


def _general_volume(rng, D, H, W, nrows):
    ncols = D * H * W
    lens = rng.integers(0, 90, nrows)
    lens[::37] = 0
    cols = [np.sort(rng.choice(ncols, n, replace=False)).astype(np.int32) for n in lens]
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return nrows, ncols, row_ptr, np.concatenate(cols).astype(np.int32), rng.random(lens.sum()) * 1.5


@pytest.mark.parametrize("kind,f16", [("rays", False), ("rays", True), ("general", False)])
def test_three_dimensional_plan_matches_oracle(kind, f16):
    """Plans over a D x H x W volume (D = 3; ragged 8 x 8 and 64 x 64 tiles): a
    stack of parallel-beam matrices (block-diagonal over the slices) and a
    general sparse A.  The block-store products, the single-pass products and
    epochs with the 3-D TV prox against the oracle, from a full plan and from
    a plan without block stores (the same store, bitwise).  For the general
    matrix, whose columns hold few entries, the single pass's A^T r is also
    allowed the rounding of its fixed-point terms (for ray matrices a column
    sum is far above its largest entry and that rounding is far below the
    FP32 bound)."""
    import paper_1812_01307_amd as bsgd
    import synth
    rng = np.random.default_rng(21)
    D, H, W = 3, 40, 70
    if kind == "rays":
        bins = 81  # covers the diagonal of a 40 x 70 slice
        nrows, ncols, row_ptr, col, val = _volume_stack(D, H, W, 24, bins)
        view_len = bins
    else:
        H = 20
        nrows, ncols, row_ptr, col, val = _general_volume(rng, D, H, W, 900)
        view_len = 0
    tp, tc, tv = synth.transpose_csr(nrows, ncols, row_ptr, col, val)
    vt = bsgd.BSGD_VAL_F16 if f16 else bsgd.BSGD_VAL_F32
    vals = f32(val).astype(np.float64)
    if f16:
        vals = vals.astype(np.float32).astype(np.float16).astype(np.float64)
    A = oracle.as_matrix(row_ptr, col, vals, ncols)
    Aabs = oracle.as_matrix(row_ptr, col, np.abs(vals), ncols)

    def make(single_pass):
        return bsgd.plan_from_host(nrows, ncols, row_ptr, col, val, tp, tc, tv, 2, 2,
                                   [0, nrows // 2, nrows], [0, ncols // 2, ncols], H, W, D,
                                   view_len=view_len, f16=f16, single_pass=single_pass)

    full, bare = make(False), make(True)
    F_full, F_bare = _fused(full), _fused(bare)
    assert bsgd.bsgd_fused_shape(F_full) == bsgd.bsgd_fused_shape(F_bare)
    assert bsgd.bsgd_fused_shape(F_full)[0] == D * ((H + 63) // 64) * 2  # tiles
    # several RHS take the 2-D prox image by image: refused for a volume plan
    with pytest.raises(bsgd.BsgdError) as e:
        bsgd.bsgd_state_create(full, 4)
    assert e.value.status == bsgd.BSGD_ERR_INVALID
    x = f32(rng.random(ncols))
    r = f32(rng.standard_normal(nrows))
    bound_f = PRODUCT_REL * (Aabs @ np.abs(x)) + 1e-30
    bound_b = PRODUCT_REL * 2 * (Aabs.T @ np.abs(r)) + 1e-30
    if not f16:
        assert np.all(np.abs(_host(bsgd.bsgd_forward(full, _dev(x))) - A @ x) <= bound_f)
        assert np.all(np.abs(_host(bsgd.bsgd_backproject(full, _dev(r))) - 2 * (A.T @ r))
                      <= bound_b)
    nz = np.diff(A.tocsc().indptr)  # entries per column
    bound_fixed = bound_b + (2 * nz * _fixed_point_step(A, r) if kind == "general" else 0.0)
    for F in (F_full, F_bare):
        ax, g = bsgd.bsgd_fused_apply(F, _dev(x), _dev(r), vt=vt)
        assert np.all(np.abs(_host(ax) - A @ x) <= bound_f)
        assert np.all(np.abs(_host(g) - 2 * (A.T @ r)) <= bound_fixed)
    mu = float(np.float32(oracle.step_size(oracle.power_umax(A))))
    y = f32(A @ rng.random(ncols) + 0.01 * rng.standard_normal(nrows))
    lam, E, K = 2.0, 5, 10
    _, _, ref = oracle.bsgd_tv(A, y.astype(np.float64), mu, lam, E, K, (D, H, W), record=True)

    def run(plan, F):
        st = bsgd.bsgd_state_create(plan, 1, vt)
        if F is not None:
            bsgd.bsgd_state_attach_fused(st, F)
        bsgd.bsgd_state_init(st, _dev(y))
        xs = []
        for _ in range(E):
            bsgd.bsgd_run_epochs(st, mu, lam, 1, K)
            xs.append(_host(bsgd.bsgd_get_x(st)))
        return xs

    runs = {"fused": run(full, F_full), "bare": run(bare, F_bare)}
    if not f16:
        runs["rows"] = run(full, None)
    for name, xs in runs.items():
        errs = [rel_l2(a, b) for a, b in zip(xs, ref)]
        assert max(errs) <= ITERATE_REL, (name, errs)
    # the prox moved the iterate by far more than the tolerance
    xhat_only, _ = oracle.bsgd_tv(A, y.astype(np.float64), mu, 0.0, 1, 1, (D, H, W))
    assert rel_l2(ref[0], xhat_only) > 100 * ITERATE_REL
    assert all(np.array_equal(a, b) for a, b in zip(runs["fused"], runs["bare"]))

"""Staged form of the fused products (BSGD_PLAN_STAGED) against the oracle (GPU)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import (ITERATE_REL, f32, matrix, mu_for, plan_for, problem, ragged_problem,
                         rel_l2)

pytestmark = pytest.mark.gpu


def _cases():
    return {
        # one stage per direction
        "c1": lambda: problem("c1_64"),
        # several stages: pixels 2 x 18432, rays 3 x 17472 (small LDS variant)
        "medium": lambda: problem(None, H=192, W=192, n_ang=180, bins=273, M=4, N=4, seed=7),
        # 8 views x 2500 bins = 20000 > 19456: the large LDS variant, 2 ray stages;
        # most rays miss the image (empty rows)
        "wide": lambda: problem(None, H=64, W=64, n_ang=16, bins=2500, M=2, N=2, seed=8),
        # non-square image, ragged tiles and view groups
        "ragged": ragged_problem,
    }


def _run(p, plan, mu, lam, epochs, K, vt=0):
    import paper_1812_01307_amd as bsgd
    st = bsgd.bsgd_state_create(plan, 1, vt)
    bsgd.bsgd_state_init(st, torch.from_numpy(f32(p.y)).cuda())
    xs = []
    for _ in range(epochs):
        bsgd.bsgd_run_epochs(st, mu, lam, 1, K)
        torch.cuda.synchronize()
        xs.append(bsgd.bsgd_get_x(st).cpu().numpy().astype(np.float64))
    return xs


@pytest.mark.parametrize("name", ["c1", "medium", "wide", "ragged"])
@pytest.mark.parametrize("view_len", [None, 0])
def test_staged_trajectory_matches_oracle(name, view_len):
    import paper_1812_01307_amd as bsgd
    p = _cases()[name]()
    plan = plan_for(p, view_len=view_len, staged=True)
    assert bsgd.bsgd_plan_staged(plan) == (4, 4)
    mu = float(np.float32(mu_for(p)))
    lam = 5.0
    E = 12
    _, _, ref = oracle.bsgd_tv(matrix(p), f32(p.y).astype(np.float64), mu, lam, E, 20,
                               (p.H, p.W), record=True)
    xs = _run(p, plan, mu, lam, E, 20)
    errs = [rel_l2(a, b) for a, b in zip(xs, ref)]
    assert max(errs) <= ITERATE_REL, (max(errs), int(np.argmax(errs)))
    # 8 lanes per row, and the row kernels on the same plan, agree to rounding
    bsgd.bsgd_plan_set_staged(plan, 8, 8)
    xs8 = _run(p, plan, mu, lam, E, 20)
    bsgd.bsgd_plan_set_staged(plan, 0, 0)
    xr = _run(p, plan, mu, lam, E, 20)
    assert max(rel_l2(a, b) for a, b in zip(xs8, xr)) <= 1e-6
    assert max(rel_l2(a, b) for a, b in zip(xs, xr)) <= 1e-6


def test_staged_fp16_values():
    import paper_1812_01307_amd as bsgd
    p = _cases()["medium"]()
    plan = plan_for(p, f16=True, staged=True)
    mu = float(np.float32(mu_for(p)))
    E = 10
    xs = _run(p, plan, mu, 5.0, E, 20, vt=bsgd.BSGD_VAL_F16)
    # against the oracle on the FP16-rounded matrix (accumulation error only)
    vals = p.val.astype(np.float32).astype(np.float16).astype(np.float64)
    A16 = oracle.as_matrix(p.row_ptr, p.col, vals, p.ncols)
    _, _, ref = oracle.bsgd_tv(A16, f32(p.y).astype(np.float64), mu, 5.0, E, 20, (p.H, p.W),
                               record=True)
    assert max(rel_l2(a, b) for a, b in zip(xs, ref)) <= ITERATE_REL
    bsgd.bsgd_plan_set_staged(plan, 0, 0)
    xr = _run(p, plan, mu, 5.0, E, 20, vt=bsgd.BSGD_VAL_F16)
    assert max(rel_l2(a, b) for a, b in zip(xs, xr)) <= 1e-6


def test_staged_runs_are_bitwise_reproducible_and_autotune():
    import paper_1812_01307_amd as bsgd
    p = _cases()["medium"]()
    plan = plan_for(p, staged=True)
    mu = float(np.float32(mu_for(p)))
    a = _run(p, plan, mu, 20.0, 6, 20)
    b = _run(p, plan, mu, 20.0, 6, 20)
    assert all(np.array_equal(u, v) for u, v in zip(a, b))
    tuned = plan_for(p, staged=True, autotune=True)
    f, bw = bsgd.bsgd_plan_staged(tuned)
    assert f in (0, 4, 8) and bw in (0, 4, 8)
    c = _run(p, tuned, mu, 20.0, 6, 20)
    assert max(rel_l2(u, v) for u, v in zip(a, c)) <= 1e-6


def test_staged_selection_is_validated():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plain = plan_for(p)
    assert bsgd.bsgd_plan_staged(plain) == (-1, -1)
    with pytest.raises(bsgd.BsgdError, match="staged"):
        bsgd.bsgd_plan_set_staged(plain, 4, 4)
    bsgd.bsgd_plan_set_staged(plain, 0, 0)
    staged = plan_for(p, staged=True)
    with pytest.raises(bsgd.BsgdError):
        bsgd.bsgd_plan_set_staged(staged, 5, 4)
    bwd_only = plan_for(p, staged="bwd")
    assert bsgd.bsgd_plan_staged(bwd_only) == (-1, 4)
    with pytest.raises(bsgd.BsgdError, match="staged"):
        bsgd.bsgd_plan_set_staged(bwd_only, 4, 4)
    with pytest.raises(bsgd.BsgdError, match="no staged form"):
        bsgd.bsgd_plan_staged_shape(bwd_only, 0)
    P, SW, ent = bsgd.bsgd_plan_staged_shape(bwd_only, 1)
    assert P == 1 and SW >= p.nrows and p.nnz <= ent <= p.nnz + 7 * p.ncols
    # a state on a staged plan needs room for the per-stage partial sums
    assert bsgd.bsgd_state_workspace_size(staged, 1) > bsgd.bsgd_state_workspace_size(plain, 1)

"""Kernel timers of a state: counts, positivity, reuse of pooled events (GPU)."""
import numpy as np
import pytest
import torch

from gpu_helpers import f32, mu_for, plan_for, problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fused", [False, True])
def test_timers_count_epochs_and_survive_state_turnover(fused):
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    y = torch.from_numpy(f32(p.y)).cuda()
    F = bsgd.bsgd_fused_create(plan, 0) if fused else None
    results = []
    for job in range(3):
        st = bsgd.bsgd_state_create(plan, 1)
        if F is not None:
            bsgd.bsgd_state_attach_fused(st, F)
        bsgd.bsgd_state_enable_timing(st, 4)
        bsgd.bsgd_state_init(st, y)
        bsgd.bsgd_run_epochs(st, mu, 5.0, 6, 10)  # only the first 4 are timed
        f, b, x, n = bsgd.bsgd_state_timing(st)
        assert n == 4
        assert f > 0.0 and b > 0.0 and x > 0.0
        # rearmed: nothing pending until epochs run again
        assert bsgd.bsgd_state_timing(st)[3] == 0
        results.append(bsgd.bsgd_get_x(st).cpu().numpy())
        del st  # its events go back to the pool for the next state
    # timing does not change the arithmetic
    assert np.array_equal(results[0], results[1]) and np.array_equal(results[1], results[2])


def test_timers_rejected_arguments():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    st = bsgd.bsgd_state_create(plan_for(p), 1)
    with pytest.raises(bsgd.BsgdError):
        bsgd.bsgd_state_enable_timing(st, -1)
    bsgd.bsgd_state_enable_timing(st, 0)  # disables
    bsgd.bsgd_state_init(st, torch.from_numpy(f32(p.y)).cuda())
    bsgd.bsgd_run_epochs(st, float(np.float32(mu_for(p))), 5.0, 2, 10)
    assert bsgd.bsgd_state_timing(st)[3] == 0


def test_sampled_timers_take_every_stride_th_epoch():
    import paper_1812_01307_amd as bsgd
    p = problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    st = bsgd.bsgd_state_create(plan, 1)
    bsgd.bsgd_state_init(st, torch.from_numpy(f32(p.y)).cuda())
    bsgd.bsgd_state_enable_timing(st, 3, stride=2)
    bsgd.bsgd_run_epochs(st, mu, 5.0, 5, 10)  # epochs 0, 2 and 4 are timed
    assert bsgd.bsgd_state_timing(st)[3] == 3
    bsgd.bsgd_run_epochs(st, mu, 5.0, 3, 10)  # rearmed: epochs 0 and 2 of this call
    assert bsgd.bsgd_state_timing(st)[3] == 2
    bsgd.bsgd_run_epochs(st, mu, 5.0, 9, 10)  # at most 3
    assert bsgd.bsgd_state_timing(st)[3] == 3
    with pytest.raises(bsgd.BsgdError):
        bsgd.bsgd_state_enable_timing(st, 3, stride=0)

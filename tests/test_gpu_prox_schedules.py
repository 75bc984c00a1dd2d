"""The three 2-D prox schedules compute the same recurrence with the same arithmetic (GPU)."""
import numpy as np
import pytest
import torch

from gpu_helpers import f32, mu_for, plan_for, problem, ragged_problem

pytestmark = pytest.mark.gpu


def _cases():
    return {
        "c1": lambda: problem("c1_64"),
        "ragged": ragged_problem,
        # 6 x 6 output tiles of the register kernel, several strips per column
        "medium": lambda: problem(None, H=192, W=192, n_ang=180, bins=273, M=4, N=4, seed=7),
    }


def _iterate(plan, y, mu, lam, K, schedule, S=1, lams=None):
    import paper_1812_01307_amd as bsgd
    st = bsgd.bsgd_state_create(plan, S)
    bsgd.bsgd_state_set_prox_schedule(st, schedule)
    bsgd.bsgd_state_init(st, y)
    if lams is not None:
        bsgd.bsgd_state_set_lambda(st, lams)
    bsgd.bsgd_run_epochs(st, mu, lam, 3, K)
    x = bsgd.bsgd_get_x(st)
    torch.cuda.synchronize()
    return x.cpu().numpy()


@pytest.mark.parametrize("name", ["c1", "ragged", "medium"])
@pytest.mark.parametrize("K", [1, 2, 3, 20, 21, 30, 41])
def test_prox_schedules_agree_bitwise(name, K):
    p = _cases()[name]()
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    y = torch.from_numpy(f32(p.y)).cuda()
    # lambda large enough that the prox moves the iterate visibly
    xs = [_iterate(plan, y, mu, 500.0, K, s) for s in (0, 1, 2)]
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    assert not np.array_equal(xs[0], _iterate(plan, y, mu, 0.0, K, 0))


def test_prox_schedules_agree_bitwise_batch():
    p = problem("c1_64")
    plan = plan_for(p)
    mu = float(np.float32(mu_for(p)))
    S = 4
    rng = np.random.default_rng(4)
    Y = f32(np.stack([p.y * (1 + 0.1 * j) + rng.standard_normal(p.nrows) for j in range(S)], 1))
    y = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    lams = [0.0, 50.0, 500.0, 5000.0]
    xs = [_iterate(plan, y, mu, -1.0, 20, s, S=S, lams=lams) for s in (0, 1, 2)]
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])

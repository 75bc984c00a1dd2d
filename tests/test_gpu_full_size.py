"""Full-size parity against the FP64 oracle, in the benchmark's launch configuration.

The 512 x 512 workload (720 angles x 729 bins, M = N = 8) runs its epochs of
Algorithm 1 (with the delay of Eq. 3) through the tile-sliced single pass,
as bench.py times it: automatic chunk count, 8 wavefronts per unit, step
mu = 0.9 / (2 u_max) with u_max from 10 Lanczos steps on the same store,
rounded to FP32 and handed to the oracle too.  Every epoch's iterate is
compared with the oracle's (relative L2 <= 1e-5 in FP32), at the workload's
lambda and at a lambda large enough that the TV prox visibly moves x.

The 1024 x 1024 workload (1440 x 1449 rays, M = N = 16, 30 FGP iterations)
checks the precision form: FP32 values against the oracle on the exact
(FP64) matrix, FP16 values against it (bar 2e-3) and against the oracle on
the FP16-dequantised matrix (accumulation error alone, bar 1e-5).  Its step
is the oracle's converged one from tests/golden/c3_1024_mu.json.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import ITERATE_REL, f32, rel_l2

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FP16_REL = 2e-3


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _plan(p, f16=False, single_pass=True):
    """The bench's plan: no block stores (the tile-sliced store is built from A's CSR)."""
    import paper_1812_01307_amd as bsgd
    tp, tc, tv = p.ensure_transpose()
    return bsgd.plan_from_host(p.nrows, p.ncols, p.row_ptr, p.col, p.val, tp, tc, tv, p.M, p.N,
                               p.row_off, p.col_off, p.H, p.W, 1, view_len=p.bins, f16=f16,
                               fwd_only=True, single_pass=single_pass)


def _store(plan):
    import paper_1812_01307_amd as bsgd
    F = bsgd.bsgd_fused_create(plan, 0)
    bsgd.bsgd_fused_set_waves(F, 8)
    return F


def _epochs(plan, F, y32, mu, lam, E, K, vt=0):
    """E single-pass epochs from x = 0; the iterate after each."""
    import paper_1812_01307_amd as bsgd
    st = bsgd.bsgd_state_create(plan, 1, vt)
    bsgd.bsgd_state_attach_fused(st, F)
    bsgd.bsgd_state_init(st, _dev(y32))
    xs = []
    for _ in range(E):
        bsgd.bsgd_run_epochs(st, mu, lam, 1, K)
        torch.cuda.synchronize()
        xs.append(bsgd.bsgd_get_x(st).cpu().numpy().astype(np.float64))
    return xs


def test_c2_512_single_pass_trajectory_matches_oracle():
    import paper_1812_01307_amd as bsgd
    print("c2_512: generating", flush=True)
    p = synth.make_problem("c2_512", dtype=np.float32)
    plan = _plan(p)
    F = _store(plan)
    tiles, chunks, segs, slices, entries, cbytes = bsgd.bsgd_fused_shape(F)
    assert (tiles, chunks, cbytes) == (64, 16, 1)
    u = bsgd.bsgd_lanczos_umax_fused(F, 10)
    # the bench's 4 steps: converged to below FP32 rounding on this geometry
    # (the FP64 recurrence from the same start is within 4e-10 after 4 steps)
    assert abs(bsgd.bsgd_lanczos_umax_fused(F, 4) - u) <= 1e-6 * u
    mu = float(np.float32(0.9 / (2.0 * u)))
    A = oracle.as_matrix(p.row_ptr, p.col, p.val, p.ncols)  # the FP32 values, in FP64
    y32 = f32(p.y)
    y64 = y32.astype(np.float64)
    # the workload's lambda (theta = mu lam ~ 1e-8: the prox barely moves x),
    # then one at which the TV correction is ~1% of x
    for lam, E in ((p.lam, 20), (2000.0, 8)):
        print(f"c2_512: lambda={lam} epochs={E}", flush=True)
        xs = _epochs(plan, F, y32, mu, lam, E, p.prox_iters)
        _, _, ref = oracle.bsgd_tv(A, y64, mu, lam, E, p.prox_iters, (p.H, p.W), record=True)
        errs = [rel_l2(a, b) for a, b in zip(xs, ref)]
        print(f"c2_512: lambda={lam} max per-epoch rel L2 {max(errs):.3e}", flush=True)
        assert max(errs) <= ITERATE_REL, errs
        if lam > 1.0:
            # the prox changed the iterate by far more than the tolerance
            xhat_only, _ = oracle.bsgd_tv(A, y64, mu, 0.0, 1, 1, (p.H, p.W))
            assert rel_l2(ref[0], xhat_only) > 100 * ITERATE_REL
    # the store built from the block store of A is the same store
    print("c2_512: store from the block store of A", flush=True)
    x_bare = _epochs(plan, F, y32, mu, 2000.0, 3, p.prox_iters)
    del F, plan
    plan_a = _plan(p, single_pass=False)
    F_a = _store(plan_a)
    assert bsgd.bsgd_fused_shape(F_a) == (tiles, chunks, segs, slices, entries, cbytes)
    assert bsgd.bsgd_lanczos_umax_fused(F_a, 10) == u
    x_a = _epochs(plan_a, F_a, y32, mu, 2000.0, 3, p.prox_iters)
    assert all(np.array_equal(a, b) for a, b in zip(x_bare, x_a))


@pytest.mark.timeout(600)
def test_c3_1024_fp32_and_fp16_values_match_oracle():
    import paper_1812_01307_amd as bsgd
    with open(os.path.join(ROOT, "tests", "golden", "c3_1024_mu.json")) as f:
        mu = float(json.load(f)["mu_f32"])
    print("c3_1024: generating (FP64 lengths)", flush=True)
    p = synth.make_problem("c3_1024", with_transpose=False)
    plan = _plan(p, f16=True)
    p.t_ptr = p.t_col = p.t_val = None  # the host transpose is not needed any more
    F = _store(plan)
    y32 = f32(p.y)
    y64 = y32.astype(np.float64)
    E, K, shape = 2, p.prox_iters, (p.H, p.W)
    print("c3_1024: device epochs", flush=True)
    x32 = _epochs(plan, F, y32, mu, p.lam, E, K, vt=bsgd.BSGD_VAL_F32)
    x16 = _epochs(plan, F, y32, mu, p.lam, E, K, vt=bsgd.BSGD_VAL_F16)
    del F, plan
    rp = p.row_ptr.astype(np.int32)  # keeps scipy from copying 1.9e9 indices to int64
    print("c3_1024: oracle on the exact matrix", flush=True)
    A = oracle.as_matrix(rp, p.col, p.val, p.ncols)
    _, _, ref = oracle.bsgd_tv(A, y64, mu, p.lam, E, K, shape, record=True)
    del A
    e32 = [rel_l2(a, b) for a, b in zip(x32, ref)]
    e16 = [rel_l2(a, b) for a, b in zip(x16, ref)]
    print("c3_1024: oracle on the FP16-dequantised matrix", flush=True)
    deq = p.val.astype(np.float32).astype(np.float16).astype(np.float64)
    A16 = oracle.as_matrix(rp, p.col, deq, p.ncols)
    _, _, ref16 = oracle.bsgd_tv(A16, y64, mu, p.lam, E, K, shape, record=True)
    e16d = [rel_l2(a, b) for a, b in zip(x16, ref16)]
    print(f"c3_1024: FP32 {max(e32):.3e}, FP16 vs exact {max(e16):.3e}, "
          f"FP16 vs dequantised {max(e16d):.3e}", flush=True)
    assert max(e32) <= ITERATE_REL, e32
    assert max(e16) <= FP16_REL, e16
    assert max(e16d) <= ITERATE_REL, e16d

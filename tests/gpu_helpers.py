"""Shared set-up for the GPU parity tests: problems, uploads, tolerances."""
import functools

import numpy as np

import oracle
import synth

# Per-element bound for an FP32 sparse dot product against the FP64 oracle:
# |gpu - ref| <= REL * sum_k |a_k| |v_k|.  FP32 rounding of the matrix values
# contributes 2^-24 per term and the FP32 accumulation over at most ~2.1e3
# terms per row (C1/C2 rows) contributes well under 2e-5 of the absolute
# sum for fixed-order pairwise-like accumulation (measured worst case below
# 2e-6); 2e-5 leaves a margin.
PRODUCT_REL = 2e-5
# Per-epoch iterate: relative L2 error of the FP32 device iterate vs the FP64
# oracle iterate.
ITERATE_REL = 1e-5


@functools.lru_cache(maxsize=None)
def problem(name=None, **kw):
    kw = dict(kw)
    return synth.make_problem(name, **kw)


def ragged_problem():
    """Non-square image, uneven blocks, lengths that are not tile multiples."""
    return problem(None, H=45, W=67, n_ang=37, bins=83, M=3, N=5, seed=21, lam=0.0)


def f32(a):
    return np.asarray(a, np.float32)


def plan_for(p, f16=False, view_len=None, autotune=False, staged=False, fwd_only=False,
             single_pass=False):
    """Plan with the view structure of the generator's rays (view_len = bins) by default."""
    import paper_1812_01307_amd as bsgd
    tp, tc, tv = p.ensure_transpose()
    vl = p.bins if view_len is None else view_len
    return bsgd.plan_from_host(p.nrows, p.ncols, p.row_ptr, p.col, p.val, tp, tc, tv, p.M, p.N,
                               p.row_off, p.col_off, p.H, p.W, 1, view_len=vl, f16=f16,
                               autotune=autotune, staged=staged, fwd_only=fwd_only,
                               single_pass=single_pass)


def matrix(p):
    return oracle.as_matrix(p.row_ptr, p.col, p.val, p.ncols)


def abs_matrix(p):
    return oracle.as_matrix(p.row_ptr, p.col, np.abs(p.val), p.ncols)


def mu_for(p):
    return oracle.step_size(oracle.power_umax(matrix(p)))


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

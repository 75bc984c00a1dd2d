"""Host-side marshalling: upload CSR arrays with torch and create a plan."""
from __future__ import annotations

import numpy as np
import torch

from . import capi


def to_device(a, dtype, device="cuda") -> torch.Tensor:
    """Copy a host array to the device with the given torch dtype."""
    np_dtype = {torch.int64: np.int64, torch.int32: np.int32, torch.float32: np.float32}[dtype]
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np_dtype)).to(device)


def plan_from_host(nrows, ncols, row_ptr, col, val, t_ptr, t_col, t_val, M, N, row_off, col_off,
                   H, W, D=1, view_len=0, f16=False, autotune=False, staged=False,
                   fwd_only=False, single_pass=False, device="cuda",
                   stream=None) -> capi.Plan:
    """Upload A and A^T (host CSR; values are rounded to FP32) and build the block store.

    The uploaded copies are released once the plan is built; the plan keeps
    only its own store.  fwd_only: BSGD_PLAN_FWD_ONLY (no A^T store; A^T's
    column indices are not uploaded).  single_pass: BSGD_PLAN_SINGLE_PASS_ONLY
    (no block store; the plan holds the uploaded A, from which the tile-sliced
    store is built).
    """
    fwd_only = fwd_only or single_pass
    A = (nrows, ncols, to_device(row_ptr, torch.int64, device), to_device(col, torch.int32, device),
         to_device(val, torch.float32, device))
    At = (ncols, nrows, to_device(t_ptr, torch.int64, device),
          None if fwd_only else to_device(t_col, torch.int32, device),
          to_device(t_val, torch.float32, device))
    flags = ((capi.BSGD_PLAN_F16 if f16 else 0) | (capi.BSGD_PLAN_AUTOTUNE if autotune else 0)
             | {False: 0, True: capi.BSGD_PLAN_STAGED, "fwd": capi.BSGD_PLAN_STAGED_FWD,
                "bwd": capi.BSGD_PLAN_STAGED_BWD}[staged]
             | (capi.BSGD_PLAN_FWD_ONLY if fwd_only else 0)
             | (capi.BSGD_PLAN_SINGLE_PASS_ONLY if single_pass else 0))
    plan = capi.bsgd_plan_create(A, At, M, N, row_off, col_off, H, W, D, view_len, flags,
                                 stream=stream)
    del A, At
    return plan

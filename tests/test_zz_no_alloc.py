"""The allocation-free prox entry point against the workspace one, through the C ABI.

bsgd_tv_prox_noalloc runs the same kernels as bsgd_tv_prox (the TV prox step of
Algorithm 1, FGP on the dual) with the duals in the library's own device array,
so its results must equal bsgd_tv_prox's bitwise; they are also checked
against the FP64 oracle to the prox bar of the parity tests.  Consecutive
calls shrink the input, so a kernel that read a dual it had not written in
the same call (the array keeps the last call's contents) would show up.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _reference(b, theta, iters):
    """bsgd_tv_prox with a NaN-filled workspace (a read of an unwritten dual shows)."""
    import paper_1812_01307_amd as bsgd
    shape = tuple(b.shape)
    D, H, W = (1,) + shape if len(shape) == 2 else shape
    ws = torch.full((bsgd.bsgd_tv_workspace_size(H, W, D) // 4 + 1,), float("nan"),
                    dtype=torch.float32, device=b.device)
    return bsgd.bsgd_tv_prox(b, theta, iters, ws=ws.view(torch.uint8))


# (shape, theta, iters), run in this order: each call after the first is smaller
SEQUENCE = [((256, 320), 0.3, 20), ((45, 67), 0.7, 13), ((1, 37), 0.05, 3),
            ((6, 40, 36), 0.05, 20), ((3, 20, 24), 0.2, 7)]


def test_noalloc_equals_workspace_prox_on_shrinking_calls():
    import paper_1812_01307_amd as bsgd
    rng = np.random.default_rng(77)
    for shape, theta, iters in SEQUENCE:
        print(f"noalloc prox {shape} theta={theta} K={iters}", flush=True)
        b = np.asarray(rng.random(shape), np.float32)
        bd = _dev(b)
        out = torch.full_like(bd, float("nan"))
        bsgd.bsgd_tv_prox_noalloc(bd, theta, iters, out)
        ref = _reference(bd, theta, iters)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref.cpu().numpy()), shape
        b64 = b.astype(np.float64)
        orc = oracle.fgp_prox2(b64, theta, iters) if len(shape) == 2 else \
            oracle.fgp_prox3(b64, theta, iters)
        ncomp = 4 if len(shape) == 2 else 6
        assert np.max(np.abs(got - orc)) <= 4e-6 + 1e-4 * ncomp * theta, shape


def test_noalloc_identity_and_size_limit():
    import paper_1812_01307_amd as bsgd
    b = _dev(np.random.default_rng(3).random((20, 24)).astype(np.float32))
    out = torch.empty_like(b)
    bsgd.bsgd_tv_prox_noalloc(b, 0.0, 20, out)
    torch.cuda.synchronize()
    assert torch.equal(out, b)
    # 2^21 pixels need 64 MiB of duals: rejected on the host before any launch
    big = torch.empty((2048, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(bsgd.BsgdError) as ei:
        bsgd.bsgd_tv_prox_noalloc(big, 0.1, 5, torch.empty_like(big))
    assert ei.value.status == bsgd.BSGD_ERR_WORKSPACE
    # the largest 2-D image the array holds runs
    edge = _dev(np.random.default_rng(4).random((1024, 1024)).astype(np.float32))
    o1 = torch.empty_like(edge)
    bsgd.bsgd_tv_prox_noalloc(edge, 0.02, 4, o1)
    ref = _reference(edge, 0.02, 4)
    torch.cuda.synchronize()
    assert torch.equal(o1, ref)


def test_noalloc_symbol_is_exported():
    import paper_1812_01307_amd as bsgd
    lib = ctypes.CDLL(bsgd.library_path())
    assert hasattr(lib, "bsgd_tv_prox_noalloc")

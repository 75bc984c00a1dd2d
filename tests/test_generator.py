"""Pins for the seeded projection-matrix generator (CPU only).

The matrix is input data, not the method, but every parity case depends on
it, so it is checked against an independent brute-force construction: the
chord of each ray clipped against each pixel square (Liang-Barsky), with the
stated edge rule applied separately.
"""
import math

import numpy as np
import pytest

import synth


def _clip_len(px, py, ex, ey, x0, x1, y0, y1):
    """Length of the line p + l e (|e| = 1) inside the box [x0,x1] x [y0,y1]."""
    lo, hi = -math.inf, math.inf
    for p0, e, a, b in ((px, ex, x0, x1), (py, ey, y0, y1)):
        if abs(e) < 1e-15:
            if p0 < a or p0 > b:
                return 0.0
        else:
            l0, l1 = (a - p0) / e, (b - p0) / e
            lo, hi = max(lo, min(l0, l1)), min(hi, max(l0, l1))
    return max(0.0, hi - lo)


def _brute_matrix(H, W, n_ang, bins):
    A = np.zeros((n_ang * bins, H * W))
    for a in range(n_ang):
        phi = a * math.pi / n_ang
        c, s = math.cos(phi), math.sin(phi)
        if abs(s) < 1e-12:
            c, s = 1.0, 0.0
        if abs(c) < 1e-12:
            c, s = 0.0, 1.0
        for b in range(bins):
            u = b - 0.5 * (bins - 1)
            px, py, ex, ey = u * c, u * s, -s, c
            for row in range(H):
                for t in range(W):
                    x0, x1 = t - W / 2, t + 1 - W / 2
                    y0, y1 = H / 2 - row - 1, H / 2 - row
                    ln = _clip_len(px, py, ex, ey, x0, x1, y0, y1)
                    if ln < 1e-12:
                        continue
                    # a line lying on an edge of this pixel is shared with the
                    # neighbour across that edge: half each
                    on_edge = (ex == 0.0 and (abs(px - x0) < 1e-12 or abs(px - x1) < 1e-12)) or \
                              (ey == 0.0 and (abs(py - y0) < 1e-12 or abs(py - y1) < 1e-12))
                    A[a * bins + b, row * W + t] = 0.5 * ln if on_edge else ln
    return A


def _dense(row_ptr, col, val, ncols):
    nrows = len(row_ptr) - 1
    A = np.zeros((nrows, ncols))
    for i in range(nrows):
        A[i, col[row_ptr[i]:row_ptr[i + 1]]] = val[row_ptr[i]:row_ptr[i + 1]]
    return A


@pytest.mark.parametrize("H,W,n_ang,bins", [(8, 8, 12, 13), (5, 7, 8, 11), (6, 6, 4, 9), (4, 4, 6, 7)])
def test_matches_brute_force_clipping(H, W, n_ang, bins):
    rp, col, val = synth.projection_matrix(H, W, n_ang, bins)
    got = _dense(rp, col, val, H * W)
    ref = _brute_matrix(H, W, n_ang, bins)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_csr_structure_and_row_sums():
    H = W = 16
    n_ang, bins = 18, 25
    rp, col, val = synth.projection_matrix(H, W, n_ang, bins)
    for i in range(n_ang * bins):
        cs = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cs) > 0)
        assert len(cs) <= H + W + 1 or (i // bins) in (0, n_ang // 2)
    assert np.all(val > 0) and np.all(val <= math.sqrt(2) + 1e-12)
    sums = np.bincount(np.repeat(np.arange(n_ang * bins), np.diff(rp)), weights=val,
                       minlength=n_ang * bins)
    # row sum = chord of the line through the image square; a line lying on
    # the square's border counts half
    for a in range(n_ang):
        phi = a * math.pi / n_ang
        c, s = math.cos(phi), math.sin(phi)
        for b in range(bins):
            u = b - 0.5 * (bins - 1)
            if abs(s) < 1e-12 or abs(c) < 1e-12:
                edge = abs(abs(u) - W / 2) < 1e-12
                full = abs(u) < W / 2
                want = (H if full else 0.0) + (0.5 * H if edge else 0.0)
            else:
                want = _clip_len(u * c, u * s, -s, c, -W / 2, W / 2, -H / 2, H / 2)
            assert abs(sums[a * bins + b] - want) < 1e-9, (a, b)


def test_transpose_is_exact():
    rp, col, val = synth.projection_matrix(9, 7, 10, 13)
    tp, tc, tv = synth.transpose_csr(130, 63, rp, col, val)
    assert np.array_equal(_dense(tp, tc, tv, 130), _dense(rp, col, val, 63).T)
    for k in range(63):
        assert np.all(np.diff(tc[tp[k]:tp[k + 1]]) > 0)


def test_phantom_and_noise_seeded():
    a = synth.ellipse_phantom(32, 32, 10, 5)
    b = synth.ellipse_phantom(32, 32, 10, 5)
    assert np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() > 0.0
    p1 = synth.make_problem(n=16, n_ang=10, bins=23, seed=3)
    p2 = synth.make_problem(n=16, n_ang=10, bins=23, seed=3)
    assert np.array_equal(p1.y, p2.y)


def test_block_offsets():
    ro, co = synth.block_offsets(90, 91, 4096, 2, 2)
    assert list(ro) == [0, 45 * 91, 90 * 91]
    assert list(co) == [0, 2048, 4096]
    ro, co = synth.block_offsets(10, 3, 35, 3, 4)
    assert list(ro) == [0, 9, 18, 30] and list(co) == [0, 8, 17, 26, 35]


def test_c1_size():
    p = synth.make_problem("c1_64", with_transpose=False)
    assert p.nrows == 8190 and p.ncols == 4096
    assert 4.5e5 < p.nnz < 5.0e5

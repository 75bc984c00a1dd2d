"""Problem instances: projection matrix, ellipse phantoms, noisy projections.

The paper's own experiment (a fan-beam Shepp-Logan scan, Section 3) gives
no image size, fan geometry or recoverable figure data, so the workloads
here are seeded parallel-beam stand-ins with the shapes below:

  name     image        angles x bins   blocks M x N   noise   lambda  epochs  prox iters
  c1_64    64 x 64      90 x 91         2 x 2          1 %     0.02    100     20
  c2_512   512 x 512    720 x 729       8 x 8          1 %     0.01    200     20
  c3_1024  1024 x 1024  1440 x 1449     16 x 16        0.5 %   0.005   300     30
  c4_vol   256 slices of 512 x 512 sharing the c2_512 matrix (3-D TV)

Angles are spread evenly over [0, pi); the step is mu = 0.9 / (2 u_max)
with u_max the largest eigenvalue of A^T A (Theorem 1 gives the bound
1 / (2 u_max)); u_max is computed by the code that runs the method, not
here.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "siddon.c")
_LIB_PATH = os.path.join(_HERE, "_libsynth.so")
_lib = None
_lib_lock = threading.Lock()


def build_native(force: bool = True) -> str:
    """Compile the generator's C code (host only, gcc + OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build_native(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
            i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
            f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
            lib.siddon_count.argtypes = [ctypes.c_int] * 4 + [i64p]
            lib.siddon_count.restype = ctypes.c_int64
            vp = ctypes.c_void_p
            lib.siddon_fill.argtypes = [ctypes.c_int] * 4 + [i64p, i32p, vp, vp, vp, vp,
                                                             ctypes.c_int]
            lib.siddon_fill.restype = ctypes.c_int
            f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
            lib.csr_transpose_f64.argtypes = [
                ctypes.c_int64, ctypes.c_int64, i64p, i32p, f64p, i64p, i32p, f64p]
            lib.csr_transpose_f64.restype = ctypes.c_int
            lib.csr_transpose_f32.argtypes = [
                ctypes.c_int64, ctypes.c_int64, i64p, i32p, f32p, i64p, i32p, f32p]
            lib.csr_transpose_f32.restype = ctypes.c_int
            lib.synth_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _vptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def projection_matrix(H: int, W: int, n_ang: int, bins: int, dtype=np.float64, x=None):
    """Parallel-beam projection matrix as CSR (row_ptr, col, val).

    Rows are rays (row index angle * bins + bin), columns are pixels
    (row-major s * W + t); entries are exact chord lengths (computed in FP64,
    stored as `dtype`), columns ascending within each row (geometry
    documented in siddon.c).  With an image x (FP64, H*W), also returns
    A x computed in FP64 from the unrounded lengths; x may also be a stack of
    images (S, H*W) or (S, H, W), then A x is returned as (S, r).
    """
    lib = _load()
    nrays = n_ang * bins
    counts = np.zeros(nrays, dtype=np.int64)
    nnz = lib.siddon_count(H, W, n_ang, bins, counts)
    if nnz < 0:
        raise RuntimeError("projection generator: internal ordering check failed")
    row_ptr = np.zeros(nrays + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    del counts
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=dtype)
    nx = 1
    xd = ax = None
    if x is not None:
        xa = np.asarray(x, np.float64)
        if xa.size == H * W:
            xd = np.ascontiguousarray(xa).ravel()
        else:
            nx = xa.shape[0]
            xd = np.ascontiguousarray(xa.reshape(nx, H * W).T)  # [pixel][image]
        ax = np.empty(nrays * nx, np.float64)
    v64 = val if val.dtype == np.float64 else None
    v32 = val if val.dtype == np.float32 else None
    if v64 is None and v32 is None:
        raise ValueError("dtype must be float64 or float32")
    if lib.siddon_fill(H, W, n_ang, bins, row_ptr, col, _vptr(v64), _vptr(v32), _vptr(xd),
                       _vptr(ax), nx) != 0:
        raise RuntimeError("projection generator: fill pass disagreed with count pass")
    if x is None:
        return row_ptr, col, val
    if nx > 1:
        ax = np.ascontiguousarray(ax.reshape(nrays, nx).T)
    return row_ptr, col, val, ax


def transpose_csr(nrows: int, ncols: int, row_ptr, col, val):
    """Stable transpose of a CSR matrix (FP64 or FP32 values; rows of the result sorted)."""
    lib = _load()
    nnz = int(row_ptr[-1])
    t_ptr = np.empty(ncols + 1, dtype=np.int64)
    t_col = np.empty(nnz, dtype=np.int32)
    if val.dtype == np.float32:
        t_val = np.empty(nnz, dtype=np.float32)
        fn = lib.csr_transpose_f32
    else:
        t_val = np.empty(nnz, dtype=np.float64)
        fn = lib.csr_transpose_f64
        val = np.ascontiguousarray(val, np.float64)
    rc = fn(nrows, ncols, np.ascontiguousarray(row_ptr, np.int64),
            np.ascontiguousarray(col, np.int32), val, t_ptr, t_col, t_val)
    if rc != 0:
        raise RuntimeError("transpose: column index out of range")
    return t_ptr, t_col, t_val


def ellipse_phantom(H: int, W: int, n_ellipses: int, seed: int) -> np.ndarray:
    """Sum of seeded random ellipses sampled at pixel centres in [-1, 1]^2.

    Per ellipse, drawn in this order from numpy's default_rng(seed):
    centre radius sqrt(U) and centre angle 2 pi U (uniform in the unit
    disk), semi-axes a, b ~ U[0.05, 0.4], rotation psi ~ U[0, pi),
    intensity ~ U[0.1, 1].  Intensities add where ellipses overlap.
    """
    rng = np.random.default_rng(seed)
    X = (np.arange(W) + 0.5) * (2.0 / W) - 1.0
    Y = 1.0 - (np.arange(H) + 0.5) * (2.0 / H)
    XX, YY = np.meshgrid(X, Y)  # YY[s, t] = Y of row s
    img = np.zeros((H, W), dtype=np.float64)
    for _ in range(n_ellipses):
        rad = np.sqrt(rng.random())
        ang = 2.0 * np.pi * rng.random()
        cx, cy = rad * np.cos(ang), rad * np.sin(ang)
        a = rng.uniform(0.05, 0.4)
        b = rng.uniform(0.05, 0.4)
        psi = rng.uniform(0.0, np.pi)
        inten = rng.uniform(0.1, 1.0)
        dx, dy = XX - cx, YY - cy
        xr = dx * np.cos(psi) + dy * np.sin(psi)
        yr = -dx * np.sin(psi) + dy * np.cos(psi)
        img[(xr / a) ** 2 + (yr / b) ** 2 <= 1.0] += inten
    return img


def block_offsets(n_ang: int, bins: int, n_pix: int, M: int, N: int):
    """Row and column block boundaries (Section 2.1's partition of A).

    Row block I_i is a contiguous group of whole angles (as even as
    possible), column block J_j a contiguous range of the row-major pixel
    index.  Returns int64 arrays row_off (M+1) and col_off (N+1).
    """
    if not (1 <= M <= n_ang) or not (1 <= N <= n_pix):
        raise ValueError("block counts out of range")
    row_off = np.array([(i * n_ang) // M * bins for i in range(M + 1)], dtype=np.int64)
    col_off = np.array([(j * n_pix) // N for j in range(N + 1)], dtype=np.int64)
    return row_off, col_off


@dataclasses.dataclass
class Problem:
    """One reconstruction instance (all arrays on the host, FP64 values)."""
    name: str
    H: int
    W: int
    n_ang: int
    bins: int
    M: int
    N: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    row_off: np.ndarray
    col_off: np.ndarray
    x_true: np.ndarray      # (H, W) or (S, H, W) for a slice stack
    y: np.ndarray           # (r,) or (r, S)
    lam: float
    epochs: int
    prox_iters: int
    noise_frac: float
    seed: int
    t_ptr: np.ndarray | None = None
    t_col: np.ndarray | None = None
    t_val: np.ndarray | None = None

    @property
    def nrows(self) -> int:
        return self.n_ang * self.bins

    @property
    def ncols(self) -> int:
        return self.H * self.W

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def ensure_transpose(self):
        if self.t_ptr is None:
            self.t_ptr, self.t_col, self.t_val = transpose_csr(
                self.nrows, self.ncols, self.row_ptr, self.col, self.val)
        return self.t_ptr, self.t_col, self.t_val


CONFIGS = {
    "c1_64": dict(n=64, n_ang=90, bins=91, M=2, N=2, noise=0.01, lam=0.02,
                  epochs=100, prox_iters=20, seed=0),
    "c2_512": dict(n=512, n_ang=720, bins=729, M=8, N=8, noise=0.01, lam=0.01,
                   epochs=200, prox_iters=20, seed=1),
    "c3_1024": dict(n=1024, n_ang=1440, bins=1449, M=16, N=16, noise=0.005,
                    lam=0.005, epochs=300, prox_iters=30, seed=2),
}


def make_problem(name: str | None = None, *, n: int | None = None, H: int | None = None,
                 W: int | None = None, n_ang: int | None = None, bins: int | None = None,
                 M: int = 1, N: int = 1, noise: float = 0.01, lam: float = 0.0,
                 epochs: int = 10, prox_iters: int = 20, seed: int = 0,
                 n_ellipses: int = 10, with_transpose: bool = True,
                 dtype=np.float64) -> Problem:
    """Build a named configuration (see the module docstring) or a custom one.

    dtype = np.float32 stores the matrix values rounded to FP32 (for the
    device path of the large workloads); the projections y are computed in
    FP64 from the unrounded lengths either way.
    """
    if name is not None:
        cfg = dict(CONFIGS[name])
        n, n_ang, bins, M, N = cfg["n"], cfg["n_ang"], cfg["bins"], cfg["M"], cfg["N"]
        noise, lam, epochs = cfg["noise"], cfg["lam"], cfg["epochs"]
        prox_iters, seed = cfg["prox_iters"], cfg["seed"]
    H = H if H is not None else n
    W = W if W is not None else n
    if bins is None:
        bins = int(np.ceil(max(H, W) * np.sqrt(2.0))) | 1
    x_true = ellipse_phantom(H, W, n_ellipses, seed)
    row_ptr, col, val, ax = projection_matrix(H, W, n_ang, bins, dtype=dtype, x=x_true)
    row_off, col_off = block_offsets(n_ang, bins, H * W, M, N)
    sigma = noise * float(np.max(ax)) if ax.size else 0.0
    rng = np.random.default_rng(seed + 10**6)
    y = ax + sigma * rng.standard_normal(ax.shape[0])
    prob = Problem(name=name or "custom", H=H, W=W, n_ang=n_ang, bins=bins, M=M, N=N,
                   row_ptr=row_ptr, col=col, val=val, row_off=row_off, col_off=col_off,
                   x_true=x_true, y=y, lam=lam, epochs=epochs, prox_iters=prox_iters,
                   noise_frac=noise, seed=seed)
    if with_transpose:
        prob.ensure_transpose()
    return prob


def seeded_vector(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded FP64 test vector U[0, scale) (shared input for parity cases)."""
    return scale * np.random.default_rng(seed).random(n)


def make_volume_problem(S: int = 256, base: str = "c2_512", first_seed: int = 1000,
                        dtype=np.float32, with_transpose: bool = True) -> Problem:
    """A stack of S slices sharing one 2-D geometry (the batched workload).

    Slice s has its own ellipse phantom (seed first_seed + s) and noise
    (seed first_seed + s + 10^6, sigma = noise * max of that slice's
    projections).  x_true is (S, H, W); y is (S, r), one sinogram per slice.
    """
    cfg = dict(CONFIGS[base])
    n, n_ang, bins = cfg["n"], cfg["n_ang"], cfg["bins"]
    X = np.stack([ellipse_phantom(n, n, 10, first_seed + s) for s in range(S)])
    row_ptr, col, val, AX = projection_matrix(n, n, n_ang, bins, dtype=dtype, x=X)
    Y = np.empty_like(AX)
    for s in range(S):
        rng = np.random.default_rng(first_seed + s + 10**6)
        Y[s] = AX[s] + cfg["noise"] * float(np.max(AX[s])) * rng.standard_normal(AX.shape[1])
    row_off, col_off = block_offsets(n_ang, bins, n * n, cfg["M"], cfg["N"])
    prob = Problem(name=f"c4_vol_{S}", H=n, W=n, n_ang=n_ang, bins=bins, M=cfg["M"], N=cfg["N"],
                   row_ptr=row_ptr, col=col, val=val, row_off=row_off, col_off=col_off,
                   x_true=X, y=Y, lam=cfg["lam"], epochs=cfg["epochs"],
                   prox_iters=cfg["prox_iters"], noise_frac=cfg["noise"], seed=first_seed)
    if with_transpose:
        prob.ensure_transpose()
    return prob


def block_subsets(iters: int, M: int, N: int, alpha: float, gamma: float, seed: int):
    """Seeded draws of the blocks that take part in each partial iteration.

    Iteration t takes max(1, round(gamma * M)) of the M row blocks and
    max(1, round(alpha * N)) of the N column blocks, uniformly without
    replacement, from numpy.random.default_rng(seed).  Returns two uint64
    arrays of length `iters` holding the draws as bit masks (bit i set when
    block i is taken); M and N are at most 64.
    """
    if not (1 <= M <= 64 and 1 <= N <= 64):
        raise ValueError("bit masks hold at most 64 blocks")
    if not (0.0 < alpha <= 1.0 and 0.0 < gamma <= 1.0):
        raise ValueError("fractions must lie in (0, 1]")
    rng = np.random.default_rng(seed)
    nr, nc = max(1, int(round(gamma * M))), max(1, int(round(alpha * N)))
    rows = np.zeros(iters, np.uint64)
    cols = np.zeros(iters, np.uint64)
    for t in range(iters):
        for i in rng.choice(M, nr, replace=False):
            rows[t] |= np.uint64(1) << np.uint64(i)
        for j in rng.choice(N, nc, replace=False):
            cols[t] |= np.uint64(1) << np.uint64(j)
    return rows, cols

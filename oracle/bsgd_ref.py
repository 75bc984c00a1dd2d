"""FP64 CPU oracle of BSGD-TV (Gao & Blumensath, arXiv 1812.01307).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
device path is checked against.  Only the test suite, the package's smoke
check and the benchmark's CPU-baseline leg may import it; the library never
does.  It shares no code with the device path: it takes problem arrays
(CSR of A, y, ...) from the seeded generator and computes everything
itself with numpy / scipy.sparse in float64.

What it computes, and where the paper defines it:

* Objective (Eq. 1 with the Alg. 1 line-9 reading below):
  F(x) = ||y - A x||^2 + lam * TV(x).
* 2-D isotropic TV (Eq. 2) with backward differences; the garbled second
  term of Eq. 2 is read as x[s,t] - x[s,t-1]; a difference that would reach
  outside the image (s = 0 or t = 0) is zero.
* One epoch of Algorithm 1 with every block pair active:
      g  = sum_i 2 (A_{I_i}^{J_j})^T r_{I_i}      (backprojection and gradient sum)
      r' = y - sum_j A_{I_i}^{J_j} x_{J_j}         (forward projection and residual)
      x^ = x + mu g                                (the gradient step)
      x  = argmin_t ||t - x^||^2 + 2 mu lam TV(t)  (the TV prox step)
      r  = r'
  The residual used in the block backprojection is one epoch old, which is Eq. 3:
  x^{k+1} = prox(x^k + 2 mu A^T (y - A x^{k-1})).  Initialisation (the
  paper ignores it): x = x0 (default 0) and r = y - A x0.
* The TV prox step is solved by the fast gradient projection (FGP) method that the
  paper cites for it (Beck & Teboulle, IEEE TIP 18(11), 2009): projected
  gradient steps with FISTA momentum on the dual of
      min_t 1/2 ||t - b||^2 + theta TV(t),   theta = mu * lam,
  which has the same minimiser as the TV prox step.  The dual step is 1/(8 theta)
  because ||D||^2 <= 8 for the 2-D difference operator (12 in 3-D).
  No constraint set is applied (no clamp), and every call starts the dual
  at zero.
* u_max = largest eigenvalue of A^T A (Theorem 1) by power iteration from
  the all-ones vector; the step used throughout is mu = 0.9 / (2 u_max).
* The M x N block partition of Section 2.1 and a blocked epoch that sums
  the block products in ascending block order (used to show that blocking
  changes rounding only).
* The Simulations section's comparison methods: ISTA (the same gradient and prox steps
  step with the current iterate's gradient, A taken whole) and gradient
  descent on f alone (ISTA with lam = 0).
* Algorithm 1 on drawn subsets of the row and column blocks (Simulations
  section, fractions gamma and alpha); the handling of the blocks left out
  of an iteration is a reading, stated at selected_iteration.

Where the paper is silent or ambiguous the readings above are used; the
design notes list them.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# ---------------------------------------------------------------------------
# Sparse products (both block products of Alg. 1, summed over blocks)
# ---------------------------------------------------------------------------


def as_matrix(row_ptr, col, val, ncols: int) -> sp.csr_matrix:
    """Wrap a CSR triple as a scipy matrix (FP64 values)."""
    nrows = len(row_ptr) - 1
    return sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col), np.asarray(row_ptr)),
                         shape=(nrows, ncols))


def forward(A: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """A x: all block forward projections z^j_{I_i} summed over j (the block forward projection of Alg. 1)."""
    return A @ np.asarray(x, np.float64)


def backproject(A: sp.csr_matrix, r: np.ndarray) -> np.ndarray:
    """2 A^T r: all block backprojections g^i_{J_j} summed over i (the block backprojection of Alg. 1)."""
    return 2.0 * (A.T @ np.asarray(r, np.float64))


# ---------------------------------------------------------------------------
# Total variation (Eq. 2) and its difference operator
# ---------------------------------------------------------------------------


def grad2(x: np.ndarray):
    """Backward differences D x of an H x W image: (vertical, horizontal)."""
    x = np.asarray(x, np.float64)
    dv = np.zeros_like(x)
    dh = np.zeros_like(x)
    dv[1:, :] = x[1:, :] - x[:-1, :]
    dh[:, 1:] = x[:, 1:] - x[:, :-1]
    return dv, dh


def grad2_adj(pv: np.ndarray, ph: np.ndarray) -> np.ndarray:
    """Adjoint D^T p of grad2 (only rows s >= 1 of pv and columns t >= 1 of ph enter)."""
    out = np.zeros_like(pv)
    out[1:, :] += pv[1:, :]
    out[:-1, :] -= pv[1:, :]
    out[:, 1:] += ph[:, 1:]
    out[:, :-1] -= ph[:, 1:]
    return out


def tv2(x: np.ndarray) -> float:
    """Isotropic TV of Eq. 2: sum over pixels of the length of (D x)[s, t]."""
    dv, dh = grad2(x)
    return float(np.sum(np.sqrt(dv * dv + dh * dh)))


def grad3(x: np.ndarray):
    """Backward differences of a D x H x W volume along (depth, rows, columns)."""
    x = np.asarray(x, np.float64)
    dd = np.zeros_like(x)
    dv = np.zeros_like(x)
    dh = np.zeros_like(x)
    dd[1:] = x[1:] - x[:-1]
    dv[:, 1:, :] = x[:, 1:, :] - x[:, :-1, :]
    dh[:, :, 1:] = x[:, :, 1:] - x[:, :, :-1]
    return dd, dv, dh


def grad3_adj(pd, pv, ph) -> np.ndarray:
    """Adjoint of grad3."""
    out = np.zeros_like(pd)
    out[1:] += pd[1:]
    out[:-1] -= pd[1:]
    out[:, 1:, :] += pv[:, 1:, :]
    out[:, :-1, :] -= pv[:, 1:, :]
    out[:, :, 1:] += ph[:, :, 1:]
    out[:, :, :-1] -= ph[:, :, 1:]
    return out


def tv3(x: np.ndarray) -> float:
    """Isotropic 3-D TV: Eq. 2 extended with a backward difference across slices."""
    dd, dv, dh = grad3(x)
    return float(np.sum(np.sqrt(dd * dd + dv * dv + dh * dh)))


# ---------------------------------------------------------------------------
# TV proximal step of Alg. 1 by FGP on the dual
# ---------------------------------------------------------------------------


def fista_tau(iters: int) -> np.ndarray:
    """Momentum sequence tau_1 = 1, tau_{k+1} = (1 + sqrt(1 + 4 tau_k^2)) / 2."""
    tau = np.empty(iters + 1)
    tau[0] = 1.0
    for k in range(iters):
        tau[k + 1] = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * tau[k] * tau[k]))
    return tau


def fgp_prox2(b: np.ndarray, theta: float, iters: int, return_dual: bool = False):
    """argmin_t 1/2||t - b||^2 + theta TV(t) by `iters` FGP iterations.

    Dual variable p = (pv, ph), one 2-vector per pixel, constrained to the
    unit disk.  Iteration k (q_1 = 0, p_0 = 0, tau_1 = 1):
        u_k     = b - theta D^T q_k
        p_k     = P(q_k + D u_k / (8 theta))      P: pointwise unit-disk projection
        q_{k+1} = p_k + (tau_k - 1)/tau_{k+1} (p_k - p_{k-1})
    and the result is b - theta D^T p_K.
    """
    b = np.asarray(b, np.float64)
    if theta == 0.0 or iters == 0:
        out = b.copy()
        zero = np.zeros_like(b)
        return (out, (zero, zero.copy())) if return_dual else out
    tau = fista_tau(iters)
    pv_old = np.zeros_like(b)
    ph_old = np.zeros_like(b)
    qv = np.zeros_like(b)
    qh = np.zeros_like(b)
    step = 1.0 / (8.0 * theta)
    for k in range(iters):
        u = b - theta * grad2_adj(qv, qh)
        gv, gh = grad2(u)
        pv = qv + step * gv
        ph = qh + step * gh
        nrm = np.maximum(1.0, np.sqrt(pv * pv + ph * ph))
        pv /= nrm
        ph /= nrm
        coef = (tau[k] - 1.0) / tau[k + 1]
        qv = pv + coef * (pv - pv_old)
        qh = ph + coef * (ph - ph_old)
        pv_old, ph_old = pv, ph
    out = b - theta * grad2_adj(pv_old, ph_old)
    return (out, (pv_old, ph_old)) if return_dual else out


def fgp_prox3(b: np.ndarray, theta: float, iters: int, return_dual: bool = False):
    """3-D version of fgp_prox2 (unit-ball projection in R^3, dual step 1/(12 theta))."""
    b = np.asarray(b, np.float64)
    if theta == 0.0 or iters == 0:
        out = b.copy()
        return (out, None) if return_dual else out
    tau = fista_tau(iters)
    old = [np.zeros_like(b) for _ in range(3)]
    q = [np.zeros_like(b) for _ in range(3)]
    step = 1.0 / (12.0 * theta)
    for k in range(iters):
        u = b - theta * grad3_adj(*q)
        g = grad3(u)
        p = [q[a] + step * g[a] for a in range(3)]
        nrm = np.maximum(1.0, np.sqrt(p[0] ** 2 + p[1] ** 2 + p[2] ** 2))
        p = [pa / nrm for pa in p]
        coef = (tau[k] - 1.0) / tau[k + 1]
        q = [p[a] + coef * (p[a] - old[a]) for a in range(3)]
        old = p
    out = b - theta * grad3_adj(*old)
    return (out, old) if return_dual else out


# ---------------------------------------------------------------------------
# Step size (Theorem 1)
# ---------------------------------------------------------------------------


def power_umax(A: sp.csr_matrix, tol: float = 1e-12, max_iter: int = 100000) -> float:
    """Largest eigenvalue of A^T A by power iteration from the all-ones vector.

    Stops when the Rayleigh quotient changes by less than `tol` (relative).
    """
    v = np.ones(A.shape[1]) / np.sqrt(A.shape[1])
    u = 0.0
    for _ in range(max_iter):
        w = A.T @ (A @ v)
        u_new = float(v @ w)
        nrm = float(np.linalg.norm(w))
        if nrm == 0.0:
            return 0.0
        v = w / nrm
        if abs(u_new - u) <= tol * abs(u_new):
            return u_new
        u = u_new
    return u


def step_size(u_max: float, factor: float = 0.9) -> float:
    """mu = factor / (2 u_max); Theorem 1 needs factor < 1 at lam = 0."""
    return factor / (2.0 * u_max)


# ---------------------------------------------------------------------------
# Algorithm 1, unblocked form
# ---------------------------------------------------------------------------


def prox(xhat: np.ndarray, theta: float, prox_iters: int, shape) -> np.ndarray:
    """The TV prox step of Alg. 1 on the image of `shape` (2-D or 3-D)."""
    if theta == 0.0:
        return xhat.copy()
    img = xhat.reshape(shape)
    if len(shape) == 2:
        return fgp_prox2(img, theta, prox_iters).ravel()
    return fgp_prox3(img, theta, prox_iters).ravel()


def bsgd_epoch(A, y, x, r, mu: float, lam: float, prox_iters: int, shape):
    """One epoch of Algorithm 1 (all block pairs); returns (x_new, r_new)."""
    g = backproject(A, r)                 # backprojection and gradient sum, stale residual
    r_new = y - forward(A, x)             # forward projection and residual, current x
    xhat = x + mu * g                     # the gradient step
    x_new = prox(xhat, mu * lam, prox_iters, shape)   # the TV prox step
    return x_new, r_new


def initial_state(A, y, x0=None):
    """x = x0 (zero by default), r = y - A x0."""
    if x0 is None:
        return np.zeros(A.shape[1]), np.asarray(y, np.float64).copy()
    x0 = np.asarray(x0, np.float64).copy()
    return x0, np.asarray(y, np.float64) - forward(A, x0)


def bsgd_tv(A, y, mu: float, lam: float, epochs: int, prox_iters: int, shape,
            x0=None, state=None, record: bool = False):
    """Run `epochs` epochs of Algorithm 1.

    Returns (x, r) after the last epoch and, with record=True, the list of
    iterates x after each epoch.  `state` = (x, r) resumes a run.
    """
    x, r = state if state is not None else initial_state(A, y, x0)
    x = np.array(x, np.float64)
    r = np.array(r, np.float64)
    hist = []
    for _ in range(epochs):
        x, r = bsgd_epoch(A, y, x, r, mu, lam, prox_iters, shape)
        if record:
            hist.append(x.copy())
    return (x, r, hist) if record else (x, r)


def objective(A, y, x, lam: float, shape) -> float:
    """F(x) = ||y - A x||^2 + lam TV(x) (the problem that the TV prox step of Alg. 1 targets)."""
    res = y - forward(A, x)
    tv = tv2(x.reshape(shape)) if len(shape) == 2 else tv3(x.reshape(shape))
    return float(res @ res) + lam * tv


def thm2_margin(A, y, x_prev, x_cur, x_next, mu: float) -> float:
    """Right side minus left side of Theorem 2's condition (Eq. 8) at one epoch.

    f(x) = ||y - A x||^2.  A positive value means the condition holds.
    """
    f = lambda v: float(np.sum((y - forward(A, v)) ** 2))  # noqa: E731
    grad_prev = -2.0 * (A.T @ (y - forward(A, x_prev)))
    d = x_next - x_cur
    rhs = f(x_cur) + float(d @ grad_prev) + float(d @ d) / (2.0 * mu)
    return rhs - f(x_next)


# ---------------------------------------------------------------------------
# Block partition (Section 2.1) and the blocked epoch
# ---------------------------------------------------------------------------


def tile(row_ptr, col, val, row_off, col_off, i: int, j: int):
    """Block A_{I_i}^{J_j} of Section 2.1's partition as a block-local CSR.

    Returns (ptr, lcol, lval): row pointers (int64, |I_i|+1 entries),
    column indices relative to the block's first column (int32, ascending
    within each row) and the values, in the order they appear in A.
    """
    r0, r1 = int(row_off[i]), int(row_off[i + 1])
    c0, c1 = int(col_off[j]), int(col_off[j + 1])
    a0, a1 = int(row_ptr[r0]), int(row_ptr[r1])
    cs = np.asarray(col[a0:a1])
    rows = np.repeat(np.arange(r1 - r0), np.diff(np.asarray(row_ptr[r0:r1 + 1])))
    sel = (cs >= c0) & (cs < c1)
    ptr = np.zeros(r1 - r0 + 1, np.int64)
    np.cumsum(np.bincount(rows[sel], minlength=r1 - r0), out=ptr[1:])
    return ptr, (cs[sel] - c0).astype(np.int32), np.asarray(val[a0:a1])[sel]


def tile_transpose(ptr, lcol, lval, ncols_block: int):
    """Transpose of a block-local CSR (rows = the block's pixels, columns = its rays)."""
    nrows_block = len(ptr) - 1
    T = sp.csr_matrix((lval, lcol, ptr), shape=(nrows_block, ncols_block)).T.tocsr()
    T.sort_indices()
    return T.indptr.astype(np.int64), T.indices.astype(np.int32), T.data.astype(lval.dtype)


def tiles(row_ptr, col, val, row_off, col_off):
    """All M x N blocks: dict (i, j) -> block CSR and ('T', i, j) -> its transpose."""
    M, N = len(row_off) - 1, len(col_off) - 1
    out = {}
    for i in range(M):
        for j in range(N):
            blk = tile(row_ptr, col, val, row_off, col_off, i, j)
            out[(i, j)] = blk
            out[("T", i, j)] = tile_transpose(*blk, int(col_off[j + 1] - col_off[j]))
    return out


def bsgd_epoch_blocked(blocks, row_off, col_off, y, x, r, mu: float, lam: float,
                       prox_iters: int, shape):
    """Algorithm 1 epoch written block by block.

    z^j_{I_i} = A_{I_i}^{J_j} x_{J_j};  g^i_{J_j} = 2 (A_{I_i}^{J_j})^T r_{I_i};
    r_{I_i} = y_{I_i} - sum_j z^j (ascending j);  g_{J_j} = sum_i g^i (ascending i).
    """
    M, N = len(row_off) - 1, len(col_off) - 1
    g = np.zeros_like(x)
    r_new = np.empty_like(r)
    z = {}
    ghat = {}
    for i in range(M):                      # the pair loop (order is irrelevant)
        r0, r1 = int(row_off[i]), int(row_off[i + 1])
        for j in range(N):
            c0, c1 = int(col_off[j]), int(col_off[j + 1])
            ptr, lcol, lval = blocks[(i, j)]
            Aij = sp.csr_matrix((lval, lcol, ptr), shape=(r1 - r0, c1 - c0))
            ghat[(i, j)] = 2.0 * (Aij.T @ r[r0:r1])
            z[(i, j)] = Aij @ x[c0:c1]
    for i in range(M):
        r0, r1 = int(row_off[i]), int(row_off[i + 1])
        acc = np.zeros(r1 - r0)
        for j in range(N):
            acc = acc + z[(i, j)]
        r_new[r0:r1] = y[r0:r1] - acc
    for j in range(N):
        c0, c1 = int(col_off[j]), int(col_off[j + 1])
        acc = np.zeros(c1 - c0)
        for i in range(M):
            acc = acc + ghat[(i, j)]
        g[c0:c1] = acc
    xhat = x + mu * g
    return prox(xhat, mu * lam, prox_iters, shape), r_new


def block_forward(blocks, row_off, col_off, i: int, j: int, x_block):
    """z^j_{I_i} = A_{I_i}^{J_j} x_{J_j} for one block (the block forward projection of Alg. 1)."""
    r0, r1 = int(row_off[i]), int(row_off[i + 1])
    c0, c1 = int(col_off[j]), int(col_off[j + 1])
    ptr, lcol, lval = blocks[(i, j)]
    return sp.csr_matrix((lval, lcol, ptr), shape=(r1 - r0, c1 - c0)) @ x_block


def block_backproject(blocks, row_off, col_off, i: int, j: int, r_block):
    """g^i_{J_j} = 2 (A_{I_i}^{J_j})^T r_{I_i} for one block (the block backprojection of Alg. 1)."""
    r0, r1 = int(row_off[i]), int(row_off[i + 1])
    c0, c1 = int(col_off[j]), int(col_off[j + 1])
    ptr, lcol, lval = blocks[(i, j)]
    return 2.0 * (sp.csr_matrix((lval, lcol, ptr), shape=(r1 - r0, c1 - c0)).T @ r_block)


# ---------------------------------------------------------------------------
# Several right-hand sides sharing A (slices of a volume, or a batch of
# independent reconstructions on one geometry)
# ---------------------------------------------------------------------------


def bsgd_epoch_multi(A, Y, X, R, mu: float, lam, prox_iters: int, shape2d, volume: bool):
    """One epoch of Algorithm 1 applied to S right-hand sides at once.

    Y, R: (S, r) arrays and X: (S, c) arrays, one row per RHS.  The products
    are those of bsgd_epoch for every RHS.  The TV prox step is either the 3-D TV prox
    of the volume whose slices are the RHS (volume=True, one lam), or the 2-D
    prox of each RHS with its own lam[j] (volume=False).
    """
    S = X.shape[0]
    H, W = shape2d
    G = 2.0 * np.asarray(A.T @ R.T).T           # backprojection and gradient sum, stale residuals
    R_new = Y - np.asarray(A @ X.T).T           # forward projection and residual
    Xhat = X + mu * G                           # the gradient step
    if volume:
        theta = mu * float(lam)
        X_new = (fgp_prox3(Xhat.reshape(S, H, W), theta, prox_iters).reshape(S, H * W)
                 if theta != 0.0 else Xhat.copy())
    else:
        lam = np.broadcast_to(np.asarray(lam, np.float64), (S,))
        X_new = np.empty_like(Xhat)
        for j in range(S):
            X_new[j] = prox(Xhat[j], mu * float(lam[j]), prox_iters, (H, W))
    return X_new, R_new


def bsgd_tv_multi(A, Y, mu: float, lam, epochs: int, prox_iters: int, shape2d, volume: bool,
                  record: bool = False):
    """Run epochs of bsgd_epoch_multi from X = 0, R = Y (the single-RHS initialisation)."""
    Y = np.asarray(Y, np.float64)
    X = np.zeros((Y.shape[0], A.shape[1]))
    R = Y.copy()
    hist = []
    for _ in range(epochs):
        X, R = bsgd_epoch_multi(A, Y, X, R, mu, lam, prox_iters, shape2d, volume)
        if record:
            hist.append(X.copy())
    return (X, R, hist) if record else (X, R)


# ---------------------------------------------------------------------------
# Comparison methods of the Simulations section (Fig. 2): ISTA and GD
# ---------------------------------------------------------------------------


def ista_epoch(A, y, x, mu: float, lam: float, prox_iters: int, shape):
    """One ISTA iteration on F (the proximal gradient method the paper compares with).

    The gradient and prox steps of Algorithm 1 with the gradient of the current
    iterate (no delay; A taken as a whole, Fig. 2 caption):
        r  = y - A x
        x' = argmin_t ||t - (x + 2 mu A^T r)||^2 + 2 mu lam TV(t).
    Returns (x', r): r is the residual of the input iterate, so the pair has
    the meaning of Algorithm 1's state (the residual one iterate behind).
    """
    r = y - forward(A, x)
    xhat = x + mu * backproject(A, r)
    return prox(xhat, mu * lam, prox_iters, shape), r


def ista_tv(A, y, mu: float, lam: float, epochs: int, prox_iters: int, shape,
            x0=None, record: bool = False):
    """Run `epochs` ISTA iterations from x0 (zero by default).

    Returns (x, r) after the last iteration (r = y - A x of the iterate
    before it) and, with record=True, the iterates after every iteration.
    """
    x = np.zeros(A.shape[1]) if x0 is None else np.array(x0, np.float64)
    r = np.asarray(y, np.float64) - forward(A, x)
    hist = []
    for _ in range(epochs):
        x, r = ista_epoch(A, y, x, mu, lam, prox_iters, shape)
        if record:
            hist.append(x.copy())
    return (x, r, hist) if record else (x, r)


def gd(A, y, mu: float, epochs: int, x0=None, record: bool = False):
    """Gradient descent on f(x) = ||y - A x||^2 with step mu (Fig. 2's GD).

    x_{k+1} = x_k + 2 mu A^T (y - A x_k): ISTA without the TV term.
    """
    shape = (A.shape[1],)
    return ista_tv(A, y, mu, 0.0, epochs, 0, shape, x0=x0, record=record)


# ---------------------------------------------------------------------------
# Algorithm 1 on drawn subsets of the blocks (Simulations section: only
# fractions alpha of {x_{J_j}} and gamma of {y_{I_i}} take part in an
# iteration)
# ---------------------------------------------------------------------------


def mask_members(mask: int, n: int):
    """Ascending indices k < n whose bit is set in `mask`."""
    return [k for k in range(n) if (int(mask) >> k) & 1]


def selected_iteration(blocks, row_off, col_off, y, x, r, Z, mu: float, lam: float,
                       prox_iters: int, shape, rows_mask: int, cols_mask: int):
    """One iteration of Algorithm 1 that runs only the pairs (i, j), i in I, j in J.

    I and J are the set bits of rows_mask and cols_mask.  Reading of what
    the paper leaves open (it states only that the method still converges
    with such subsets):
      * every pair keeps the last product z^j_{I_i} it computed, in Z[j]
        (a full-length ray vector per column block);
      * both block products run for the selected pairs: g^i_{J_j} from the kept
        residual r_{I_i}, and z^j_{I_i} from the current x_{J_j} (stored in Z);
      * the residual update refreshes r_{I_i} for i in I from y and the kept products of
        all column blocks, ascending j; other rows keep their residual;
      * the gradient sum sums g^i over i in I only (no rescaling); the gradient step moves the
        selected column blocks; the other blocks of x stay as they are;
      * the TV prox step runs on the whole image with theta = mu * lam, as written.
    With every bit set this is bsgd_epoch_blocked.  Returns (x, r, Z) as new
    arrays.
    """
    M, N = len(row_off) - 1, len(col_off) - 1
    I, J = mask_members(rows_mask, M), mask_members(cols_mask, N)
    Z = Z.copy()
    r_new = r.copy()
    g = np.zeros_like(x)
    for j in J:                                   # backprojection and gradient sum over i in I
        c0, c1 = int(col_off[j]), int(col_off[j + 1])
        acc = np.zeros(c1 - c0)
        for i in I:
            r0, r1 = int(row_off[i]), int(row_off[i + 1])
            acc = acc + block_backproject(blocks, row_off, col_off, i, j, r[r0:r1])
        g[c0:c1] = acc
    for i in I:                                   # the block forward projection, then the residual update for I_i
        r0, r1 = int(row_off[i]), int(row_off[i + 1])
        for j in J:
            c0, c1 = int(col_off[j]), int(col_off[j + 1])
            Z[j, r0:r1] = block_forward(blocks, row_off, col_off, i, j, x[c0:c1])
        acc = np.zeros(r1 - r0)
        for j in range(N):
            acc = acc + Z[j, r0:r1]
        r_new[r0:r1] = y[r0:r1] - acc
    xhat = x + mu * g                             # the gradient step (zero outside J)
    return prox(xhat, mu * lam, prox_iters, shape), r_new, Z


def selected_initial_state(blocks, row_off, col_off, y, x0=None):
    """x = x0 (zero by default); Z[j] = the block products of x0; r = y - sum_j Z[j]."""
    M, N = len(row_off) - 1, len(col_off) - 1
    nrows, ncols = int(row_off[-1]), int(col_off[-1])
    x = np.zeros(ncols) if x0 is None else np.array(x0, np.float64)
    Z = np.zeros((N, nrows))
    for i in range(M):
        r0, r1 = int(row_off[i]), int(row_off[i + 1])
        for j in range(N):
            c0, c1 = int(col_off[j]), int(col_off[j + 1])
            Z[j, r0:r1] = block_forward(blocks, row_off, col_off, i, j, x[c0:c1])
    r = np.asarray(y, np.float64) - Z.sum(axis=0) if x0 is not None else \
        np.asarray(y, np.float64).copy()
    return x, r, Z


def bsgd_selected(blocks, row_off, col_off, y, mu: float, lam: float, prox_iters: int, shape,
                  rows_masks, cols_masks, x0=None, state=None, record: bool = False):
    """Iterations of selected_iteration, one per (rows_masks[t], cols_masks[t]).

    Returns (x, r, Z) and, with record=True, the iterates after every
    iteration.  `state` = (x, r, Z) resumes a run.
    """
    x, r, Z = state if state is not None else selected_initial_state(blocks, row_off, col_off,
                                                                     y, x0)
    hist = []
    for rm, cm in zip(rows_masks, cols_masks):
        x, r, Z = selected_iteration(blocks, row_off, col_off, y, x, r, Z, mu, lam, prox_iters,
                                     shape, int(rm), int(cm))
        if record:
            hist.append(x.copy())
    return (x, r, Z, hist) if record else (x, r, Z)


def selected_epochs(rows_masks, cols_masks, M: int, N: int) -> np.ndarray:
    """Epoch count after each iteration: the fraction of the M x N pairs run, summed."""
    frac = [bin(int(a)).count("1") * bin(int(b)).count("1") / (M * N)
            for a, b in zip(rows_masks, cols_masks)]
    return np.cumsum(frac)

/*
 * bsgd.h — C ABI of the BSGD-TV device library (gfx950 / MI355X).
 *
 * BSGD-TV (Gao & Blumensath, "BSGD-TV: A parallel algorithm solving total
 * variation constrained image reconstruction problems", arXiv 1812.01307)
 * minimises ||y - A x||^2 + (TV term) for a sparse X-ray projection matrix A
 * (r rays x c pixels) split into M row blocks I_i and N column blocks J_j
 * (Section 2.1).  Each epoch of Algorithm 1 computes, for every block pair,
 *     g^i_{J_j} = 2 (A_{I_i}^{J_j})^T r_{I_i}      (the block backprojection)
 *     z^j_{I_i} = A_{I_i}^{J_j} x_{J_j}             (the block forward projection)
 * then r = y - sum_j z^j (the residual update), g = sum_i g^i (the gradient sum), x = x + mu g
 * (the gradient step) and x = argmin_t ||t - x||^2 + 2 mu lam TV(t) (the TV prox step), the last
 * solved by fast gradient projection (FGP) on the dual (the method the
 * paper cites for the TV prox step).
 *
 * Conventions for every call:
 *   - Pointers documented as "device" point to HIP device memory owned by
 *     the caller; the library never frees them and never keeps them beyond
 *     the object that borrows them (plan or state).  "host" pointers are
 *     read during the call only.
 *   - Calls that take a stream enqueue work on it and return without
 *     waiting, unless the description says "synchronises".
 *   - Every call returns a bsgd_status; on failure nothing has been
 *     enqueued (argument errors) or the HIP error is reported
 *     (BSGD_ERR_HIP), and bsgd_last_error() gives a message (thread-local).
 *   - The library allocates no device memory: plans and states live in
 *     caller-provided workspaces whose sizes the *_workspace_size calls
 *     return.  It allocates small host structures only.
 *   - Vectors are FP32.  Images are row-major H x W (pixel index s*W + t,
 *     row s from the top); a D-slice volume is D consecutive images.
 */
#ifndef BSGD_H
#define BSGD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BSGD_OK = 0,
  BSGD_ERR_INVALID = -1,     /* bad argument or inconsistent input data     */
  BSGD_ERR_WORKSPACE = -2,   /* workspace smaller than the size query gave  */
  BSGD_ERR_HIP = -3,         /* a HIP runtime call failed                   */
  BSGD_ERR_UNSUPPORTED = -4, /* valid request the library does not implement */
  BSGD_ERR_DIVERGED = -5     /* residual norm is not finite                 */
} bsgd_status;

/* Element type of the stored matrix values; accumulation is always FP32. */
typedef enum { BSGD_VAL_F32 = 0, BSGD_VAL_F16 = 1 } bsgd_valtype;

/* Plan flags. */
#define BSGD_PLAN_F16 1u      /* also keep an FP16 (round-to-nearest-even) copy of the values */
#define BSGD_PLAN_AUTOTUNE 2u /* time the row kernels per store and keep the fastest launch */
#define BSGD_PLAN_STAGED_FWD 4u /* also build the staged form of the forward store (A) */
#define BSGD_PLAN_STAGED_BWD 8u /* also build the staged form of the backward store (A^T) */
#define BSGD_PLAN_STAGED 12u    /* both staged forms */
/*
 * Build the block store of A only, not that of A^T: for plans whose epochs
 * run on the tile-sliced store (bsgd_fused_create), which yields A x and
 * A^T r from one read of A.  Calls that need the A^T store return
 * BSGD_ERR_UNSUPPORTED (bsgd_backproject, bsgd_backproject_block,
 * bsgd_tile_export with transposed = 1, bsgd_power_umax, bsgd_lanczos_umax,
 * block-selection states, and bsgd_run_epochs unless the state has a
 * tile-sliced store attached and is not an ISTA state with nrhs > 1).
 * Excludes BSGD_PLAN_STAGED_BWD.
 */
#define BSGD_PLAN_FWD_ONLY 16u
/*
 * Build no block store at all: for plans whose epochs run only on the
 * tile-sliced store, which bsgd_fused_create then builds straight from A's
 * CSR.  The plan keeps the device pointers of A's row_ptr, col and val (not
 * copies): the caller keeps those arrays alive and unchanged while the plan
 * exists.  A's columns are validated (in range, strictly ascending) when the
 * tile-sliced store is built.  Implies BSGD_PLAN_FWD_ONLY; also refused
 * (BSGD_ERR_UNSUPPORTED): bsgd_forward, bsgd_forward_block, bsgd_tile_nnz,
 * bsgd_tile_export, bsgd_state_init with x0 and bsgd_state_set_rhs with x0.
 * Excludes the staged forms and BSGD_PLAN_AUTOTUNE; with BSGD_PLAN_F16 the
 * tile-sliced store's FP16 copy is rounded from A's FP32 values, as the block
 * store's would be.
 */
#define BSGD_PLAN_SINGLE_PASS_ONLY 32u

/*
 * A sparse matrix in CSR form, in device memory.  Columns must be strictly
 * ascending within each row and lie in [0, ncols); row_ptr[0] = 0 and
 * row_ptr[nrows] = nnz.  nnz < 2^31.
 */
typedef struct {
  int64_t nrows;
  int64_t ncols;
  int64_t nnz;
  const int64_t* row_ptr; /* device, nrows + 1 */
  const int32_t* col;     /* device, nnz */
  const float* val;       /* device, nnz */
} bsgd_csr;

typedef struct bsgd_plan bsgd_plan;   /* block store of A and A^T (opaque) */
typedef struct bsgd_state bsgd_state; /* iterate, residual and prox buffers (opaque) */
typedef struct bsgd_graph bsgd_graph; /* captured epochs of one state (opaque) */
typedef struct bsgd_fused bsgd_fused; /* tile-sliced store for single-pass epochs (opaque) */

/* ------------------------------------------------------------------------
 * Block store (Section 2.1: A divided into M row blocks and N column blocks)
 * ---------------------------------------------------------------------- */

/*
 * Upper bound of the plan workspace for a matrix of this size (host only,
 * no device access).  Arguments as for bsgd_plan_create.
 */
bsgd_status bsgd_plan_workspace_size(int64_t nrows, int64_t ncols, int64_t nnz, int M, int N,
                                     int H, int W, int D, int64_t view_len, unsigned flags,
                                     size_t* bytes);

/*
 * Build the block store of A (Section 2.1) in `workspace` (device, at least
 * bsgd_plan_workspace_size bytes, 256-byte aligned).
 *
 *   A       the whole matrix (rays x pixels), device CSR, FP32 values.
 *   At      its transpose (pixels x rays), device CSR; the caller guarantees
 *           that it is the transpose of A (same nnz is checked).
 *   M, N    number of row and column blocks, 1 <= M <= nrows, 1 <= N <= ncols.
 *   row_off host, M+1 ascending ray offsets, row_off[0] = 0, row_off[M] = r:
 *           row block I_i = rays [row_off[i], row_off[i+1]).
 *   col_off host, N+1 ascending pixel offsets, col_off[N] = c: column block
 *           J_j = pixels [col_off[j], col_off[j+1]).
 *   H, W, D image shape with H*W*D = c (D = 1 for a 2-D image).
 *   view_len number of consecutive rays that form one view (one projection
 *           angle), or 0 if the rows have no such structure.  Only the
 *           internal vector order depends on it (rays of 8 consecutive views
 *           are interleaved bin by bin, pixels are stored in 8 x 8 tiles, so
 *           the gathers of the products stay within few cache lines); every
 *           vector crossing this interface is in natural order.
 *   flags   BSGD_PLAN_F16, BSGD_PLAN_AUTOTUNE, BSGD_PLAN_STAGED_FWD,
 *           BSGD_PLAN_STAGED_BWD and/or BSGD_PLAN_FWD_ONLY.  With
 *           BSGD_PLAN_FWD_ONLY only the row pointers and values of At are
 *           read (row_ptr is validated; its columns are not).
 *
 * The store keeps every block A_{I_i}^{J_j} and its transpose addressable
 * (bsgd_tile_export) in a row-interleaved layout: the entries of ray rho for
 * column block j follow those for block j-1, and likewise for each pixel's
 * row of A^T over the row blocks.  It also keeps the largest column sum of
 * |A| and the largest |a| (FP64, from At), which bound the fixed-point sums
 * of the tile-sliced store.  The A/At arrays are only read during the
 * call.  Synchronises `stream` at the end (to validate the input: sorted
 * columns, indices in range, row_ptr consistent with nnz).
 * *out is released with bsgd_plan_destroy; the workspace must outlive it.
 */
bsgd_status bsgd_plan_create(const bsgd_csr* A, const bsgd_csr* At, int M, int N,
                             const int64_t* row_off, const int64_t* col_off, int H, int W, int D,
                             int64_t view_len, unsigned flags, void* workspace,
                             size_t workspace_bytes, hipStream_t stream, bsgd_plan** out);

void bsgd_plan_destroy(bsgd_plan* plan);

/*
 * Launch choice of the fused row kernels of the forward store (A) and the
 * backward store (A^T): the number of lanes of a wavefront that share one
 * row (2, 4, 8, 16, 32 or 64), or-ed with BSGD_LAUNCH_NT when the matrix
 * streams are read with non-temporal loads.  Chosen from the mean row length
 * (plain loads), or by timing every choice when the plan was created with
 * BSGD_PLAN_AUTOTUNE; set_lanes overrides it (for instance with values an
 * earlier autotuned plan of the same matrix reported).  Results change only
 * by summation order.
 */
#define BSGD_LAUNCH_NT 128
bsgd_status bsgd_plan_lanes(const bsgd_plan* plan, int* fwd_launch, int* bwd_launch);
bsgd_status bsgd_plan_set_lanes(bsgd_plan* plan, int fwd_launch, int bwd_launch);

/*
 * Staged form (plans created with BSGD_PLAN_STAGED_FWD / _BWD).  The same fused sums of
 * The block products, block sums and gradient step of Algorithm 1 as the row kernels, reorganised for the epochs of
 * one-RHS states: the internal column space is cut into stages of at most
 * 32768 columns (whole 8-pixel tile rows, or whole groups of 8 views), each
 * row's entries are regrouped by stage with 16-bit stage-local column
 * indices (6 bytes per entry with FP32 values, 4 with FP16), and a
 * workgroup per (2048-row chunk, stage) serves its gathers from a copy of the
 * stage's slice of x or r in LDS.  Per-stage row sums are added in stage
 * order: deterministic, different rounding from the row kernels.
 *   staged      lanes per row of each direction's staged kernel (4 or 8), 0
 *               when the epochs of that direction use the row kernels, -1
 *               when the direction has no staged form.  Built plans default
 *               to 4; BSGD_PLAN_AUTOTUNE keeps the staged form only where it
 *               timed faster than the best row-kernel launch.
 *   set_staged  0, 4 or 8 per direction (4 / 8 only where built).
 *   staged_shape  stages P, stage width and stored entries (with padding) of
 *               the forward (transposed = 0) or backward (1) staged store.
 * States created on the plan reserve the per-stage partial sums (P x rows
 * floats per direction); bsgd_forward / bsgd_backproject, the block products
 * and the power iteration always use the row kernels.
 */
bsgd_status bsgd_plan_staged(const bsgd_plan* plan, int* fwd_lanes, int* bwd_lanes);
bsgd_status bsgd_plan_set_staged(bsgd_plan* plan, int fwd_lanes, int bwd_lanes);
bsgd_status bsgd_plan_staged_shape(const bsgd_plan* plan, int transposed, int* stages,
                                   int* stage_width, int64_t* entries);

/*
 * Number of stored entries of block (i, j) (identical for the block and its
 * transpose).  Synchronises `stream`.
 */
bsgd_status bsgd_tile_nnz(const bsgd_plan* plan, int i, int j, hipStream_t stream, int64_t* nnz);

/*
 * Write block A_{I_i}^{J_j} (transposed = 0) or its transpose (transposed = 1)
 * as a block-local CSR: ptr (device, rows+1 int64), col (device, nnz int32,
 * column indices relative to the block's first column, ascending) and val
 * (device, nnz FP32).  rows = |I_i| (|J_j| when transposed); nnz from
 * bsgd_tile_nnz.
 */
bsgd_status bsgd_tile_export(const bsgd_plan* plan, int i, int j, int transposed, int64_t* ptr,
                             int32_t* col, float* val, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Step-level products of Algorithm 1 (block products, block sums, gradient step).  The whole-matrix
 * calls stage their operands in the plan's scratch vectors, so calls on one
 * plan must not overlap (serialise them on one stream).
 * ---------------------------------------------------------------------- */

/*
 * Forward projection over all blocks (forward projection and residual):
 *   y == NULL:  out = A x             (sum over j of z^j = A_{I_i}^{J_j} x_{J_j})
 *   y != NULL:  out = y - A x         (the residual update)
 * x: device, c floats; y, out: device, r floats.  vt selects the value copy.
 */
bsgd_status bsgd_forward(const bsgd_plan* plan, bsgd_valtype vt, const float* x, const float* y,
                         float* out, hipStream_t stream);

/*
 * Backprojection over all blocks (backprojection, gradient sum and step):
 *   x == NULL:  out = 2 A^T r                    (g = sum_i 2 (A_{I_i}^{J_j})^T r_{I_i})
 *   x != NULL:  out = x + mu * 2 A^T r           (the gradient step)
 * r: device, r floats; x, out: device, c floats.
 */
bsgd_status bsgd_backproject(const bsgd_plan* plan, bsgd_valtype vt, const float* r,
                             const float* x, float mu, float* out, hipStream_t stream);

/*
 * One block's forward product z^j_{I_i} = A_{I_i}^{J_j} x_{J_j} (the block forward projection).
 * xj: device, |J_j| floats; z: device, |I_i| floats.
 */
bsgd_status bsgd_forward_block(const bsgd_plan* plan, bsgd_valtype vt, int i, int j,
                               const float* xj, float* z, hipStream_t stream);

/*
 * One block's backprojection g^i_{J_j} = 2 (A_{I_i}^{J_j})^T r_{I_i} (the block backprojection).
 * ri: device, |I_i| floats; g: device, |J_j| floats.
 */
bsgd_status bsgd_backproject_block(const bsgd_plan* plan, bsgd_valtype vt, int i, int j,
                                   const float* ri, float* g, hipStream_t stream);

/* ------------------------------------------------------------------------
 * TV proximal step of Algorithm 1 and TV value (Eq. 2)
 * ---------------------------------------------------------------------- */

/* Workspace bytes for bsgd_tv_prox / bsgd_tv_value on an H x W x D image. */
bsgd_status bsgd_tv_workspace_size(int H, int W, int D, size_t* bytes);

/*
 * out = argmin_t 1/2 ||t - b||^2 + theta TV(t) approximated by `iters` FGP
 * iterations started from a zero dual (the TV prox step with theta = mu * lam).  TV is
 * the isotropic TV of Eq. 2 with backward differences (zero where a
 * difference would leave the image); D > 1 adds the difference across
 * slices (3-D TV, dual step 1/(12 theta) instead of 1/(8 theta)).
 * b, out: device, H*W*D floats (out may not alias b); ws: device workspace.
 * theta = 0 or iters = 0 copies b.
 */
bsgd_status bsgd_tv_prox(int H, int W, int D, const float* b, float theta, int iters, float* out,
                         void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * bsgd_tv_prox without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, kernels and results (bitwise) as
 * bsgd_tv_prox; the FGP duals live in a scratch array of 32 MiB that the
 * library holds on every GPU it runs on until the process ends.  Images
 * needing more (2-D above 1048576 pixels, volumes above 645277 voxels) are
 * rejected with BSGD_ERR_WORKSPACE.  The stream must belong to the current
 * device.  Makes no allocation (device or host).  Calls that overlap on one
 * GPU share the array and race: serialise them (one stream, or events).
 */
bsgd_status bsgd_tv_prox_noalloc(int H, int W, int D, const float* b, float theta, int iters,
                                 float* out, hipStream_t stream);

/* TV(x) of Eq. 2 (3-D when D > 1), accumulated in FP64.  Synchronises. */
bsgd_status bsgd_tv_value(int H, int W, int D, const float* x, void* ws, size_t ws_bytes,
                          hipStream_t stream, double* tv);

/* ------------------------------------------------------------------------
 * Step size (Theorem 1: mu < 1 / (2 u_max), u_max = largest eigenvalue of A^T A)
 * ---------------------------------------------------------------------- */

/* Workspace bytes for bsgd_power_umax. */
bsgd_status bsgd_power_workspace_size(const bsgd_plan* plan, size_t* bytes);

/*
 * u_max by `iters` power-iteration steps v <- A^T A v / ||A^T A v|| from the
 * all-ones vector; *umax is the last Rayleigh quotient ||A v||^2 / ||v||^2.
 * Synchronises.
 */
bsgd_status bsgd_power_umax(const bsgd_plan* plan, bsgd_valtype vt, int iters, void* ws,
                            size_t ws_bytes, hipStream_t stream, float* umax);

/*
 * u_max by `steps` steps of Golub-Kahan-Lanczos bidiagonalisation of A from
 * the all-ones vector (each step one product with A and one with A^T, like a
 * power step): the largest eigenvalue of B^T B, B the steps x steps upper
 * bidiagonal of the recurrence, is the largest Ritz value of A^T A in the
 * Krylov space, which approaches u_max from below far faster than the
 * power iteration.  Synchronises; BSGD_ERR_DIVERGED if a value is not
 * finite.  1 <= steps <= 4096; workspace from bsgd_lanczos_workspace_size.
 */
bsgd_status bsgd_lanczos_workspace_size(const bsgd_plan* plan, int steps, size_t* bytes);
bsgd_status bsgd_lanczos_umax(const bsgd_plan* plan, bsgd_valtype vt, int steps, void* ws,
                              size_t ws_bytes, hipStream_t stream, float* umax);

/* ------------------------------------------------------------------------
 * Whole epochs (Algorithm 1)
 * ---------------------------------------------------------------------- */

/*
 * State flags.  A state holds nrhs right-hand sides that share the plan's A:
 * nrhs = 1, or a power of two from 4 to 1024 (several RHS need a 2-D plan,
 * D = 1: BSGD_ERR_INVALID otherwise).  With several RHS every vector
 * crossing this interface is a row-major matrix [rows][nrhs] (the RHS index
 * fastest), the products become sparse-times-dense products that read A once
 * for all RHS, and the prox is either
 *   - per RHS (default): independent 2-D reconstructions, each with its own
 *     lambda (bsgd_state_set_lambda) -- batches of requests on one geometry;
 *   - BSGD_STATE_VOLUME: the RHS are the slices of one volume and the TV prox step uses
 *     the isotropic 3-D TV across them (needs a 2-D plan, D = 1).
 */
#define BSGD_STATE_VOLUME 1u
/*
 * BSGD_STATE_BLOCK_SELECT: the state can also run iterations in which only
 * drawn subsets of the row and column blocks take part (bsgd_run_selected).
 * It adds one kept product z^j_{I_i} per (ray, column block), N x r floats,
 * to the workspace.  Needs nrhs = 1 and at most 64 row and column blocks.
 */
#define BSGD_STATE_BLOCK_SELECT 2u

/* Workspace bytes of a state. */
bsgd_status bsgd_state_workspace_size(const bsgd_plan* plan, int nrhs, unsigned flags,
                                      size_t* bytes);

/*
 * Create a state in `workspace` (device).  The state borrows the plan.  It
 * holds one extra HIP stream and two events (default priority) that let the
 * forward product overlap the prox inside an epoch; they come from a pool
 * the library keeps per device for the life of the process.
 */
bsgd_status bsgd_state_create(const bsgd_plan* plan, int nrhs, bsgd_valtype vt, unsigned flags,
                              void* workspace, size_t workspace_bytes, bsgd_state** out);

/* Waits for the state's extra stream, returns it and the events to the pool. */
void bsgd_state_destroy(bsgd_state* state);

/*
 * Start a reconstruction: copy y (device, r x nrhs floats); x = x0 (device,
 * c x nrhs floats) or 0 when x0 == NULL; r = y - A x0 (r = y when x0 ==
 * NULL), the initialisation that Algorithm 1 leaves open.  Resets the epoch
 * count and the per-RHS lambdas (to 0).  With BSGD_STATE_BLOCK_SELECT the
 * kept products become the block products of x0 (0 when x0 == NULL) and r
 * their residual y - sum_j z^j.
 */
bsgd_status bsgd_state_init(bsgd_state* state, const float* y, const float* x0, hipStream_t stream);

/*
 * Resume from a saved state: x (device, c floats), r (device, r floats, the
 * residual y - A x_prev of the previous epoch; Eq. 3 makes it part of the
 * state) and the epoch count.  y must have been set by bsgd_state_init.
 * With BSGD_STATE_BLOCK_SELECT the kept products are recomputed from x.
 */
bsgd_status bsgd_state_load(bsgd_state* state, const float* x, const float* r, int64_t epoch,
                            hipStream_t stream);

/*
 * Run `epochs` epochs of Algorithm 1 with every block pair active:
 *   g = 2 A^T r; r' = y - A x; x^ = x + mu g; x = FGP(x^, theta = mu * lam,
 *   prox_iters); r = r'.
 * mu > 0, lam >= 0 (the same for every RHS), epochs >= 0, prox_iters >= 1
 * when lam != 0.  lam = 0 skips the prox (x = x^).  On a batch state,
 * lam < 0 selects the per-RHS values of bsgd_state_set_lambda.  Enqueued on
 * `stream` (the state's own stream joins it); no allocation and no host
 * synchronisation, so a call can be captured in a HIP graph (capture an even
 * number of epochs: the iterate buffers alternate).
 */
bsgd_status bsgd_run_epochs(bsgd_state* state, float mu, float lam, int epochs, int prox_iters,
                            hipStream_t stream);

/*
 * Update rule of bsgd_run_epochs (the Simulations section compares
 * BSGD-TV with ISTA and with gradient descent, Fig. 2):
 *   BSGD_METHOD_BSGD (default): Algorithm 1 as above; the block backprojection uses the
 *     residual of the previous iterate (Eq. 3), so both products read x and
 *     r of the epoch's start.
 *   BSGD_METHOD_ISTA: r = y - A x, then x = FGP(x + 2 mu A^T r): the
 *     gradient of the current iterate (no delay), so the backprojection
 *     waits for the forward pass.  lam = 0 gives gradient descent on
 *     ||y - A x||^2 (Fig. 2's GD).
 * Both keep r = y - A x of the iterate before the current one, so the
 * methods can alternate on one state.  With an attached single-pass store an
 * ISTA epoch reads that store twice (A x, then A^T of the new residual);
 * without one it runs the block store's row kernels.
 */
#define BSGD_METHOD_BSGD 0
#define BSGD_METHOD_ISTA 1
bsgd_status bsgd_state_set_method(bsgd_state* state, int method);

/*
 * `iters` iterations of Algorithm 1 in which only drawn blocks take part
 * (Simulations section: fractions gamma of {y_{I_i}} and alpha of
 * {x_{J_j}} per iteration).  Iteration t runs the pairs (i, j) with bit i
 * of rows_sel[t] and bit j of cols_sel[t] set (host arrays of iters masks,
 * each non-zero and within M resp. N bits; the caller draws them):
 *   backprojection, gradient sum and step: x_{J_j} += 2 mu sum over drawn i of (A_{I_i}^{J_j})^T
 *     r_{I_i} for drawn j (kept r, no rescaling); other blocks of x stay;
 *   the block forward projection: z^j_{I_i} = A_{I_i}^{J_j} x_{J_j} for drawn pairs, kept;
 *   the residual update: r_{I_i} = y_{I_i} - sum over all j of the kept z^j_{I_i}
 *     (ascending j) for drawn i; other rows keep r;
 *   the TV prox step: the prox of the whole image with theta = mu * lam.
 * With every bit set an iteration is an epoch of Algorithm 1 (up to
 * rounding).  Needs a state created with BSGD_STATE_BLOCK_SELECT; counts
 * iterations in bsgd_get_stats.  The epoch of the Simulations section is
 * the sum over iterations of the fraction of pairs drawn.  Enqueued on
 * `stream`, no allocation and no synchronisation.
 */
bsgd_status bsgd_run_selected(bsgd_state* state, float mu, float lam, int iters, int prox_iters,
                              const uint64_t* rows_sel, const uint64_t* cols_sel,
                              hipStream_t stream);

/*
 * Epoch schedule.  The forward pass (forward projection, residual) does not depend on the
 * backprojection (backprojection, gradient sum and step) or the prox of the same epoch
 * (Eq. 3: the block backprojection uses the previous epoch's residual), so it runs on the
 * state's second stream: mode 0 starts it together with the backprojection,
 * mode 1 after the backprojection (it then overlaps the prox only; faster on
 * MI355X since both passes are bandwidth-bound); mode 2 runs everything on
 * the caller's stream in order (backprojection, prox, forward pass), which
 * gives each kernel the whole GPU.  With an attached single-pass store,
 * modes 0 and 1 run the ray half of the reduce (the residual update: the next residual,
 * needed only by the next pass) on the second stream, concurrently with the
 * pixel half and the prox; mode 2 keeps it on the caller's stream.  Results
 * do not depend on the mode.  Default 1.
 */
bsgd_status bsgd_state_set_overlap(bsgd_state* state, int mode);

/*
 * Schedule of the 2-D prox kernels: 0 splits the FGP iterations
 * into equal launches of at most 12 on 32 x 32 tiles, recomputing a halo as
 * wide as the launch's iteration count (few launches, redundant work), with
 * each thread keeping a strip of
 * pixels' duals in registers; 2 is the same schedule with the duals in LDS;
 * 1 runs one iteration per launch (no redundant work, small LDS footprint).
 * Same arithmetic per pixel, so all three give identical results.
 * Default 0.
 */
bsgd_status bsgd_state_set_prox_schedule(bsgd_state* state, int schedule);

/*
 * Launch shapes of the state's epochs that do not change results:
 *   pass_waves  wavefronts per workgroup of the single pass: 2, 4 or 8 for
 *               one RHS, 8 or 16 for several (0: the store's choice, resp. 16).
 *               Row sums are per segment in a fixed order and the column sums
 *               exact fixed-point integers, so results are the same for all.
 *   prox_split  most FGP iterations per launch of the prox (2-D: 1 to 10,
 *               volumes: 1 to 3; 0 or more than that: the most).  Each pixel's
 *               arithmetic is the same whatever the split.
 * bsgd_state_autotune chooses both by timing them on this state (every epoch
 * of Algorithm 1 runs the same kernels, so a few epochs measure a choice):
 * `reps` epochs per candidate with the given mu, lam and prox_iters (pass wavefronts 4 or 8 for one RHS, 8 or 16 for several; prox
 * split 5, 7 or 10 in 2-D, 1, 2 or 3 for volumes).  It runs on zero data and
 * must be called before bsgd_state_init (it overwrites the state's vectors
 * and leaves the state uninitialised); choice (host, 2 ints, may be NULL)
 * receives the pass wavefronts (0 without a store) and the split (0 when lam
 * = 0).  Synchronises.
 */
bsgd_status bsgd_state_set_launch(bsgd_state* state, int pass_waves, int prox_split);
bsgd_status bsgd_state_launch(const bsgd_state* state, int* pass_waves, int* prox_split);
bsgd_status bsgd_state_autotune(bsgd_state* state, float mu, float lam, int prox_iters, int reps,
                                hipStream_t stream, int* choice);

/* Copy the current iterate x (c floats) / residual r (r floats) to device memory. */
bsgd_status bsgd_get_x(const bsgd_state* state, float* x, hipStream_t stream);
bsgd_status bsgd_get_r(const bsgd_state* state, float* r, hipStream_t stream);

/*
 * ||r||^2 of the current residual (FP64 sum of FP32 squares, fixed order)
 * and the number of epochs run since init.  Synchronises.  Returns
 * BSGD_ERR_DIVERGED (with the values filled in) when ||r||^2 is not finite.
 */
bsgd_status bsgd_get_stats(const bsgd_state* state, hipStream_t stream, double* res_norm2,
                           int64_t* epochs_done);

/*
 * Kernel timers (measurement).  After bsgd_state_enable_timing(state,
 * max_epochs), each of the next max_epochs epochs run by bsgd_run_epochs
 * (or iterations run by bsgd_run_selected) records HIP events (on the stream each kernel runs on) around its forward
 * pass (forward projection and residual), its backprojection pass (backprojection, gradient sum and step) and its prox
 * (the TV prox step).  bsgd_state_timing synchronises, returns the summed durations in
 * milliseconds and the number of timed epochs, and rearms the timers.
 * max_epochs = 0 disables timing.  bsgd_state_enable_timing_sampled times
 * one epoch in every `stride` (the first, then every stride-th), up to
 * max_epochs timed epochs: each timed epoch records 5 events between its
 * kernels, and every event leaves the GPU idle for a few microseconds, so a
 * throughput measurement that also samples kernel durations should not time
 * every epoch.  The events come from a per-device pool
 * that the library keeps for the life of the process (destroying the state
 * returns them to it), so timing a fresh state per job costs no event
 * creation after the first.
 */
bsgd_status bsgd_state_enable_timing(bsgd_state* state, int max_epochs);
bsgd_status bsgd_state_enable_timing_sampled(bsgd_state* state, int max_epochs, int stride);
bsgd_status bsgd_state_timing(bsgd_state* state, double* fwd_ms, double* bwd_ms, double* prox_ms,
                              int64_t* epochs_timed);

/*
 * Batch states (several RHS, no BSGD_STATE_VOLUME): per-slot operations for
 * serving independent reconstructions on one geometry.
 *   set_rhs     (re)start slot k with y (device, r floats, natural order) and
 *               x0 (device, c floats, or NULL for 0); y == NULL empties the
 *               slot (all its vectors become zero and stay zero).  Other
 *               slots are untouched.
 *   set_lambda  per-slot lambda (host, nrhs floats >= 0), used by
 *               bsgd_run_epochs with lam < 0.  Synchronises.
 *   get_x_rhs   slot k's iterate (device, c floats, natural order).
 *   get_stats_rhs  ||r_k||^2 per slot (host, nrhs doubles, FP64 sums in a
 *               fixed order).  Synchronises; BSGD_ERR_DIVERGED if any is
 *               not finite.
 *   get_res_change_rhs  the squared residual norms of the last two epochs per
 *               slot: now[j] = ||r_{k+1}||^2 (the residual that the next
 *               epoch's backprojection uses) and prev[j] = ||r_k||^2 (the one
 *               the last epoch used), read from the two residual buffers
 *               (the two block products of Algorithm 1 keep both).  prev is meaningful once
 *               an epoch has run since init, load or the slot's set_rhs.
 *               Any state, also nrhs = 1.  Synchronises; BSGD_ERR_DIVERGED if
 *               a value is not finite.  This is what a stopping rule on the
 *               relative change of ||r|| needs.
 */
bsgd_status bsgd_state_set_rhs(bsgd_state* state, int k, const float* y, const float* x0,
                               hipStream_t stream);
bsgd_status bsgd_state_set_lambda(bsgd_state* state, const float* lam, hipStream_t stream);
bsgd_status bsgd_get_x_rhs(const bsgd_state* state, int k, float* x, hipStream_t stream);
bsgd_status bsgd_get_stats_rhs(const bsgd_state* state, hipStream_t stream, double* res_norm2);
bsgd_status bsgd_get_res_change_rhs(const bsgd_state* state, hipStream_t stream, double* now,
                                    double* prev);

/*
 * Capture `epochs` epochs of bsgd_run_epochs (same arguments; epochs even,
 * >= 2) as a HIP graph on `stream` (not the null stream) and instantiate it.
 * bsgd_graph_launch replays them on `stream`: the same kernels, so results
 * equal bsgd_run_epochs bitwise.  The graph belongs to the state (destroy it
 * first); mu, lam and the iteration count are fixed at capture.
 */
bsgd_status bsgd_graph_create(bsgd_state* state, float mu, float lam, int epochs, int prox_iters,
                              hipStream_t stream, bsgd_graph** out);
bsgd_status bsgd_graph_launch(bsgd_graph* graph, hipStream_t stream);
void bsgd_graph_destroy(bsgd_graph* graph);

/* ------------------------------------------------------------------------
 * Single-pass epochs (the block products, block sums and gradient step of Algorithm 1, with the delay of Eq. 3)
 *
 * The block backprojection of an epoch uses the previous epoch's residual r_k and the block forward projection the
 * current iterate x_k, so both products can be taken in one pass over the
 * stored entries: z[rho] += a x_k[p] and g[p] += a r_k[rho] for every entry
 * a = A[rho, p].  An epoch then reads the matrix once instead of once as A
 * and once as A^T.
 *
 * The tile-sliced store regroups the plan's forward store: pixels in 64 x 64
 * tiles, rays in `chunks` chunks of whole ray groups (8 interleaved views when
 * the plan has view_len > 0); the part of one ray inside one tile (a
 * segment) is one lane's list of (16-bit tile-local column, value) entries.
 * Columns are 8-bit steps between a segment's successive tile-local pixel
 * addresses (with a 16-bit start per segment) when every step is below 256,
 * which holds for rays (5 bytes per entry with FP32 values, 3 with FP16),
 * else 16-bit addresses (flag BSGD_FUSED_WIDE forces them).  One workgroup
 * per (tile, chunk) keeps the tile of x in LDS for the row sums of A x and
 * adds the terms of A^T r into the tile in LDS as 32-bit fixed-point numbers
 * (integer additions, exact in any order; the scale is set from max |r|, the
 * largest column sum of |A| and the largest |a| so that sums stay below 2^30
 * and terms below 2^21: a term's rounding is below 2^-31 of the largest
 * possible sum, or 2^-22 of the largest possible term when the second bound
 * is the tighter one);
 * per-segment sums of A x and per-chunk sums of A^T r are added in a fixed
 * order by a second kernel, so results are bitwise reproducible for a given
 * store (and differ from the row kernels by summation order only).  FP16
 * values are available when the plan has BSGD_PLAN_F16.  Images wider than
 * 4096 pixels are not supported (BSGD_ERR_UNSUPPORTED).
 *
 *   fused_workspace_size  counts the segments of `plan` (device pass over the
 *               forward store, or over A's CSR for a BSGD_PLAN_SINGLE_PASS_ONLY
 *               plan, which is also where A's columns are checked:
 *               BSGD_ERR_INVALID for a column out of range or out of order;
 *               such plans also need slices of at most 2^24 pixels, else
 *               BSGD_ERR_UNSUPPORTED; uses the plan's scratch vectors: no
 *               other call on the plan may overlap it) and returns the
 *               workspace bytes for bsgd_fused_create with the same chunks and
 *               flags.  chunks = 0 picks at least about 1024 (tile, chunk)
 *               units and chunks of at most 131072 rays; chunks <= number of
 *               ray groups.  Synchronises `stream`.
 *   fused_create  builds the store in `workspace` (device, 256-byte aligned,
 *               at least the size returned above) from the plan's forward
 *               store (from A's CSR for a BSGD_PLAN_SINGLE_PASS_ONLY plan:
 *               the same store, bitwise); the plan must outlive it.  The same
 *               errors as above.  Synchronises.
 *   fused_shape   tiles, chunks, segments, slices (64 segments each),
 *               stored entries (with padding) and bytes per stored column (1:
 *               8-bit steps, 2: 16-bit addresses).
 *   fused_set_waves  wavefronts per (tile, chunk) workgroup of one-RHS
 *               passes: 2, 4 or 8 (default); a state can override it
 *               (bsgd_state_set_launch).  Results do not depend on it
 *               (per-segment row sums in a fixed order, exact fixed-point
 *               column sums).
 *   fused_partials_size  bytes of the partial-sum buffer (device) that every
 *               pass needs: the row sums of the segments (one float per
 *               slot, or per ray and rank, whichever needs more) and
 *               chunks x pixels.
 *   fused_apply   one pass in natural orders:
 *                   out_r = y - A x      (A x when y == NULL)      (forward projection, residual)
 *                   out_x = xadd + mu * 2 A^T r   (2 A^T r when xadd == NULL)
 *                                                               (backprojection, gradient sum and step)
 *               x, xadd, out_x: c floats; y, r, out_r: r floats (device).
 *               Uses the store's internal scratch vectors: calls on one store
 *               must not overlap.
 *   state_attach_fused  epochs of a state on the same plan use the
 *               single-pass form (pass, then the reduce that writes r' and x^,
 *               then the prox, all on the caller's stream); `partials` (device,
 *               fused_partials_size_rhs bytes for the state's nrhs) belongs to
 *               the state while attached.  fused == NULL detaches (the row
 *               kernels again).  The state's value type must be available in
 *               the store.  States with several RHS (batches, volumes; nrhs a
 *               multiple of 4) take the pass four RHS per workgroup: the tile
 *               of x for those RHS in LDS as 4-vectors, two lanes per segment
 *               with two RHS each, the terms of A^T r added as 32-bit
 *               fixed-point integers per RHS (scale from that RHS's max |r|:
 *               sums below 2^30, terms below 2^21), two RHS per 64-bit atomic;
 *               results are bitwise reproducible and each RHS's are
 *               independent of the others.  ISTA epochs of such
 *               states, and block-select states, use the block store.
 */
#define BSGD_FUSED_WIDE 1u /* 16-bit column addresses even where 8-bit steps would do */
bsgd_status bsgd_fused_workspace_size(const bsgd_plan* plan, int chunks, unsigned flags,
                                      hipStream_t stream, size_t* bytes);
bsgd_status bsgd_fused_create(const bsgd_plan* plan, int chunks, unsigned flags, void* workspace,
                              size_t workspace_bytes, hipStream_t stream, bsgd_fused** out);
void bsgd_fused_destroy(bsgd_fused* fused);
bsgd_status bsgd_fused_shape(const bsgd_fused* fused, int* tiles, int* chunks, int64_t* segments,
                             int64_t* slices, int64_t* entries, int* col_bytes);
bsgd_status bsgd_fused_set_waves(bsgd_fused* fused, int waves);
bsgd_status bsgd_fused_partials_size(const bsgd_fused* fused, size_t* bytes);
/*
 * Partial-sum buffer of a state with nrhs right-hand sides (1, or a multiple
 * of 4): nrhs floats per segment slot and per (chunk, pixel), 2 nrhs words of
 * max |r|.
 */
bsgd_status bsgd_fused_partials_size_rhs(const bsgd_fused* fused, int nrhs, size_t* bytes);
bsgd_status bsgd_fused_apply(const bsgd_fused* fused, bsgd_valtype vt, const float* x,
                             const float* y, const float* r, const float* xadd, float mu,
                             float* out_r, float* out_x, void* partials, size_t partials_bytes,
                             hipStream_t stream);
bsgd_status bsgd_state_attach_fused(bsgd_state* state, const bsgd_fused* fused, void* partials,
                                    size_t partials_bytes);

/*
 * u_max (S0', the bound of Theorem 1 on the step) by the Lanczos steps of
 * bsgd_lanczos_umax, with the products A v and A^T u taken from the
 * tile-sliced store: one single-direction pass each (about 0.55 times the
 * time of a row-kernel product at 512^2).  A^T u is summed in the store's
 * fixed-point form, scaled from max |u|.  The result differs from the
 * row-kernel form only by summation order.  Workspace (device, 256-byte
 * aligned) from bsgd_lanczos_workspace_size_fused; the store's plan must not
 * run other calls meanwhile (none of its scratch is used, but the store reads
 * its arrays).  Synchronises; BSGD_ERR_DIVERGED if a value is not finite.
 */
bsgd_status bsgd_lanczos_workspace_size_fused(const bsgd_fused* fused, int steps, size_t* bytes);
bsgd_status bsgd_lanczos_umax_fused(const bsgd_fused* fused, bsgd_valtype vt, int steps,
                                    void* ws, size_t ws_bytes, hipStream_t stream, float* umax);

/* Message for the last failed call on this thread ("" if none). */
const char* bsgd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BSGD_H */

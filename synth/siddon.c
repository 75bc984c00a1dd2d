/*
 * Seeded-input generator: 2-D parallel-beam X-ray projection matrix.
 *
 * This file builds the sparse matrix A of the problem y ~= A x_true (the
 * paper's introduction: A is an X-ray projection model, r x c).  It holds
 * none of the reconstruction method's arithmetic; both the FP64 oracle and
 * the device path take its output as input.
 *
 * Geometry (the paper's experiment geometry is not recoverable, so a
 * parallel-beam geometry is used):
 *   image H rows x W columns of unit pixels centred on the origin, row s
 *   counted from the top;  pixel (s,t) covers
 *       X in [t - W/2, t + 1 - W/2],   Y in [H/2 - s - 1, H/2 - s],
 *   and has column index s*W + t (row-major vectorisation of the image).
 *   Ray (a, b), a in [0, n_ang), b in [0, bins): angle phi = a*pi/n_ang,
 *   detector offset u = b - (bins-1)/2 (unit spacing); the ray is the line
 *   { p : p . (cos phi, sin phi) = u } and has row index a*bins + b.
 *   Entry A[ray][pixel] = length of the ray's chord inside the pixel square.
 *   A ray lying exactly on a pixel edge has its length split equally
 *   between the two pixels sharing that edge (on the image border only the
 *   inside pixel exists and receives the half).  Lengths below 1e-12 are
 *   dropped.  Within each row, entries are sorted by ascending column.
 *
 * The chord lengths are computed with Siddon's method (R. L. Siddon,
 * "Fast calculation of the exact radiological path for a three-dimensional
 * CT array", Med. Phys. 12(2), 1985): the parameters at which the line
 * crosses the vertical and horizontal grid lines are merged, and each
 * interval between consecutive crossings is one pixel's chord.
 *
 * Exported (C ABI, used from Python through ctypes):
 *   siddon_count     per-ray entry counts
 *   siddon_fill      CSR column indices and lengths (FP64 or FP32), and
 *                    optionally the FP64 projections of an image
 *   csr_transpose_f64 / _f32  stable counting-sort transpose (rows of A^T
 *                    sorted by ray index)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EDGE_TOL 1e-12
#define LEN_TOL 1e-12

typedef struct {
  int32_t col;
  double len;
} entry_t;

/* Reverse entries [lo, hi). */
static void rev(entry_t* e, int lo, int hi) {
  for (int i = lo, j = hi - 1; i < j; ++i, --j) {
    entry_t tmp = e[i];
    e[i] = e[j];
    e[j] = tmp;
  }
}

/*
 * Entries of one ray, written to out (capacity >= 2*(H+W)+4), sorted by
 * column.  lam is scratch of capacity >= H+W+4.  Returns the count, or -1
 * if the sortedness check fails (never expected).
 */
static int ray_entries(int H, int W, double phi, double u, entry_t* out,
                       double* lam, double* lam2) {
  const double c = cos(phi), s = sin(phi);
  const double halfW = 0.5 * W, halfH = 0.5 * H;
  int n = 0;

  if (fabs(s) < EDGE_TOL) {
    /* Vertical line X = u*c (phi = 0). */
    const double X = u * c;
    const double tt = X + halfW; /* column coordinate */
    const double tr = nearbyint(tt);
    if (fabs(tt - tr) < EDGE_TOL) {
      const int t0 = (int)tr; /* on the grid line between t0-1 and t0 */
      for (int row = 0; row < H; ++row) {
        if (t0 - 1 >= 0 && t0 - 1 < W) {
          out[n].col = row * W + (t0 - 1);
          out[n].len = 0.5;
          ++n;
        }
        if (t0 >= 0 && t0 < W) {
          out[n].col = row * W + t0;
          out[n].len = 0.5;
          ++n;
        }
      }
    } else {
      const int t = (int)floor(tt);
      if (t >= 0 && t < W)
        for (int row = 0; row < H; ++row) {
          out[n].col = row * W + t;
          out[n].len = 1.0;
          ++n;
        }
    }
    return n;
  }
  if (fabs(c) < EDGE_TOL) {
    /* Horizontal line Y = u*s (phi = pi/2). */
    const double Y = u * s;
    const double ss = halfH - Y; /* row coordinate */
    const double sr = nearbyint(ss);
    if (fabs(ss - sr) < EDGE_TOL) {
      const int s0 = (int)sr; /* on the grid line between rows s0-1 and s0 */
      if (s0 - 1 >= 0 && s0 - 1 < H)
        for (int t = 0; t < W; ++t) {
          out[n].col = (s0 - 1) * W + t;
          out[n].len = 0.5;
          ++n;
        }
      if (s0 >= 0 && s0 < H)
        for (int t = 0; t < W; ++t) {
          out[n].col = s0 * W + t;
          out[n].len = 0.5;
          ++n;
        }
    } else {
      const int row = (int)floor(ss);
      if (row >= 0 && row < H)
        for (int t = 0; t < W; ++t) {
          out[n].col = row * W + t;
          out[n].len = 1.0;
          ++n;
        }
    }
    return n;
  }

  /* General direction: p(l) = u*(c, s) + l*(-s, c); l is arc length. */
  const double px = u * c, py = u * s, ex = -s, ey = c;
  double lx0 = (-halfW - px) / ex, lx1 = (halfW - px) / ex;
  double ly0 = (-halfH - py) / ey, ly1 = (halfH - py) / ey;
  if (lx0 > lx1) { double t = lx0; lx0 = lx1; lx1 = t; }
  if (ly0 > ly1) { double t = ly0; ly0 = ly1; ly1 = t; }
  const double lmin = lx0 > ly0 ? lx0 : ly0;
  const double lmax = lx1 < ly1 ? lx1 : ly1;
  if (!(lmax - lmin > LEN_TOL)) return 0;

  /* Crossings with vertical grid lines X = k - W/2, increasing in l. */
  int nx = 0;
  for (int k = 0; k <= W; ++k) {
    const int kk = ex > 0 ? k : W - k;
    const double l = (kk - halfW - px) / ex;
    if (l > lmin && l < lmax) lam[nx++] = l;
  }
  /* Crossings with horizontal grid lines Y = H/2 - k, increasing in l. */
  int ny = 0;
  for (int k = 0; k <= H; ++k) {
    const int kk = ey > 0 ? H - k : k;
    const double l = (halfH - kk - py) / ey;
    if (l > lmin && l < lmax) lam2[ny++] = l;
  }
  /* Merge into one increasing sequence bracketed by lmin and lmax. */
  double prev = lmin;
  int i = 0, j = 0;
  for (;;) {
    double next;
    if (i < nx && (j >= ny || lam[i] <= lam2[j]))
      next = lam[i++];
    else if (j < ny)
      next = lam2[j++];
    else
      next = lmax;
    const double len = next - prev;
    if (len >= LEN_TOL) {
      const double m = 0.5 * (prev + next);
      int t = (int)floor(px + m * ex + halfW);
      int row = (int)floor(halfH - (py + m * ey));
      if (t < 0) t = 0;
      if (t >= W) t = W - 1;
      if (row < 0) row = 0;
      if (row >= H) row = H - 1;
      out[n].col = row * W + t;
      out[n].len = len;
      ++n;
    }
    if (next == lmax && i >= nx && j >= ny) break;
    prev = next;
  }

  /* Along l the row index and the column index are each monotone.  Put the
   * row index in ascending order, then the column index within each row. */
  if (n > 1) {
    if (out[0].col / W > out[n - 1].col / W) rev(out, 0, n);
    int tdesc = 0;
    for (int k = 1; k < n; ++k)
      if (out[k].col / W == out[k - 1].col / W) {
        tdesc = (out[k].col % W) < (out[k - 1].col % W);
        break;
      }
    if (tdesc) {
      int lo = 0;
      for (int k = 1; k <= n; ++k)
        if (k == n || out[k].col / W != out[lo].col / W) {
          rev(out, lo, k);
          lo = k;
        }
    }
    for (int k = 1; k < n; ++k)
      if (out[k].col <= out[k - 1].col) return -1;
  }
  return n;
}

static int ray_capacity(int H, int W) { return 2 * (H + W) + 8; }

/* Per-ray entry counts.  Returns total nnz, or -1 on an internal error. */
int64_t siddon_count(int H, int W, int n_ang, int bins, int64_t* counts) {
  const int64_t nrays = (int64_t)n_ang * bins;
  int err = 0;
#pragma omp parallel reduction(| : err)
  {
    const int cap = ray_capacity(H, W);
    entry_t* buf = (entry_t*)malloc(sizeof(entry_t) * cap);
    double* lam = (double*)malloc(sizeof(double) * cap);
    double* lam2 = (double*)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 64)
    for (int64_t ray = 0; ray < nrays; ++ray) {
      const int a = (int)(ray / bins), b = (int)(ray % bins);
      const double phi = (double)a * M_PI / (double)n_ang;
      const double u = (double)b - 0.5 * (double)(bins - 1);
      const int n = ray_entries(H, W, phi, u, buf, lam, lam2);
      if (n < 0) err |= 1;
      counts[ray] = n < 0 ? 0 : n;
    }
    free(buf);
    free(lam);
    free(lam2);
  }
  if (err) return -1;
  int64_t total = 0;
  for (int64_t ray = 0; ray < nrays; ++ray) total += counts[ray];
  return total;
}

/*
 * Fill CSR columns and lengths given row_ptr (nrays+1) from the counts.
 * Lengths go to val64 (FP64) or, when val64 is NULL, to val32 (rounded to
 * FP32).  When x is not NULL it holds nx images as a [H*W][nx] matrix and
 * ax[ray*nx + j] = sum of length * x[col*nx + j] over the row in column
 * order, in FP64 (the noiseless projections of the images).
 */
int siddon_fill(int H, int W, int n_ang, int bins, const int64_t* row_ptr,
                int32_t* col, double* val64, float* val32, const double* x, double* ax,
                int nx) {
  const int64_t nrays = (int64_t)n_ang * bins;
  int err = 0;
#pragma omp parallel reduction(| : err)
  {
    const int cap = ray_capacity(H, W);
    entry_t* buf = (entry_t*)malloc(sizeof(entry_t) * cap);
    double* lam = (double*)malloc(sizeof(double) * cap);
    double* lam2 = (double*)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 64)
    for (int64_t ray = 0; ray < nrays; ++ray) {
      const int a = (int)(ray / bins), b = (int)(ray % bins);
      const double phi = (double)a * M_PI / (double)n_ang;
      const double u = (double)b - 0.5 * (double)(bins - 1);
      const int n = ray_entries(H, W, phi, u, buf, lam, lam2);
      if (n < 0 || n != row_ptr[ray + 1] - row_ptr[ray]) {
        err |= 1;
        continue;
      }
      const int64_t base = row_ptr[ray];
      for (int k = 0; k < n; ++k) {
        col[base + k] = buf[k].col;
        if (val64)
          val64[base + k] = buf[k].len;
        else
          val32[base + k] = (float)buf[k].len;
      }
      if (x && ax) {
        double* out = ax + ray * (int64_t)nx;
        for (int j = 0; j < nx; ++j) out[j] = 0.0;
        for (int k = 0; k < n; ++k) {
          const double* xr = x + (int64_t)buf[k].col * nx;
          const double len = buf[k].len;
          for (int j = 0; j < nx; ++j) out[j] += len * xr[j];
        }
      }
    }
    free(buf);
    free(lam);
    free(lam2);
  }
  return err ? -1 : 0;
}

/*
 * Stable counting-sort transpose of a CSR matrix (nrows x ncols): row k of
 * the result lists the original rows holding column k in ascending order.
 * t_ptr has ncols+1 entries.  Threads own contiguous row ranges; per-thread
 * column histograms give each thread its write offsets, so the result is
 * the same as a serial pass.  Returns 0, or -1 if a column index is out of
 * range.
 */
#define DEFINE_TRANSPOSE(NAME, T)                                                      \
  int NAME(int64_t nrows, int64_t ncols, const int64_t* row_ptr, const int32_t* col,    \
           const T* val, int64_t* t_ptr, int32_t* t_col, T* t_val) {                    \
    int nth = 1;                                                                        \
    _Pragma("omp parallel") _Pragma("omp single") nth = synth_threads_();               \
    int64_t* hist = (int64_t*)calloc((size_t)nth * (size_t)ncols, sizeof(int64_t));     \
    if (!hist) return -2;                                                               \
    int bad = 0;                                                                        \
    _Pragma("omp parallel num_threads(nth) reduction(| : bad)") {                       \
      const int t = synth_thread_id_();                                                 \
      const int64_t r0 = nrows * t / nth, r1 = nrows * (t + 1) / nth;                   \
      int64_t* h = hist + (size_t)t * ncols;                                            \
      for (int64_t e = row_ptr[r0]; e < row_ptr[r1]; ++e) {                             \
        if (col[e] < 0 || col[e] >= ncols)                                              \
          bad = 1;                                                                      \
        else                                                                            \
          h[col[e]]++;                                                                  \
      }                                                                                 \
    }                                                                                   \
    if (bad) {                                                                          \
      free(hist);                                                                       \
      return -1;                                                                        \
    }                                                                                   \
    int64_t run = 0;                                                                    \
    for (int64_t k = 0; k < ncols; ++k) {                                               \
      t_ptr[k] = run;                                                                   \
      for (int t = 0; t < nth; ++t) {                                                   \
        const int64_t c = hist[(size_t)t * ncols + k];                                  \
        hist[(size_t)t * ncols + k] = run;                                              \
        run += c;                                                                       \
      }                                                                                 \
    }                                                                                   \
    t_ptr[ncols] = run;                                                                 \
    _Pragma("omp parallel num_threads(nth)") {                                          \
      const int t = synth_thread_id_();                                                 \
      const int64_t r0 = nrows * t / nth, r1 = nrows * (t + 1) / nth;                   \
      int64_t* cur = hist + (size_t)t * ncols;                                          \
      for (int64_t row = r0; row < r1; ++row)                                           \
        for (int64_t e = row_ptr[row]; e < row_ptr[row + 1]; ++e) {                     \
          const int64_t dst = cur[col[e]]++;                                            \
          t_col[dst] = (int32_t)row;                                                    \
          t_val[dst] = val[e];                                                          \
        }                                                                               \
    }                                                                                   \
    free(hist);                                                                         \
    return 0;                                                                           \
  }

static int synth_threads_(void) {
#ifdef _OPENMP
  return omp_get_num_threads();
#else
  return 1;
#endif
}

static int synth_thread_id_(void) {
#ifdef _OPENMP
  return omp_get_thread_num();
#else
  return 0;
#endif
}

DEFINE_TRANSPOSE(csr_transpose_f32, float)
DEFINE_TRANSPOSE(csr_transpose_f64, double)

int synth_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

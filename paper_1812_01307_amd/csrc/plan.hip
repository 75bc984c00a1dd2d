// Block store of A and A^T (Section 2.1: A split into M row blocks I_i of
// rays and N column blocks J_j of pixels).
//
// Layout in HBM (one "Store" per direction):
//   ptr[row]        int64, start of the row, a multiple of kPad entries;
//   col[e], val[e]  int32 global column index, FP32 value (and an optional
//                   FP16 copy), the row's entries in ascending column order
//                   followed by zero-valued padding;
//   seg[row][k]     int32, offset within the row of the first entry whose
//                   column is in block k (k = 0..nseg), seg[row][nseg] = the
//                   row's unpadded length.
// A ray's entries are therefore grouped by column block (its pieces of the
// blocks A_{I_i}^{J_j}, j ascending) and a pixel's entries in A^T by row
// block, so every block is addressable while a whole row streams as one
// contiguous run.
#include <algorithm>
#include <cstring>

#include "bsgd_internal.h"

namespace bsgd {

enum : int {
  kErrRowPtr = 1,     // row_ptr not ascending / out of [0, nnz] / row_ptr[n] != nnz
  kErrColRange = 2,   // column index outside [0, ncols)
  kErrColOrder = 4,   // columns not strictly ascending within a row
};

// Padded row lengths and row_ptr validation.
__global__ void k_padlen(const int64_t* __restrict__ row_ptr, int64_t nrows, int64_t nnz,
                         int64_t* __restrict__ plen, int* __restrict__ err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = row_ptr[i], b = row_ptr[i + 1];
    bool bad = a < 0 || b < a || b > nnz;
    if (i == 0 && a != 0) bad = true;
    if (i == nrows - 1 && b != nnz) bad = true;
    if (bad) {
      atomicOr(err, kErrRowPtr);
      plen[i] = 0;
    } else {
      plen[i] = (b - a + kPad - 1) / kPad * kPad;
    }
  }
}

// Copy rows into the padded store and compute the segment table.  One
// wavefront per row.  Invalid columns are replaced by 0 and flagged.
__global__ __launch_bounds__(256) void k_fill(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_in,
    const float* __restrict__ val_in, int64_t nrows, int64_t ncols,
    const int64_t* __restrict__ ptr, int32_t* __restrict__ col, float* __restrict__ val,
    __half* __restrict__ val16, int32_t* __restrict__ seg, const int64_t* __restrict__ seg_off,
    int nseg, int* __restrict__ err) {
  const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  if (row >= nrows) return;
  const int64_t a = row_ptr[row];
  const int64_t len = row_ptr[row + 1] - a;
  const int64_t dst = ptr[row];
  const int64_t plen = ptr[row + 1] - dst;
  int bad = 0;
  for (int64_t k = lane; k < plen; k += 64) {
    int32_t c;
    float v;
    if (k < len) {
      c = col_in[a + k];
      v = val_in[a + k];
      if (c < 0 || c >= ncols) {
        bad |= kErrColRange;
        c = 0;
      }
      if (k > 0 && col_in[a + k - 1] >= col_in[a + k]) bad |= kErrColOrder;
    } else {
      // padding: repeat the last real column (an address already touched by
      // the row) with a zero value
      int32_t last = col_in[a + len - 1];
      c = (last >= 0 && last < ncols) ? last : 0;
      v = 0.0f;
    }
    col[dst + k] = c;
    val[dst + k] = v;
    if (val16) val16[dst + k] = __float2half_rn(v);
  }
  // seg[k] = number of entries with column < seg_off[k] (binary search)
  int32_t* sg = seg + row * (int64_t)(nseg + 1);
  for (int k = lane; k <= nseg; k += 64) {
    const int64_t bound = seg_off[k];
    int64_t lo = 0, hi = len;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)col_in[a + mid] < bound)
        lo = mid + 1;
      else
        hi = mid;
    }
    sg[k] = (int32_t)lo;
  }
  if (bad) atomicOr(err, bad);
}

static int choose_lanes(int64_t nnz, int64_t nrows) {
  // aim for about two 4-entry chunks per lane on an average row
  const double avg = nrows > 0 ? (double)nnz / (double)nrows : 0.0;
  int lpr = 8;
  while (lpr < 64 && lpr * 8 < avg) lpr *= 2;
  return lpr;
}

static void carve_store(Carver& cv, Store& st, int64_t nrows, int64_t nnz, int nseg,
                        bool f16) {
  st.nrows = nrows;
  st.nnz = nnz;
  st.cap = nnz + (int64_t)(kPad - 1) * nrows;
  st.nseg = nseg;
  st.ptr = cv.take<int64_t>(nrows + 1);
  st.seg = cv.take<int32_t>((size_t)nrows * (nseg + 1));
  st.col = cv.take<int32_t>(st.cap);
  st.val = cv.take<float>(st.cap);
  st.val16 = f16 ? cv.take<__half>(st.cap) : nullptr;
}

static size_t plan_layout(bsgd_plan* p, void* ws, int64_t nrows, int64_t ncols, int64_t nnz,
                          int M, int N, unsigned flags) {
  Carver cv(ws);
  const bool f16 = (flags & BSGD_PLAN_F16) != 0;
  carve_store(cv, p->fwd, nrows, nnz, N, f16);
  carve_store(cv, p->bwd, ncols, nnz, M, f16);
  const int64_t mx = std::max(nrows, ncols);
  p->scratch64 = cv.take<int64_t>(mx + 1);
  p->scan_tmp = cv.take<int64_t>(scan_tmp_count(mx) + 1);
  p->err = cv.take<int>(64);
  // device copy of the segment bounds (block offsets) used by k_fill
  p->seg_dev = cv.take<int64_t>((size_t)std::max(M, N) + 1);
  return align_up(cv.off, kAlign);
}

static bsgd_status build_store(Store& st, const bsgd_csr& src, int64_t ncols,
                               const std::vector<int64_t>& seg_off, int64_t* seg_dev,
                               int64_t* scratch, int64_t* scan_tmp, int* err, hipStream_t s,
                               const char* what) {
  st.ncols = ncols;
  st.seg_off = seg_off;
  st.lanes_per_row = choose_lanes(st.nnz, st.nrows);
  BSGD_HIP(hipMemcpyAsync(seg_dev, seg_off.data(), sizeof(int64_t) * seg_off.size(),
                          hipMemcpyHostToDevice, s));
  BSGD_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
  if (st.nrows > 0) {
    int64_t blocks = std::min<int64_t>((st.nrows + 255) / 256, 65535);
    k_padlen<<<(unsigned)blocks, 256, 0, s>>>(src.row_ptr, st.nrows, src.nnz, scratch, err);
    BSGD_LAUNCH_CHECK();
  }
  int h_err = 0;
  BSGD_HIP(hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s));
  BSGD_HIP(hipStreamSynchronize(s));
  BSGD_REQUIRE(!(h_err & kErrRowPtr),
               "%s: row_ptr is not ascending within [0, nnz] or row_ptr[nrows] != nnz", what);
  BSGD_HIP(exclusive_scan_i64(scratch, st.ptr, st.nrows, scan_tmp, s));
  if (st.nrows > 0) {
    const unsigned blocks = (unsigned)((st.nrows * 64 + 255) / 256);
    k_fill<<<blocks, 256, 0, s>>>(src.row_ptr, src.col, src.val, st.nrows, ncols, st.ptr,
                                  st.col, st.val, st.val16, st.seg, seg_dev, st.nseg, err);
    BSGD_LAUNCH_CHECK();
  }
  BSGD_HIP(hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s));
  BSGD_HIP(hipStreamSynchronize(s));
  BSGD_REQUIRE(!(h_err & kErrColRange), "%s: column index out of range", what);
  BSGD_REQUIRE(!(h_err & kErrColOrder), "%s: columns not strictly ascending within a row", what);
  return BSGD_OK;
}

// ---------------------------------------------------------------------------
// Block export
// ---------------------------------------------------------------------------
__global__ void k_tile_len(const int32_t* __restrict__ seg, int nseg, int64_t row0,
                           int64_t nrows, int segk, int64_t* __restrict__ len) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t* sg = seg + (row0 + r) * (int64_t)(nseg + 1);
    len[r] = sg[segk + 1] - sg[segk];
  }
}

__global__ __launch_bounds__(256) void k_tile_copy(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ seg, int nseg,
    const int32_t* __restrict__ col, const float* __restrict__ val, int64_t row0, int64_t nrows,
    int segk, int64_t col_base, const int64_t* __restrict__ optr, int32_t* __restrict__ ocol,
    float* __restrict__ oval) {
  const int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  if (r >= nrows) return;
  const int32_t* sg = seg + (row0 + r) * (int64_t)(nseg + 1);
  const int64_t beg = ptr[row0 + r] + sg[segk], n = sg[segk + 1] - sg[segk];
  const int64_t dst = optr[r];
  for (int64_t k = lane; k < n; k += 64) {
    ocol[dst + k] = (int32_t)(col[beg + k] - col_base);
    oval[dst + k] = val[beg + k];
  }
}

}  // namespace bsgd

using namespace bsgd;

extern "C" bsgd_status bsgd_plan_workspace_size(int64_t nrows, int64_t ncols, int64_t nnz, int M,
                                                int N, unsigned flags, size_t* bytes) {
  clear_error();
  BSGD_REQUIRE(bytes != nullptr, "bytes is NULL");
  BSGD_REQUIRE(nrows >= 1 && ncols >= 1 && nnz >= 0, "bad matrix size");
  BSGD_REQUIRE(nnz < ((int64_t)1 << 31) - (int64_t)kPad * std::max(nrows, ncols),
               "nnz too large for int32 row offsets");
  BSGD_REQUIRE(M >= 1 && N >= 1 && M <= nrows && N <= ncols, "bad block counts M=%d N=%d", M, N);
  bsgd_plan tmp;
  *bytes = plan_layout(&tmp, nullptr, nrows, ncols, nnz, M, N, flags);
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_plan_create(const bsgd_csr* A, const bsgd_csr* At, int M, int N,
                                        const int64_t* row_off, const int64_t* col_off, int H,
                                        int W, int D, unsigned flags, void* workspace,
                                        size_t workspace_bytes, hipStream_t stream,
                                        bsgd_plan** out) {
  clear_error();
  BSGD_REQUIRE(A && At && row_off && col_off && workspace && out, "NULL argument");
  BSGD_REQUIRE((flags & ~BSGD_PLAN_F16) == 0, "unknown plan flags 0x%x", flags);
  BSGD_REQUIRE(((uintptr_t)workspace % kAlign) == 0, "workspace must be 256-byte aligned");
  BSGD_REQUIRE(A->row_ptr && A->col && A->val && At->row_ptr && At->col && At->val,
               "NULL CSR array");
  BSGD_REQUIRE(At->nrows == A->ncols && At->ncols == A->nrows, "At is not shaped as A^T");
  BSGD_REQUIRE(At->nnz == A->nnz, "At has %lld entries, A has %lld", (long long)At->nnz,
               (long long)A->nnz);
  BSGD_REQUIRE(H >= 1 && W >= 1 && D >= 1 && (int64_t)H * W * D == A->ncols,
               "image shape %d x %d x %d does not match %lld columns", H, W, D,
               (long long)A->ncols);
  size_t need = 0;
  bsgd_status st = bsgd_plan_workspace_size(A->nrows, A->ncols, A->nnz, M, N, flags, &need);
  if (st != BSGD_OK) return st;
  if (workspace_bytes < need) {
    set_error("plan workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return BSGD_ERR_WORKSPACE;
  }
  BSGD_REQUIRE(row_off[0] == 0 && row_off[M] == A->nrows, "row_off must run from 0 to r");
  BSGD_REQUIRE(col_off[0] == 0 && col_off[N] == A->ncols, "col_off must run from 0 to c");
  for (int i = 0; i < M; ++i)
    BSGD_REQUIRE(row_off[i] < row_off[i + 1], "row_off not strictly ascending at %d", i);
  for (int j = 0; j < N; ++j)
    BSGD_REQUIRE(col_off[j] < col_off[j + 1], "col_off not strictly ascending at %d", j);

  bsgd_plan* p = new bsgd_plan();
  p->M = M;
  p->N = N;
  p->H = H;
  p->W = W;
  p->D = D;
  p->flags = flags;
  p->row_off.assign(row_off, row_off + M + 1);
  p->col_off.assign(col_off, col_off + N + 1);
  plan_layout(p, workspace, A->nrows, A->ncols, A->nnz, M, N, flags);
  int64_t* seg_dev = p->seg_dev;
  st = build_store(p->fwd, *A, A->ncols, p->col_off, seg_dev, p->scratch64, p->scan_tmp, p->err,
                   stream, "A");
  if (st == BSGD_OK)
    st = build_store(p->bwd, *At, At->ncols, p->row_off, seg_dev, p->scratch64, p->scan_tmp,
                     p->err, stream, "At");
  if (st == BSGD_OK) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      set_error("plan build failed: %s", hipGetErrorString(e));
      st = BSGD_ERR_HIP;
    }
  }
  if (st != BSGD_OK) {
    delete p;
    return st;
  }
  *out = p;
  return BSGD_OK;
}

extern "C" void bsgd_plan_destroy(bsgd_plan* plan) { delete plan; }

static bsgd_status tile_rows(const bsgd_plan* plan, int i, int j, int transposed,
                             const Store** st, int64_t* row0, int64_t* nrows, int* segk,
                             int64_t* col_base) {
  BSGD_REQUIRE(plan != nullptr, "plan is NULL");
  BSGD_REQUIRE(i >= 0 && i < plan->M && j >= 0 && j < plan->N, "block (%d, %d) out of range", i,
               j);
  if (!transposed) {
    *st = &plan->fwd;
    *row0 = plan->row_off[i];
    *nrows = plan->row_off[i + 1] - plan->row_off[i];
    *segk = j;
    *col_base = plan->col_off[j];
  } else {
    *st = &plan->bwd;
    *row0 = plan->col_off[j];
    *nrows = plan->col_off[j + 1] - plan->col_off[j];
    *segk = i;
    *col_base = plan->row_off[i];
  }
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_tile_nnz(const bsgd_plan* plan, int i, int j, hipStream_t stream,
                                     int64_t* nnz) {
  clear_error();
  const Store* st;
  int64_t row0, nrows, col_base;
  int segk;
  bsgd_status s = tile_rows(plan, i, j, 0, &st, &row0, &nrows, &segk, &col_base);
  if (s != BSGD_OK) return s;
  BSGD_REQUIRE(nnz != nullptr, "nnz is NULL");
  const unsigned blocks = (unsigned)std::min<int64_t>((nrows + 255) / 256, 65535);
  k_tile_len<<<blocks, 256, 0, stream>>>(st->seg, st->nseg, row0, nrows, segk, plan->scratch64);
  BSGD_LAUNCH_CHECK();
  // per-row lengths are summed on the host (this call synchronises anyway)
  std::vector<int64_t> h(nrows);
  BSGD_HIP(hipMemcpyAsync(h.data(), plan->scratch64, sizeof(int64_t) * nrows,
                          hipMemcpyDeviceToHost, stream));
  BSGD_HIP(hipStreamSynchronize(stream));
  int64_t tot = 0;
  for (int64_t k = 0; k < nrows; ++k) tot += h[k];
  *nnz = tot;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_tile_export(const bsgd_plan* plan, int i, int j, int transposed,
                                        int64_t* ptr, int32_t* col, float* val,
                                        hipStream_t stream) {
  clear_error();
  const Store* st;
  int64_t row0, nrows, col_base;
  int segk;
  bsgd_status s = tile_rows(plan, i, j, transposed, &st, &row0, &nrows, &segk, &col_base);
  if (s != BSGD_OK) return s;
  BSGD_REQUIRE(ptr && col && val, "NULL output");
  const unsigned blocks = (unsigned)std::min<int64_t>((nrows + 255) / 256, 65535);
  k_tile_len<<<blocks, 256, 0, stream>>>(st->seg, st->nseg, row0, nrows, segk, plan->scratch64);
  BSGD_LAUNCH_CHECK();
  BSGD_HIP(exclusive_scan_i64(plan->scratch64, ptr, nrows, plan->scan_tmp, stream));
  const unsigned cblocks = (unsigned)((nrows * 64 + 255) / 256);
  k_tile_copy<<<cblocks, 256, 0, stream>>>(st->ptr, st->seg, st->nseg, st->col, st->val, row0,
                                           nrows, segk, col_base, ptr, col, val);
  BSGD_LAUNCH_CHECK();
  return BSGD_OK;
}

// Block store of A and A^T (Section 2.1: A split into M row blocks I_i of
// rays and N column blocks J_j of pixels).
//
// Layout in HBM (one Store per direction, rows in the internal order of
// bsgd::Layout):
//   ptr[row]        int64, start of the row, a multiple of kPad entries;
//   col[e], val[e]  int32 internal column index (pixel index for A, ray index
//                   for A^T), FP32 value (and an optional FP16 copy); the
//                   row's entries in ascending natural column order, then
//                   zero-valued padding;
//   seg[row][k]     int32, offset within the row of the first entry whose
//                   natural column is in block k (k = 0..nseg), seg[row][nseg]
//                   = the row's unpadded length.
// A ray's entries are therefore grouped by column block (its pieces of
// A_{I_i}^{J_1}, ..., A_{I_i}^{J_N}, in that order) and a pixel's entries in
// A^T by row block, so every block is addressable while a whole row streams
// as one contiguous run.
#include <algorithm>
#include <cstring>

#include "bsgd_internal.h"

namespace bsgd {

Layout make_layout(int64_t nrows, int64_t view_len, int H, int W, int D) {
  Layout L;
  L.nrows = nrows;
  if (view_len > 0 && nrows % view_len == 0) {
    L.view_len = view_len;
    L.nviews = nrows / view_len;
    L.r_int = (L.nviews + kViewTile - 1) / kViewTile * kViewTile * view_len;
  } else {
    L.view_len = 0;
    L.nviews = 0;
    L.r_int = nrows;
  }
  L.H = H;
  L.W = W;
  L.D = D;
  L.Ht = (H + kPixTile - 1) / kPixTile;
  L.Wt = (W + kPixTile - 1) / kPixTile;
  L.c_int = (int64_t)D * L.Ht * L.Wt * 64;
  return L;
}

enum : int {
  kErrRowPtr = 1,     // row_ptr not ascending / out of [0, nnz] / row_ptr[n] != nnz
  kErrColRange = 2,   // column index outside [0, ncols)
  kErrColOrder = 4,   // columns not strictly ascending within a row
};

__global__ void k_check_rowptr(const int64_t* __restrict__ row_ptr, int64_t nrows, int64_t nnz,
                               int* __restrict__ err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = row_ptr[i], b = row_ptr[i + 1];
    bool bad = a < 0 || b < a || b > nnz;
    if (i == 0 && a != 0) bad = true;
    if (i == nrows - 1 && b != nnz) bad = true;
    if (bad) atomicOr(err, kErrRowPtr);
  }
}

// Largest sum of |a| over one row of At (a column sum of |A|) into out[0] and
// the largest |a| into out[1], FP64, as bit patterns of non-negative doubles
// (which order like the values).  One wavefront per row; lane-strided sums
// combined by a butterfly, so the result does not depend on the launch.
__global__ __launch_bounds__(256) void k_col_abs_sums(const int64_t* __restrict__ row_ptr,
                                                      const float* __restrict__ val, int64_t n,
                                                      unsigned long long* __restrict__ out) {
  const int64_t k = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (k >= n) return;  // uniform per wavefront
  const int64_t beg = row_ptr[k], len = row_ptr[k + 1] - beg;
  double acc = 0.0, amax = 0.0;
#pragma unroll 4
  for (int64_t e = lane; e < len; e += 64) {
    const double a = fabs((double)val[beg + e]);
    acc += a;
    amax = fmax(amax, a);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc += __shfl_xor(acc, off);
    amax = fmax(amax, __shfl_xor(amax, off));
  }
  const unsigned long long bits = (unsigned long long)__double_as_longlong(acc);
  const unsigned long long abits = (unsigned long long)__double_as_longlong(amax);
  if (lane == 0 && bits > __atomic_load_n(out, __ATOMIC_RELAXED)) atomicMax(out, bits);
  if (lane == 0 && abits > __atomic_load_n(out + 1, __ATOMIC_RELAXED)) atomicMax(out + 1, abits);
}

template <bool FWD>
__device__ __forceinline__ int64_t nat_row(const Layout& L, int64_t k) {
  return FWD ? L.ray_out(k) : L.pix_out(k);
}
template <bool FWD>
__device__ __forceinline__ int64_t int_row(const Layout& L, int64_t n) {
  return FWD ? L.ray_in(n) : L.pix_in(n);
}
// stored column index of a natural column
template <bool FWD>
__device__ __forceinline__ int64_t col_in(const Layout& L, int64_t c) {
  return FWD ? L.pix_in(c) : L.ray_in(c);
}
// natural column of a stored column index
template <bool FWD>
__device__ __forceinline__ int64_t col_out(const Layout& L, int64_t c) {
  return FWD ? L.pix_out(c) : L.ray_out(c);
}

// Padded lengths of the rows in internal order (holes are empty).
template <bool FWD>
__global__ void k_padlen(const int64_t* __restrict__ row_ptr, Layout L, int64_t n_int,
                         int64_t* __restrict__ plen) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_int;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = nat_row<FWD>(L, k);
    const int64_t len = n >= 0 ? row_ptr[n + 1] - row_ptr[n] : 0;
    plen[k] = (len + kPad - 1) / kPad * kPad;
  }
}

// Copy rows into the padded store (internal row order, internal column
// indices) and compute the segment table from the natural columns.  One
// wavefront per internal row.  Invalid columns are replaced by a valid one
// and flagged (the plan is then rejected).
template <bool FWD>
__global__ __launch_bounds__(256) void k_fill(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_src,
    const float* __restrict__ val_src, Layout L, int64_t n_int, int64_t ncols,
    const int64_t* __restrict__ ptr, int32_t* __restrict__ col, float* __restrict__ val,
    __half* __restrict__ val16, int32_t* __restrict__ seg, const int64_t* __restrict__ seg_off,
    int nseg, int* __restrict__ err) {
  const int64_t k = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  if (k >= n_int) return;
  int32_t* sg = seg + k * (int64_t)(nseg + 1);
  const int64_t n = nat_row<FWD>(L, k);
  if (n < 0) {
    for (int q = lane; q <= nseg; q += 64) sg[q] = 0;
    return;
  }
  const int64_t a = row_ptr[n];
  const int64_t len = row_ptr[n + 1] - a;
  const int64_t dst = ptr[k];
  const int64_t plen = ptr[k + 1] - dst;
  // seg[b] = number of entries whose natural column is < seg_off[b].  With
  // fewer than 64 blocks, lane b holds the inner bound seg_off[b] (below
  // ncols < 2^31), each entry finds its block by comparing with them, and the
  // first entry of each block writes the table; otherwise a binary search
  // per bound follows the copy.
  const bool few = nseg < 64;
  const int32_t bnd = few && lane < nseg ? (int32_t)seg_off[lane] : 0;
  auto block_of = [&](int64_t c) {
    int blk = 0;
    for (int b = 1; b < nseg; ++b) blk += c >= (int64_t)__builtin_amdgcn_readlane(bnd, b);
    return blk;
  };
  int bad = 0;
#pragma unroll 4
  for (int64_t q = lane; q < plen; q += 64) {
    int64_t c;
    float v;
    if (q < len) {
      c = col_src[a + q];
      v = val_src[a + q];
      if (c < 0 || c >= ncols) {
        bad |= kErrColRange;
        c = 0;
      }
      const int64_t cp = q > 0 ? (int64_t)col_src[a + q - 1] : 0;
      if (q > 0 && cp >= c) bad |= kErrColOrder;
      if (few) {
        // blocks (block of the previous entry, this entry's] start here
        const int hi = block_of(c);
        for (int b = q > 0 ? block_of(cp) + 1 : 1; b <= hi; ++b) sg[b] = (int32_t)q;
      }
    } else {
      // padding: repeat the last real column (already touched by the row)
      c = col_src[a + len - 1];
      if (c < 0 || c >= ncols) c = 0;
      v = 0.0f;
    }
    col[dst + q] = (int32_t)col_in<FWD>(L, c);
    val[dst + q] = v;
    if (val16) val16[dst + q] = __float2half_rn(v);
  }
  if (few) {
    // blocks after the last entry's start at len (all of them when empty)
    const int last = len > 0 ? block_of(col_src[a + len - 1]) : 0;
    for (int b = lane; b <= nseg; b += 64)
      if (b == 0 || b > last) sg[b] = b == 0 ? 0 : (int32_t)len;
    if (bad) atomicOr(err, bad);
    return;
  }
  for (int q = lane; q <= nseg; q += 64) {
    const int64_t bound = seg_off[q];
    int64_t lo = 0, hi = len;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)col_src[a + mid] < bound)
        lo = mid + 1;
      else
        hi = mid;
    }
    sg[q] = (int32_t)lo;
  }
  if (bad) atomicOr(err, bad);
}

static int heuristic_lanes(int64_t nnz, int64_t nrows) {
  // measured on gfx950: about ten or more 4-entry chunks per lane group keep
  // enough loads in flight; short rows want narrow groups
  const double avg = nrows > 0 ? (double)nnz / (double)nrows : 0.0;
  if (avg >= 160) return 8;
  if (avg >= 48) return 4;
  return 2;
}

static void carve_store(Carver& cv, Store& st, int64_t nrows, int64_t nnz, int nseg, bool f16) {
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

static void carve_staged(Carver& cv, Staged& st, const Layout& L, bool fwd, int64_t nnz,
                         bool f16) {
  if (!stage_geometry(L, fwd, st)) return;
  // every non-empty segment adds at most kStageVec - 1 padding entries
  st.cap = nnz + (int64_t)(kStageVec - 1) * std::min<int64_t>(nnz, st.nrows * st.P) + kStageVec;
  st.wbase = cv.take<int64_t>(st.nW + 1);
  st.segp = cv.take<int32_t>((size_t)st.nW * st.P * (st.RW + 1));
  st.col = cv.take<uint16_t>(st.cap);
  st.val = cv.take<float>(st.cap);
  st.val16 = f16 ? cv.take<__half>(st.cap) : nullptr;
}

static size_t plan_layout(bsgd_plan* p, void* ws, const Layout& L, int64_t nnz, int M, int N,
                          unsigned flags) {
  Carver cv(ws);
  const bool f16 = (flags & BSGD_PLAN_F16) != 0;
  if (!(flags & BSGD_PLAN_SINGLE_PASS_ONLY)) carve_store(cv, p->fwd, L.r_int, nnz, N, f16);
  if (!(flags & (BSGD_PLAN_FWD_ONLY | BSGD_PLAN_SINGLE_PASS_ONLY)))
    carve_store(cv, p->bwd, L.c_int, nnz, M, f16);
  if (flags & BSGD_PLAN_STAGED) {
    if (flags & BSGD_PLAN_STAGED_FWD) carve_staged(cv, p->sfwd, L, true, nnz, f16);
    if (flags & BSGD_PLAN_STAGED_BWD) carve_staged(cv, p->sbwd, L, false, nnz, f16);
    p->stage_cnt = cv.take<int64_t>(stage_cnt_count(L));
    if (flags & BSGD_PLAN_AUTOTUNE)
      p->stage_z = cv.take<float>((size_t)std::max(p->sfwd.P * L.r_int, p->sbwd.P * L.c_int));
  }
  const int64_t mx = std::max(L.r_int, L.c_int);
  p->scratch64 = cv.take<int64_t>(mx + 1);
  p->scan_tmp = cv.take<int64_t>(scan_tmp_count(mx) + 1);
  p->err = cv.take<int>(64);
  p->colmax = cv.take<unsigned long long>(2);
  p->seg_dev = cv.take<int64_t>((size_t)std::max(M, N) + 1);
  p->vin = cv.take<float>(mx);
  p->vaux = cv.take<float>(mx);
  p->vout = cv.take<float>(mx);
  return align_up(cv.off, kAlign);
}

// Validates row_ptr (ascending within [0, nnz], from 0 to nnz) before any
// kernel indexes the entries through it.  Synchronises.
static bsgd_status check_row_ptr(const bsgd_csr& src, int* err, hipStream_t s, const char* what) {
  BSGD_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
  {
    const int64_t blocks = std::min<int64_t>((src.nrows + 255) / 256, 65535);
    k_check_rowptr<<<(unsigned)blocks, 256, 0, s>>>(src.row_ptr, src.nrows, src.nnz, err);
    BSGD_LAUNCH_CHECK();
  }
  int h_err = 0;
  BSGD_HIP(hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s));
  BSGD_HIP(hipStreamSynchronize(s));
  BSGD_REQUIRE(!(h_err & kErrRowPtr),
               "%s: row_ptr is not ascending within [0, nnz] or row_ptr[nrows] != nnz", what);
  return BSGD_OK;
}

template <bool FWD>
static bsgd_status build_store(Store& st, const bsgd_csr& src, const Layout& L,
                               const std::vector<int64_t>& seg_off, int64_t* seg_dev,
                               int64_t* scratch, int64_t* scan_tmp, int* err, hipStream_t s,
                               const char* what) {
  st.ncols = src.ncols;
  st.seg_off = seg_off;
  st.lanes_per_row = heuristic_lanes(st.nnz, src.nrows);
  BSGD_HIP(hipMemcpyAsync(seg_dev, seg_off.data(), sizeof(int64_t) * seg_off.size(),
                          hipMemcpyHostToDevice, s));
  {
    const bsgd_status rs = check_row_ptr(src, err, s, what);
    if (rs != BSGD_OK) return rs;
  }
  {
    const int64_t blocks = std::min<int64_t>((st.nrows + 255) / 256, 65535);
    k_padlen<FWD><<<(unsigned)blocks, 256, 0, s>>>(src.row_ptr, L, st.nrows, scratch);
    BSGD_LAUNCH_CHECK();
  }
  BSGD_HIP(exclusive_scan_i64(scratch, st.ptr, st.nrows, scan_tmp, s));
  {
    const unsigned blocks = (unsigned)((st.nrows * 64 + 255) / 256);
    k_fill<FWD><<<blocks, 256, 0, s>>>(src.row_ptr, src.col, src.val, L, st.nrows, src.ncols,
                                       st.ptr, st.col, st.val, st.val16, st.seg, seg_dev,
                                       st.nseg, err);
    BSGD_LAUNCH_CHECK();
  }
  int h_err = 0;
  BSGD_HIP(hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s));
  BSGD_HIP(hipStreamSynchronize(s));
  BSGD_REQUIRE(!(h_err & kErrColRange), "%s: column index out of range", what);
  BSGD_REQUIRE(!(h_err & kErrColOrder), "%s: columns not strictly ascending within a row", what);
  return BSGD_OK;
}

// Time the fused row kernel for each candidate (lane count, load kind) and
// keep the fastest.
static bsgd_status autotune_store(Store& st, const float* v, float* out, hipStream_t s,
                                  float* best_ms) {
  static const int cand[] = {2, 4, 8, 16, 32};
  hipEvent_t e0, e1;
  BSGD_HIP(hipEventCreate(&e0));
  BSGD_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_l = st.lanes_per_row;
  bool best_nt = st.nontemporal;
  for (int k = 0; k < 10; ++k) {
    const int l = cand[k % 5];
    const int nt = k / 5;
    hipError_t e = launch_rows(st, BSGD_VAL_F32, kPlain, v, nullptr, nullptr, 1.f, out, s, l, nt);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
      e = launch_rows(st, BSGD_VAL_F32, kPlain, v, nullptr, nullptr, 1.f, out, s, l, nt);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      set_error("autotune failed: %s", hipGetErrorString(e));
      return BSGD_ERR_HIP;
    }
    if (ms < best) {
      best = ms;
      best_l = l;
      best_nt = nt != 0;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  st.lanes_per_row = best_l;
  st.nontemporal = best_nt;
  *best_ms = best;
  return BSGD_OK;
}

// Time the staged form (4 and 8 lanes per row) against the row kernel's best
// time and keep whichever is fastest (lanes = 0: the row kernel).
static bsgd_status autotune_staged(Staged& st, const float* v, int64_t nv, float* out,
                                   float* zpart, hipStream_t s, float rows_ms) {
  hipEvent_t e0, e1;
  BSGD_HIP(hipEventCreate(&e0));
  BSGD_HIP(hipEventCreate(&e1));
  float best = rows_ms;
  int best_l = 0;
  for (int l : {4, 8}) {
    st.lanes = l;
    hipError_t e = launch_staged(st, BSGD_VAL_F32, kPlain, v, nv, nullptr, nullptr, 1.f, out,
                                 zpart, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
      e = launch_staged(st, BSGD_VAL_F32, kPlain, v, nv, nullptr, nullptr, 1.f, out, zpart, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      set_error("autotune failed: %s", hipGetErrorString(e));
      return BSGD_ERR_HIP;
    }
    if (ms < best) {
      best = ms;
      best_l = l;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  st.lanes = best_l;
  return BSGD_OK;
}

// ---------------------------------------------------------------------------
// Block export (natural orders, block-local indices)
// ---------------------------------------------------------------------------
template <bool FWD>
__global__ void k_tile_len(const int32_t* __restrict__ seg, int nseg, Layout L, int64_t row0,
                           int64_t nrows, int segk, int64_t* __restrict__ len) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t* sg = seg + int_row<FWD>(L, row0 + r) * (int64_t)(nseg + 1);
    len[r] = sg[segk + 1] - sg[segk];
  }
}

template <bool FWD>
__global__ __launch_bounds__(256) void k_tile_copy(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ seg, int nseg,
    const int32_t* __restrict__ col, const float* __restrict__ val, Layout L, int64_t row0,
    int64_t nrows, int segk, int64_t col_base, const int64_t* __restrict__ optr,
    int32_t* __restrict__ ocol, float* __restrict__ oval) {
  const int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  if (r >= nrows) return;
  const int64_t k = int_row<FWD>(L, row0 + r);
  const int32_t* sg = seg + k * (int64_t)(nseg + 1);
  const int64_t beg = ptr[k] + sg[segk], n = sg[segk + 1] - sg[segk];
  const int64_t dst = optr[r];
  for (int64_t q = lane; q < n; q += 64) {
    ocol[dst + q] = (int32_t)(col_out<FWD>(L, col[beg + q]) - col_base);
    oval[dst + q] = val[beg + q];
  }
}

// ---------------------------------------------------------------------------
// Vector permutations (whole rows of S values move together)
// ---------------------------------------------------------------------------
__global__ void k_permute_in(Layout L, int kind, const float* __restrict__ nat,
                             float* __restrict__ out, int64_t n_int, int S) {
  const int64_t tot = n_int * S;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = q / S;
    const int j = (int)(q - k * S);
    const int64_t src = kind == kPixels ? L.pix_out(k) : L.ray_out(k);
    out[q] = src >= 0 ? nat[src * S + j] : 0.f;
  }
}

__global__ void k_permute_out(Layout L, int kind, const float* __restrict__ in,
                              float* __restrict__ nat, int64_t n, int S) {
  const int64_t tot = n * S;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / S;
    const int j = (int)(q - i * S);
    nat[q] = in[(kind == kPixels ? L.pix_in(i) : L.ray_in(i)) * S + j];
  }
}

__global__ void k_scatter_col(Layout L, int kind, const float* __restrict__ nat,
                              float* __restrict__ mat, int64_t n_int, int S, int j) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_int;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t src = kind == kPixels ? L.pix_out(k) : L.ray_out(k);
    mat[k * S + j] = (nat && src >= 0) ? nat[src] : 0.f;
  }
}

__global__ void k_gather_col(Layout L, int kind, const float* __restrict__ mat,
                             float* __restrict__ nat, int64_t n, int S, int j) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    nat[i] = mat[(kind == kPixels ? L.pix_in(i) : L.ray_in(i)) * S + j];
}

__global__ void k_fill_pixels_one(Layout L, float* __restrict__ v) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < L.c_int;
       k += (int64_t)gridDim.x * blockDim.x)
    v[k] = L.pix_out(k) >= 0 ? 1.f : 0.f;
}

static unsigned grid_of(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

static int64_t nat_len(const Layout& L, VecKind kind) {
  return kind == kPixels ? (int64_t)L.H * L.W * L.D : L.nrows;
}
static int64_t int_len(const Layout& L, VecKind kind) {
  return kind == kPixels ? L.c_int : L.r_int;
}

hipError_t permute_in(const Layout& L, VecKind kind, const float* nat, float* internal,
                      hipStream_t s, int S) {
  const int64_t n = int_len(L, kind);
  k_permute_in<<<grid_of(n * S), 256, 0, s>>>(L, kind, nat, internal, n, S);
  return hipGetLastError();
}

hipError_t permute_out(const Layout& L, VecKind kind, const float* internal, float* nat,
                       hipStream_t s, int S) {
  const int64_t n = nat_len(L, kind);
  k_permute_out<<<grid_of(n * S), 256, 0, s>>>(L, kind, internal, nat, n, S);
  return hipGetLastError();
}

hipError_t scatter_column(const Layout& L, VecKind kind, const float* nat, float* internal,
                          int S, int j, hipStream_t s) {
  const int64_t n = int_len(L, kind);
  k_scatter_col<<<grid_of(n), 256, 0, s>>>(L, kind, nat, internal, n, S, j);
  return hipGetLastError();
}

hipError_t gather_column(const Layout& L, VecKind kind, const float* internal, float* nat, int S,
                         int j, hipStream_t s) {
  const int64_t n = nat_len(L, kind);
  k_gather_col<<<grid_of(n), 256, 0, s>>>(L, kind, internal, nat, n, S, j);
  return hipGetLastError();
}

__global__ void k_set_col(const float* __restrict__ v, float* __restrict__ mat, int64_t n, int S,
                          int j) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    mat[k * S + j] = v[k];
}

hipError_t set_column(const float* v, float* mat, int64_t n, int S, int j, hipStream_t s) {
  k_set_col<<<grid_of(n), 256, 0, s>>>(v, mat, n, S, j);
  return hipGetLastError();
}

hipError_t fill_pixels_one(const Layout& L, float* v, hipStream_t s) {
  k_fill_pixels_one<<<grid_of(L.c_int), 256, 0, s>>>(L, v);
  return hipGetLastError();
}

}  // namespace bsgd

using namespace bsgd;

static bsgd_status check_sizes(int64_t nrows, int64_t ncols, int64_t nnz, int M, int N, int H,
                               int W, int D, int64_t view_len) {
  BSGD_REQUIRE(nrows >= 1 && ncols >= 1 && nnz >= 0, "bad matrix size");
  BSGD_REQUIRE(M >= 1 && N >= 1 && M <= nrows && N <= ncols, "bad block counts M=%d N=%d", M, N);
  BSGD_REQUIRE(H >= 1 && W >= 1 && D >= 1 && (int64_t)H * W * D == ncols,
               "image shape %d x %d x %d does not match %lld columns", H, W, D, (long long)ncols);
  BSGD_REQUIRE(view_len >= 0, "view_len must be >= 0");
  const Layout L = make_layout(nrows, view_len, H, W, D);
  BSGD_REQUIRE(L.r_int < ((int64_t)1 << 31) && L.c_int < ((int64_t)1 << 31),
               "vector lengths must stay below 2^31");
  BSGD_REQUIRE(nnz < ((int64_t)1 << 31) - (int64_t)kPad * std::max(L.r_int, L.c_int),
               "nnz too large for int32 row offsets");
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_plan_workspace_size(int64_t nrows, int64_t ncols, int64_t nnz, int M,
                                                int N, int H, int W, int D, int64_t view_len,
                                                unsigned flags, size_t* bytes) {
  clear_error();
  BSGD_REQUIRE(bytes != nullptr, "bytes is NULL");
  BSGD_REQUIRE((flags & ~(BSGD_PLAN_F16 | BSGD_PLAN_AUTOTUNE | BSGD_PLAN_STAGED |
                          BSGD_PLAN_FWD_ONLY | BSGD_PLAN_SINGLE_PASS_ONLY)) == 0,
               "unknown plan flags 0x%x", flags);
  BSGD_REQUIRE(!((flags & BSGD_PLAN_FWD_ONLY) && (flags & BSGD_PLAN_STAGED_BWD)),
               "BSGD_PLAN_FWD_ONLY excludes BSGD_PLAN_STAGED_BWD");
  BSGD_REQUIRE(!((flags & BSGD_PLAN_SINGLE_PASS_ONLY) &&
                 (flags & (BSGD_PLAN_STAGED | BSGD_PLAN_AUTOTUNE))),
               "BSGD_PLAN_SINGLE_PASS_ONLY excludes the staged forms and BSGD_PLAN_AUTOTUNE");
  bsgd_status st = check_sizes(nrows, ncols, nnz, M, N, H, W, D, view_len);
  if (st != BSGD_OK) return st;
  bsgd_plan tmp;
  *bytes = plan_layout(&tmp, nullptr, make_layout(nrows, view_len, H, W, D), nnz, M, N, flags);
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_plan_create(const bsgd_csr* A, const bsgd_csr* At, int M, int N,
                                        const int64_t* row_off, const int64_t* col_off, int H,
                                        int W, int D, int64_t view_len, unsigned flags,
                                        void* workspace, size_t workspace_bytes,
                                        hipStream_t stream, bsgd_plan** out) {
  clear_error();
  BSGD_REQUIRE(A && At && row_off && col_off && workspace && out, "NULL argument");
  BSGD_REQUIRE((flags & ~(BSGD_PLAN_F16 | BSGD_PLAN_AUTOTUNE | BSGD_PLAN_STAGED |
                          BSGD_PLAN_FWD_ONLY | BSGD_PLAN_SINGLE_PASS_ONLY)) == 0,
               "unknown plan flags 0x%x", flags);
  BSGD_REQUIRE(!((flags & BSGD_PLAN_FWD_ONLY) && (flags & BSGD_PLAN_STAGED_BWD)),
               "BSGD_PLAN_FWD_ONLY excludes BSGD_PLAN_STAGED_BWD");
  BSGD_REQUIRE(!((flags & BSGD_PLAN_SINGLE_PASS_ONLY) &&
                 (flags & (BSGD_PLAN_STAGED | BSGD_PLAN_AUTOTUNE))),
               "BSGD_PLAN_SINGLE_PASS_ONLY excludes the staged forms and BSGD_PLAN_AUTOTUNE");
  BSGD_REQUIRE(((uintptr_t)workspace % kAlign) == 0, "workspace must be 256-byte aligned");
  const bool no_store = (flags & BSGD_PLAN_SINGLE_PASS_ONLY) != 0;
  if (no_store) flags |= BSGD_PLAN_FWD_ONLY;  // refuses every call that needs A^T's store
  const bool fwd_only = (flags & BSGD_PLAN_FWD_ONLY) != 0;
  BSGD_REQUIRE(A->row_ptr && A->col && A->val && At->row_ptr && (At->col || fwd_only) &&
                   At->val,
               "NULL CSR array");
  BSGD_REQUIRE(At->nrows == A->ncols && At->ncols == A->nrows, "At is not shaped as A^T");
  BSGD_REQUIRE(At->nnz == A->nnz, "At has %lld entries, A has %lld", (long long)At->nnz,
               (long long)A->nnz);
  size_t need = 0;
  bsgd_status st = bsgd_plan_workspace_size(A->nrows, A->ncols, A->nnz, M, N, H, W, D, view_len,
                                            flags, &need);
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
  p->L = make_layout(A->nrows, view_len, H, W, D);
  p->row_off.assign(row_off, row_off + M + 1);
  p->col_off.assign(col_off, col_off + N + 1);
  plan_layout(p, workspace, p->L, A->nnz, M, N, flags);
  if (no_store) {
    // the tile-sliced store is built straight from A (its columns are
    // checked then); the row pointers are checked here
    st = check_row_ptr(*A, p->err, stream, "A");
    p->src_ptr = A->row_ptr;
    p->src_col = A->col;
    p->src_val = A->val;
    p->src_nnz = A->nnz;
  } else {
    st = build_store<true>(p->fwd, *A, p->L, p->col_off, p->seg_dev, p->scratch64, p->scan_tmp,
                           p->err, stream, "A");
  }
  if (st == BSGD_OK && !fwd_only)
    st = build_store<false>(p->bwd, *At, p->L, p->row_off, p->seg_dev, p->scratch64, p->scan_tmp,
                            p->err, stream, "At");
  if (st == BSGD_OK && fwd_only) st = check_row_ptr(*At, p->err, stream, "At");
  if (st == BSGD_OK) {
    // column sums of |A| and max |a| from the (validated) rows of At
    hipError_t e = hipMemsetAsync(p->colmax, 0, 2 * sizeof(unsigned long long), stream);
    if (e == hipSuccess && At->nrows > 0) {
      k_col_abs_sums<<<(unsigned)((At->nrows * 64 + 255) / 256), 256, 0, stream>>>(
          At->row_ptr, At->val, At->nrows, p->colmax);
      e = hipGetLastError();
    }
    if (e != hipSuccess) {
      set_error("column sums: %s", hipGetErrorString(e));
      st = BSGD_ERR_HIP;
    }
  }
  if (st == BSGD_OK && p->sfwd.P > 0)
    st = build_staged<true>(p->sfwd, *A, p->L, p->stage_cnt, stream);
  if (st == BSGD_OK && p->sbwd.P > 0)
    st = build_staged<false>(p->sbwd, *At, p->L, p->stage_cnt, stream);
  if (st == BSGD_OK && (flags & BSGD_PLAN_AUTOTUNE)) {
    hipError_t e = fill_pixels_one(p->L, p->vin, stream);
    if (e == hipSuccess) e = fill_f32(p->vaux, p->L.r_int, 1.f, stream);
    if (e != hipSuccess) {
      set_error("autotune setup failed: %s", hipGetErrorString(e));
      st = BSGD_ERR_HIP;
    }
    float tf = 0.f, tb = 0.f;
    if (st == BSGD_OK) st = autotune_store(p->fwd, p->vin, p->vout, stream, &tf);
    if (st == BSGD_OK && !fwd_only) st = autotune_store(p->bwd, p->vaux, p->vout, stream, &tb);
    if (st == BSGD_OK && p->sfwd.built)
      st = autotune_staged(p->sfwd, p->vin, p->L.c_int, p->vout, p->stage_z, stream, tf);
    if (st == BSGD_OK && p->sbwd.built)
      st = autotune_staged(p->sbwd, p->vaux, p->L.r_int, p->vout, p->stage_z, stream, tb);
  }
  if (st == BSGD_OK) {
    unsigned long long bits[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(bits, p->colmax, sizeof(bits), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      set_error("plan build failed: %s", hipGetErrorString(e));
      st = BSGD_ERR_HIP;
    }
    std::memcpy(&p->smax, &bits[0], sizeof(double));
    std::memcpy(&p->amax, &bits[1], sizeof(double));
  }
  if (st != BSGD_OK) {
    delete p;
    return st;
  }
  *out = p;
  return BSGD_OK;
}

extern "C" void bsgd_plan_destroy(bsgd_plan* plan) { delete plan; }

// Launch choice encoding: lanes | (non-temporal ? BSGD_LAUNCH_NT : 0)
extern "C" bsgd_status bsgd_plan_lanes(const bsgd_plan* plan, int* fwd_launch, int* bwd_launch) {
  clear_error();
  BSGD_REQUIRE(plan && fwd_launch && bwd_launch, "NULL argument");
  *fwd_launch = plan->fwd.lanes_per_row | (plan->fwd.nontemporal ? BSGD_LAUNCH_NT : 0);
  *bwd_launch = plan->bwd.lanes_per_row | (plan->bwd.nontemporal ? BSGD_LAUNCH_NT : 0);
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_plan_staged(const bsgd_plan* plan, int* fwd_lanes, int* bwd_lanes) {
  clear_error();
  BSGD_REQUIRE(plan && fwd_lanes && bwd_lanes, "NULL argument");
  *fwd_lanes = plan->sfwd.built ? plan->sfwd.lanes : -1;
  *bwd_lanes = plan->sbwd.built ? plan->sbwd.lanes : -1;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_plan_staged_shape(const bsgd_plan* plan, int transposed, int* stages,
                                              int* stage_width, int64_t* entries) {
  clear_error();
  BSGD_REQUIRE(plan && stages && stage_width && entries, "NULL argument");
  const Staged& st = transposed ? plan->sbwd : plan->sfwd;
  BSGD_REQUIRE(st.built, "this direction has no staged form");
  *stages = st.P;
  *stage_width = st.SW;
  *entries = st.total;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_plan_set_staged(bsgd_plan* plan, int fwd_lanes, int bwd_lanes) {
  clear_error();
  BSGD_REQUIRE(plan != nullptr, "plan is NULL");
  auto ok = [](const Staged& st, int l) {
    return l == 0 || ((l == 4 || l == 8) && st.built);
  };
  BSGD_REQUIRE(ok(plan->sfwd, fwd_lanes) && ok(plan->sbwd, bwd_lanes),
               "staged lanes must be 0 (row kernel) or 4 / 8 on a direction built staged");
  plan->sfwd.lanes = fwd_lanes;
  plan->sbwd.lanes = bwd_lanes;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_plan_set_lanes(bsgd_plan* plan, int fwd_launch, int bwd_launch) {
  clear_error();
  BSGD_REQUIRE(plan != nullptr, "plan is NULL");
  auto ok = [](int v) {
    const int l = v & ~BSGD_LAUNCH_NT;
    return (v & ~(BSGD_LAUNCH_NT | 127)) == 0 &&
           (l == 2 || l == 4 || l == 8 || l == 16 || l == 32 || l == 64);
  };
  BSGD_REQUIRE(ok(fwd_launch) && ok(bwd_launch),
               "launch must be 2, 4, 8, 16, 32 or 64 lanes, optionally | BSGD_LAUNCH_NT");
  plan->fwd.lanes_per_row = fwd_launch & ~BSGD_LAUNCH_NT;
  plan->fwd.nontemporal = (fwd_launch & BSGD_LAUNCH_NT) != 0;
  plan->bwd.lanes_per_row = bwd_launch & ~BSGD_LAUNCH_NT;
  plan->bwd.nontemporal = (bwd_launch & BSGD_LAUNCH_NT) != 0;
  return BSGD_OK;
}

static bsgd_status tile_rows(const bsgd_plan* plan, int i, int j, int transposed,
                             int64_t* row0, int64_t* nrows, int* segk, int64_t* col_base) {
  BSGD_REQUIRE(plan != nullptr, "plan is NULL");
  BSGD_REQUIRE(i >= 0 && i < plan->M && j >= 0 && j < plan->N, "block (%d, %d) out of range", i,
               j);
  if (!transposed) {
    *row0 = plan->row_off[i];
    *nrows = plan->row_off[i + 1] - plan->row_off[i];
    *segk = j;
    *col_base = plan->col_off[j];
  } else {
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
  int64_t row0, nrows, col_base;
  int segk;
  bsgd_status s = tile_rows(plan, i, j, 0, &row0, &nrows, &segk, &col_base);
  if (s != BSGD_OK) return s;
  BSGD_REQUIRE(nnz != nullptr, "nnz is NULL");
  BSGD_NEED_FWD(plan, "bsgd_tile_nnz");
  const Store& st = plan->fwd;
  const unsigned blocks = (unsigned)std::min<int64_t>((nrows + 255) / 256, 65535);
  plan->fz_count.valid = false;  // scratch64 is overwritten
  k_tile_len<true><<<blocks, 256, 0, stream>>>(st.seg, st.nseg, plan->L, row0, nrows, segk,
                                               plan->scratch64);
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
  int64_t row0, nrows, col_base;
  int segk;
  bsgd_status s = tile_rows(plan, i, j, transposed, &row0, &nrows, &segk, &col_base);
  if (s != BSGD_OK) return s;
  BSGD_REQUIRE(ptr && col && val, "NULL output");
  BSGD_NEED_FWD(plan, "bsgd_tile_export");
  if (transposed) BSGD_NEED_BWD(plan, "bsgd_tile_export (transposed)");
  const Store& st = transposed ? plan->bwd : plan->fwd;
  const unsigned blocks = (unsigned)std::min<int64_t>((nrows + 255) / 256, 65535);
  const unsigned cblocks = (unsigned)((nrows * 64 + 255) / 256);
  plan->fz_count.valid = false;  // scratch64 is overwritten
  if (!transposed)
    k_tile_len<true><<<blocks, 256, 0, stream>>>(st.seg, st.nseg, plan->L, row0, nrows, segk,
                                                 plan->scratch64);
  else
    k_tile_len<false><<<blocks, 256, 0, stream>>>(st.seg, st.nseg, plan->L, row0, nrows, segk,
                                                  plan->scratch64);
  BSGD_LAUNCH_CHECK();
  BSGD_HIP(exclusive_scan_i64(plan->scratch64, ptr, nrows, plan->scan_tmp, stream));
  if (!transposed)
    k_tile_copy<true><<<cblocks, 256, 0, stream>>>(st.ptr, st.seg, st.nseg, st.col, st.val,
                                                   plan->L, row0, nrows, segk, col_base, ptr,
                                                   col, val);
  else
    k_tile_copy<false><<<cblocks, 256, 0, stream>>>(st.ptr, st.seg, st.nseg, st.col, st.val,
                                                    plan->L, row0, nrows, segk, col_base, ptr,
                                                    col, val);
  BSGD_LAUNCH_CHECK();
  return BSGD_OK;
}

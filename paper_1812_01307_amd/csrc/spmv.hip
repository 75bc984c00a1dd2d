// Sparse products over the block store (the block products, block sums and gradient step of Algorithm 1).
//
// A row of the store (a ray of A, or a pixel of A^T) lists the row's entries
// of all its blocks back to back, so one pass over the row computes the sum
// over blocks of the block products: sum_j z^j for a ray (forward projection and residual) and
// sum_i g^i for a pixel (backprojection and gradient sum).  A group of LPR lanes of one
// wavefront walks a row with 16-byte loads of column indices and values
// (rows are padded to a multiple of 8 entries, so loads are aligned), gathers
// the vector entries (x or r, in the internal tiled orders, L2-resident), and
// reduces across the group with cross-lane shuffles.  No atomics: every
// output element is written once by one lane, and the summation order is
// fixed for a given LPR.  Narrow groups (8 lanes on the 512^2 workload)
// keep many rows in flight per wavefront and measured fastest on gfx950.
#include "bsgd_internal.h"

namespace bsgd {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Matrix streams are read once per pass; NT = true marks the loads
// non-temporal so they do not evict the gathered vector from L2.
template <bool NT, typename T>
__device__ __forceinline__ T ld(const T* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// Sum of val[e] * v[col[e]] over the lane's share of [beg, end).
template <int LPR, bool NT>
__device__ __forceinline__ float row_dot_f32(const int32_t* __restrict__ col,
                                             const float* __restrict__ val,
                                             const float* __restrict__ v, int64_t beg, int64_t end,
                                             int lane) {
  float acc0 = 0.f, acc1 = 0.f;
  int64_t e = beg + 4 * lane;
  // two chunks in flight per lane
  for (; e + 4 * LPR < end; e += 8 * LPR) {
    const i32x4 c0 = ld<NT>(reinterpret_cast<const i32x4*>(col + e));
    const f32x4 a0 = ld<NT>(reinterpret_cast<const f32x4*>(val + e));
    const i32x4 c1 = ld<NT>(reinterpret_cast<const i32x4*>(col + e + 4 * LPR));
    const f32x4 a1 = ld<NT>(reinterpret_cast<const f32x4*>(val + e + 4 * LPR));
    acc0 = fmaf(a0.x, v[c0.x], acc0);
    acc1 = fmaf(a1.x, v[c1.x], acc1);
    acc0 = fmaf(a0.y, v[c0.y], acc0);
    acc1 = fmaf(a1.y, v[c1.y], acc1);
    acc0 = fmaf(a0.z, v[c0.z], acc0);
    acc1 = fmaf(a1.z, v[c1.z], acc1);
    acc0 = fmaf(a0.w, v[c0.w], acc0);
    acc1 = fmaf(a1.w, v[c1.w], acc1);
  }
  if (e < end) {
    const i32x4 c0 = ld<NT>(reinterpret_cast<const i32x4*>(col + e));
    const f32x4 a0 = ld<NT>(reinterpret_cast<const f32x4*>(val + e));
    acc0 = fmaf(a0.x, v[c0.x], acc0);
    acc0 = fmaf(a0.y, v[c0.y], acc0);
    acc0 = fmaf(a0.z, v[c0.z], acc0);
    acc0 = fmaf(a0.w, v[c0.w], acc0);
  }
  return acc0 + acc1;
}

// FP16 values: 8 entries per lane per chunk (32 B of columns, 16 B of
// values), two chunks in flight per lane.
template <int LPR, bool NT>
__device__ __forceinline__ float row_dot_f16(const int32_t* __restrict__ col,
                                             const __half* __restrict__ val,
                                             const float* __restrict__ v, int64_t beg, int64_t end,
                                             int lane) {
  float acc0 = 0.f, acc1 = 0.f;
  int64_t e = beg + 8 * lane;
  for (; e + 8 * LPR < end; e += 16 * LPR) {
    const int64_t e1 = e + 8 * LPR;
    const i32x4 c0 = ld<NT>(reinterpret_cast<const i32x4*>(col + e));
    const i32x4 c1 = ld<NT>(reinterpret_cast<const i32x4*>(col + e + 4));
    const f16x8 a = ld<NT>(reinterpret_cast<const f16x8*>(val + e));
    const i32x4 d0 = ld<NT>(reinterpret_cast<const i32x4*>(col + e1));
    const i32x4 d1 = ld<NT>(reinterpret_cast<const i32x4*>(col + e1 + 4));
    const f16x8 b = ld<NT>(reinterpret_cast<const f16x8*>(val + e1));
    acc0 = fmaf((float)a[0], v[c0.x], acc0);
    acc1 = fmaf((float)b[0], v[d0.x], acc1);
    acc0 = fmaf((float)a[1], v[c0.y], acc0);
    acc1 = fmaf((float)b[1], v[d0.y], acc1);
    acc0 = fmaf((float)a[2], v[c0.z], acc0);
    acc1 = fmaf((float)b[2], v[d0.z], acc1);
    acc0 = fmaf((float)a[3], v[c0.w], acc0);
    acc1 = fmaf((float)b[3], v[d0.w], acc1);
    acc0 = fmaf((float)a[4], v[c1.x], acc0);
    acc1 = fmaf((float)b[4], v[d1.x], acc1);
    acc0 = fmaf((float)a[5], v[c1.y], acc0);
    acc1 = fmaf((float)b[5], v[d1.y], acc1);
    acc0 = fmaf((float)a[6], v[c1.z], acc0);
    acc1 = fmaf((float)b[6], v[d1.z], acc1);
    acc0 = fmaf((float)a[7], v[c1.w], acc0);
    acc1 = fmaf((float)b[7], v[d1.w], acc1);
  }
  if (e < end) {
    const i32x4 c0 = ld<NT>(reinterpret_cast<const i32x4*>(col + e));
    const i32x4 c1 = ld<NT>(reinterpret_cast<const i32x4*>(col + e + 4));
    const f16x8 a = ld<NT>(reinterpret_cast<const f16x8*>(val + e));
    acc0 = fmaf((float)a[0], v[c0.x], acc0);
    acc1 = fmaf((float)a[4], v[c1.x], acc1);
    acc0 = fmaf((float)a[1], v[c0.y], acc0);
    acc1 = fmaf((float)a[5], v[c1.y], acc1);
    acc0 = fmaf((float)a[2], v[c0.z], acc0);
    acc1 = fmaf((float)a[6], v[c1.z], acc1);
    acc0 = fmaf((float)a[3], v[c0.w], acc0);
    acc1 = fmaf((float)a[7], v[c1.w], acc1);
  }
  return acc0 + acc1;
}

template <int LPR>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, LPR);
  return x;
}

template <typename VT, int LPR, int MODE, bool NT>
__global__ __launch_bounds__(256) void k_rows(const int64_t* __restrict__ ptr,
                                              const int32_t* __restrict__ col,
                                              const VT* __restrict__ val,
                                              const float* __restrict__ v,
                                              const float* __restrict__ y,
                                              const float* __restrict__ xadd, float scale,
                                              float* __restrict__ out, int64_t nrows) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = gid / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  float acc = 0.f;
  if (row < nrows) {
    const int64_t beg = ptr[row], end = ptr[row + 1];
    if constexpr (sizeof(VT) == 4)
      acc = row_dot_f32<LPR, NT>(col, reinterpret_cast<const float*>(val), v, beg, end, lane);
    else
      acc = row_dot_f16<LPR, NT>(col, reinterpret_cast<const __half*>(val), v, beg, end, lane);
  }
  acc = group_sum<LPR>(acc);
  if (row < nrows && lane == 0) {
    if constexpr (MODE == kPlain)
      out[row] = scale * acc;
    else if constexpr (MODE == kResidual)
      out[row] = y[row] - acc;
    else
      out[row] = fmaf(scale, acc, xadd[row]);
  }
}

template <typename VT, int MODE, int LPR>
static void launch_lpr(const Store& st, bool nt, const VT* val, const float* v, const float* y,
                       const float* xadd, float scale, float* out, hipStream_t s) {
  const unsigned blocks = (unsigned)((st.nrows * LPR + 255) / 256);
  if (!blocks) return;
  if (nt)
    k_rows<VT, LPR, MODE, true><<<blocks, 256, 0, s>>>(st.ptr, st.col, val, v, y, xadd, scale,
                                                       out, st.nrows);
  else
    k_rows<VT, LPR, MODE, false><<<blocks, 256, 0, s>>>(st.ptr, st.col, val, v, y, xadd, scale,
                                                        out, st.nrows);
}

template <typename VT, int MODE>
static hipError_t launch_rows_vt(const Store& st, int lanes, bool nt, const VT* val,
                                 const float* v, const float* y, const float* xadd, float scale,
                                 float* out, hipStream_t s) {
  switch (lanes) {
    case 2: launch_lpr<VT, MODE, 2>(st, nt, val, v, y, xadd, scale, out, s); break;
    case 4: launch_lpr<VT, MODE, 4>(st, nt, val, v, y, xadd, scale, out, s); break;
    case 8: launch_lpr<VT, MODE, 8>(st, nt, val, v, y, xadd, scale, out, s); break;
    case 16: launch_lpr<VT, MODE, 16>(st, nt, val, v, y, xadd, scale, out, s); break;
    case 32: launch_lpr<VT, MODE, 32>(st, nt, val, v, y, xadd, scale, out, s); break;
    default: launch_lpr<VT, MODE, 64>(st, nt, val, v, y, xadd, scale, out, s); break;
  }
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_rows_mode(const Store& st, int lanes, bool nt, bsgd_valtype vt,
                                   const float* v, const float* y, const float* xadd,
                                   float scale, float* out, hipStream_t s) {
  if (vt == BSGD_VAL_F16)
    return launch_rows_vt<__half, MODE>(st, lanes, nt, st.val16, v, y, xadd, scale, out, s);
  return launch_rows_vt<float, MODE>(st, lanes, nt, st.val, v, y, xadd, scale, out, s);
}

hipError_t launch_rows(const Store& st, bsgd_valtype vt, RowMode mode, const float* v,
                       const float* y, const float* xadd, float scale, float* out,
                       hipStream_t s, int lanes, int nt) {
  if (lanes <= 0) lanes = st.lanes_per_row;
  const bool n = nt < 0 ? st.nontemporal : nt != 0;
  switch (mode) {
    case kPlain:
      return launch_rows_mode<kPlain>(st, lanes, n, vt, v, y, xadd, scale, out, s);
    case kResidual:
      return launch_rows_mode<kResidual>(st, lanes, n, vt, v, y, xadd, scale, out, s);
    default:
      return launch_rows_mode<kStep>(st, lanes, n, vt, v, y, xadd, scale, out, s);
  }
}

// ---------------------------------------------------------------------------
// One block's product in natural orders: rows nat_row0 .. nat_row0+nrows-1
// (rays of I_i, or pixels of J_j), the entries of segment `segk`, gathering
// v[natural column - col_base].  One wavefront per row, scalar loads (used
// for per-block checks, not on the epoch path).
// ---------------------------------------------------------------------------
template <typename VT, bool FWD>
__global__ __launch_bounds__(256) void k_segment_rows(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ seg, int nseg,
    const int32_t* __restrict__ col, const VT* __restrict__ val, Layout L, int64_t row0,
    int64_t nrows, int segk, int64_t col_base, const float* __restrict__ v, float scale,
    float* __restrict__ out) {
  const int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  float acc = 0.f;
  if (r < nrows) {
    const int64_t k = FWD ? L.ray_in(row0 + r) : L.pix_in(row0 + r);
    const int32_t* sg = seg + k * (nseg + 1);
    const int64_t beg = ptr[k] + sg[segk], end = ptr[k] + sg[segk + 1];
    for (int64_t e = beg + lane; e < end; e += 64) {
      const int64_t nat = FWD ? L.pix_out(col[e]) : L.ray_out(col[e]);
      acc = fmaf((float)val[e], v[nat - col_base], acc);
    }
  }
  acc = group_sum<64>(acc);
  if (r < nrows && lane == 0) out[r] = scale * acc;
}

hipError_t launch_segment_rows(const bsgd_plan* p, bool fwd, bsgd_valtype vt, int64_t nat_row0,
                               int64_t nrows, int segk, int64_t col_base, const float* v,
                               float scale, float* out, hipStream_t s) {
  const unsigned blocks = (unsigned)((nrows * 64 + 255) / 256);
  if (blocks == 0) return hipSuccess;
  const Store& st = fwd ? p->fwd : p->bwd;
  if (fwd) {
    if (vt == BSGD_VAL_F16)
      k_segment_rows<__half, true><<<blocks, 256, 0, s>>>(st.ptr, st.seg, st.nseg, st.col,
                                                          st.val16, p->L, nat_row0, nrows, segk,
                                                          col_base, v, scale, out);
    else
      k_segment_rows<float, true><<<blocks, 256, 0, s>>>(st.ptr, st.seg, st.nseg, st.col, st.val,
                                                         p->L, nat_row0, nrows, segk, col_base, v,
                                                         scale, out);
  } else {
    if (vt == BSGD_VAL_F16)
      k_segment_rows<__half, false><<<blocks, 256, 0, s>>>(st.ptr, st.seg, st.nseg, st.col,
                                                           st.val16, p->L, nat_row0, nrows, segk,
                                                           col_base, v, scale, out);
    else
      k_segment_rows<float, false><<<blocks, 256, 0, s>>>(st.ptr, st.seg, st.nseg, st.col,
                                                          st.val, p->L, nat_row0, nrows, segk,
                                                          col_base, v, scale, out);
  }
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Iterations over drawn block subsets (Simulations section: fractions gamma
// of the row blocks and alpha of the column blocks take part).  A row of a
// store lists its entries block by block (segment k = block k), so a drawn
// subset is a choice of segments: the kernels read only the drawn segments
// of the drawn rows.  Block sets are bit masks (at most 64 blocks a side).
// ---------------------------------------------------------------------------
struct BlockBounds {
  int64_t v[kMaxSelBlocks + 1];
  int n;
};

typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

// Four matrix values at a 4-aligned entry index as FP32 (FP16 values load as
// bits).  Ordinary loads, not non-temporal ones: a group's 128-byte step
// rarely starts on a cache line, so each line is read by two successive
// steps, and with the non-temporal hint the line was often gone before the
// second (1.78x the algorithmic bytes from L2 to memory, against 1.20x with
// ordinary loads, and 15% slower, measured on gfx950).
template <typename VT>
__device__ __forceinline__ f32x4 ld_val4(const VT* p) {
  if constexpr (sizeof(VT) == 4) {
    return ld<false>(reinterpret_cast<const f32x4*>(p));
  } else {
    const u16x4 h = ld<false>(reinterpret_cast<const u16x4*>(p));
    return f32x4{__half2float(__ushort_as_half(h.x)), __half2float(__ushort_as_half(h.y)),
                 __half2float(__ushort_as_half(h.z)), __half2float(__ushort_as_half(h.w))};
  }
}

// Sum of val[e] * v[col[e]] over the entries [beg, end) of one segment, by
// a group of LPR lanes: each lane takes the 4-aligned chunks (16-byte loads)
// that overlap the range, LPR chunks apart, and zeroes the entries outside
// it.  Segments of the block-major copy start at multiples of 4 entries and
// are padded to one with a real column, so every chunk lies inside the
// segment's storage and every gathered index is valid.
template <typename VT, int LPR>
__device__ __forceinline__ float seg_dot(const int32_t* __restrict__ col,
                                         const VT* __restrict__ val, const float* __restrict__ v,
                                         int64_t beg, int64_t end, int lane) {
  float acc0 = 0.f, acc1 = 0.f;
  for (int64_t e = (beg & ~(int64_t)3) + 4 * lane; e < end; e += 4 * LPR) {
    const i32x4 c = ld<false>(reinterpret_cast<const i32x4*>(col + e));
    const f32x4 a = ld_val4(val + e);
    const float a0 = (e >= beg) ? a.x : 0.f;
    const float a1 = (e + 1 >= beg && e + 1 < end) ? a.y : 0.f;
    const float a2 = (e + 2 >= beg && e + 2 < end) ? a.z : 0.f;
    const float a3 = (e + 3 < end) ? a.w : 0.f;
    acc0 = fmaf(a0, v[c.x], acc0);
    acc1 = fmaf(a1, v[c.y], acc1);
    acc0 = fmaf(a2, v[c.z], acc0);
    acc1 = fmaf(a3, v[c.w], acc1);
  }
  return acc0 + acc1;
}

// id[k] = block of internal row k (0xFF for a hole of the internal order).
template <bool RAYS>
__global__ __launch_bounds__(256) void k_block_ids(Layout L, BlockBounds b, uint8_t* __restrict__ id,
                                                   int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * 256) {
    const int64_t nat = RAYS ? L.ray_out(k) : L.pix_out(k);
    int blk = 0;
#pragma unroll
    for (int q = 1; q < kMaxSelBlocks; ++q) blk += (q < b.n && nat >= b.v[q]) ? 1 : 0;
    id[k] = nat < 0 ? (uint8_t)0xFF : (uint8_t)blk;
  }
}

// Block-major copy of one direction of the block store.  Segment j of row
// k (the entries of block j in that row) moves to bm.off[j * nrows + k],
// padded with zero values to a multiple of 4 entries on a column the row
// already uses; the segments of one block j lie back to back in internal
// row order, so the drawn blocks of consecutive rows are contiguous.
__global__ __launch_bounds__(256) void k_bm_len(const int32_t* __restrict__ seg, int nseg,
                                                int64_t nrows, int64_t* __restrict__ len4) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nrows * nseg;
       i += (int64_t)gridDim.x * 256) {
    const int j = (int)(i / nrows);
    const int64_t k = i - (int64_t)j * nrows;
    const int32_t* sg = seg + k * (nseg + 1);
    len4[i] = (sg[j + 1] - sg[j] + 3) & ~3;
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_bm_copy(const int64_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ seg, int nseg,
                                                 const int32_t* __restrict__ col,
                                                 const VT* __restrict__ val, int64_t nrows,
                                                 const int64_t* __restrict__ off,
                                                 int32_t* __restrict__ ocol, VT* __restrict__ oval) {
  // one wavefront per (row, block) segment
  const int64_t w = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (w >= nrows * nseg) return;
  const int j = (int)(w / nrows);
  const int64_t k = w - (int64_t)j * nrows;
  const int32_t* sg = seg + k * (nseg + 1);
  const int64_t src = ptr[k] + sg[j], len = sg[j + 1] - sg[j];
  const int64_t dst = off[w], len4 = off[w + 1] - dst;
  for (int64_t e = lane; e < len4; e += 64) {
    if (e < len) {
      ocol[dst + e] = col[src + e];
      oval[dst + e] = val[src + e];
    } else {
      ocol[dst + e] = col[src + len - 1];  // len4 > len implies len >= 1
      oval[dst + e] = VT(0.f);
    }
  }
}

// Forward projection and residual for the drawn pairs.  A ray of a drawn row block computes
// z^j (its segment j) for every drawn column block j and keeps it in
// Z[j * nrows + ray]; its residual becomes y - sum_j Z[j] over all column
// blocks, ascending j (kept products for the others).  Other rays copy
// r_in to r_out.  Segments are read from the block-major copy.
template <typename VT, int LPR>
__global__ __launch_bounds__(256) void k_sel_forward(
    const int32_t* __restrict__ seg, int nseg, const int64_t* __restrict__ off,
    const int32_t* __restrict__ col, const VT* __restrict__ val, const uint8_t* __restrict__ blk,
    uint64_t rows, uint64_t cols, const float* __restrict__ x, const float* __restrict__ y,
    const float* __restrict__ r_in, float* __restrict__ r_out, float* __restrict__ Z,
    int64_t nrows) {
  const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  if (row >= nrows) return;  // uniform over the lane group
  const unsigned b = blk[row];
  if (b == 0xFFu || !((rows >> b) & 1)) {
    if (lane == 0) r_out[row] = r_in[row];
    return;
  }
  const int32_t* sg = seg + row * (nseg + 1);
  float tot = 0.f;
  for (int j = 0; j < nseg; ++j) {
    float zj;
    if ((cols >> j) & 1) {
      const int64_t beg = off[(int64_t)j * nrows + row];
      zj = group_sum<LPR>(seg_dot<VT, LPR>(col, val, x, beg, beg + (sg[j + 1] - sg[j]), lane));
      if (lane == 0) Z[j * nrows + row] = zj;
    } else {
      zj = Z[j * nrows + row];
    }
    tot += zj;
  }
  if (lane == 0) r_out[row] = y[row] - tot;
}

// Backprojection, gradient sum and step for the drawn pairs.  A pixel of a drawn column block
// sums its segments i (rows of A^T restricted to I_i) over the drawn row
// blocks: out = xadd + scale * sum; other pixels copy xadd.
template <typename VT, int LPR>
__global__ __launch_bounds__(256) void k_sel_backward(
    const int32_t* __restrict__ seg, int nseg, const int64_t* __restrict__ off,
    const int32_t* __restrict__ col, const VT* __restrict__ val, const uint8_t* __restrict__ blk,
    uint64_t rows, uint64_t cols, const float* __restrict__ r, const float* __restrict__ xadd,
    float scale, float* __restrict__ out, int64_t nrows) {
  const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  if (row >= nrows) return;  // uniform over the lane group
  const unsigned b = blk[row];
  if (b == 0xFFu || !((cols >> b) & 1)) {
    if (lane == 0) out[row] = xadd[row];
    return;
  }
  const int32_t* sg = seg + row * (nseg + 1);
  float acc = 0.f;
  for (int i = 0; i < nseg; ++i)
    if ((rows >> i) & 1) {
      const int64_t beg = off[(int64_t)i * nrows + row];
      acc += seg_dot<VT, LPR>(col, val, r, beg, beg + (sg[i + 1] - sg[i]), lane);
    }
  acc = group_sum<LPR>(acc);
  if (lane == 0) out[row] = fmaf(scale, acc, xadd[row]);
}

static BlockBounds block_bounds(const std::vector<int64_t>& off) {
  BlockBounds b{};
  b.n = (int)off.size() - 1;
  for (size_t k = 0; k < off.size() && k <= (size_t)kMaxSelBlocks; ++k) b.v[k] = off[k];
  return b;
}

hipError_t launch_block_ids(const bsgd_plan* p, uint8_t* blk_r, uint8_t* blk_c, hipStream_t s) {
  const Layout& L = p->L;
  k_block_ids<true><<<1024, 256, 0, s>>>(L, block_bounds(p->row_off), blk_r, L.r_int);
  k_block_ids<false><<<1024, 256, 0, s>>>(L, block_bounds(p->col_off), blk_c, L.c_int);
  return hipGetLastError();
}

size_t block_major_entries(const Store& st) {
  return (size_t)(st.nnz + 3 * st.nrows * (int64_t)st.nseg + 4);
}

hipError_t build_block_major(const Store& st, BlockMajor& bm, int64_t* scan_tmp, hipStream_t s) {
  const int64_t n = st.nrows * st.nseg;
  bm.nrows = st.nrows;
  bm.nseg = st.nseg;
  k_bm_len<<<std::max<unsigned>(1, std::min<unsigned>((unsigned)((n + 255) / 256), 4096)), 256,
             0, s>>>(st.seg, st.nseg, st.nrows, bm.off);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = exclusive_scan_i64(bm.off, bm.off, n, scan_tmp, s);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)((n * 64 + 255) / 256);
  if (blocks == 0) return hipSuccess;
  k_bm_copy<float><<<blocks, 256, 0, s>>>(st.ptr, st.seg, st.nseg, st.col, st.val, st.nrows,
                                           bm.off, bm.col, bm.val);
  if (bm.val16)
    k_bm_copy<__half><<<blocks, 256, 0, s>>>(st.ptr, st.seg, st.nseg, st.col, st.val16,
                                              st.nrows, bm.off, bm.col, bm.val16);
  return hipGetLastError();
}

constexpr int kSelLanes = 8;

hipError_t launch_sel_forward(const Store& st, const BlockMajor& bm, bsgd_valtype vt,
                              const uint8_t* blk, uint64_t rows, uint64_t cols, const float* x,
                              const float* y, const float* r_in, float* r_out, float* Z,
                              hipStream_t s) {
  const unsigned blocks = (unsigned)((st.nrows * kSelLanes + 255) / 256);
  if (!blocks) return hipSuccess;
  if (vt == BSGD_VAL_F16)
    k_sel_forward<__half, kSelLanes><<<blocks, 256, 0, s>>>(
        st.seg, st.nseg, bm.off, bm.col, bm.val16, blk, rows, cols, x, y, r_in, r_out, Z,
        st.nrows);
  else
    k_sel_forward<float, kSelLanes><<<blocks, 256, 0, s>>>(
        st.seg, st.nseg, bm.off, bm.col, bm.val, blk, rows, cols, x, y, r_in, r_out, Z,
        st.nrows);
  return hipGetLastError();
}

hipError_t launch_sel_backward(const Store& st, const BlockMajor& bm, bsgd_valtype vt,
                               const uint8_t* blk, uint64_t rows, uint64_t cols, const float* r,
                               const float* xadd, float scale, float* out, hipStream_t s) {
  const unsigned blocks = (unsigned)((st.nrows * kSelLanes + 255) / 256);
  if (!blocks) return hipSuccess;
  if (vt == BSGD_VAL_F16)
    k_sel_backward<__half, kSelLanes><<<blocks, 256, 0, s>>>(
        st.seg, st.nseg, bm.off, bm.col, bm.val16, blk, rows, cols, r, xadd, scale, out,
        st.nrows);
  else
    k_sel_backward<float, kSelLanes><<<blocks, 256, 0, s>>>(
        st.seg, st.nseg, bm.off, bm.col, bm.val, blk, rows, cols, r, xadd, scale, out,
        st.nrows);
  return hipGetLastError();
}

}  // namespace bsgd

// ---------------------------------------------------------------------------
// C ABI: step-level products (natural orders; the plan's scratch vectors
// carry the permuted operands, so calls on one plan must not overlap)
// ---------------------------------------------------------------------------
using namespace bsgd;

static bsgd_status check_vt(const bsgd_plan* plan, bsgd_valtype vt) {
  BSGD_REQUIRE(plan != nullptr, "plan is NULL");
  BSGD_REQUIRE(vt == BSGD_VAL_F32 || vt == BSGD_VAL_F16, "unknown value type %d", (int)vt);
  if (vt == BSGD_VAL_F16 && !(plan->flags & BSGD_PLAN_F16)) {
    set_error("plan was created without BSGD_PLAN_F16");
    return BSGD_ERR_INVALID;
  }
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_forward(const bsgd_plan* plan, bsgd_valtype vt, const float* x,
                                    const float* y, float* out, hipStream_t stream) {
  clear_error();
  bsgd_status st = check_vt(plan, vt);
  if (st != BSGD_OK) return st;
  BSGD_REQUIRE(x != nullptr && out != nullptr, "x and out must be non-NULL");
  BSGD_NEED_FWD(plan, "bsgd_forward");
  const Layout& L = plan->L;
  BSGD_HIP(permute_in(L, kPixels, x, plan->vin, stream));
  if (y) BSGD_HIP(permute_in(L, kRays, y, plan->vaux, stream));
  BSGD_HIP(launch_rows(plan->fwd, vt, y ? kResidual : kPlain, plan->vin, plan->vaux, nullptr,
                       1.0f, plan->vout, stream));
  BSGD_HIP(permute_out(L, kRays, plan->vout, out, stream));
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_backproject(const bsgd_plan* plan, bsgd_valtype vt, const float* r,
                                        const float* x, float mu, float* out,
                                        hipStream_t stream) {
  clear_error();
  bsgd_status st = check_vt(plan, vt);
  if (st != BSGD_OK) return st;
  BSGD_REQUIRE(r != nullptr && out != nullptr, "r and out must be non-NULL");
  BSGD_NEED_BWD(plan, "bsgd_backproject");
  const Layout& L = plan->L;
  BSGD_HIP(permute_in(L, kRays, r, plan->vin, stream));
  if (x) {
    BSGD_HIP(permute_in(L, kPixels, x, plan->vaux, stream));
    BSGD_HIP(launch_rows(plan->bwd, vt, kStep, plan->vin, nullptr, plan->vaux, 2.0f * mu,
                         plan->vout, stream));
  } else {
    BSGD_HIP(launch_rows(plan->bwd, vt, kPlain, plan->vin, nullptr, nullptr, 2.0f, plan->vout,
                         stream));
  }
  BSGD_HIP(permute_out(L, kPixels, plan->vout, out, stream));
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_forward_block(const bsgd_plan* plan, bsgd_valtype vt, int i, int j,
                                          const float* xj, float* z, hipStream_t stream) {
  clear_error();
  bsgd_status st = check_vt(plan, vt);
  if (st != BSGD_OK) return st;
  BSGD_REQUIRE(i >= 0 && i < plan->M && j >= 0 && j < plan->N, "block (%d, %d) out of range", i,
               j);
  BSGD_REQUIRE(xj != nullptr && z != nullptr, "xj and z must be non-NULL");
  BSGD_NEED_FWD(plan, "bsgd_forward_block");
  const int64_t r0 = plan->row_off[i], r1 = plan->row_off[i + 1];
  BSGD_HIP(launch_segment_rows(plan, true, vt, r0, r1 - r0, j, plan->col_off[j], xj, 1.0f, z,
                               stream));
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_backproject_block(const bsgd_plan* plan, bsgd_valtype vt, int i,
                                              int j, const float* ri, float* g,
                                              hipStream_t stream) {
  clear_error();
  bsgd_status st = check_vt(plan, vt);
  if (st != BSGD_OK) return st;
  BSGD_REQUIRE(i >= 0 && i < plan->M && j >= 0 && j < plan->N, "block (%d, %d) out of range", i,
               j);
  BSGD_REQUIRE(ri != nullptr && g != nullptr, "ri and g must be non-NULL");
  BSGD_NEED_BWD(plan, "bsgd_backproject_block");
  const int64_t c0 = plan->col_off[j], c1 = plan->col_off[j + 1];
  BSGD_HIP(launch_segment_rows(plan, false, vt, c0, c1 - c0, i, plan->row_off[i], ri, 2.0f, g,
                               stream));
  return BSGD_OK;
}

// ---------------------------------------------------------------------------
// Several right-hand sides (slices of a volume, or a batch of reconstructions
// sharing A): V is [ncols_int][S], Y / XADD / OUT are [nrows_int][S], the RHS
// index fastest.  Each lane owns 4 consecutive RHS, so L = min(S/4, 16) lanes
// cover a chunk of 4L RHS (one 16-byte gather per lane and entry, 16L bytes
// contiguous per entry).  Chunks of at most 64 RHS keep the rows gathered by
// one chunk (256 bytes per vector row: 67 MB for a 512 x 512 image) inside
// the 256 MB last-level cache: 256 RHS at once (268 MB) made the 256-slice
// volume's epochs 16% slower on gfx950, although A is read once per chunk.  When S is small the row's entries are split over G
// groups of L lanes (G = 8 for L <= 8, else 64/L): group g takes the 4-entry
// chunks g, g + G, ... (rows are padded to a multiple of 8 entries, so chunks
// never straddle the row end), and the G partial sums are added with xor
// shuffles in a fixed order.  A row uses L*G lanes; a wavefront holds 64/(L*G)
// rows.  blockIdx.y selects the RHS chunk when S > 64 (the chunks run in
// order: blockIdx.x varies fastest in the launch).  No atomics; the
// summation order depends only on S.
// ---------------------------------------------------------------------------
namespace bsgd {

__device__ __forceinline__ f32x4 load_vals(const float* __restrict__ val, int64_t e) {
  return *reinterpret_cast<const f32x4*>(val + e);
}

__device__ __forceinline__ f32x4 load_vals(const __half* __restrict__ val, int64_t e) {
  typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
  const f16x4 h = *reinterpret_cast<const f16x4*>(val + e);
  return f32x4{(float)h.x, (float)h.y, (float)h.z, (float)h.w};
}

template <typename VT, int MODE, int L>
__global__ __launch_bounds__(256) void k_spmm(const int64_t* __restrict__ ptr,
                                              const int32_t* __restrict__ col,
                                              const VT* __restrict__ val,
                                              const float* __restrict__ V,
                                              const float* __restrict__ Y,
                                              const float* __restrict__ XADD, float scale,
                                              float* __restrict__ OUT, int64_t nrows, int S) {
  constexpr int G = L <= 8 ? 8 : 64 / L;  // entry groups per row
  constexpr int LPR = L * G;              // lanes per row
  constexpr int RPW = 64 / LPR;           // rows per wavefront
  const int lane = threadIdx.x & 63;
  const int li = lane % LPR, g = li / L, l = li % L;
  const int64_t row = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW + lane / LPR;
  const int j = blockIdx.y * (4 * L) + 4 * l;  // < S: the host launches S / (4L) chunks
  // rows past the end keep an empty range; every lane reaches the shuffles
  int64_t beg = 0, end = 0;
  if (row < nrows) {
    beg = ptr[row];
    end = ptr[row + 1];
  }
  f32x4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0, a2 = a0, a3 = a0;
  for (int64_t e = beg + 4 * g; e < end; e += 4 * G) {
    const i32x4 c = *reinterpret_cast<const i32x4*>(col + e);
    const f32x4 w = load_vals(val, e);
    const f32x4 v0 = *reinterpret_cast<const f32x4*>(V + (int64_t)c.x * S + j);
    const f32x4 v1 = *reinterpret_cast<const f32x4*>(V + (int64_t)c.y * S + j);
    const f32x4 v2 = *reinterpret_cast<const f32x4*>(V + (int64_t)c.z * S + j);
    const f32x4 v3 = *reinterpret_cast<const f32x4*>(V + (int64_t)c.w * S + j);
    a0 += w.x * v0;
    a1 += w.y * v1;
    a2 += w.z * v2;
    a3 += w.w * v3;
  }
  f32x4 acc = (a0 + a1) + (a2 + a3);
#pragma unroll
  for (int off = L; off < LPR; off <<= 1) {
    acc.x += __shfl_xor(acc.x, off);
    acc.y += __shfl_xor(acc.y, off);
    acc.z += __shfl_xor(acc.z, off);
    acc.w += __shfl_xor(acc.w, off);
  }
  if (g != 0 || row >= nrows) return;
  const int64_t o = row * S + j;
  f32x4 res;
  if constexpr (MODE == kPlain) {
    res = scale * acc;
  } else if constexpr (MODE == kResidual) {
    res = *reinterpret_cast<const f32x4*>(Y + o) - acc;
  } else {
    const f32x4 xa = *reinterpret_cast<const f32x4*>(XADD + o);
    res.x = fmaf(scale, acc.x, xa.x);
    res.y = fmaf(scale, acc.y, xa.y);
    res.z = fmaf(scale, acc.z, xa.z);
    res.w = fmaf(scale, acc.w, xa.w);
  }
  *reinterpret_cast<f32x4*>(OUT + o) = res;
}

template <int MODE, int L>
static hipError_t launch_spmm_l(const Store& st, bsgd_valtype vt, const float* V, const float* Y,
                                const float* XADD, float scale, float* OUT, int S,
                                hipStream_t s) {
  constexpr int G = L <= 8 ? 8 : 64 / L;
  constexpr int rows_per_block = 4 * (64 / (L * G));
  dim3 grid((unsigned)((st.nrows + rows_per_block - 1) / rows_per_block),
            (unsigned)(S / (4 * L)));
  if (grid.x == 0) return hipSuccess;
  if (vt == BSGD_VAL_F16)
    k_spmm<__half, MODE, L><<<grid, 256, 0, s>>>(st.ptr, st.col, st.val16, V, Y, XADD, scale,
                                                 OUT, st.nrows, S);
  else
    k_spmm<float, MODE, L><<<grid, 256, 0, s>>>(st.ptr, st.col, st.val, V, Y, XADD, scale, OUT,
                                                st.nrows, S);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_spmm_mode(const Store& st, bsgd_valtype vt, const float* V,
                                   const float* Y, const float* XADD, float scale, float* OUT,
                                   int S, hipStream_t s) {
  // S is 4 .. 1024 and a power of two (checked when the state is created)
  switch (std::min(S / 4, 16)) {
    case 1: return launch_spmm_l<MODE, 1>(st, vt, V, Y, XADD, scale, OUT, S, s);
    case 2: return launch_spmm_l<MODE, 2>(st, vt, V, Y, XADD, scale, OUT, S, s);
    case 4: return launch_spmm_l<MODE, 4>(st, vt, V, Y, XADD, scale, OUT, S, s);
    case 8: return launch_spmm_l<MODE, 8>(st, vt, V, Y, XADD, scale, OUT, S, s);
    case 16: return launch_spmm_l<MODE, 16>(st, vt, V, Y, XADD, scale, OUT, S, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spmm(const Store& st, bsgd_valtype vt, RowMode mode, const float* V,
                       const float* Y, const float* XADD, float scale, float* OUT, int S,
                       hipStream_t s) {
  switch (mode) {
    case kPlain:
      return launch_spmm_mode<kPlain>(st, vt, V, Y, XADD, scale, OUT, S, s);
    case kResidual:
      return launch_spmm_mode<kResidual>(st, vt, V, Y, XADD, scale, OUT, S, s);
    default:
      return launch_spmm_mode<kStep>(st, vt, V, Y, XADD, scale, OUT, S, s);
  }
}

}  // namespace bsgd

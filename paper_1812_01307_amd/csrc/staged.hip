// Staged form of the fused products (the block products, block sums and gradient step of Algorithm 1 over the whole
// block store): the same sums as the row kernels, with every gather served
// from LDS.
//
// The internal column space (pixels for A, rays for A^T) is cut into P
// stages of SW columns, aligned to whole tile rows of the pixel order (8
// image rows) or whole groups of 8 views of the ray order, so that a stage is
// also a contiguous range of natural columns and a row's entries of one stage
// are contiguous in the source CSR.  Rows are grouped into chunks of RW.  One
// workgroup per (chunk, stage) copies the stage's slice of the vector (x or
// r, at most 128 KB) into LDS with coalesced loads and walks the chunk's row
// segments for that stage: 8 entries per lane and load (16-bit stage-local
// columns, so 6 bytes per entry with FP32 values, 4 with FP16), two loads in
// flight, groups of 4 or 8 lanes per row reduced with xor shuffles.  The
// per-stage row sums go to a partial buffer; a second pass adds the P
// partials of each row in stage order and applies the epilogue (residual or
// gradient step).  No atomics, fixed summation order: results are bitwise
// reproducible.
#include <algorithm>

#include "bsgd_internal.h"

namespace bsgd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
bool stage_geometry(const Layout& L, bool fwd, Staged& st) {
  const int64_t ncols_int = fwd ? L.c_int : L.r_int;
  const int64_t nrows_int = fwd ? L.r_int : L.c_int;
  // alignment unit: one tile row of one slice (pixels) or one group of views (rays)
  const int64_t U = fwd ? 64 * (int64_t)L.Wt : (L.view_len > 0 ? kViewTile * L.view_len : 4);
  auto width = [&](int64_t maxw) { return (maxw / U) * U; };
  int64_t sw = width(kStageSmall);
  if (sw == 0 || (ncols_int + sw - 1) / sw > 32) sw = width(kStageLarge);
  if (sw == 0) return false;
  st.SW = (int)sw;
  st.P = (int)((ncols_int + sw - 1) / sw);
  st.RW = kStageRows;
  st.nrows = nrows_int;
  st.nW = (nrows_int + st.RW - 1) / st.RW;
  st.bnd.assign(st.P + 1, 0);
  const int64_t hw = (int64_t)L.H * L.W;
  for (int s = 0; s <= st.P; ++s) {
    const int64_t q = std::min<int64_t>((int64_t)s * sw, ncols_int);
    const int64_t units = q / U;
    int64_t nat;
    if (fwd) {
      const int64_t d = units / L.Ht, tr = units % L.Ht;
      nat = d * hw + std::min<int64_t>(8 * tr, L.H) * L.W;
    } else if (L.view_len > 0) {
      nat = std::min<int64_t>(units * kViewTile * L.view_len, L.nrows);
    } else {
      nat = std::min<int64_t>(q, L.nrows);
    }
    st.bnd[s] = nat;
  }
  return true;
}

static int64_t stage_segments(const Staged& st) { return st.nW * st.P * st.RW; }

size_t stage_cnt_count(const Layout& L) {
  size_t mx = 0;
  for (int f = 0; f < 2; ++f) {
    Staged st;
    if (!stage_geometry(L, f == 0, st)) continue;
    const int64_t n = stage_segments(st);
    mx = std::max(mx, (size_t)(n + 1) + scan_tmp_count(n) + 1 + (size_t)(st.P + 1));
  }
  return mx;
}

// ---------------------------------------------------------------------------
// Build
// ---------------------------------------------------------------------------
__global__ void k_fill_i64(int64_t* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0;
}

template <bool FWD>
__device__ __forceinline__ int64_t srow(const Layout& L, int64_t k) {
  return FWD ? L.ray_out(k) : L.pix_out(k);
}
template <bool FWD>
__device__ __forceinline__ int64_t scol_in(const Layout& L, int64_t c) {
  return FWD ? L.pix_in(c) : L.ray_in(c);
}

__device__ __forceinline__ int64_t lower(const int32_t* __restrict__ c, int64_t len, int64_t b) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)c[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// cnt[(w*P + s)*RW + k] = padded length of row (w*RW + k)'s segment in stage s
template <bool FWD>
__global__ __launch_bounds__(256) void k_stage_count(const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_src,
                                                     Layout L, int64_t n_int, int P, int RW,
                                                     const int64_t* __restrict__ bnd,
                                                     int64_t* __restrict__ cnt) {
  const int64_t k = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  if (k >= n_int) return;
  const int64_t n = srow<FWD>(L, k);
  if (n < 0) return;  // a hole: counts stay 0
  const int64_t a = row_ptr[n], len = row_ptr[n + 1] - a;
  const int64_t w = k / RW, rl = k % RW;
  for (int s = lane; s < P; s += 64) {
    const int64_t lo = lower(col_src + a, len, bnd[s]);
    const int64_t hi = lower(col_src + a, len, bnd[s + 1]);
    cnt[(w * P + s) * RW + rl] = (hi - lo + kStageVec - 1) / kStageVec * kStageVec;
  }
}

// One wavefront per internal row: the lanes find the row's bounds of 64
// stages at a time (one binary search each, shared with shuffles), then the
// wavefront copies the stages' entries in turn.
template <bool FWD>
__global__ __launch_bounds__(256) void k_stage_fill(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_src,
    const float* __restrict__ val_src, Layout L, int64_t n_int, int P, int RW, int SW,
    const int64_t* __restrict__ bnd, const int64_t* __restrict__ off,
    uint16_t* __restrict__ col, float* __restrict__ val, __half* __restrict__ val16) {
  const int64_t k = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  if (k >= n_int) return;  // uniform per wavefront
  const int64_t n = srow<FWD>(L, k);
  if (n < 0) return;
  const int64_t a = row_ptr[n], len = row_ptr[n + 1] - a;
  const int64_t w = k / RW, rl = k % RW;
  for (int s0 = 0; s0 < P; s0 += 64) {
    const int ns = min(64, P - s0);
    const int mine = lane <= ns ? (int)lower(col_src + a, len, bnd[s0 + lane]) : 0;
    const int last = (int)lower(col_src + a, len, bnd[s0 + ns]);
    for (int j = 0; j < ns; ++j) {
      const int lo = __shfl(mine, j);
      const int hi = j + 1 < ns ? __shfl(mine, j + 1) : last;
      const int64_t idx = (w * P + s0 + j) * RW + rl;
      const int64_t dst = off[idx], plen = off[idx + 1] - dst;
      const int64_t base = (int64_t)(s0 + j) * SW;
      for (int64_t q = lane; q < plen; q += 64) {
        uint16_t c = 0;
        float v = 0.f;
        if (lo + q < hi) {
          c = (uint16_t)(scol_in<FWD>(L, col_src[a + lo + q]) - base);
          v = val_src[a + lo + q];
        }
        col[dst + q] = c;
        val[dst + q] = v;
        if (val16) val16[dst + q] = __float2half_rn(v);
      }
    }
  }
}

// segp[(w*P + s)*(RW+1) + k] = off[(w*P + s)*RW + k] - off[w*P*RW]; wbase[w] = off[w*P*RW]
__global__ void k_stage_segp(const int64_t* __restrict__ off, int64_t nW, int P, int RW,
                             int32_t* __restrict__ segp, int64_t* __restrict__ wbase) {
  const int64_t tot = nW * P * (int64_t)(RW + 1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ws = i / (RW + 1), k = i % (RW + 1);
    const int64_t w = ws / P;
    segp[i] = (int32_t)(off[ws * RW + k] - off[w * P * RW]);
  }
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w <= nW;
       w += (int64_t)gridDim.x * blockDim.x)
    wbase[w] = off[w * P * RW];
}

static unsigned grid_n(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
}

template <bool FWD>
bsgd_status build_staged(Staged& st, const bsgd_csr& src, const Layout& L, int64_t* scratch,
                         hipStream_t s) {
  const int64_t nseg = stage_segments(st);
  // scratch (stage_cnt_count(L) entries): counts/offsets, scan block sums, stage bounds
  int64_t* cnt = scratch;
  int64_t* scan_tmp = cnt + (nseg + 1);
  int64_t* bnd_dev = scan_tmp + scan_tmp_count(nseg) + 1;
  BSGD_HIP(hipMemcpyAsync(bnd_dev, st.bnd.data(), sizeof(int64_t) * st.bnd.size(),
                          hipMemcpyHostToDevice, s));
  k_fill_i64<<<grid_n(nseg + 1), 256, 0, s>>>(cnt, nseg + 1);
  BSGD_LAUNCH_CHECK();
  const unsigned blocks = (unsigned)((st.nrows * 64 + 255) / 256);
  k_stage_count<FWD><<<blocks, 256, 0, s>>>(src.row_ptr, src.col, L, st.nrows, st.P, st.RW,
                                            bnd_dev, cnt);
  BSGD_LAUNCH_CHECK();
  BSGD_HIP(exclusive_scan_i64(cnt, cnt, nseg, scan_tmp, s));  // in place: offsets
  int64_t total = 0;
  BSGD_HIP(hipMemcpyAsync(&total, cnt + nseg, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BSGD_HIP(hipStreamSynchronize(s));
  if (total > st.cap) {
    set_error("staged store needs %lld entries, capacity %lld", (long long)total,
              (long long)st.cap);
    return BSGD_ERR_INVALID;
  }
  k_stage_fill<FWD><<<blocks, 256, 0, s>>>(src.row_ptr, src.col, src.val, L, st.nrows, st.P,
                                           st.RW, st.SW, bnd_dev, cnt, st.col, st.val, st.val16);
  BSGD_LAUNCH_CHECK();
  k_stage_segp<<<grid_n(nseg + st.nW * st.P), 256, 0, s>>>(cnt, st.nW, st.P, st.RW, st.segp,
                                                            st.wbase);
  BSGD_LAUNCH_CHECK();
  st.total = total;
  st.built = true;
  st.lanes = 4;
  return BSGD_OK;
}

template bsgd_status build_staged<true>(Staged&, const bsgd_csr&, const Layout&, int64_t*,
                                        hipStream_t);
template bsgd_status build_staged<false>(Staged&, const bsgd_csr&, const Layout&, int64_t*,
                                         hipStream_t);

// ---------------------------------------------------------------------------
// Products
// ---------------------------------------------------------------------------
constexpr int kStageThreads = 1024;

template <typename VT>
__device__ __forceinline__ void stage_chunk(const uint16_t* __restrict__ cw,
                                            const VT* __restrict__ vw, int32_t k, u16x8& c,
                                            float (&a)[8]) {
  c = *reinterpret_cast<const u16x8*>(cw + k);
  if constexpr (sizeof(VT) == 4) {
    const f32x4 a0 = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(vw) + k);
    const f32x4 a1 = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(vw) + k + 4);
    a[0] = a0.x; a[1] = a0.y; a[2] = a0.z; a[3] = a0.w;
    a[4] = a1.x; a[5] = a1.y; a[6] = a1.z; a[7] = a1.w;
  } else {
    const f16x8 h = *reinterpret_cast<const f16x8*>(reinterpret_cast<const _Float16*>(vw) + k);
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = (float)h[q];
  }
}

template <typename VT, int LPR, int SWMAX>
__global__ __launch_bounds__(kStageThreads) void k_staged(
    const int64_t* __restrict__ wbase, const int32_t* __restrict__ segp,
    const uint16_t* __restrict__ col, const VT* __restrict__ val, const float* __restrict__ v,
    int64_t nv, int P, int RW, int SW, float* __restrict__ zpart, int64_t nrows) {
  __shared__ float sx[SWMAX];
  constexpr int NG = kStageThreads / LPR;
  constexpr int STEP = LPR * kStageVec;
  const int w = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int g = tid / LPR, l = tid % LPR;
  const int64_t base = wbase[w];
  const uint16_t* cw = col + base;
  const VT* vw = val + base;
  const int32_t* spp = segp + ((int64_t)w * P + s) * (RW + 1);
  // the stage's slice of v (SW is a multiple of 4; the tail past nv reads 0)
  const int64_t v0 = (int64_t)s * SW;
  for (int i = tid * 4; i < SW; i += kStageThreads * 4) {
    f32x4 q;
    if (v0 + i + 3 < nv) {
      q = *reinterpret_cast<const f32x4*>(v + v0 + i);
    } else {
      q.x = v0 + i < nv ? v[v0 + i] : 0.f;
      q.y = v0 + i + 1 < nv ? v[v0 + i + 1] : 0.f;
      q.z = v0 + i + 2 < nv ? v[v0 + i + 2] : 0.f;
      q.w = 0.f;
    }
    *reinterpret_cast<f32x4*>(sx + i) = q;
  }
  __syncthreads();
  const int64_t r0 = (int64_t)w * RW;
  const int rows = (int)std::min<int64_t>(RW, nrows - r0);
  for (int rl = g; rl < rows; rl += NG) {
    const int32_t b = spp[rl], e = spp[rl + 1];
    float acc0 = 0.f, acc1 = 0.f;
    int32_t k = b + l * kStageVec;
    for (; k + STEP < e; k += 2 * STEP) {
      u16x8 c0, c1;
      float a0[8], a1[8];
      stage_chunk<VT>(cw, vw, k, c0, a0);
      stage_chunk<VT>(cw, vw, k + STEP, c1, a1);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        acc0 = fmaf(a0[q], sx[c0[q]], acc0);
        acc1 = fmaf(a1[q], sx[c1[q]], acc1);
      }
    }
    if (k < e) {
      u16x8 c0;
      float a0[8];
      stage_chunk<VT>(cw, vw, k, c0, a0);
#pragma unroll
      for (int q = 0; q < 8; ++q) acc0 = fmaf(a0[q], sx[c0[q]], acc0);
    }
    float acc = acc0 + acc1;
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
    if (l == 0) zpart[(int64_t)s * nrows + r0 + rl] = acc;
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_staged_sum(const float* __restrict__ zpart, int P,
                                                    int64_t nrows, const float* __restrict__ y,
                                                    const float* __restrict__ xadd, float scale,
                                                    float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nrows;
       i += (int64_t)gridDim.x * 256) {
    float a = 0.f;
    for (int s = 0; s < P; ++s) a += zpart[(int64_t)s * nrows + i];
    if constexpr (MODE == kPlain)
      out[i] = scale * a;
    else if constexpr (MODE == kResidual)
      out[i] = y[i] - a;
    else
      out[i] = fmaf(scale, a, xadd[i]);
  }
}

template <typename VT, int LPR>
static void launch_staged_vt(const Staged& st, const VT* val, const float* v, int64_t nv,
                             float* zpart, hipStream_t s) {
  const dim3 grid((unsigned)st.nW, (unsigned)st.P);
  if (st.SW <= kStageSmall)
    k_staged<VT, LPR, kStageSmall><<<grid, kStageThreads, 0, s>>>(
        st.wbase, st.segp, st.col, val, v, nv, st.P, st.RW, st.SW, zpart, st.nrows);
  else
    k_staged<VT, LPR, kStageLarge><<<grid, kStageThreads, 0, s>>>(
        st.wbase, st.segp, st.col, val, v, nv, st.P, st.RW, st.SW, zpart, st.nrows);
}

hipError_t launch_staged(const Staged& st, bsgd_valtype vt, RowMode mode, const float* v,
                         int64_t nv, const float* y, const float* xadd, float scale, float* out,
                         float* zpart, hipStream_t s) {
  if (!st.built || (st.lanes != 4 && st.lanes != 8) || st.SW > kStageLarge)
    return hipErrorInvalidValue;
  if (st.nrows == 0) return hipSuccess;
  if (vt == BSGD_VAL_F16) {
    if (!st.val16) return hipErrorInvalidValue;
    if (st.lanes == 4)
      launch_staged_vt<__half, 4>(st, st.val16, v, nv, zpart, s);
    else
      launch_staged_vt<__half, 8>(st, st.val16, v, nv, zpart, s);
  } else {
    if (st.lanes == 4)
      launch_staged_vt<float, 4>(st, st.val, v, nv, zpart, s);
    else
      launch_staged_vt<float, 8>(st, st.val, v, nv, zpart, s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned blocks = grid_n(st.nrows);
  switch (mode) {
    case kPlain:
      k_staged_sum<kPlain><<<blocks, 256, 0, s>>>(zpart, st.P, st.nrows, y, xadd, scale, out);
      break;
    case kResidual:
      k_staged_sum<kResidual><<<blocks, 256, 0, s>>>(zpart, st.P, st.nrows, y, xadd, scale, out);
      break;
    default:
      k_staged_sum<kStep><<<blocks, 256, 0, s>>>(zpart, st.P, st.nrows, y, xadd, scale, out);
      break;
  }
  return hipGetLastError();
}

}  // namespace bsgd

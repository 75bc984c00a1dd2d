// Error reporting, scans, fills and deterministic reductions.
#include <cstdio>
#include <string>

#include "bsgd_internal.h"

namespace bsgd {

static thread_local std::string g_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
}

void clear_error() { g_error.clear(); }

// ---------------------------------------------------------------------------
// Exclusive scan of int64 (out has n + 1 entries; out[n] = total).
// Three passes: per-block sums, a single-block scan of the block sums, then
// per-block scans offset by the scanned block sums.
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;  // elements per thread
constexpr int kScanTile = kScanBlock * kScanItems;

size_t scan_tmp_count(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

__device__ inline int64_t block_inclusive_scan(int64_t v, int64_t* sh) {
  // sh: kScanBlock entries of LDS.  Hillis-Steele over the block.
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < kScanBlock; d <<= 1) {
    int64_t add = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  return sh[t];
}

__global__ __launch_bounds__(kScanBlock) void k_scan_block_sums(const int64_t* __restrict__ in,
                                                                int64_t n,
                                                                int64_t* __restrict__ sums) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += in[base + k];
  int64_t inc = block_inclusive_scan(s, sh);
  if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = inc;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int64_t* __restrict__ sums,
                                                          int64_t nb) {
  // exclusive scan of nb block sums in place, one block, sequential chunks
  __shared__ int64_t sh[kScanBlock];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kScanBlock) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nb ? sums[i] : 0;
    const int64_t inc = block_inclusive_scan(v, sh);
    const int64_t total = sh[kScanBlock - 1];
    if (i < nb) sums[i] = carry + inc - v;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const int64_t* __restrict__ in,
                                                           int64_t n,
                                                           const int64_t* __restrict__ sums,
                                                           int64_t* __restrict__ out) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t loc[kScanItems];
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    loc[k] = base + k < n ? in[base + k] : 0;
    s += loc[k];
  }
  const int64_t inc = block_inclusive_scan(s, sh);
  int64_t run = sums[blockIdx.x] + inc - s;
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += loc[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = sums[gridDim.x];
}

hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp,
                              hipStream_t s) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) {
    // n == 0: out[0] = 0
    k_scan_sums<<<1, kScanBlock, 0, s>>>(tmp, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(out, tmp, sizeof(int64_t), hipMemcpyDeviceToDevice, s);
  }
  k_scan_block_sums<<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, tmp);
  k_scan_sums<<<1, kScanBlock, 0, s>>>(tmp, nb);
  k_scan_apply<<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, tmp, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fill
// ---------------------------------------------------------------------------
__global__ void k_fill_f32(float* __restrict__ x, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

hipError_t fill_f32(float* x, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill_f32<<<(unsigned)blocks, 256, 0, s>>>(x, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deterministic FP64 sum of squares: kReduceBlocks partials over a
// grid-stride loop, then one block adds them in a fixed tree order.
// ---------------------------------------------------------------------------
__device__ inline double block_sum_f64(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = blockDim.x / 2; d > 0; d >>= 1) {
    if (t < d) sh[t] += sh[t + d];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(256) void k_sumsq_partial(const float* __restrict__ x, int64_t n,
                                                       double* __restrict__ partial) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = x[i];
    acc += v * v;
  }
  const double s = block_sum_f64(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ partial, int nparts,
                                                   double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) acc += partial[i];
  const double s = block_sum_f64(acc, sh);
  if (threadIdx.x == 0) *out = s;
}

hipError_t launch_sumsq(const float* x, int64_t n, double* partial, double* out, hipStream_t s) {
  k_sumsq_partial<<<kReduceBlocks, 256, 0, s>>>(x, n, partial);
  k_sum_final<<<1, 256, 0, s>>>(partial, kReduceBlocks, out);
  return hipGetLastError();
}

// Per-column sums of squares of an [n][S] matrix (S a power of two).  Block
// b covers rows b, b + kColBlocks, ...; with S <= 256 each thread keeps one
// column (thread t: column t mod S) and the block adds its 256/S partials per
// column in a fixed order; with S > 256 each thread keeps S/256 columns.  A
// second kernel adds the kColBlocks partials of each column in order.
__global__ __launch_bounds__(256) void k_colsumsq_partial(const float* __restrict__ X, int64_t n,
                                                          int S, double* __restrict__ partial) {
  __shared__ double sh[256];
  const int t = threadIdx.x;
  if (S <= 256) {
    const int j = t & (S - 1), per = 256 / S;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * per + t / S; i < n; i += (int64_t)kColBlocks * per) {
      const double v = X[i * S + j];
      acc += v * v;
    }
    sh[t] = acc;
    __syncthreads();
    if (t < S) {
      double s = 0.0;
      for (int m = 0; m < per; ++m) s += sh[t + m * S];
      partial[(int64_t)blockIdx.x * S + t] = s;
    }
  } else {
    for (int j = t; j < S; j += 256) {
      double acc = 0.0;
      for (int64_t i = blockIdx.x; i < n; i += kColBlocks) {
        const double v = X[i * S + j];
        acc += v * v;
      }
      partial[(int64_t)blockIdx.x * S + j] = acc;
    }
  }
}

__global__ __launch_bounds__(256) void k_colsumsq_final(const double* __restrict__ partial, int S,
                                                        double* __restrict__ out) {
  for (int j = blockIdx.x * 256 + threadIdx.x; j < S; j += gridDim.x * 256) {
    double acc = 0.0;
    for (int b = 0; b < kColBlocks; ++b) acc += partial[(int64_t)b * S + j];
    out[j] = acc;
  }
}

hipError_t launch_colsumsq(const float* X, int64_t n, int S, double* partial, double* out,
                           hipStream_t s) {
  k_colsumsq_partial<<<kColBlocks, 256, 0, s>>>(X, n, S, partial);
  k_colsumsq_final<<<(S + 255) / 256, 256, 0, s>>>(partial, S, out);
  return hipGetLastError();
}

}  // namespace bsgd

extern "C" const char* bsgd_last_error(void) { return bsgd::g_error.c_str(); }

// TV proximal step (Algorithm 1 line 9) by fast gradient projection on the
// dual, and the TV value of Eq. 2.
//
// The prox argmin_t 1/2 ||t - b||^2 + theta TV(t) (line 9 with theta = mu lam)
// is solved on the dual variable p (one 2-vector per pixel, in the unit
// disk).  With D the backward-difference operator of Eq. 2 (zero where a
// difference would leave the image) and D^T its adjoint, iteration k is
//     q_k     = p_{k-1} + c_k (p_{k-1} - p_{k-2}),  c_k = (tau_{k-1} - 1) / tau_k
//     u_k     = b - theta D^T q_k
//     p_k     = P(q_k + D u_k / (8 theta))          (P: unit-disk projection)
// with tau_1 = 1, tau_{k+1} = (1 + sqrt(1 + 4 tau_k^2)) / 2 and q_1 = 0; the
// result is b - theta D^T p_K.
//
// One kernel per iteration: a 32 x 8 tile of output pixels stages q on the
// tile plus a one-pixel halo and u on the tile plus its upper/left halo in
// LDS, so each input element is read from memory (L2 for these image-sized
// buffers) once per iteration.  The dual lives in three rotating buffer
// pairs (pv, ph); nothing needs zero-initialising because iteration 1 takes
// q = 0 and iteration 2 takes q = p_1 without reading p_0.
#include <cmath>
#include <vector>

#include "bsgd_internal.h"

namespace bsgd {

constexpr int kTW = 32;  // tile width (columns)
constexpr int kTH = 8;   // tile height (rows)

enum QMode { kQZero = 0, kQCopy = 1, kQMomentum = 2 };

__global__ __launch_bounds__(kTW* kTH) void k_fgp_iter2(
    int H, int W, const float* __restrict__ b, float theta, float step, float coef, int qmode,
    const float* __restrict__ p1v, const float* __restrict__ p1h, const float* __restrict__ p2v,
    const float* __restrict__ p2h, float* __restrict__ ov, float* __restrict__ oh) {
  __shared__ float sqv[kTH + 2][kTW + 2];
  __shared__ float sqh[kTH + 2][kTW + 2];
  __shared__ float su[kTH + 1][kTW + 1];
  const int s0 = blockIdx.y * kTH, t0 = blockIdx.x * kTW;
  const int tid = threadIdx.y * kTW + threadIdx.x;

  // q on rows s0-1 .. s0+kTH, columns t0-1 .. t0+kTW (zero outside the image)
  for (int k = tid; k < (kTH + 2) * (kTW + 2); k += kTW * kTH) {
    const int ls = k / (kTW + 2), lt = k % (kTW + 2);
    const int s = s0 - 1 + ls, t = t0 - 1 + lt;
    float qv = 0.f, qh = 0.f;
    if (qmode != kQZero && s >= 0 && s < H && t >= 0 && t < W) {
      const size_t i = (size_t)s * W + t;
      const float av = p1v[i], ah = p1h[i];
      if (qmode == kQCopy) {
        qv = av;
        qh = ah;
      } else {
        qv = fmaf(coef, av - p2v[i], av);
        qh = fmaf(coef, ah - p2h[i], ah);
      }
    }
    sqv[ls][lt] = qv;
    sqh[ls][lt] = qh;
  }
  __syncthreads();

  // u = b - theta D^T q on rows s0-1 .. s0+kTH-1, columns t0-1 .. t0+kTW-1
  for (int k = tid; k < (kTH + 1) * (kTW + 1); k += kTW * kTH) {
    const int ls = k / (kTW + 1), lt = k % (kTW + 1);
    const int s = s0 - 1 + ls, t = t0 - 1 + lt;
    float u = 0.f;
    if (s >= 0 && s < H && t >= 0 && t < W) {
      // D^T q at (s, t): qv(s,t) - qv(s+1,t) + qh(s,t) - qh(s,t+1)
      const float dtq = (sqv[ls][lt] - sqv[ls + 1][lt]) + (sqh[ls][lt] - sqh[ls][lt + 1]);
      u = b[(size_t)s * W + t] - theta * dtq;
    }
    su[ls][lt] = u;
  }
  __syncthreads();

  const int s = s0 + threadIdx.y, t = t0 + threadIdx.x;
  if (s < H && t < W) {
    const int ls = threadIdx.y + 1, lt = threadIdx.x + 1;
    const float uc = su[ls][lt];
    const float gv = s >= 1 ? uc - su[ls - 1][lt] : 0.f;
    const float gh = t >= 1 ? uc - su[ls][lt - 1] : 0.f;
    const float av = fmaf(step, gv, sqv[ls][lt]);
    const float ah = fmaf(step, gh, sqh[ls][lt]);
    const float nrm = fmaxf(1.f, sqrtf(av * av + ah * ah));
    const size_t i = (size_t)s * W + t;
    ov[i] = av / nrm;
    oh[i] = ah / nrm;
  }
}

// out = b - theta D^T p
__global__ __launch_bounds__(256) void k_fgp_out2(int H, int W, const float* __restrict__ b,
                                                  float theta, const float* __restrict__ pv,
                                                  const float* __restrict__ ph,
                                                  float* __restrict__ out) {
  const int64_t n = (int64_t)H * W;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const int s = (int)(i / W), t = (int)(i % W);
    const float dn = s + 1 < H ? pv[i + W] : 0.f;
    const float rt = t + 1 < W ? ph[i + 1] : 0.f;
    const float dtp = (pv[i] - dn) + (ph[i] - rt);
    out[i] = b[i] - theta * dtp;
  }
}

// 3-D: D x H x W volume, dual (pd, pv, ph), step 1/(12 theta).  One kernel
// per iteration without LDS staging (neighbour reads hit the caches).
// q = momentum combination of the last two duals (three planes each).
__global__ __launch_bounds__(256) void k_fgp_q3(int64_t n, float coef, int qmode,
                                                const float* __restrict__ p1,
                                                const float* __restrict__ p2,
                                                float* __restrict__ q) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < 3 * n;
       i += (int64_t)gridDim.x * 256) {
    float v = 0.f;
    if (qmode == kQCopy)
      v = p1[i];
    else if (qmode == kQMomentum)
      v = fmaf(coef, p1[i] - p2[i], p1[i]);
    q[i] = v;
  }
}

// u = b - theta D^T q
__global__ __launch_bounds__(256) void k_fgp_u3(int D, int H, int W, const float* __restrict__ b,
                                                 float theta, const float* __restrict__ q,
                                                 float* __restrict__ u) {
  const int64_t n = (int64_t)D * H * W;
  const int64_t hw = (int64_t)H * W;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const int d = (int)(i / hw);
    const int64_t rem = i % hw;
    const int s = (int)(rem / W), t = (int)(rem % W);
    const float nd = d + 1 < D ? q[i + hw] : 0.f;
    const float nv = s + 1 < H ? q[n + i + W] : 0.f;
    const float nh = t + 1 < W ? q[2 * n + i + 1] : 0.f;
    const float dtq = (q[i] - nd) + (q[n + i] - nv) + (q[2 * n + i] - nh);
    u[i] = b[i] - theta * dtq;
  }
}

__global__ __launch_bounds__(256) void k_fgp_p3(int D, int H, int W, float step,
                                                const float* __restrict__ q,
                                                const float* __restrict__ u,
                                                float* __restrict__ p) {
  const int64_t n = (int64_t)D * H * W;
  const int64_t hw = (int64_t)H * W;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const int d = (int)(i / hw);
    const int64_t rem = i % hw;
    const int s = (int)(rem / W), t = (int)(rem % W);
    const float uc = u[i];
    const float gd = d >= 1 ? uc - u[i - hw] : 0.f;
    const float gv = s >= 1 ? uc - u[i - W] : 0.f;
    const float gh = t >= 1 ? uc - u[i - 1] : 0.f;
    const float ad = fmaf(step, gd, q[i]);
    const float av = fmaf(step, gv, q[n + i]);
    const float ah = fmaf(step, gh, q[2 * n + i]);
    const float nrm = fmaxf(1.f, sqrtf(ad * ad + av * av + ah * ah));
    p[i] = ad / nrm;
    p[n + i] = av / nrm;
    p[2 * n + i] = ah / nrm;
  }
}

__global__ __launch_bounds__(256) void k_fgp_out3(int D, int H, int W, const float* __restrict__ b,
                                                  float theta, const float* __restrict__ p,
                                                  float* __restrict__ out) {
  const int64_t n = (int64_t)D * H * W;
  const int64_t hw = (int64_t)H * W;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const int d = (int)(i / hw);
    const int64_t rem = i % hw;
    const int s = (int)(rem / W), t = (int)(rem % W);
    const float nd = d + 1 < D ? p[i + hw] : 0.f;
    const float nv = s + 1 < H ? p[n + i + W] : 0.f;
    const float nh = t + 1 < W ? p[2 * n + i + 1] : 0.f;
    const float dtp = (p[i] - nd) + (p[n + i] - nv) + (p[2 * n + i] - nh);
    out[i] = b[i] - theta * dtp;
  }
}

__global__ void k_copy_f32(const float* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

size_t tv_ws_floats(int H, int W, int D) {
  const size_t n = (size_t)H * W * D;
  // 2-D: three rotating dual pairs; 3-D: three rotating triples plus q and u
  return D == 1 ? 6 * n : 9 * n + 3 * n + n;
}

static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// Momentum coefficients c_k = (tau_{k-1} - 1) / tau_k for k = 1..iters
// (c_1 = c_2 = 0), evaluated in double and rounded once to float.
static void momentum(int iters, std::vector<float>& c) {
  c.assign(iters + 1, 0.f);
  double tau = 1.0;  // tau_1
  for (int k = 2; k <= iters; ++k) {
    const double tau_next = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tau * tau));  // tau_k
    c[k] = (float)((tau - 1.0) / tau_next);
    tau = tau_next;
  }
}

hipError_t tv_prox_run(int H, int W, int D, const float* b, float theta, int iters, float* out,
                       float* ws, hipStream_t s) {
  const int64_t n = (int64_t)H * W * D;
  if (theta == 0.f || iters == 0) {
    k_copy_f32<<<grid_for(n), 256, 0, s>>>(b, out, n);
    return hipGetLastError();
  }
  std::vector<float> c;
  momentum(iters, c);
  if (D == 1) {
    float* buf[3] = {ws, ws + 2 * n, ws + 4 * n};  // (pv, ph) pairs
    const float step = 1.0f / (8.0f * theta);
    dim3 grid((W + kTW - 1) / kTW, (H + kTH - 1) / kTH);
    dim3 block(kTW, kTH);
    int cur = 0;  // buffer receiving p_k
    for (int k = 1; k <= iters; ++k) {
      float* o = buf[cur];
      const float* p1 = buf[(cur + 2) % 3];  // p_{k-1}
      const float* p2 = buf[(cur + 1) % 3];  // p_{k-2}
      const int qm = k == 1 ? kQZero : (k == 2 ? kQCopy : kQMomentum);
      k_fgp_iter2<<<grid, block, 0, s>>>(H, W, b, theta, step, c[k], qm, p1, p1 + n, p2, p2 + n, o,
                                         o + n);
      cur = (cur + 1) % 3;
    }
    const float* pk = buf[(cur + 2) % 3];
    k_fgp_out2<<<grid_for(n), 256, 0, s>>>(H, W, b, theta, pk, pk + n, out);
    return hipGetLastError();
  }
  float* buf[3] = {ws, ws + 3 * n, ws + 6 * n};  // (pd, pv, ph) triples
  float* q = ws + 9 * n;
  float* u = ws + 12 * n;
  const float step = 1.0f / (12.0f * theta);
  int cur = 0;
  for (int k = 1; k <= iters; ++k) {
    float* o = buf[cur];
    const float* p1 = buf[(cur + 2) % 3];
    const float* p2 = buf[(cur + 1) % 3];
    const int qm = k == 1 ? kQZero : (k == 2 ? kQCopy : kQMomentum);
    k_fgp_q3<<<grid_for(3 * n), 256, 0, s>>>(n, c[k], qm, p1, p2, q);
    k_fgp_u3<<<grid_for(n), 256, 0, s>>>(D, H, W, b, theta, q, u);
    k_fgp_p3<<<grid_for(n), 256, 0, s>>>(D, H, W, step, q, u, o);
    cur = (cur + 1) % 3;
  }
  k_fgp_out3<<<grid_for(n), 256, 0, s>>>(D, H, W, b, theta, buf[(cur + 2) % 3], out);
  return hipGetLastError();
}

// TV value: per-element isotropic difference length, FP64 partials.
__global__ __launch_bounds__(256) void k_tv_partial(int D, int H, int W,
                                                    const float* __restrict__ x,
                                                    double* __restrict__ partial) {
  __shared__ double sh[256];
  const int64_t n = (int64_t)D * H * W;
  const int64_t hw = (int64_t)H * W;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const int d = (int)(i / hw);
    const int64_t rem = i % hw;
    const int s = (int)(rem / W), t = (int)(rem % W);
    const double xc = x[i];
    const double gd = d >= 1 ? xc - (double)x[i - hw] : 0.0;
    const double gv = s >= 1 ? xc - (double)x[i - W] : 0.0;
    const double gh = t >= 1 ? xc - (double)x[i - 1] : 0.0;
    acc += sqrt(gd * gd + gv * gv + gh * gh);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int dd = 128; dd > 0; dd >>= 1) {
    if ((int)threadIdx.x < dd) sh[threadIdx.x] += sh[threadIdx.x + dd];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int n,
                                                      double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int dd = 128; dd > 0; dd >>= 1) {
    if ((int)threadIdx.x < dd) sh[threadIdx.x] += sh[threadIdx.x + dd];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

}  // namespace bsgd

using namespace bsgd;

static size_t tv_bytes(int H, int W, int D) {
  return align_up(tv_ws_floats(H, W, D) * sizeof(float), kAlign) +
         align_up((kReduceBlocks + 1) * sizeof(double), kAlign);
}

extern "C" bsgd_status bsgd_tv_workspace_size(int H, int W, int D, size_t* bytes) {
  clear_error();
  BSGD_REQUIRE(bytes != nullptr, "bytes is NULL");
  BSGD_REQUIRE(H >= 1 && W >= 1 && D >= 1, "bad image shape %d x %d x %d", H, W, D);
  *bytes = tv_bytes(H, W, D);
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_tv_prox(int H, int W, int D, const float* b, float theta, int iters,
                                    float* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(H >= 1 && W >= 1 && D >= 1, "bad image shape %d x %d x %d", H, W, D);
  BSGD_REQUIRE(b && out && ws, "NULL argument");
  BSGD_REQUIRE(b != out, "out may not alias b");
  BSGD_REQUIRE(std::isfinite(theta) && theta >= 0.f, "theta must be finite and >= 0");
  BSGD_REQUIRE(iters >= 0, "iters must be >= 0");
  if (ws_bytes < tv_bytes(H, W, D)) {
    set_error("tv workspace has %zu bytes, needs %zu", ws_bytes, tv_bytes(H, W, D));
    return BSGD_ERR_WORKSPACE;
  }
  BSGD_HIP(tv_prox_run(H, W, D, b, theta, iters, out, static_cast<float*>(ws), stream));
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_tv_value(int H, int W, int D, const float* x, void* ws,
                                     size_t ws_bytes, hipStream_t stream, double* tv) {
  clear_error();
  BSGD_REQUIRE(H >= 1 && W >= 1 && D >= 1, "bad image shape %d x %d x %d", H, W, D);
  BSGD_REQUIRE(x && ws && tv, "NULL argument");
  if (ws_bytes < tv_bytes(H, W, D)) {
    set_error("tv workspace has %zu bytes, needs %zu", ws_bytes, tv_bytes(H, W, D));
    return BSGD_ERR_WORKSPACE;
  }
  double* partial = reinterpret_cast<double*>(
      static_cast<char*>(ws) + align_up(tv_ws_floats(H, W, D) * sizeof(float), kAlign));
  k_tv_partial<<<kReduceBlocks, 256, 0, stream>>>(D, H, W, x, partial);
  BSGD_LAUNCH_CHECK();
  k_sum_partials<<<1, 256, 0, stream>>>(partial, kReduceBlocks, partial + kReduceBlocks);
  BSGD_LAUNCH_CHECK();
  BSGD_HIP(hipMemcpyAsync(tv, partial + kReduceBlocks, sizeof(double), hipMemcpyDeviceToHost,
                          stream));
  BSGD_HIP(hipStreamSynchronize(stream));
  return BSGD_OK;
}

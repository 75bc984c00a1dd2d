// TV proximal step of Algorithm 1 by fast gradient projection on the
// dual, and the TV value of Eq. 2.
//
// The prox argmin_t 1/2 ||t - b||^2 + theta TV(t) (the TV prox step with theta = mu lam)
// is solved on the dual variable p (one 2-vector per pixel, in the unit
// disk).  With D the backward-difference operator of Eq. 2 (zero where a
// difference would leave the image) and D^T its adjoint, iteration k is
//     q_k     = p_{k-1} + c_k (p_{k-1} - p_{k-2}),  c_k = (tau_{k-1} - 1) / tau_k
//     u_k     = b - theta D^T q_k
//     p_k     = P(q_k + D u_k / (8 theta))          (P: unit-disk projection)
// with tau_1 = 1, tau_{k+1} = (1 + sqrt(1 + 4 tau_k^2)) / 2 and q_1 = 0; the
// result is b - theta D^T p_K.  Volumes (D > 1 slices) add the difference
// across slices, project onto the unit ball of R^3 and step 1/(12 theta).
//
// 2-D: up to 20 iterations per launch (k_fgp_fused2, below): a 32 x 32
// output tile plus a halo one pixel wider than the iteration count lives in
// LDS, and the halo is recomputed rather than exchanged.  Nothing needs zero-initialising: iteration 1 takes q = 0 and iteration 2
// takes q = p_1 without reading p_0.  Images are addressed either in natural
// row-major order or in the library's internal 8 x 8-tiled pixel order.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "bsgd_internal.h"

namespace bsgd {

enum QMode { kQZero = 0, kQCopy = 1, kQMomentum = 2 };

// Projection onto the unit disk (2-D) or ball (3-D), applied in place: a
// dual vector longer than 1 is scaled by the hardware reciprocal square
// root of its squared length (within about 1 ulp of the division by the
// length; one transcendental instead of a square root and two or three
// IEEE divisions).  Every prox kernel uses these, so all schedules keep
// identical per-pixel arithmetic.
__device__ __forceinline__ void project2(float& av, float& ah) {
  const float s2 = fmaf(av, av, ah * ah);
  if (s2 > 1.f) {
    const float sc = __builtin_amdgcn_rsqf(s2);
    av *= sc;
    ah *= sc;
  }
}

__device__ __forceinline__ void project3(float& ad, float& av, float& ah) {
  const float s2 = fmaf(ad, ad, fmaf(av, av, ah * ah));
  if (s2 > 1.f) {
    const float sc = __builtin_amdgcn_rsqf(s2);
    ad *= sc;
    av *= sc;
    ah *= sc;
  }
}

template <bool TILED>
__device__ __forceinline__ int64_t pidx(const Layout& L, int d, int s, int t) {
  if constexpr (TILED)
    return L.pix_st(d, s, t);
  else
    return ((int64_t)d * L.H + s) * L.W + t;
}

// ---------------------------------------------------------------------------
// One 2-D FGP iteration per launch: a 32 x 8 tile of output pixels stages q on
// the tile plus a one-pixel halo and u on the tile plus its upper/left halo
// in LDS (no redundant work, 5 KB of LDS, so blocks co-reside with the
// concurrently running forward pass).  Batch layout and per-image theta as
// for k_fgp_fused2 (blockIdx.z = image).
// ---------------------------------------------------------------------------
constexpr int kTW = 32;  // tile width (columns)
constexpr int kTH = 8;   // tile height (rows)

template <bool TILED>
__global__ __launch_bounds__(kTW* kTH) void k_fgp_iter2(
    Layout L, int S, const float* __restrict__ lam, float mu, float theta0,
    const float* __restrict__ b, float coef, int qmode, const float* __restrict__ p1v,
    const float* __restrict__ p1h, const float* __restrict__ p2v, const float* __restrict__ p2h,
    float* __restrict__ ov, float* __restrict__ oh) {
  __shared__ float sqv[kTH + 2][kTW + 2];
  __shared__ float sqh[kTH + 2][kTW + 2];
  __shared__ float su[kTH + 1][kTW + 1];
  const int H = L.H, W = L.W;
  const int img = blockIdx.z;
  const float theta = lam ? mu * lam[img] : theta0;
  if (theta == 0.f) return;  // identity prox: the output kernel copies b
  const float step = 1.0f / (8.0f * theta);
  const int s0 = blockIdx.y * kTH, t0 = blockIdx.x * kTW;
  const int tid = threadIdx.y * kTW + threadIdx.x;

  // q on rows s0-1 .. s0+kTH, columns t0-1 .. t0+kTW (zero outside the image)
  for (int k = tid; k < (kTH + 2) * (kTW + 2); k += kTW * kTH) {
    const int ls = k / (kTW + 2), lt = k % (kTW + 2);
    const int s = s0 - 1 + ls, t = t0 - 1 + lt;
    float qv = 0.f, qh = 0.f;
    if (qmode != kQZero && s >= 0 && s < H && t >= 0 && t < W) {
      const int64_t i = pidx<TILED>(L, 0, s, t) * S + img;
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
      const float dtq = (sqv[ls][lt] - sqv[ls + 1][lt]) + (sqh[ls][lt] - sqh[ls][lt + 1]);
      u = b[pidx<TILED>(L, 0, s, t) * S + img] - theta * dtq;
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
    float av = fmaf(step, gv, sqv[ls][lt]);
    float ah = fmaf(step, gh, sqh[ls][lt]);
    project2(av, ah);
    const int64_t i = pidx<TILED>(L, 0, s, t) * S + img;
    ov[i] = av;
    oh[i] = ah;
  }
}

// out = b - theta D^T p (2-D, batch layout; theta_j = 0 copies b)
template <bool TILED>
__global__ __launch_bounds__(256) void k_fgp_out2b(Layout L, int S, const float* __restrict__ lam,
                                                   float mu, float theta0,
                                                   const float* __restrict__ b,
                                                   const float* __restrict__ pv,
                                                   const float* __restrict__ ph,
                                                   float* __restrict__ out) {
  const int H = L.H, W = L.W;
  const int64_t tot = (int64_t)H * W * S;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < tot;
       q += (int64_t)gridDim.x * 256) {
    const int img = (int)(q % S);
    const int64_t pix = q / S;
    const int s = (int)(pix / W), t = (int)(pix % W);
    const int64_t c = pidx<TILED>(L, 0, s, t) * S + img;
    const float theta = lam ? mu * lam[img] : theta0;
    if (theta == 0.f) {
      out[c] = b[c];
      continue;
    }
    const float dn = s + 1 < H ? pv[pidx<TILED>(L, 0, s + 1, t) * S + img] : 0.f;
    const float rt = t + 1 < W ? ph[pidx<TILED>(L, 0, s, t + 1) * S + img] : 0.f;
    const float dtp = (pv[c] - dn) + (ph[c] - rt);
    out[c] = b[c] - theta * dtp;
  }
}

// ---------------------------------------------------------------------------
// Fused 2-D FGP: up to kFuseMax iterations in one launch.  Each block owns a
// kFT x kFT output tile and keeps b and the last two duals on the tile plus a
// halo of (iterations + 1) pixels in LDS.  Every iteration shrinks the region
// on which the duals are exact by one pixel per side (D and D^T are one-pixel
// stencils), so after L iterations the tile and one extra row/column are
// exact; the halo work is recomputed redundantly by neighbouring blocks
// instead of exchanged.  Pixels outside the image are held at zero and the
// same boundary rules as the per-iteration kernel apply, so the arithmetic
// per pixel is the same.
// ---------------------------------------------------------------------------
constexpr int kFT = 32;
constexpr int kFuseMax = 20;    // most iterations one launch can hold (LDS sizing)
constexpr int kFuseSplit = 10;  // launches take equal chunks of at most this many
static_assert(kFuseSplit <= kFuseMax, "chunks must fit the LDS regions");
constexpr int kFR = kFT + 2 * (kFuseMax + 1);  // 74
constexpr int kFThreads = 512;

struct FuseArgs {
  float coef[kFuseMax + 1];  // coef[m] = c_{k0+m}
};

// A batch of S images shares the launch (blockIdx.z = image j, pixel (s, t)
// of image j at index(s, t) * S + j); image j uses theta_j = mu * lam[j], or
// theta0 when lam is null.  theta_j = 0 copies b (the prox is the identity).
template <bool TILED>
__global__ __launch_bounds__(kFThreads) void k_fgp_fused2(
    Layout L, int S, const float* __restrict__ lam, float mu, float theta0,
    const float* __restrict__ b, int k0, int iters, FuseArgs ca, const float* __restrict__ in1v,
    const float* __restrict__ in1h, const float* __restrict__ in2v,
    const float* __restrict__ in2h, float* __restrict__ out_x, float* __restrict__ o1v,
    float* __restrict__ o1h, float* __restrict__ o2v, float* __restrict__ o2h) {
  __shared__ float sb[kFR * kFR];
  __shared__ float sav[kFR * kFR], sah[kFR * kFR];  // dual slot A
  __shared__ float sbv[kFR * kFR], sbh[kFR * kFR];  // dual slot B
  __shared__ float su[kFR * kFR];
  const int H = L.H, W = L.W;
  const int h = iters + 1;
  const int R = kFT + 2 * h;
  const int s0 = blockIdx.y * kFT - h, t0 = blockIdx.x * kFT - h;  // image coords of LDS (0,0)
  const int tid = threadIdx.x;
  const int img = blockIdx.z;
  const float theta = lam ? mu * lam[img] : theta0;
  if (theta == 0.f) {
    if (out_x)
      for (int q = tid; q < kFT * kFT; q += kFThreads) {
        const int s = s0 + h + q / kFT, t = t0 + h + q % kFT;
        if (s < H && t < W) {
          const int64_t i = pidx<TILED>(L, 0, s, t) * S + img;
          out_x[i] = b[i];
        }
      }
    return;
  }
  const float step = 1.0f / (8.0f * theta);

  // load b and the incoming duals (p_{k0} -> slot A, p_{k0-1} -> slot B)
  for (int q = tid; q < R * R; q += kFThreads) {
    const int ls = q / R, lt = q - ls * R;
    const int s = s0 + ls, t = t0 + lt;
    float vb = 0.f, a1 = 0.f, a2 = 0.f, b1 = 0.f, b2 = 0.f;
    if (s >= 0 && s < H && t >= 0 && t < W) {
      const int64_t i = pidx<TILED>(L, 0, s, t) * S + img;
      vb = b[i];
      if (k0 >= 1) {
        a1 = in1v[i];
        a2 = in1h[i];
      }
      if (k0 >= 2) {
        b1 = in2v[i];
        b2 = in2h[i];
      }
    }
    const int o = ls * kFR + lt;
    sb[o] = vb;
    sav[o] = a1;
    sah[o] = a2;
    sbv[o] = b1;
    sbh[o] = b2;
  }
  __syncthreads();

  float* p1v = sav;  // p_{k-1}
  float* p1h = sah;
  float* p2v = sbv;  // p_{k-2}
  float* p2h = sbh;
  for (int m = 1; m <= iters; ++m) {
    const int k = k0 + m;
    const int qm = k == 1 ? kQZero : (k == 2 ? kQCopy : kQMomentum);
    const float coef = ca.coef[m];
    // q at an LDS offset from the two dual slots
    auto qv_at = [&](int o) {
      return qm == kQZero ? 0.f : (qm == kQCopy ? p1v[o] : fmaf(coef, p1v[o] - p2v[o], p1v[o]));
    };
    auto qh_at = [&](int o) {
      return qm == kQZero ? 0.f : (qm == kQCopy ? p1h[o] : fmaf(coef, p1h[o] - p2h[o], p1h[o]));
    };
    // u on [m-1, R-m) x [m-1, R-m)
    {
      const int lo = m - 1, wdt = R - m - lo;
      for (int q = tid; q < wdt * wdt; q += kFThreads) {
        const int ls = lo + q / wdt, lt = lo + q % wdt;
        const int s = s0 + ls, t = t0 + lt;
        float u = 0.f;
        if (s >= 0 && s < H && t >= 0 && t < W) {
          const int o = ls * kFR + lt;
          const float dtq = (qv_at(o) - qv_at(o + kFR)) + (qh_at(o) - qh_at(o + 1));
          u = sb[o] - theta * dtq;
        }
        su[ls * kFR + lt] = u;
      }
    }
    __syncthreads();
    // p_k on [m, R-m) x [m, R-m), written over p_{k-2}
    {
      const int lo = m, wdt = R - m - lo;
      for (int q = tid; q < wdt * wdt; q += kFThreads) {
        const int ls = lo + q / wdt, lt = lo + q % wdt;
        const int s = s0 + ls, t = t0 + lt;
        if (s >= 0 && s < H && t >= 0 && t < W) {
          const int o = ls * kFR + lt;
          const float uc = su[o];
          const float gv = s >= 1 ? uc - su[o - kFR] : 0.f;
          const float gh = t >= 1 ? uc - su[o - 1] : 0.f;
          float av = fmaf(step, gv, qv_at(o));
          float ah = fmaf(step, gh, qh_at(o));
          project2(av, ah);
          p2v[o] = av;
          p2h[o] = ah;
        }
      }
    }
    __syncthreads();
    float* tv = p1v;
    float* th = p1h;
    p1v = p2v;
    p1h = p2h;
    p2v = tv;
    p2h = th;
  }

  // outputs on the kFT x kFT tile
  for (int q = tid; q < kFT * kFT; q += kFThreads) {
    const int ls = h + q / kFT, lt = h + q % kFT;
    const int s = s0 + ls, t = t0 + lt;
    if (s >= H || t >= W) continue;
    const int o = ls * kFR + lt;
    const int64_t i = pidx<TILED>(L, 0, s, t) * S + img;
    if (out_x) {
      const float dn = s + 1 < H ? p1v[o + kFR] : 0.f;
      const float rt = t + 1 < W ? p1h[o + 1] : 0.f;
      const float dtp = (p1v[o] - dn) + (p1h[o] - rt);
      out_x[i] = sb[o] - theta * dtp;
    } else {
      o1v[i] = p1v[o];
      o1h[i] = p1h[o];
      o2v[i] = p2v[o];
      o2h[i] = p2h[o];
    }
  }
}

// Register-resident fused 2-D FGP (the default schedule): the same chunks,
// tiles, halo and per-pixel arithmetic as k_fgp_fused2, with each thread
// owning a strip of kRNP rows of one column of the tile-plus-halo region.
// b and the last two duals stay in registers; an iteration publishes q_h
// (all rows) and q_v (the strip's first row) to LDS for the D^T q stencil,
// then u (all rows; the strip's last row separately) for the D u stencil,
// with two barriers.  Vertical neighbours inside a strip come from
// registers, so an iteration costs about four LDS accesses per pixel
// instead of about twenty.  Region-edge pixels read zeros for their missing
// neighbours; like the LDS-resident kernel, errors from the edge move one
// pixel per iteration and stay inside the halo.
constexpr int kRNP = 3;                                  // rows per thread
constexpr int kRThreads = 1024;
constexpr int kRMax = kFT + 2 * (kFuseSplit + 1);        // 54: launches hold at most kFuseSplit
constexpr int kRP = kRMax + 2;                           // LDS pitch: a pad column each side
constexpr int kRNS = (kRMax + kRNP - 1) / kRNP;          // 18 strips
static_assert(kRMax * kRNS <= kRThreads, "every strip of the largest region needs a thread");

template <bool TILED>
__global__ __launch_bounds__(kRThreads) void k_fgp_reg2(
    Layout L, int S, const float* __restrict__ lam, float mu, float theta0,
    const float* __restrict__ b, int k0, int iters, FuseArgs ca, const float* __restrict__ in1v,
    const float* __restrict__ in1h, const float* __restrict__ in2v,
    const float* __restrict__ in2h, float* __restrict__ out_x, float* __restrict__ o1v,
    float* __restrict__ o1h, float* __restrict__ o2v, float* __restrict__ o2h) {
  __shared__ float sqh[kRMax * kRP];           // q_h, then p_h for the output stencil
  __shared__ float su[kRMax * kRP];            // u
  __shared__ float sqv[(kRNS + 1) * kRP];      // q_v (then p_v) of each strip's first row
  __shared__ float sub[(kRNS + 1) * kRP];      // u of strip k-1's last row at k
  const int H = L.H, W = L.W;
  const int h = iters + 1;
  const int R = kFT + 2 * h;
  const int NS = (R + kRNP - 1) / kRNP;
  const int s0 = blockIdx.y * kFT - h, t0 = blockIdx.x * kFT - h;
  const int tid = threadIdx.x;
  const int img = blockIdx.z;
  const float theta = lam ? mu * lam[img] : theta0;
  if (theta == 0.f) {
    if (out_x)
      for (int q = tid; q < kFT * kFT; q += kRThreads) {
        const int s = s0 + h + q / kFT, t = t0 + h + q % kFT;
        if (s < H && t < W) {
          const int64_t i = pidx<TILED>(L, 0, s, t) * S + img;
          out_x[i] = b[i];
        }
      }
    return;
  }
  const float step = 1.0f / (8.0f * theta);
  const bool active = tid < R * NS;
  const int col = active ? tid % R : 0, strip = active ? tid / R : 0;
  // cells no thread writes (pads, rows past the region) read as zero
  for (int q = tid; q < kRMax * kRP; q += kRThreads) {
    sqh[q] = 0.f;
    su[q] = 0.f;
  }
  for (int q = tid; q < (kRNS + 1) * kRP; q += kRThreads) {
    sqv[q] = 0.f;
    sub[q] = 0.f;
  }
  __syncthreads();
  const int row0 = strip * kRNP;
  const int t = t0 + col;
  const int lc = col + 1;  // LDS column
  float vb[kRNP], p1v[kRNP], p1h[kRNP], p2v[kRNP], p2h[kRNP];
  unsigned inside = 0;  // bit r: row0 + r is in the region and the pixel in the image
#pragma unroll
  for (int r = 0; r < kRNP; ++r) {
    const int ls = row0 + r, s = s0 + ls;
    vb[r] = p1v[r] = p1h[r] = p2v[r] = p2h[r] = 0.f;
    if (active && ls < R && s >= 0 && s < H && t >= 0 && t < W) {
      inside |= 1u << r;
      const int64_t i = pidx<TILED>(L, 0, s, t) * S + img;
      vb[r] = b[i];
      if (k0 >= 1) {
        p1v[r] = in1v[i];
        p1h[r] = in1h[i];
      }
      if (k0 >= 2) {
        p2v[r] = in2v[i];
        p2h[r] = in2h[i];
      }
    }
  }
  for (int m = 1; m <= iters; ++m) {
    const int k = k0 + m;
    const int qm = k == 1 ? kQZero : (k == 2 ? kQCopy : kQMomentum);
    const float coef = ca.coef[m];
    float qv[kRNP], qh[kRNP], u[kRNP];
#pragma unroll
    for (int r = 0; r < kRNP; ++r) {
      qv[r] = qm == kQZero ? 0.f : (qm == kQCopy ? p1v[r] : fmaf(coef, p1v[r] - p2v[r], p1v[r]));
      qh[r] = qm == kQZero ? 0.f : (qm == kQCopy ? p1h[r] : fmaf(coef, p1h[r] - p2h[r], p1h[r]));
    }
    if (active) {
#pragma unroll
      for (int r = 0; r < kRNP; ++r)
        if (row0 + r < R) sqh[(row0 + r) * kRP + lc] = qh[r];
      sqv[strip * kRP + lc] = qv[0];
    }
    __syncthreads();
    // u = b - theta D^T q
    const float qv_next = sqv[(strip + 1) * kRP + lc];  // first row of the strip below
#pragma unroll
    for (int r = 0; r < kRNP; ++r) {
      u[r] = 0.f;
      if (inside & (1u << r)) {
        const int ls = row0 + r;
        const float below = r + 1 < kRNP ? qv[r + 1] : qv_next;
        const float right = sqh[ls * kRP + lc + 1];
        const float dtq = (qv[r] - below) + (qh[r] - right);
        u[r] = vb[r] - theta * dtq;
      }
    }
    if (active) {
#pragma unroll
      for (int r = 0; r < kRNP; ++r)
        if (row0 + r < R) su[(row0 + r) * kRP + lc] = u[r];
      sub[(strip + 1) * kRP + lc] = u[kRNP - 1];
    }
    __syncthreads();
    // p = P(q + D u / (8 theta))
    const float u_prev = sub[strip * kRP + lc];  // last row of the strip above
#pragma unroll
    for (int r = 0; r < kRNP; ++r) {
      if (inside & (1u << r)) {
        const int ls = row0 + r, s = s0 + ls;
        const float uc = u[r];
        const float above = r > 0 ? u[r - 1] : u_prev;
        const float left = su[ls * kRP + lc - 1];
        const float gv = s >= 1 ? uc - above : 0.f;
        const float gh = t >= 1 ? uc - left : 0.f;
        float av = fmaf(step, gv, qv[r]);
        float ah = fmaf(step, gh, qh[r]);
        project2(av, ah);
        p2v[r] = p1v[r];
        p2h[r] = p1h[r];
        p1v[r] = av;
        p1h[r] = ah;
      }
    }
  }
  if (out_x) {
    // out = b - theta D^T p_K on the output tile: p_v of the row below, p_h
    // of the column to the right
    __syncthreads();
    if (active) {
#pragma unroll
      for (int r = 0; r < kRNP; ++r)
        if (row0 + r < R) sqh[(row0 + r) * kRP + lc] = p1h[r];
      sqv[strip * kRP + lc] = p1v[0];
    }
    __syncthreads();
    const float pv_next = sqv[(strip + 1) * kRP + lc];
#pragma unroll
    for (int r = 0; r < kRNP; ++r) {
      const int ls = row0 + r, s = s0 + ls;
      if (!active || ls < h || ls >= h + kFT || col < h || col >= h + kFT || s >= H || t >= W)
        continue;
      const float below = r + 1 < kRNP ? p1v[r + 1] : pv_next;
      const float dn = s + 1 < H ? below : 0.f;
      const float rt = t + 1 < W ? sqh[ls * kRP + lc + 1] : 0.f;
      const float dtp = (p1v[r] - dn) + (p1h[r] - rt);
      out_x[pidx<TILED>(L, 0, s, t) * S + img] = vb[r] - theta * dtp;
    }
  } else {
#pragma unroll
    for (int r = 0; r < kRNP; ++r) {
      const int ls = row0 + r, s = s0 + ls;
      if (!active || ls < h || ls >= h + kFT || col < h || col >= h + kFT || s >= H || t >= W)
        continue;
      const int64_t i = pidx<TILED>(L, 0, s, t) * S + img;
      o1v[i] = p1v[r];
      o1h[i] = p1h[r];
      o2v[i] = p2v[r];
      o2h[i] = p2h[r];
    }
  }
}

// out = b - theta D^T p (2-D)
template <bool TILED>
__global__ __launch_bounds__(256) void k_fgp_out2(Layout L, const float* __restrict__ b,
                                                  float theta, const float* __restrict__ pv,
                                                  const float* __restrict__ ph,
                                                  float* __restrict__ out) {
  const int H = L.H, W = L.W;
  const int64_t n = (int64_t)H * W;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const int s = (int)(i / W), t = (int)(i % W);
    const int64_t c = pidx<TILED>(L, 0, s, t);
    const float dn = s + 1 < H ? pv[pidx<TILED>(L, 0, s + 1, t)] : 0.f;
    const float rt = t + 1 < W ? ph[pidx<TILED>(L, 0, s, t + 1)] : 0.f;
    const float dtp = (pv[c] - dn) + (ph[c] - rt);
    out[c] = b[c] - theta * dtp;
  }
}

// 3-D (D slices): q = momentum combination of the last two duals (3 planes
// of length n each, element-wise, so the order of the planes' elements does
// not matter).
__global__ __launch_bounds__(256) void k_fgp_q3(int64_t n3, float coef, int qmode,
                                                const float* __restrict__ p1,
                                                const float* __restrict__ p2,
                                                float* __restrict__ q) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n3;
       i += (int64_t)gridDim.x * 256) {
    float v = 0.f;
    if (qmode == kQCopy)
      v = p1[i];
    else if (qmode == kQMomentum)
      v = fmaf(coef, p1[i] - p2[i], p1[i]);
    q[i] = v;
  }
}

// u = b - theta D^T q (3-D); n = plane length (vector length)
template <bool TILED>
__global__ __launch_bounds__(256) void k_fgp_u3(Layout L, int64_t n, const float* __restrict__ b,
                                                float theta, const float* __restrict__ q,
                                                float* __restrict__ u) {
  const int D = L.D, H = L.H, W = L.W;
  const int64_t hw = (int64_t)H * W, tot = hw * D;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * 256) {
    const int d = (int)(i / hw);
    const int64_t rem = i - d * hw;
    const int s = (int)(rem / W), t = (int)(rem % W);
    const int64_t c = pidx<TILED>(L, d, s, t);
    const float nd = d + 1 < D ? q[pidx<TILED>(L, d + 1, s, t)] : 0.f;
    const float nv = s + 1 < H ? q[n + pidx<TILED>(L, d, s + 1, t)] : 0.f;
    const float nh = t + 1 < W ? q[2 * n + pidx<TILED>(L, d, s, t + 1)] : 0.f;
    const float dtq = (q[c] - nd) + (q[n + c] - nv) + (q[2 * n + c] - nh);
    u[c] = b[c] - theta * dtq;
  }
}

template <bool TILED>
__global__ __launch_bounds__(256) void k_fgp_p3(Layout L, int64_t n, float step,
                                                const float* __restrict__ q,
                                                const float* __restrict__ u,
                                                float* __restrict__ p) {
  const int D = L.D, H = L.H, W = L.W;
  const int64_t hw = (int64_t)H * W, tot = hw * D;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * 256) {
    const int d = (int)(i / hw);
    const int64_t rem = i - d * hw;
    const int s = (int)(rem / W), t = (int)(rem % W);
    const int64_t c = pidx<TILED>(L, d, s, t);
    const float uc = u[c];
    const float gd = d >= 1 ? uc - u[pidx<TILED>(L, d - 1, s, t)] : 0.f;
    const float gv = s >= 1 ? uc - u[pidx<TILED>(L, d, s - 1, t)] : 0.f;
    const float gh = t >= 1 ? uc - u[pidx<TILED>(L, d, s, t - 1)] : 0.f;
    float ad = fmaf(step, gd, q[c]);
    float av = fmaf(step, gv, q[n + c]);
    float ah = fmaf(step, gh, q[2 * n + c]);
    project3(ad, av, ah);
    p[c] = ad;
    p[n + c] = av;
    p[2 * n + c] = ah;
  }
}

template <bool TILED>
__global__ __launch_bounds__(256) void k_fgp_out3(Layout L, int64_t n,
                                                  const float* __restrict__ b, float theta,
                                                  const float* __restrict__ p,
                                                  float* __restrict__ out) {
  const int D = L.D, H = L.H, W = L.W;
  const int64_t hw = (int64_t)H * W, tot = hw * D;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * 256) {
    const int d = (int)(i / hw);
    const int64_t rem = i - d * hw;
    const int s = (int)(rem / W), t = (int)(rem % W);
    const int64_t c = pidx<TILED>(L, d, s, t);
    const float nd = d + 1 < D ? p[pidx<TILED>(L, d + 1, s, t)] : 0.f;
    const float nv = s + 1 < H ? p[n + pidx<TILED>(L, d, s + 1, t)] : 0.f;
    const float nh = t + 1 < W ? p[2 * n + pidx<TILED>(L, d, s, t + 1)] : 0.f;
    const float dtp = (p[c] - nd) + (p[n + c] - nv) + (p[2 * n + c] - nh);
    out[c] = b[c] - theta * dtp;
  }
}

__global__ void k_copy_f32v(const float* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

template <bool TILED>
__global__ void k_copy_img(Layout L, const float* __restrict__ a, float* __restrict__ b) {
  const int64_t hw = (int64_t)L.H * L.W, tot = hw * L.D;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int d = (int)(i / hw);
    const int64_t rem = i - d * hw;
    const int64_t c = pidx<TILED>(L, d, (int)(rem / L.W), (int)(rem % L.W));
    b[c] = a[c];
  }
}

size_t tv_ws_floats(int64_t n, int D) {
  // 2-D: two dual pairs in, two out (fused chunks); 3-D: three rotating
  // triples plus q and u
  return D == 1 ? 8 * (size_t)n : 13 * (size_t)n;
}

static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// Momentum coefficients c_k = (tau_{k-1} - 1) / tau_k for k = 1, 2, ...
// (c_1 = c_2 = 0), evaluated in double and rounded once to float.  next()
// returns c_1, c_2, ... in turn; kept on the stack so that the prox makes no
// host allocation either.
struct Momentum {
  double tau = 1.0;  // tau_{k-1}
  int k = 0;
  float next() {
    if (++k == 1) return 0.f;
    const double tau_next = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tau * tau));  // tau_k
    const float c = (float)((tau - 1.0) / tau_next);
    tau = tau_next;
    return c;
  }
};

// 2-D FGP over S images ([n][S] with n the per-image vector length) in chunks
// of up to kFuseMax iterations, one fused launch each.  A chunk reads p_{k0}
// and p_{k0-1} (every block reads a halo, so the outputs cannot overwrite
// them) and writes p_{k0+L}, p_{k0+L-1} into the other two of four (pv, ph)
// buffer pairs; the last chunk writes the result.
template <bool TILED>
static hipError_t fgp2_per_iteration(const Layout& L, int S, const float* b, float theta0,
                                     const float* lam, float mu, int iters, Momentum& mom,
                                     float* out, float* ws,
                                     int64_t n, hipStream_t s) {
  const int64_t m = n * S;
  float* buf[3] = {ws, ws + 2 * m, ws + 4 * m};  // rotating (pv, ph) pairs
  dim3 grid((L.W + kTW - 1) / kTW, (L.H + kTH - 1) / kTH, S);
  dim3 block(kTW, kTH);
  int cur = 0;  // buffer receiving p_k
  for (int k = 1; k <= iters; ++k) {
    float* o = buf[cur];
    const float* p1 = buf[(cur + 2) % 3];  // p_{k-1}
    const float* p2 = buf[(cur + 1) % 3];  // p_{k-2}
    const int qm = k == 1 ? kQZero : (k == 2 ? kQCopy : kQMomentum);
    k_fgp_iter2<TILED><<<grid, block, 0, s>>>(L, S, lam, mu, theta0, b, mom.next(), qm, p1,
                                              p1 + m, p2, p2 + m, o, o + m);
    cur = (cur + 1) % 3;
  }
  const float* pk = buf[(cur + 2) % 3];
  k_fgp_out2b<TILED><<<grid_for((int64_t)L.H * L.W * S), 256, 0, s>>>(L, S, lam, mu, theta0, b,
                                                                       pk, pk + m, out);
  return hipGetLastError();
}

// Prox schedule: kFgpFused = up to 20 iterations per launch with recomputed
// halos, state in registers (k_fgp_reg2); kFgpFusedLds = the same chunks
// with the state in LDS (k_fgp_fused2); kFgpPerIteration = one launch per
// iteration.  All compute the same recurrence with the same arithmetic.
template <bool TILED>
static hipError_t fgp2_chunks(const Layout& L, int S, const float* b, float theta0,
                              const float* lam, float mu, int iters, float* out, float* ws,
                              int64_t n, hipStream_t s, int schedule, int split = 0) {
  Momentum mom;
  if (schedule == kFgpPerIteration && iters >= 1)
    return fgp2_per_iteration<TILED>(L, S, b, theta0, lam, mu, iters, mom, out, ws, n, s);
  const int64_t m = n * S;
  float* buf[4] = {ws, ws + 2 * m, ws + 4 * m, ws + 6 * m};
  dim3 grid((L.W + kFT - 1) / kFT, (L.H + kFT - 1) / kFT, S);
  int in = 0;  // p_{k0} in buf[in], p_{k0-1} in buf[in + 1]
  // Equal chunks of at most kFuseSplit iterations: a launch recomputes a
  // halo one pixel wider per iteration, so two launches of 10 cost less than
  // one of 20 (measured on gfx950: 63 vs 84 us at 512^2, 337 vs 388 us for
  // 30 iterations at 1024^2).  The per-pixel arithmetic does not depend on
  // the split.
  const int most = split >= 1 && split < kFuseSplit ? split : kFuseSplit;
  const int nl = (iters + most - 1) / most;
  for (int k0 = 0, li = 0; k0 < iters; ++li) {
    const int chunk = iters / nl + (li < iters % nl ? 1 : 0);
    FuseArgs ca{};
    for (int q = 1; q <= chunk; ++q) ca.coef[q] = mom.next();  // c_{k0+q}
    const float* i1 = buf[in];
    const float* i2 = buf[in + 1];
    float* o1 = buf[2 - in];
    float* o2 = buf[3 - in];
    const bool last = k0 + chunk == iters;
    if (schedule == kFgpFusedLds)
      k_fgp_fused2<TILED><<<grid, kFThreads, 0, s>>>(L, S, lam, mu, theta0, b, k0, chunk, ca, i1,
                                                     i1 + m, i2, i2 + m, last ? out : nullptr, o1,
                                                     o1 + m, o2, o2 + m);
    else
      k_fgp_reg2<TILED><<<grid, kRThreads, 0, s>>>(L, S, lam, mu, theta0, b, k0, chunk, ca, i1,
                                                   i1 + m, i2, i2 + m, last ? out : nullptr, o1,
                                                   o1 + m, o2, o2 + m);
    in = 2 - in;
    k0 += chunk;
  }
  return hipGetLastError();
}

template <bool TILED>
static hipError_t tv_prox_impl(const Layout& L, const float* b, float theta, int iters,
                               float* out, float* ws, hipStream_t s, int schedule, int split) {
  const int64_t n = TILED ? L.c_int : (int64_t)L.H * L.W * L.D;
  const int64_t npix = (int64_t)L.H * L.W * L.D;
  if (theta == 0.f || iters == 0) {
    k_copy_img<TILED><<<grid_for(npix), 256, 0, s>>>(L, b, out);
    return hipGetLastError();
  }
  if (L.D == 1)
    return fgp2_chunks<TILED>(L, 1, b, theta, nullptr, 1.f, iters, out, ws, n, s, schedule,
                              split);
  Momentum mom;
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
    k_fgp_q3<<<grid_for(3 * n), 256, 0, s>>>(3 * n, mom.next(), qm, p1, p2, q);
    k_fgp_u3<TILED><<<grid_for(npix), 256, 0, s>>>(L, n, b, theta, q, u);
    k_fgp_p3<TILED><<<grid_for(npix), 256, 0, s>>>(L, n, step, q, u, o);
    cur = (cur + 1) % 3;
  }
  k_fgp_out3<TILED><<<grid_for(npix), 256, 0, s>>>(L, n, b, theta, buf[(cur + 2) % 3], out);
  return hipGetLastError();
}

hipError_t tv_prox_run(const Layout& L, bool tiled, const float* b, float theta, int iters,
                       float* out, float* ws, hipStream_t s, int schedule, int split) {
  return tiled ? tv_prox_impl<true>(L, b, theta, iters, out, ws, s, schedule, split)
               : tv_prox_impl<false>(L, b, theta, iters, out, ws, s, schedule, split);
}

hipError_t tv_prox_batch(const Layout& L, int S, const float* b, float mu, const float* lam,
                         float lam0, int iters, float* out, float* ws, hipStream_t s,
                         int schedule, int split) {
  if (iters == 0) {
    // identity for every image: one chunk-free copy through the theta = 0 path
    return fgp2_chunks<true>(L, S, b, 0.f, nullptr, mu, 1, out, ws, L.c_int, s, kFgpFused);
  }
  return fgp2_chunks<true>(L, S, b, mu * lam0, lam, mu, iters, out, ws, L.c_int, s, schedule,
                          split);
}

// ---------------------------------------------------------------------------
// 3-D FGP for a volume of S slices stored slice-minor in the internal pixel
// order: voxel (d, s, t) at pix_st(s, t) * S + d.  One kernel per iteration
// (the same recurrence as the 2-D kernels, with the difference across slices
// added and step 1/(12 theta)).  A block owns one 8 x 8 memory tile of
// pixels and walks down its slices in chunks of kVC = 32 (one 128-byte line
// of a pixel's slices).  Chunk c0 loads q and b on slices c0 .. c0 + 31,
// whole lines, for the tile plus a one-pixel halo; u on a slice needs q on
// the next slice, so the chunk forms u and the new dual one slice behind,
// on slices c0 - 1 .. c0 + 30, and carries the last q, u and b slices to the
// next chunk.  Every line of the block's columns is read once (the halo
// columns belong to neighbouring tiles).  LDS holds slices fastest (pitch
// kVC + 1 floats), so a wavefront's lanes address consecutive words.
// ---------------------------------------------------------------------------
constexpr int kVS = 8;                       // pixel tile side
constexpr int kVC = 32;                      // slices per chunk
constexpr int kVQP = (kVS + 2) * (kVS + 2);  // q pixels: tile plus one-pixel halo
constexpr int kVUP = (kVS + 1) * (kVS + 1);  // u pixels: tile plus upper/left halo
constexpr int kVThreads = 512;
static_assert(kVThreads % kVC == 0 && kVC == 32, "u phase: one pixel per 32 lanes");

__global__ __launch_bounds__(kVThreads) void k_fgp_iter3v(
    Layout L, int S, const float* __restrict__ b, float theta, float step, float coef, int qmode,
    const float* __restrict__ p1, const float* __restrict__ p2, float* __restrict__ po,
    int64_t n) {
  // In chunk c0: sq[c][qp][j] = component c (depth, vertical, horizontal) of
  // q on slice c0 - 1 + j of halo pixel qp = (s - s0 + 1) * 10 + (t - t0 + 1);
  // su[up][j] = u on slice c0 - 2 + j of pixel up = (s - s0 + 1) * 9 + (t - t0 + 1);
  // sb[c0 / kVC % 2][up] = b on slice c0 - 1.  Zero outside the volume.
  __shared__ float sq[3][kVQP][kVC + 1];
  __shared__ float su[kVUP][kVC + 1];
  __shared__ float sb[2][kVUP];
  const int H = L.H, W = L.W;
  const int tile = blockIdx.x;
  const int s0 = (tile / L.Wt) * kVS, t0 = (tile % L.Wt) * kVS;
  const int tid = threadIdx.x;
  for (int k = tid; k < kVQP + kVUP; k += kVThreads) {
    if (k < kVQP) {
      sq[0][k][0] = 0.f;
      sq[1][k][0] = 0.f;
      sq[2][k][0] = 0.f;
    } else {
      su[k - kVQP][0] = 0.f;
      sb[0][k - kVQP] = 0.f;
    }
  }
  for (int c0 = 0, par = 0; c0 - 1 < S; c0 += kVC, par ^= 1) {
    // q on slices c0 .. c0 + 31
    for (int k = tid; k < kVQP * kVC; k += kVThreads) {
      const int qp = k / kVC, j = k % kVC;
      const int s = s0 - 1 + qp / (kVS + 2), t = t0 - 1 + qp % (kVS + 2), d = c0 + j;
      float qa = 0.f, qb = 0.f, qc = 0.f;
      if (qmode != kQZero && d < S && s >= 0 && s < H && t >= 0 && t < W) {
        const int64_t i = L.pix_st(0, s, t) * S + d;
        const float a1 = p1[i], b1 = p1[n + i], c1 = p1[2 * n + i];
        if (qmode == kQCopy) {
          qa = a1;
          qb = b1;
          qc = c1;
        } else {
          qa = fmaf(coef, a1 - p2[i], a1);
          qb = fmaf(coef, b1 - p2[n + i], b1);
          qc = fmaf(coef, c1 - p2[2 * n + i], c1);
        }
      }
      sq[0][qp][j + 1] = qa;
      sq[1][qp][j + 1] = qb;
      sq[2][qp][j + 1] = qc;
    }
    __syncthreads();
    // u = b - theta D^T q on slices e = c0 - 1 + j.  Each group of 32 lanes
    // holds one pixel; lane j loads b on slice c0 + j and takes b on e from
    // lane j - 1 (lane 0 from the previous chunk's slice c0 - 1).
    for (int k = tid; k < kVUP * kVC; k += kVThreads) {
      const int up = k / kVC, j = k % kVC;
      const int ls = up / (kVS + 1), lt = up % (kVS + 1);
      const int s = s0 - 1 + ls, t = t0 - 1 + lt, e = c0 - 1 + j;
      const bool pix = s >= 0 && s < H && t >= 0 && t < W;
      const float bn = (pix && e + 1 < S) ? b[L.pix_st(0, s, t) * S + e + 1] : 0.f;
      float be = __shfl_up(bn, 1, kVC);
      if (j == 0) be = sb[par][up];
      if (j == kVC - 1) sb[par ^ 1][up] = bn;
      float u = 0.f;
      if (pix && e >= 0 && e < S) {
        const int c = ls * (kVS + 2) + lt;
        const float dtq = (sq[0][c][j] - sq[0][c][j + 1]) +
                          (sq[1][c][j] - sq[1][c + kVS + 2][j]) +
                          (sq[2][c][j] - sq[2][c + 1][j]);
        u = be - theta * dtq;
      }
      su[up][j + 1] = u;
    }
    __syncthreads();
    // p = P(q + step D u) on the tile, slices e = c0 - 1 + j
    for (int k = tid; k < kVS * kVS * kVC; k += kVThreads) {
      const int tp = k / kVC, j = k % kVC;
      const int ls = tp / kVS, lt = tp % kVS;
      const int s = s0 + ls, t = t0 + lt, e = c0 - 1 + j;
      if (s >= H || t >= W || e < 0 || e >= S) continue;
      const int uc = (ls + 1) * (kVS + 1) + lt + 1;
      const float u0 = su[uc][j + 1];
      const float gd = e >= 1 ? u0 - su[uc][j] : 0.f;
      const float gv = s >= 1 ? u0 - su[uc - (kVS + 1)][j + 1] : 0.f;
      const float gh = t >= 1 ? u0 - su[uc - 1][j + 1] : 0.f;
      const int c = (ls + 1) * (kVS + 2) + lt + 1;
      float ad = fmaf(step, gd, sq[0][c][j]);
      float av = fmaf(step, gv, sq[1][c][j]);
      float ah = fmaf(step, gh, sq[2][c][j]);
      project3(ad, av, ah);
      const int64_t i = L.pix_st(0, s, t) * S + e;
      po[i] = ad;
      po[n + i] = av;
      po[2 * n + i] = ah;
    }
    __syncthreads();
    // the chunk's last q and u slices become the next chunk's first
    for (int k = tid; k < kVQP + kVUP; k += kVThreads) {
      if (k < kVQP) {
        sq[0][k][0] = sq[0][k][kVC];
        sq[1][k][0] = sq[1][k][kVC];
        sq[2][k][0] = sq[2][k][kVC];
      } else {
        su[k - kVQP][0] = su[k - kVQP][kVC];
      }
    }
    __syncthreads();
  }
}

// out = b - theta D^T p (volume, slice-minor)
__global__ __launch_bounds__(256) void k_fgp_out3v(Layout L, int S, const float* __restrict__ b,
                                                   float theta, const float* __restrict__ p,
                                                   float* __restrict__ out, int64_t n) {
  const int64_t tot = (int64_t)L.H * L.W * S;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < tot;
       q += (int64_t)gridDim.x * 256) {
    const int d = (int)(q % S);
    const int64_t pix = q / S;
    const int s = (int)(pix / L.W), t = (int)(pix % L.W);
    const int64_t c = L.pix_st(0, s, t) * S + d;
    const float nd = d + 1 < S ? p[c + 1] : 0.f;
    const float nv = s + 1 < L.H ? p[n + L.pix_st(0, s + 1, t) * S + d] : 0.f;
    const float nh = t + 1 < L.W ? p[2 * n + L.pix_st(0, s, t + 1) * S + d] : 0.f;
    const float dtp = (p[c] - nd) + (p[n + c] - nv) + (p[2 * n + c] - nh);
    out[c] = b[c] - theta * dtp;
  }
}

// ---------------------------------------------------------------------------
// Temporally blocked 3-D FGP (volumes; the default schedule).  One launch runs
// KL consecutive iterations.  Block (bx, by, bz) owns the columns t in
// [bx T, bx T + T), the slices d in [by T, by T + T) and the image rows s in
// [bz R, bz R + R), T = 32 - 2 KL, on a region of 32 x 32 (t, d) cells times
// R + 2 KL rows: the owned ones plus a halo of KL on each side, recomputed
// rather than exchanged (a value from the region edge is wrong by one more
// cell per iteration, so after KL iterations the owned cells are exact).
// One thread per (t, d) cell; the 32 cells of a thread column are
// consecutive slices of one pixel, consecutive in memory.  The block streams
// down its rows: at step tau, level m (global iteration k0 + m) works on
// local row tau - 2m, so what level m needs of
// level m - 1 (its dual on the next row) was made one step earlier and the
// levels of one step are independent.  A step has three phases separated by
// two barriers: (A) every level forms q on its next row from the two
// previous levels' duals (registers) and publishes its current row's slice
// and column components of q to LDS; (B) u = b - theta D^T q, with the row
// neighbour from registers and the t and d neighbours from LDS, published to
// LDS; (C) p = P(q + step D u), with u of the previous row from registers.
// Each level keeps its last four row outputs in registers (the next level
// reads them one step later, the one after that three steps later); b and the
// launch's input duals are read once per row at the leading edge.  The
// per-voxel arithmetic is that of k_fgp_iter3v, so both schedules agree
// bitwise.
// ---------------------------------------------------------------------------
constexpr int kBR = 32;                       // region cells along t and along d
constexpr int kTB3Rows = 64;                  // owned image rows per block
constexpr int kBRing = 8;                     // b ring: rows tau .. tau - 2 KL

template <int KL>
__global__ __launch_bounds__(kBR* kBR) void k_fgp_tb3(
    Layout L, int S, const float* __restrict__ b, float theta, float step, int k0, FuseArgs ca,
    const float* __restrict__ in1, const float* __restrict__ in2, float* __restrict__ o1,
    float* __restrict__ o2, int64_t n, int R) {
  static_assert(KL >= 1 && 2 * KL + 1 <= kBRing, "levels per launch");
  constexpr int T = kBR - 2 * KL;
  constexpr int LP = kBR + 2;  // LDS pitch: cell (x, z) at [x + 1][z + 1], pads read as zero
  __shared__ float sqd[KL][LP][LP];
  __shared__ float sqh[KL][LP][LP];
  __shared__ float su[KL][LP][LP];
  const int tid = threadIdx.x;
  const int dz = tid % kBR, tx = tid / kBR;
  const int t = (int)blockIdx.x * T - KL + tx, d = (int)blockIdx.y * T - KL + dz;
  // rows [lo, hi) are streamed, [own0, own1) written; rows outside [lo, hi)
  // read as zero (the image border where lo = 0 or hi = H)
  const int own0 = (int)blockIdx.z * R, own1 = min(own0 + R, L.H);
  const int lo = max(own0 - KL, 0), hi = min(own1 + KL, L.H);
  const bool inside = t >= 0 && t < L.W && d >= 0 && d < S;
  const bool owner = inside && tx >= KL && tx < KL + T && dz >= KL && dz < KL + T;
  for (int q = tid; q < KL * LP * LP; q += kBR * kBR) {
    (&sqd[0][0][0])[q] = 0.f;
    (&sqh[0][0][0])[q] = 0.f;
    (&su[0][0][0])[q] = 0.f;
  }
  float br[kBRing];
  float pr[KL + 1][4][3];  // pr[m][row % 4]: level m's dual (m = 0: the input p_{k0})
  float pm[2][3];          // the input p_{k0-1}, [row % 2]
  float qc[KL][3], qn[KL][3], up[KL];
#pragma unroll
  for (int i = 0; i < kBRing; ++i) br[i] = 0.f;
#pragma unroll
  for (int m = 0; m <= KL; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) pr[m][r][0] = pr[m][r][1] = pr[m][r][2] = 0.f;
#pragma unroll
  for (int r = 0; r < 2; ++r) pm[r][0] = pm[r][1] = pm[r][2] = 0.f;
#pragma unroll
  for (int m = 0; m < KL; ++m) {
    qc[m][0] = qc[m][1] = qc[m][2] = 0.f;
    qn[m][0] = qn[m][1] = qn[m][2] = 0.f;
    up[m] = 0.f;
  }
  __syncthreads();
  const int steps = (hi - lo + 2 * KL + kBRing - 1) / kBRing * kBRing;
  for (int tau0 = 0; tau0 < steps; tau0 += kBRing) {
#pragma unroll
    for (int u = 0; u < kBRing; ++u) {
      const int tau = tau0 + u;
      // leading edge: b and the input duals on row tau
      {
        float bv = 0.f, a[3] = {0.f, 0.f, 0.f}, c[3] = {0.f, 0.f, 0.f};
        if (inside && lo + tau < hi) {
          const int64_t i = L.pix_st(0, lo + tau, t) * S + d;
          bv = b[i];
          if (k0 >= 1) {
            a[0] = in1[i];
            a[1] = in1[n + i];
            a[2] = in1[2 * n + i];
          }
          if (k0 >= 2) {
            c[0] = in2[i];
            c[1] = in2[n + i];
            c[2] = in2[2 * n + i];
          }
        }
        br[u] = bv;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          pr[0][u % 4][k] = a[k];
          pm[u % 2][k] = c[k];
        }
      }
      // (A) q of level m on row tau - 2m + 1; publish q on row tau - 2m
#pragma unroll
      for (int m = 1; m <= KL; ++m) {
        const int j = k0 + m;
        const float coef = ca.coef[m];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float p1 = pr[m - 1][(u + 3) % 4][k];                       // made at tau - 1
          const float p2 = m >= 2 ? pr[m - 2][(u + 1) % 4][k] : pm[(u + 1) % 2][k];  // tau - 3
          qn[m - 1][k] = j == 1 ? 0.f : (j == 2 ? p1 : fmaf(coef, p1 - p2, p1));
        }
        sqd[m - 1][tx + 1][dz + 1] = qc[m - 1][0];
        sqh[m - 1][tx + 1][dz + 1] = qc[m - 1][2];
      }
      __syncthreads();
      // (B) u = b - theta D^T q on row tau - 2m
      float uu[KL];
#pragma unroll
      for (int m = 1; m <= KL; ++m) {
        const int s = lo + tau - 2 * m;
        uu[m - 1] = 0.f;
        if (inside && s >= lo && s < hi) {
          const float dtq = (qc[m - 1][0] - sqd[m - 1][tx + 1][dz + 2]) +
                            (qc[m - 1][1] - qn[m - 1][1]) +
                            (qc[m - 1][2] - sqh[m - 1][tx + 2][dz + 1]);
          uu[m - 1] = br[(u + kBRing - 2 * m) % kBRing] - theta * dtq;
        }
        su[m - 1][tx + 1][dz + 1] = uu[m - 1];
      }
      __syncthreads();
      // (C) p = P(q + step D u) on row tau - 2m
#pragma unroll
      for (int m = 1; m <= KL; ++m) {
        const int s = lo + tau - 2 * m;
        float ad = 0.f, av = 0.f, ah = 0.f;
        const bool live = inside && s >= lo && s < hi;
        if (live) {
          const float u0 = uu[m - 1];
          const float gd = d >= 1 ? u0 - su[m - 1][tx + 1][dz] : 0.f;
          const float gv = s >= 1 ? u0 - up[m - 1] : 0.f;
          const float gh = t >= 1 ? u0 - su[m - 1][tx][dz + 1] : 0.f;
          ad = fmaf(step, gd, qc[m - 1][0]);
          av = fmaf(step, gv, qc[m - 1][1]);
          ah = fmaf(step, gh, qc[m - 1][2]);
          project3(ad, av, ah);
        }
        pr[m][u % 4][0] = ad;
        pr[m][u % 4][1] = av;
        pr[m][u % 4][2] = ah;
        up[m - 1] = uu[m - 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) qc[m - 1][k] = qn[m - 1][k];
        if (owner && s >= own0 && s < own1) {
          const int64_t i = L.pix_st(0, s, t) * S + d;
          if (m == KL) {
            o1[i] = ad;
            o1[n + i] = av;
            o1[2 * n + i] = ah;
          }
          if (m == KL - 1) {
            o2[i] = ad;
            o2[n + i] = av;
            o2[2 * n + i] = ah;
          }
        }
      }
      if constexpr (KL == 1) {
        // the launch's second output is its input p_{k0} on the same row
        const int s = lo + tau - 2;
        if (owner && s >= own0 && s < own1) {
          const int64_t i = L.pix_st(0, s, t) * S + d;
          o2[i] = pr[0][(u + 2) % 4][0];
          o2[n + i] = pr[0][(u + 2) % 4][1];
          o2[2 * n + i] = pr[0][(u + 2) % 4][2];
        }
      }
    }
  }
}

template <int KL>
static void launch_tb3(const Layout& L, int S, const float* b, float theta, float step, int k0,
                       const FuseArgs& ca, const float* i1, const float* i2, float* o1,
                       float* o2, int64_t n, hipStream_t s) {
  constexpr int T = kBR - 2 * KL;
  dim3 grid((L.W + T - 1) / T, (S + T - 1) / T, (L.H + kTB3Rows - 1) / kTB3Rows);
  k_fgp_tb3<KL><<<grid, kBR * kBR, 0, s>>>(L, S, b, theta, step, k0, ca, i1, i2, o1, o2, n,
                                            kTB3Rows);
}

constexpr int kTB3Levels = 3;  // most iterations one launch of k_fgp_tb3 runs

hipError_t tv_prox_volume(const Layout& L, int S, const float* b, float theta, int iters,
                          float* out, float* ws, hipStream_t s, int schedule, int split) {
  const int64_t n = L.c_int * S;
  if (theta == 0.f || iters == 0) {
    k_copy_f32v<<<grid_for(n), 256, 0, s>>>(b, out, n);
    return hipGetLastError();
  }
  Momentum mom;
  const float step = 1.0f / (12.0f * theta);
  if (schedule != kFgpPerIteration) {
    // equal launches of at most kTB3Levels iterations; p_{k0} in buf[in],
    // p_{k0-1} in buf[in + 1], outputs to the other pair
    float* buf[4] = {ws, ws + 3 * n, ws + 6 * n, ws + 9 * n};
    const int most = split >= 1 && split < kTB3Levels ? split : kTB3Levels;
    const int nl = (iters + most - 1) / most;
    int in = 0;
    for (int k0 = 0, li = 0; k0 < iters; ++li) {
      const int chunk = iters / nl + (li < iters % nl ? 1 : 0);
      FuseArgs ca{};
      for (int q = 1; q <= chunk; ++q) ca.coef[q] = mom.next();  // c_{k0+q}
      const float* i1 = buf[in];
      const float* i2 = buf[in + 1];
      float* o1 = buf[2 - in];
      float* o2 = buf[3 - in];
      switch (chunk) {
        case 1: launch_tb3<1>(L, S, b, theta, step, k0, ca, i1, i2, o1, o2, n, s); break;
        case 2: launch_tb3<2>(L, S, b, theta, step, k0, ca, i1, i2, o1, o2, n, s); break;
        default: launch_tb3<3>(L, S, b, theta, step, k0, ca, i1, i2, o1, o2, n, s); break;
      }
      in = 2 - in;
      k0 += chunk;
    }
    k_fgp_out3v<<<grid_for((int64_t)L.H * L.W * S), 256, 0, s>>>(L, S, b, theta, buf[in], out,
                                                                 n);
    return hipGetLastError();
  }
  float* buf[3] = {ws, ws + 3 * n, ws + 6 * n};  // (pd, pv, ph) triples
  const unsigned grid = (unsigned)(L.Ht * L.Wt);
  int cur = 0;
  for (int k = 1; k <= iters; ++k) {
    float* o = buf[cur];
    const float* p1 = buf[(cur + 2) % 3];
    const float* p2 = buf[(cur + 1) % 3];
    const int qm = k == 1 ? kQZero : (k == 2 ? kQCopy : kQMomentum);
    k_fgp_iter3v<<<grid, kVThreads, 0, s>>>(L, S, b, theta, step, mom.next(), qm, p1, p2, o,
                                             n);
    cur = (cur + 1) % 3;
  }
  k_fgp_out3v<<<grid_for((int64_t)L.H * L.W * S), 256, 0, s>>>(L, S, b, theta,
                                                               buf[(cur + 2) % 3], out, n);
  return hipGetLastError();
}

// TV value (natural order): per-element isotropic difference length, FP64 partials.
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
  return align_up(tv_ws_floats((int64_t)H * W * D, D) * sizeof(float), kAlign) +
         align_up((kReduceBlocks + 1) * sizeof(double), kAlign);
}

static Layout natural_layout(int H, int W, int D) {
  Layout L;
  L.H = H;
  L.W = W;
  L.D = D;
  return L;
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
  BSGD_HIP(tv_prox_run(natural_layout(H, W, D), false, b, theta, iters, out,
                       static_cast<float*>(ws), stream, kFgpFused));
  return BSGD_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free prox, for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops).  The FGP duals live in a
// file-scope device array instead of a caller workspace; every GPU the
// library runs on holds its own copy of it until the process ends.  In host
// code the array's name is not a device address: its address on each device
// is taken once, with that device current, by hipGetSymbolAddress, and only
// that pointer is passed to kernels.  The FGP reads no dual it has not
// written in the same call (iteration 1 takes q = 0, iteration 2 q = p_1),
// so the array needs no clearing between calls; calls that overlap on one
// GPU share it and race.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = (size_t)32 << 20;  // 2-D up to 2^20 pixels, 3-D 645277 voxels
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) float scratch[kNoAllocBytes / sizeof(float)];

static std::mutex g_scratch_mu;
static float* g_scratch_ptr[kNoAllocDevices] = {};

// Device address of `scratch` on device `dev` (the current device).
static bsgd_status scratch_on_device(int dev, float** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                hipGetErrorString(e));
      return BSGD_ERR_HIP;
    }
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_tv_prox_noalloc(int H, int W, int D, const float* b, float theta,
                                            int iters, float* out, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(H >= 1 && W >= 1 && D >= 1, "bad image shape %d x %d x %d", H, W, D);
  BSGD_REQUIRE(b && out, "NULL argument");
  BSGD_REQUIRE(b != out, "out may not alias b");
  BSGD_REQUIRE(std::isfinite(theta) && theta >= 0.f, "theta must be finite and >= 0");
  BSGD_REQUIRE(iters >= 0, "iters must be >= 0");
  const int64_t n = (int64_t)H * W * D;
  const size_t need = tv_ws_floats(n, D) * sizeof(float);
  if (need > kNoAllocBytes) {
    set_error("bsgd_tv_prox_noalloc: a %d x %d x %d image needs %zu bytes of scratch, the "
              "library holds %zu (2-D images up to 1048576 pixels, volumes up to 645277 voxels)",
              H, W, D, need, kNoAllocBytes);
    return BSGD_ERR_WORKSPACE;
  }
  int dev = -1;
  BSGD_HIP(hipGetDevice(&dev));
  BSGD_REQUIRE(dev >= 0 && dev < kNoAllocDevices, "device %d out of range", dev);
  if (stream) {
    int sdev = -1;
    BSGD_HIP(hipStreamGetDevice(stream, &sdev));
    BSGD_REQUIRE(sdev == dev, "stream belongs to device %d, current device is %d", sdev, dev);
  }
  float* ws = nullptr;
  const bsgd_status st = scratch_on_device(dev, &ws);
  if (st != BSGD_OK) return st;
  BSGD_HIP(tv_prox_run(natural_layout(H, W, D), false, b, theta, iters, out, ws, stream,
                       kFgpFused));
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
      static_cast<char*>(ws) +
      align_up(tv_ws_floats((int64_t)H * W * D, D) * sizeof(float), kAlign));
  k_tv_partial<<<kReduceBlocks, 256, 0, stream>>>(D, H, W, x, partial);
  BSGD_LAUNCH_CHECK();
  k_sum_partials<<<1, 256, 0, stream>>>(partial, kReduceBlocks, partial + kReduceBlocks);
  BSGD_LAUNCH_CHECK();
  BSGD_HIP(hipMemcpyAsync(tv, partial + kReduceBlocks, sizeof(double), hipMemcpyDeviceToHost,
                          stream));
  BSGD_HIP(hipStreamSynchronize(stream));
  return BSGD_OK;
}


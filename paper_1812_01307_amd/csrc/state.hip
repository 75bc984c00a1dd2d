// Step size (Theorem 1) and whole epochs of Algorithm 1.
//
// Epoch schedule.  The block backprojection uses the residual r_k of the previous epoch and
// the block forward projection the current iterate x_k, so within one epoch
//     S2: x^ = x_k + mu * 2 A^T r_k     (backprojection, gradient sum and step; one fused pass over A^T)
//     S1: r_{k+1} = y - A x_k           (forward projection, residual;    one fused pass over A)
//     S5: x_{k+1} = FGP(x^)             (the TV prox step)
// S1 depends on nothing produced in the epoch, so it runs on the state's
// second stream while S2 and then the prox run on the caller's stream; the
// prox (many short launches) hides under the forward pass.  x and r are
// double-buffered; events order the buffer reuse across epochs.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "bsgd_internal.h"

struct bsgd_state {
  const bsgd_plan* plan = nullptr;
  int nrhs = 1;            // right-hand sides (vectors are [rows][nrhs], RHS fastest)
  unsigned flags = 0;      // BSGD_STATE_VOLUME: the RHS are slices of one volume (3-D TV)
  bsgd_valtype vt = BSGD_VAL_F32;
  float* lam = nullptr;    // nrhs per-RHS lambdas (batches of independent images)
  float* tmp_r = nullptr;  // r_int: one-RHS scratch (slot initialisation)
  float* tmp_c = nullptr;  // c_int
  float* y = nullptr;
  float* x[2] = {nullptr, nullptr};
  float* r[2] = {nullptr, nullptr};
  float* xhat = nullptr;
  float* tv_ws = nullptr;
  double* partial = nullptr;  // kReduceBlocks + 1 (last = result)
  float* zf = nullptr;        // per-stage partials of the staged forward product
  float* zb = nullptr;        // ... and of the staged backprojection
  const bsgd_fused* fz = nullptr;  // single-pass form (attached), with its partial sums
  bsgd::FusedPartials fzp;
  int cur = 0;
  int overlap = 1;  // 0: forward pass concurrent with backprojection + prox; 1: with the prox only
  int prox_schedule = bsgd::kFgpFused;  // 2-D prox: fused chunks or one launch per iteration
  int method = BSGD_METHOD_BSGD;        // update rule of bsgd_run_epochs
  int pass_waves = 0;   // wavefronts per single-pass workgroup (0: the default)
  int prox_split = 0;   // most FGP iterations per prox launch (0: the most)
  float* zt = nullptr;                  // BSGD_STATE_BLOCK_SELECT: kept products, [N][r_int]
  uint8_t* blk_r = nullptr;             // ... row block of each internal ray (0xFF: hole)
  uint8_t* blk_c = nullptr;             // ... column block of each internal pixel
  bsgd::BlockMajor bmf, bmb;            // ... block-major copies of A and A^T
  int64_t* bm_scan = nullptr;           // ... scan scratch for building them
  bool bm_built = false;
  int64_t epochs_done = 0;
  bool initialised = false;
  hipStream_t aux = nullptr;
  hipEvent_t ev_main = nullptr, ev_aux = nullptr;
  // optional kernel timers: 5 events per timed epoch, taken from the event
  // pool of device tev_dev
  std::vector<hipEvent_t> tev;
  int tev_dev = 0;
  int aux_dev = 0;                      // device of the pooled aux stream and events
  int t_cap = 0, t_used = 0;
  int t_stride = 1;         // time one epoch in every t_stride ...
  int64_t t_seen = 0;       // ... counting epochs since the timers were armed
};

namespace bsgd {

// ---------------------------------------------------------------------------
// Power iteration helpers
// ---------------------------------------------------------------------------
__global__ void k_scale_by_rsqrt(float* __restrict__ v, const float* __restrict__ w, int64_t n,
                                 const double* __restrict__ nrm2) {
  const double s = *nrm2 > 0.0 ? 1.0 / sqrt(*nrm2) : 0.0;
  const float fs = (float)s;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = w[i] * fs;
}

__global__ void k_ratio(const double* __restrict__ num, const double* __restrict__ den,
                        float* __restrict__ out) {
  *out = *den > 0.0 ? (float)(*num / *den) : 0.f;
}

// Golub-Kahan-Lanczos helpers: x -= sqrt(*s2) * y (s2 a sum of squares)
__global__ void k_sub_scaled(float* __restrict__ x, const float* __restrict__ y, int64_t n,
                             const double* __restrict__ s2) {
  const float a = (float)sqrt(*s2);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = fmaf(-a, y[i], x[i]);
}

static size_t lanczos_layout(const bsgd_plan* p, int steps, void* ws, float** v, float** w,
                             float** u0, float** u1, double** part, double** sc) {
  Carver cv(ws);
  *v = cv.take<float>(p->L.c_int);
  *w = cv.take<float>(p->L.c_int);
  *u0 = cv.take<float>(p->L.r_int);
  *u1 = cv.take<float>(p->L.r_int);
  *part = cv.take<double>(kReduceBlocks);
  *sc = cv.take<double>(2 * (size_t)std::max(steps, 1));
  return align_up(cv.off, kAlign);
}

// Largest eigenvalue of the symmetric tridiagonal matrix (d, e) by bisection
// on Sturm counts.
static double tridiag_max_eig(const std::vector<double>& d, const std::vector<double>& e) {
  const int n = (int)d.size();
  double lo = 0.0, hi = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    hi = std::max(hi, d[i] + r);
    lo = std::min(lo, d[i] - r);
  }
  auto count_below = [&](double x) {  // eigenvalues < x
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
      const double off = i > 0 ? e[i - 1] * e[i - 1] : 0.0;
      q = d[i] - x - (i > 0 ? off / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0.0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) == n)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

static size_t power_layout(const bsgd_plan* p, void* ws, float** v, float** z, float** w,
                           double** part, double** sc, float** res) {
  Carver cv(ws);
  *v = cv.take<float>(p->L.c_int);
  *w = cv.take<float>(p->L.c_int);
  *z = cv.take<float>(p->L.r_int);
  *part = cv.take<double>(kReduceBlocks);
  *sc = cv.take<double>(4);
  *res = cv.take<float>(4);
  return align_up(cv.off, kAlign);
}

// All state vectors are in the plan's internal orders (see bsgd::Layout),
// [rows][nrhs] with the RHS index fastest.
static size_t state_layout(const bsgd_plan* p, int S, unsigned flags, void* ws, bsgd_state* st) {
  Carver cv(ws);
  const int64_t r = p->L.r_int * S, c = p->L.c_int * S;
  st->y = cv.take<float>(r);
  st->x[0] = cv.take<float>(c);
  st->x[1] = cv.take<float>(c);
  st->r[0] = cv.take<float>(r);
  st->r[1] = cv.take<float>(r);
  st->xhat = cv.take<float>(c);
  const size_t tvf = S == 1 ? tv_ws_floats(p->L.c_int, p->D)
                            : tv_ws_floats(c, (flags & BSGD_STATE_VOLUME) ? 2 : 1);
  st->tv_ws = cv.take<float>(tvf);
  st->partial = cv.take<double>(std::max<size_t>(kReduceBlocks + 1, (size_t)(kColBlocks + 1) * S));
  st->lam = cv.take<float>(S);
  st->tmp_r = cv.take<float>(p->L.r_int);
  st->tmp_c = cv.take<float>(p->L.c_int);
  if (S == 1 && p->sfwd.P > 0) st->zf = cv.take<float>((size_t)p->sfwd.P * p->L.r_int);
  if (S == 1 && p->sbwd.P > 0) st->zb = cv.take<float>((size_t)p->sbwd.P * p->L.c_int);
  if (flags & BSGD_STATE_BLOCK_SELECT) {
    st->zt = cv.take<float>((size_t)p->N * p->L.r_int);
    st->blk_r = cv.take<uint8_t>(p->L.r_int);
    st->blk_c = cv.take<uint8_t>(p->L.c_int);
    const bool f16 = p->fwd.val16 != nullptr;
    for (int d = 0; d < 2; ++d) {
      const Store& so = d == 0 ? p->fwd : p->bwd;
      BlockMajor& bm = d == 0 ? st->bmf : st->bmb;
      const size_t cap = block_major_entries(so);
      bm.off = cv.take<int64_t>((size_t)so.nrows * so.nseg + 1);
      bm.col = cv.take<int32_t>(cap);
      bm.val = cv.take<float>(cap);
      bm.val16 = f16 ? cv.take<__half>(cap) : nullptr;
    }
    st->bm_scan = cv.take<int64_t>(
        scan_tmp_count(std::max(p->fwd.nrows * p->fwd.nseg, p->bwd.nrows * p->bwd.nseg)));
  }
  return align_up(cv.off, kAlign);
}

static bool valid_nrhs(int S) {
  return S == 1 || (S >= 4 && S <= 1024 && (S & (S - 1)) == 0);
}

}  // namespace bsgd

using namespace bsgd;

extern "C" bsgd_status bsgd_power_workspace_size(const bsgd_plan* plan, size_t* bytes) {
  clear_error();
  BSGD_REQUIRE(plan && bytes, "NULL argument");
  float *v, *z, *w, *res;
  double *part, *sc;
  *bytes = power_layout(plan, nullptr, &v, &z, &w, &part, &sc, &res);
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_power_umax(const bsgd_plan* plan, bsgd_valtype vt, int iters,
                                       void* ws, size_t ws_bytes, hipStream_t stream,
                                       float* umax) {
  clear_error();
  BSGD_REQUIRE(plan && ws && umax, "NULL argument");
  BSGD_REQUIRE(iters >= 1, "iters must be >= 1");
  BSGD_NEED_BWD(plan, "bsgd_power_umax");
  BSGD_REQUIRE(vt == BSGD_VAL_F32 || (vt == BSGD_VAL_F16 && (plan->flags & BSGD_PLAN_F16)),
               "value type not available in this plan");
  float *v, *z, *w, *res;
  double *part, *sc;
  const size_t need = power_layout(plan, ws, &v, &z, &w, &part, &sc, &res);
  if (ws_bytes < need) {
    set_error("power workspace has %zu bytes, needs %zu", ws_bytes, need);
    return BSGD_ERR_WORKSPACE;
  }
  const int64_t c = plan->L.c_int, r = plan->L.r_int;
  BSGD_HIP(fill_pixels_one(plan->L, v, stream));
  for (int it = 0; it < iters; ++it) {
    BSGD_HIP(launch_rows(plan->fwd, vt, kPlain, v, nullptr, nullptr, 1.0f, z, stream));  // A v
    BSGD_HIP(launch_rows(plan->bwd, vt, kPlain, z, nullptr, nullptr, 1.0f, w, stream));  // A^T A v
    BSGD_HIP(launch_sumsq(z, r, part, sc + 0, stream));   // ||A v||^2
    BSGD_HIP(launch_sumsq(v, c, part, sc + 1, stream));   // ||v||^2
    BSGD_HIP(launch_sumsq(w, c, part, sc + 2, stream));   // ||A^T A v||^2
    k_ratio<<<1, 1, 0, stream>>>(sc + 0, sc + 1, res);
    BSGD_LAUNCH_CHECK();
    k_scale_by_rsqrt<<<1024, 256, 0, stream>>>(v, w, c, sc + 2);
    BSGD_LAUNCH_CHECK();
  }
  BSGD_HIP(hipMemcpyAsync(umax, res, sizeof(float), hipMemcpyDeviceToHost, stream));
  BSGD_HIP(hipStreamSynchronize(stream));
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_lanczos_workspace_size(const bsgd_plan* plan, int steps,
                                                   size_t* bytes) {
  clear_error();
  BSGD_REQUIRE(plan && bytes, "NULL argument");
  BSGD_REQUIRE(steps >= 1 && steps <= 4096, "steps must be in [1, 4096]");
  float *v, *w, *u0, *u1;
  double *part, *sc;
  *bytes = lanczos_layout(plan, steps, nullptr, &v, &w, &u0, &u1, &part, &sc);
  return BSGD_OK;
}

// Golub-Kahan-Lanczos recurrence with the two products given as callables:
// fwd(v, out) = A v (r_int floats), bwd(u, out) = A^T u (c_int floats), both
// in the internal orders on `stream`.
template <class Fwd, class Bwd>
static bsgd_status lanczos_run(const bsgd_plan* plan, int steps, void* ws, size_t ws_bytes,
                               hipStream_t stream, float* umax, Fwd fwd, Bwd bwd) {
  float *v, *w, *u[2];
  double *part, *sc;
  const size_t need = lanczos_layout(plan, steps, ws, &v, &w, &u[0], &u[1], &part, &sc);
  if (ws_bytes < need) {
    set_error("lanczos workspace has %zu bytes, needs %zu", ws_bytes, need);
    return BSGD_ERR_WORKSPACE;
  }
  const int64_t c = plan->L.c_int, r = plan->L.r_int;
  // v_1 = ones / ||ones|| (holes of the internal order stay 0)
  BSGD_HIP(fill_pixels_one(plan->L, w, stream));
  BSGD_HIP(launch_sumsq(w, c, part, sc, stream));
  k_scale_by_rsqrt<<<1024, 256, 0, stream>>>(v, w, c, sc);
  BSGD_LAUNCH_CHECK();
  for (int j = 0; j < steps; ++j) {
    float* un = u[j & 1];
    const float* up = u[(j + 1) & 1];
    // alpha_j u_j = A v_j - beta_{j-1} u_{j-1}
    BSGD_HIP(fwd(v, un));
    if (j > 0) {
      k_sub_scaled<<<1024, 256, 0, stream>>>(un, up, r, sc + 2 * (j - 1) + 1);
      BSGD_LAUNCH_CHECK();
    }
    BSGD_HIP(launch_sumsq(un, r, part, sc + 2 * j, stream));
    k_scale_by_rsqrt<<<1024, 256, 0, stream>>>(un, un, r, sc + 2 * j);
    BSGD_LAUNCH_CHECK();
    // beta_j v_{j+1} = A^T u_j - alpha_j v_j
    BSGD_HIP(bwd(un, w));
    k_sub_scaled<<<1024, 256, 0, stream>>>(w, v, c, sc + 2 * j);
    BSGD_LAUNCH_CHECK();
    BSGD_HIP(launch_sumsq(w, c, part, sc + 2 * j + 1, stream));
    k_scale_by_rsqrt<<<1024, 256, 0, stream>>>(v, w, c, sc + 2 * j + 1);
    BSGD_LAUNCH_CHECK();
  }
  std::vector<double> h(2 * (size_t)steps);
  BSGD_HIP(hipMemcpyAsync(h.data(), sc, sizeof(double) * h.size(), hipMemcpyDeviceToHost, stream));
  BSGD_HIP(hipStreamSynchronize(stream));
  // B: diagonal alpha_j, superdiagonal beta_j; B^T B is tridiagonal with
  // diagonal alpha_j^2 + beta_{j-1}^2 and off-diagonal alpha_j beta_j
  std::vector<double> d(steps), e(std::max(steps - 1, 0));
  for (int j = 0; j < steps; ++j) {
    const double a2 = h[2 * j], b2p = j > 0 ? h[2 * (j - 1) + 1] : 0.0;
    d[j] = a2 + b2p;
    if (j + 1 < steps) e[j] = std::sqrt(a2 * h[2 * j + 1]);
  }
  for (double x : h)
    if (!std::isfinite(x)) {
      set_error("lanczos produced a non-finite value");
      return BSGD_ERR_DIVERGED;
    }
  *umax = (float)tridiag_max_eig(d, e);
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_lanczos_umax(const bsgd_plan* plan, bsgd_valtype vt, int steps,
                                         void* ws, size_t ws_bytes, hipStream_t stream,
                                         float* umax) {
  clear_error();
  BSGD_REQUIRE(plan && ws && umax, "NULL argument");
  BSGD_REQUIRE(steps >= 1 && steps <= 4096, "steps must be in [1, 4096]");
  BSGD_REQUIRE(vt == BSGD_VAL_F32 || (vt == BSGD_VAL_F16 && (plan->flags & BSGD_PLAN_F16)),
               "value type not available in this plan");
  BSGD_NEED_BWD(plan, "bsgd_lanczos_umax");
  return lanczos_run(
      plan, steps, ws, ws_bytes, stream, umax,
      [&](const float* v, float* out) {
        return launch_rows(plan->fwd, vt, kPlain, v, nullptr, nullptr, 1.0f, out, stream);
      },
      [&](const float* u, float* out) {
        return launch_rows(plan->bwd, vt, kPlain, u, nullptr, nullptr, 1.0f, out, stream);
      });
}

extern "C" bsgd_status bsgd_lanczos_workspace_size_fused(const bsgd_fused* F, int steps,
                                                         size_t* bytes) {
  clear_error();
  BSGD_REQUIRE(F && bytes, "NULL argument");
  BSGD_REQUIRE(steps >= 1 && steps <= 4096, "steps must be in [1, 4096]");
  float *v, *w, *u0, *u1;
  double *part, *sc;
  const size_t a = lanczos_layout(fused_plan(F), steps, nullptr, &v, &w, &u0, &u1, &part, &sc);
  *bytes = a + align_up(fused_partials(F, 1, nullptr, nullptr), kAlign);
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_lanczos_umax_fused(const bsgd_fused* F, bsgd_valtype vt, int steps,
                                               void* ws, size_t ws_bytes, hipStream_t stream,
                                               float* umax) {
  clear_error();
  BSGD_REQUIRE(F && ws && umax, "NULL argument");
  BSGD_REQUIRE(steps >= 1 && steps <= 4096, "steps must be in [1, 4096]");
  BSGD_REQUIRE(vt == BSGD_VAL_F32 || (vt == BSGD_VAL_F16 && fused_has_f16(F)),
               "value type not available in this store");
  const bsgd_plan* plan = fused_plan(F);
  float *v, *w, *u0, *u1;
  double *part, *sc;
  const size_t a = lanczos_layout(plan, steps, nullptr, &v, &w, &u0, &u1, &part, &sc);
  const size_t b = align_up(fused_partials(F, 1, nullptr, nullptr), kAlign);
  if (ws_bytes < a + b) {
    set_error("lanczos workspace has %zu bytes, needs %zu", ws_bytes, a + b);
    return BSGD_ERR_WORKSPACE;
  }
  FusedPartials fp;
  fused_partials(F, 1, &fp, static_cast<char*>(ws) + a);
  const int64_t r = plan->L.r_int;
  return lanczos_run(
      plan, steps, ws, a, stream, umax,
      [&](const float* x, float* out) -> hipError_t {
        // A x: the pass's row sums, then the ray half of the reduce (no y)
        hipError_t e =
            launch_fused_pass(F, vt, x, nullptr, nullptr, nullptr, fp.zp, fp.gp, stream, kPassA);
        if (e != hipSuccess) return e;
        return launch_fused_reduce(F, fp.zp, fp.gp, nullptr, out, nullptr, nullptr, 1.0f,
                                   nullptr, stream, kReduceRays);
      },
      [&](const float* u, float* out) -> hipError_t {
        // A^T u: max |u| sets the fixed-point scale of the pass's LDS sums
        hipError_t e = launch_fused_absmax(u, r, fp.rmax, stream);
        if (e != hipSuccess) return e;
        e = launch_fused_pass(F, vt, nullptr, u, fp.rmax, nullptr, fp.zp, fp.gp, stream,
                              kPassAt);
        if (e != hipSuccess) return e;
        return launch_fused_reduce(F, fp.zp, fp.gp, nullptr, nullptr, nullptr, nullptr, 1.0f,
                                   out, stream, kReducePixels);
      });
}

extern "C" bsgd_status bsgd_state_workspace_size(const bsgd_plan* plan, int nrhs, unsigned flags,
                                                 size_t* bytes) {
  clear_error();
  BSGD_REQUIRE(plan && bytes, "NULL argument");
  BSGD_REQUIRE(valid_nrhs(nrhs), "nrhs must be 1 or a power of two from 4 to 1024");
  BSGD_REQUIRE((flags & ~(BSGD_STATE_VOLUME | BSGD_STATE_BLOCK_SELECT)) == 0,
               "unknown state flags 0x%x", flags);
  BSGD_REQUIRE(!(flags & BSGD_STATE_VOLUME) || (nrhs > 1 && plan->D == 1),
               "a volume state needs nrhs > 1 slices and a 2-D plan");
  // the batch prox is the 2-D one, image by image
  BSGD_REQUIRE(nrhs == 1 || plan->D == 1, "states with several RHS need a 2-D plan (D = 1)");
  BSGD_REQUIRE(!(flags & BSGD_STATE_BLOCK_SELECT) ||
                   (nrhs == 1 && plan->M <= kMaxSelBlocks && plan->N <= kMaxSelBlocks),
               "block selection needs nrhs = 1 and at most %d row and column blocks",
               kMaxSelBlocks);
  if (flags & BSGD_STATE_BLOCK_SELECT) BSGD_NEED_BWD(plan, "a block-selection state");
  bsgd_state tmp;
  *bytes = state_layout(plan, nrhs, flags, nullptr, &tmp);
  return BSGD_OK;
}

// The second stream and the two ordering events of a state are pooled per
// device for the life of the process, like the timing events below: a job
// that creates a state per reconstruction spent hundreds of microseconds of
// host time creating a stream.  A state returns them after its stream has
// drained.
struct AuxSet {
  hipStream_t aux = nullptr;
  hipEvent_t ev_main = nullptr, ev_aux = nullptr;
};
static std::mutex g_aux_mu;
static std::vector<std::vector<AuxSet>> g_aux_pool;  // [device]

static hipError_t take_aux(bsgd_state* st) {
  int dev = 0;
  hipError_t r = hipGetDevice(&dev);
  if (r != hipSuccess) return r;
  st->aux_dev = dev;
  {
    std::lock_guard<std::mutex> lk(g_aux_mu);
    if ((int)g_aux_pool.size() > dev && !g_aux_pool[dev].empty()) {
      const AuxSet a = g_aux_pool[dev].back();
      g_aux_pool[dev].pop_back();
      st->aux = a.aux;
      st->ev_main = a.ev_main;
      st->ev_aux = a.ev_aux;
      return hipSuccess;
    }
  }
  AuxSet a;
  r = hipStreamCreateWithFlags(&a.aux, hipStreamNonBlocking);
  if (r == hipSuccess) r = hipEventCreateWithFlags(&a.ev_main, hipEventDisableTiming);
  if (r == hipSuccess) r = hipEventCreateWithFlags(&a.ev_aux, hipEventDisableTiming);
  if (r != hipSuccess) {
    if (a.ev_main) (void)hipEventDestroy(a.ev_main);
    if (a.aux) (void)hipStreamDestroy(a.aux);
    return r;
  }
  st->aux = a.aux;
  st->ev_main = a.ev_main;
  st->ev_aux = a.ev_aux;
  return hipSuccess;
}

static void give_aux(bsgd_state* st) {
  if (!st->aux) return;
  (void)hipStreamSynchronize(st->aux);
  std::lock_guard<std::mutex> lk(g_aux_mu);
  if ((int)g_aux_pool.size() <= st->aux_dev) g_aux_pool.resize(st->aux_dev + 1);
  g_aux_pool[st->aux_dev].push_back(AuxSet{st->aux, st->ev_main, st->ev_aux});
  st->aux = nullptr;
  st->ev_main = st->ev_aux = nullptr;
}

extern "C" bsgd_status bsgd_state_create(const bsgd_plan* plan, int nrhs, bsgd_valtype vt,
                                         unsigned flags, void* workspace, size_t workspace_bytes,
                                         bsgd_state** out) {
  clear_error();
  BSGD_REQUIRE(plan && workspace && out, "NULL argument");
  BSGD_REQUIRE(((uintptr_t)workspace % kAlign) == 0, "workspace must be 256-byte aligned");
  BSGD_REQUIRE(vt == BSGD_VAL_F32 || (vt == BSGD_VAL_F16 && (plan->flags & BSGD_PLAN_F16)),
               "value type not available in this plan");
  size_t need = 0;
  bsgd_status s = bsgd_state_workspace_size(plan, nrhs, flags, &need);
  if (s != BSGD_OK) return s;
  if (workspace_bytes < need) {
    set_error("state workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return BSGD_ERR_WORKSPACE;
  }
  bsgd_state* st = new bsgd_state();
  st->plan = plan;
  st->nrhs = nrhs;
  st->flags = flags;
  st->vt = vt;
  state_layout(plan, nrhs, flags, workspace, st);
  const hipError_t e = take_aux(st);
  if (e != hipSuccess) {
    set_error("state stream/event creation failed: %s", hipGetErrorString(e));
    delete st;
    return BSGD_ERR_HIP;
  }
  *out = st;
  return BSGD_OK;
}

// Timing events are pooled per device for the life of the process and
// reused by later states: a state timing every epoch of a job needs
// thousands, and creating and destroying them took milliseconds of host time
// per job.  An event handed back may still be pending; recording it again
// re-arms it.
static std::mutex g_event_mu;
static std::vector<std::vector<hipEvent_t>> g_event_pool;  // [device]

static void destroy_timers(bsgd_state* st) {
  if (!st->tev.empty()) {
    std::lock_guard<std::mutex> lk(g_event_mu);
    if ((int)g_event_pool.size() <= st->tev_dev) g_event_pool.resize(st->tev_dev + 1);
    auto& pool = g_event_pool[st->tev_dev];
    pool.insert(pool.end(), st->tev.begin(), st->tev.end());
  }
  st->tev.clear();
  st->t_cap = st->t_used = 0;
}

// Events of the epoch about to run, or NULL when it is not timed.
static hipEvent_t* next_timers(bsgd_state* st) {
  if (st->t_used >= st->t_cap) return nullptr;
  if (st->t_seen++ % st->t_stride != 0) return nullptr;
  return &st->tev[5 * (size_t)st->t_used++];
}

// n events on the current device into st->tev (pooled ones first).
static hipError_t take_timers(bsgd_state* st, size_t n) {
  int dev = 0;
  hipError_t r = hipGetDevice(&dev);
  if (r != hipSuccess) return r;
  st->tev_dev = dev;
  st->tev.reserve(n);
  {
    std::lock_guard<std::mutex> lk(g_event_mu);
    if ((int)g_event_pool.size() > dev) {
      auto& pool = g_event_pool[dev];
      while (st->tev.size() < n && !pool.empty()) {
        st->tev.push_back(pool.back());
        pool.pop_back();
      }
    }
  }
  while (st->tev.size() < n) {
    hipEvent_t e = nullptr;
    r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    st->tev.push_back(e);
  }
  return hipSuccess;
}

extern "C" void bsgd_state_destroy(bsgd_state* st) {
  if (!st) return;
  give_aux(st);
  destroy_timers(st);
  delete st;
}

extern "C" bsgd_status bsgd_state_init(bsgd_state* st, const float* y, const float* x0,
                                       hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(st && y, "NULL argument");
  const bsgd_plan* p = st->plan;
  if (x0) BSGD_NEED_FWD(p, "bsgd_state_init with x0");
  const int S = st->nrhs;
  const int64_t r = p->L.r_int * S, c = p->L.c_int * S;
  BSGD_HIP(permute_in(p->L, kRays, y, st->y, stream, S));
  st->cur = 0;
  BSGD_HIP(fill_f32(st->x[1], c, 0.0f, stream));
  BSGD_HIP(fill_f32(st->xhat, c, 0.0f, stream));
  BSGD_HIP(fill_f32(st->r[1], r, 0.0f, stream));
  BSGD_HIP(fill_f32(st->lam, S, 0.0f, stream));
  if (x0) {
    BSGD_HIP(permute_in(p->L, kPixels, x0, st->x[0], stream, S));
    if (S == 1)
      BSGD_HIP(launch_rows(p->fwd, st->vt, kResidual, st->x[0], st->y, nullptr, 1.0f, st->r[0],
                           stream));
    else
      BSGD_HIP(launch_spmm(p->fwd, st->vt, kResidual, st->x[0], st->y, nullptr, 1.0f, st->r[0],
                           S, stream));
  } else {
    BSGD_HIP(fill_f32(st->x[0], c, 0.0f, stream));
    BSGD_HIP(hipMemcpyAsync(st->r[0], st->y, sizeof(float) * r, hipMemcpyDeviceToDevice, stream));
  }
  if (st->zt) {
    if (!st->bm_built) {  // block ids and block-major copies: once per state
      BSGD_HIP(launch_block_ids(p, st->blk_r, st->blk_c, stream));
      BSGD_HIP(build_block_major(p->fwd, st->bmf, st->bm_scan, stream));
      BSGD_HIP(build_block_major(p->bwd, st->bmb, st->bm_scan, stream));
      st->bm_built = true;
    }
    if (x0)  // kept products of x0 and their residual
      BSGD_HIP(launch_sel_forward(p->fwd, st->bmf, st->vt, st->blk_r, ~0ull, ~0ull, st->x[0],
                                  st->y, st->r[0], st->r[0], st->zt, stream));
    else
      BSGD_HIP(fill_f32(st->zt, (int64_t)p->N * p->L.r_int, 0.0f, stream));
  }
  st->epochs_done = 0;
  st->initialised = true;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_state_load(bsgd_state* st, const float* x, const float* r,
                                       int64_t epoch, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(st && x && r, "NULL argument");
  BSGD_REQUIRE(st->initialised, "state_init must be called first (it sets y)");
  BSGD_REQUIRE(epoch >= 0, "epoch must be >= 0");
  const bsgd_plan* p = st->plan;
  st->cur = 0;
  BSGD_HIP(permute_in(p->L, kPixels, x, st->x[0], stream, st->nrhs));
  BSGD_HIP(permute_in(p->L, kRays, r, st->r[0], stream, st->nrhs));
  if (st->zt)  // kept products of the loaded x (their residual goes to scratch)
    BSGD_HIP(launch_sel_forward(p->fwd, st->bmf, st->vt, st->blk_r, ~0ull, ~0ull, st->x[0],
                                st->y, st->r[0], st->tmp_r, st->zt, stream));
  st->epochs_done = epoch;
  return BSGD_OK;
}

// Forward projection and residual (out = y - A x) and backprojection, gradient sum and step (out = xadd + scale A^T r)
// over the block store, in the state's launch form (staged, row kernel, or
// the several-RHS product), and the TV prox step into `out`.
static hipError_t forward_residual(const bsgd_state* st, const float* x, float* out,
                                   hipStream_t s) {
  const bsgd_plan* p = st->plan;
  const int S = st->nrhs;
  if (S == 1 && p->sfwd.lanes && st->zf)
    return launch_staged(p->sfwd, st->vt, kResidual, x, p->L.c_int, st->y, nullptr, 1.0f, out,
                         st->zf, s);
  if (S == 1) return launch_rows(p->fwd, st->vt, kResidual, x, st->y, nullptr, 1.0f, out, s);
  return launch_spmm(p->fwd, st->vt, kResidual, x, st->y, nullptr, 1.0f, out, S, s);
}

static hipError_t backward_step(const bsgd_state* st, const float* r, const float* xadd,
                                float scale, float* out, hipStream_t s) {
  const bsgd_plan* p = st->plan;
  const int S = st->nrhs;
  if (S == 1 && p->sbwd.lanes && st->zb)
    return launch_staged(p->sbwd, st->vt, kStep, r, p->L.r_int, nullptr, xadd, scale, out,
                         st->zb, s);
  if (S == 1) return launch_rows(p->bwd, st->vt, kStep, r, nullptr, xadd, scale, out, s);
  return launch_spmm(p->bwd, st->vt, kStep, r, nullptr, xadd, scale, out, S, s);
}

static hipError_t prox_step(const bsgd_state* st, float mu, float lam, bool per_rhs,
                            int prox_iters, float* out, hipStream_t s) {
  const bsgd_plan* p = st->plan;
  const int S = st->nrhs;
  if (S == 1)
    return tv_prox_run(p->L, true, st->xhat, mu * lam, prox_iters, out, st->tv_ws, s,
                       st->prox_schedule, st->prox_split);
  if (st->flags & BSGD_STATE_VOLUME)
    return tv_prox_volume(p->L, S, st->xhat, mu * lam, prox_iters, out, st->tv_ws, s,
                          st->prox_schedule, st->prox_split);
  return tv_prox_batch(p->L, S, st->xhat, mu, per_rhs ? st->lam : nullptr, lam, prox_iters, out,
                       st->tv_ws, s, st->prox_schedule, st->prox_split);
}

extern "C" bsgd_status bsgd_run_epochs(bsgd_state* st, float mu, float lam, int epochs,
                                       int prox_iters, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(st != nullptr, "state is NULL");
  BSGD_REQUIRE(st->initialised, "state_init must be called first");
  BSGD_REQUIRE(std::isfinite(mu) && mu > 0.f, "mu must be finite and > 0");
  BSGD_REQUIRE(std::isfinite(lam), "lam must be finite");
  const bool per_rhs = lam < 0.f;
  BSGD_REQUIRE(!per_rhs || (st->nrhs > 1 && !(st->flags & BSGD_STATE_VOLUME)),
               "lam < 0 (per-RHS lambdas) needs a batch state");
  BSGD_REQUIRE(epochs >= 0, "epochs must be >= 0");
  BSGD_REQUIRE(lam == 0.f || prox_iters >= 1, "prox_iters must be >= 1 when lam != 0");
  const bsgd_plan* p = st->plan;
  const int S = st->nrhs;
  // every epoch below reads A^T from the block store unless a tile-sliced
  // store serves both products (ISTA with several RHS excepted)
  if (!st->fz || (st->method == BSGD_METHOD_ISTA && S > 1))
    BSGD_NEED_BWD(p, "bsgd_run_epochs without a tile-sliced store");
  const float theta = per_rhs ? -1.f : mu * lam;  // -1: per-RHS thetas from st->lam
  for (int e = 0; e < epochs; ++e) {
    const int c = st->cur, n = 1 - c;
    hipEvent_t* tv = next_timers(st);
    // S2 (+S4) on `stream`; S1 on the aux stream after everything queued on
    // `stream` before this epoch (overlap 0) or after S2 (overlap 1), or on
    // `stream` after the prox (overlap 2: no concurrency)
    float* step_out = theta == 0.f ? st->x[n] : st->xhat;
    if (st->method == BSGD_METHOD_ISTA) {
      // r' = y - A x, then x^ = x + 2 mu A^T r' (current gradient), then
      // the TV prox step; in order on `stream`.  With a single-pass store the two
      // products are two passes over it (A x only, then A^T r' only: the
      // second needs the first's residual), each with its half of the reduce.
      if (tv) BSGD_HIP(hipEventRecord(tv[0], stream));
      if (st->fz && S == 1) {
        const FusedPartials& fp = st->fzp;
        BSGD_HIP(launch_fused_pass(st->fz, st->vt, st->x[c], nullptr, nullptr, fp.rmax + n,
                                   fp.zp, fp.gp, stream, kPassA));
        if (tv) BSGD_HIP(hipEventRecord(tv[1], stream));
        BSGD_HIP(launch_fused_reduce(st->fz, fp.zp, fp.gp, st->y, st->r[n], fp.rmax + n,
                                     nullptr, 0.f, nullptr, stream, kReduceRays));
        if (tv) BSGD_HIP(hipEventRecord(tv[2], stream));
        BSGD_HIP(launch_fused_pass(st->fz, st->vt, nullptr, st->r[n], fp.rmax + n, nullptr,
                                   fp.zp, fp.gp, stream, kPassAt));
        BSGD_HIP(launch_fused_reduce(st->fz, fp.zp, fp.gp, nullptr, nullptr, nullptr, st->x[c],
                                     2.0f * mu, step_out, stream, kReducePixels));
      } else {
        BSGD_HIP(forward_residual(st, st->x[c], st->r[n], stream));
        if (tv) BSGD_HIP(hipEventRecord(tv[1], stream));
        if (tv) BSGD_HIP(hipEventRecord(tv[2], stream));
        BSGD_HIP(backward_step(st, st->r[n], st->x[c], 2.0f * mu, step_out, stream));
      }
      if (tv) BSGD_HIP(hipEventRecord(tv[3], stream));
      if (theta != 0.f) BSGD_HIP(prox_step(st, mu, lam, per_rhs, prox_iters, st->x[n], stream));
      if (tv) BSGD_HIP(hipEventRecord(tv[4], stream));
      st->cur = n;
      st->epochs_done++;
      continue;
    }
    if (st->fz && S > 1) {
      // several RHS: the same schedule as below with the several-RHS pass and
      // reduce (per-RHS max |r| words at rmax + c * S and rmax + n * S), and
      // the batch or volume prox
      const FusedPartials& fp = st->fzp;
      const bool split = st->overlap != 2;
      if (e == 0)
        BSGD_HIP(launch_fused_absmax_mr(st->r[c], p->L.r_int, S, fp.rmax + (size_t)c * S,
                                        stream));
      if (tv) BSGD_HIP(hipEventRecord(tv[0], stream));
      BSGD_HIP(launch_fused_pass_mr(st->fz, st->vt, S, st->x[c], st->r[c],
                                    fp.rmax + (size_t)c * S, fp.zp, fp.gp, stream,
                                    st->pass_waves));
      if (tv) BSGD_HIP(hipEventRecord(tv[1], stream));
      // the next residual's maxima start from zero (after the pass read this one's)
      BSGD_HIP(launch_fused_zero(fp.rmax + (size_t)n * S, S, stream));
      if (split) {
        BSGD_HIP(hipEventRecord(st->ev_main, stream));
        BSGD_HIP(hipStreamWaitEvent(st->aux, st->ev_main, 0));
        BSGD_HIP(launch_fused_reduce_mr(st->fz, S, fp.zp, fp.gp, st->y, st->r[n],
                                        fp.rmax + (size_t)n * S, nullptr, 0.f, nullptr, st->aux,
                                        kReduceRays));
        BSGD_HIP(hipEventRecord(st->ev_aux, st->aux));
      }
      if (tv) BSGD_HIP(hipEventRecord(tv[2], stream));
      BSGD_HIP(launch_fused_reduce_mr(st->fz, S, fp.zp, fp.gp, st->y, st->r[n],
                                      fp.rmax + (size_t)n * S, st->x[c], 2.0f * mu, step_out,
                                      stream, split ? kReducePixels : kReduceAll));
      if (tv) BSGD_HIP(hipEventRecord(tv[3], stream));
      if (theta != 0.f) BSGD_HIP(prox_step(st, mu, lam, per_rhs, prox_iters, st->x[n], stream));
      if (tv) BSGD_HIP(hipEventRecord(tv[4], stream));
      if (split) BSGD_HIP(hipStreamWaitEvent(stream, st->ev_aux, 0));
      st->cur = n;
      st->epochs_done++;
      continue;
    }
    if (st->fz) {
      // single pass over the tile-sliced store (both block products together), then the
      // reduce (block sums and gradient step), then the prox (the TV prox step) on `stream`.  The ray half
      // of the reduce (the residual update: the next residual and its max |r|) is needed
      // only by the next pass, so with overlap modes 0 and 1 it runs on the
      // state's second stream, concurrently with the pixel half and the prox
      // (starting it after the pixel half, beside the prox only, measured
      // slower: the prox lost more than the pixel half gained).  max |r| of
      // the residual the pass reads: computed at the start of each call, then
      // carried by the reduce (which writes the next residual)
      const FusedPartials& fp = st->fzp;
      const bool split = st->overlap != 2;
      // with the ray half of the reduce off the critical path, the pass stores
      // its row sums in slot order (coalesced) and that half gathers them
      const bool slotz = split && fused_slot_partials(st->fz);
      if (e == 0) BSGD_HIP(launch_fused_absmax(st->r[c], p->L.r_int, fp.rmax + c, stream));
      if (tv) BSGD_HIP(hipEventRecord(tv[0], stream));
      BSGD_HIP(launch_fused_pass(st->fz, st->vt, st->x[c], st->r[c], fp.rmax + c, fp.rmax + n,
                                 fp.zp, fp.gp, stream, kPassBoth, st->pass_waves, slotz));
      if (tv) BSGD_HIP(hipEventRecord(tv[1], stream));
      if (split) {
        BSGD_HIP(hipEventRecord(st->ev_main, stream));
        BSGD_HIP(hipStreamWaitEvent(st->aux, st->ev_main, 0));
        BSGD_HIP(launch_fused_reduce(st->fz, fp.zp, fp.gp, st->y, st->r[n], fp.rmax + n,
                                     nullptr, 0.f, nullptr, st->aux, kReduceRays, slotz));
        BSGD_HIP(hipEventRecord(st->ev_aux, st->aux));
      }
      if (tv) BSGD_HIP(hipEventRecord(tv[2], stream));
      BSGD_HIP(launch_fused_reduce(st->fz, fp.zp, fp.gp, st->y, st->r[n], fp.rmax + n, st->x[c],
                                   2.0f * mu, step_out, stream,
                                   split ? kReducePixels : kReduceAll));
      if (tv) BSGD_HIP(hipEventRecord(tv[3], stream));
      if (theta != 0.f)
        BSGD_HIP(tv_prox_run(p->L, true, st->xhat, theta, prox_iters, st->x[n], st->tv_ws,
                             stream, st->prox_schedule, st->prox_split));
      if (tv) BSGD_HIP(hipEventRecord(tv[4], stream));
      if (split) BSGD_HIP(hipStreamWaitEvent(stream, st->ev_aux, 0));
      st->cur = n;
      st->epochs_done++;
      continue;
    }
    if (st->overlap == 0) BSGD_HIP(hipEventRecord(st->ev_main, stream));
    if (tv) BSGD_HIP(hipEventRecord(tv[2], stream));
    BSGD_HIP(backward_step(st, st->r[c], st->x[c], 2.0f * mu, step_out, stream));
    if (tv) BSGD_HIP(hipEventRecord(tv[3], stream));
    if (st->overlap == 1) BSGD_HIP(hipEventRecord(st->ev_main, stream));
    hipStream_t fs = st->overlap == 2 ? stream : st->aux;
    auto forward = [&]() -> bsgd_status {
      if (tv) BSGD_HIP(hipEventRecord(tv[0], fs));
      BSGD_HIP(forward_residual(st, st->x[c], st->r[n], fs));
      if (tv) BSGD_HIP(hipEventRecord(tv[1], fs));
      return BSGD_OK;
    };
    if (st->overlap != 2) {
      BSGD_HIP(hipStreamWaitEvent(st->aux, st->ev_main, 0));
      bsgd_status fst = forward();
      if (fst != BSGD_OK) return fst;
      BSGD_HIP(hipEventRecord(st->ev_aux, st->aux));
    }
    // S5 on `stream`
    if (theta != 0.f) BSGD_HIP(prox_step(st, mu, lam, per_rhs, prox_iters, st->x[n], stream));
    if (tv) BSGD_HIP(hipEventRecord(tv[4], stream));
    if (st->overlap == 2) {
      bsgd_status fst = forward();
      if (fst != BSGD_OK) return fst;
    } else {
      BSGD_HIP(hipStreamWaitEvent(stream, st->ev_aux, 0));
    }
    st->cur = n;
    st->epochs_done++;
  }
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_get_x(const bsgd_state* st, float* x, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(st && x, "NULL argument");
  BSGD_HIP(permute_out(st->plan->L, kPixels, st->x[st->cur], x, stream, st->nrhs));
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_get_r(const bsgd_state* st, float* r, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(st && r, "NULL argument");
  BSGD_HIP(permute_out(st->plan->L, kRays, st->r[st->cur], r, stream, st->nrhs));
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_get_stats(const bsgd_state* st, hipStream_t stream, double* res_norm2,
                                      int64_t* epochs_done) {
  clear_error();
  BSGD_REQUIRE(st && res_norm2 && epochs_done, "NULL argument");
  BSGD_HIP(launch_sumsq(st->r[st->cur], st->plan->L.r_int * st->nrhs, st->partial,
                        st->partial + kReduceBlocks, stream));
  BSGD_HIP(hipMemcpyAsync(res_norm2, st->partial + kReduceBlocks, sizeof(double),
                          hipMemcpyDeviceToHost, stream));
  BSGD_HIP(hipStreamSynchronize(stream));
  *epochs_done = st->epochs_done;
  if (!std::isfinite(*res_norm2)) {
    set_error("residual norm is not finite after %lld epochs", (long long)st->epochs_done);
    return BSGD_ERR_DIVERGED;
  }
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_state_enable_timing(bsgd_state* st, int max_epochs) {
  return bsgd_state_enable_timing_sampled(st, max_epochs, 1);
}

extern "C" bsgd_status bsgd_state_enable_timing_sampled(bsgd_state* st, int max_epochs,
                                                        int stride) {
  clear_error();
  BSGD_REQUIRE(st != nullptr, "state is NULL");
  BSGD_REQUIRE(max_epochs >= 0, "max_epochs must be >= 0");
  BSGD_REQUIRE(stride >= 1, "stride must be >= 1");
  destroy_timers(st);
  hipError_t r = take_timers(st, 5 * (size_t)max_epochs);
  if (r != hipSuccess) {
    destroy_timers(st);
    set_error("timer event creation failed: %s", hipGetErrorString(r));
    return BSGD_ERR_HIP;
  }
  st->t_cap = max_epochs;
  st->t_used = 0;
  st->t_stride = stride;
  st->t_seen = 0;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_state_timing(bsgd_state* st, double* fwd_ms, double* bwd_ms,
                                         double* prox_ms, int64_t* epochs_timed) {
  clear_error();
  BSGD_REQUIRE(st && fwd_ms && bwd_ms && prox_ms && epochs_timed, "NULL argument");
  double f = 0, b = 0, x = 0;
  for (int k = 0; k < st->t_used; ++k) {
    hipEvent_t* e = &st->tev[5 * (size_t)k];
    BSGD_HIP(hipEventSynchronize(e[4]));
    BSGD_HIP(hipEventSynchronize(e[1]));
    float ms = 0.f;
    BSGD_HIP(hipEventElapsedTime(&ms, e[0], e[1]));
    f += ms;
    BSGD_HIP(hipEventElapsedTime(&ms, e[2], e[3]));
    b += ms;
    BSGD_HIP(hipEventElapsedTime(&ms, e[3], e[4]));
    x += ms;
  }
  *fwd_ms = f;
  *bwd_ms = b;
  *prox_ms = x;
  *epochs_timed = st->t_used;
  st->t_used = 0;
  st->t_seen = 0;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_state_set_overlap(bsgd_state* st, int mode) {
  clear_error();
  BSGD_REQUIRE(st != nullptr, "state is NULL");
  BSGD_REQUIRE(mode >= 0 && mode <= 2, "overlap mode must be 0, 1 or 2");
  st->overlap = mode;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_state_set_method(bsgd_state* st, int method) {
  clear_error();
  BSGD_REQUIRE(st != nullptr, "state is NULL");
  BSGD_REQUIRE(method == BSGD_METHOD_BSGD || method == BSGD_METHOD_ISTA,
               "method must be BSGD_METHOD_BSGD (0) or BSGD_METHOD_ISTA (1)");
  st->method = method;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_run_selected(bsgd_state* st, float mu, float lam, int iters,
                                         int prox_iters, const uint64_t* rows_sel,
                                         const uint64_t* cols_sel, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(st != nullptr, "state is NULL");
  BSGD_REQUIRE(st->initialised, "state_init must be called first");
  BSGD_REQUIRE(st->zt != nullptr, "the state was created without BSGD_STATE_BLOCK_SELECT");
  BSGD_REQUIRE(std::isfinite(mu) && mu > 0.f, "mu must be finite and > 0");
  BSGD_REQUIRE(std::isfinite(lam) && lam >= 0.f, "lam must be finite and >= 0");
  BSGD_REQUIRE(iters >= 0, "iters must be >= 0");
  BSGD_REQUIRE(lam == 0.f || prox_iters >= 1, "prox_iters must be >= 1 when lam != 0");
  BSGD_REQUIRE(iters == 0 || (rows_sel && cols_sel), "NULL block masks");
  const bsgd_plan* p = st->plan;
  const uint64_t row_bits = p->M == 64 ? ~0ull : ((1ull << p->M) - 1);
  const uint64_t col_bits = p->N == 64 ? ~0ull : ((1ull << p->N) - 1);
  for (int t = 0; t < iters; ++t) {
    BSGD_REQUIRE(rows_sel[t] != 0 && (rows_sel[t] & ~row_bits) == 0,
                 "rows_sel[%d] = 0x%llx: needs a non-empty subset of the %d row blocks", t,
                 (unsigned long long)rows_sel[t], p->M);
    BSGD_REQUIRE(cols_sel[t] != 0 && (cols_sel[t] & ~col_bits) == 0,
                 "cols_sel[%d] = 0x%llx: needs a non-empty subset of the %d column blocks", t,
                 (unsigned long long)cols_sel[t], p->N);
  }
  const float theta = mu * lam;
  for (int t = 0; t < iters; ++t) {
    const int c = st->cur, n = 1 - c;
    float* step_out = theta == 0.f ? st->x[n] : st->xhat;
    hipEvent_t* tv = next_timers(st);
    // forward projection and residual with the current x; backprojection, gradient sum and step with the kept residual
    if (tv) BSGD_HIP(hipEventRecord(tv[0], stream));
    BSGD_HIP(launch_sel_forward(p->fwd, st->bmf, st->vt, st->blk_r, rows_sel[t], cols_sel[t],
                                st->x[c], st->y, st->r[c], st->r[n], st->zt, stream));
    if (tv) BSGD_HIP(hipEventRecord(tv[1], stream));
    if (tv) BSGD_HIP(hipEventRecord(tv[2], stream));
    BSGD_HIP(launch_sel_backward(p->bwd, st->bmb, st->vt, st->blk_c, rows_sel[t], cols_sel[t],
                                 st->r[c], st->x[c], 2.0f * mu, step_out, stream));
    if (tv) BSGD_HIP(hipEventRecord(tv[3], stream));
    if (theta != 0.f) BSGD_HIP(prox_step(st, mu, lam, false, prox_iters, st->x[n], stream));
    if (tv) BSGD_HIP(hipEventRecord(tv[4], stream));
    st->cur = n;
    st->epochs_done++;
  }
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_state_attach_fused(bsgd_state* st, const bsgd_fused* fused,
                                               void* partials, size_t partials_bytes) {
  clear_error();
  BSGD_REQUIRE(st != nullptr, "state is NULL");
  if (!fused) {
    st->fz = nullptr;
    st->fzp = FusedPartials();
    return BSGD_OK;
  }
  BSGD_REQUIRE(partials != nullptr, "partials is NULL");
  BSGD_REQUIRE(fused_plan(fused) == st->plan, "the store belongs to another plan");
  BSGD_REQUIRE(st->nrhs == 1 || st->nrhs % 4 == 0,
               "single-pass epochs need one RHS or a multiple of 4");
  BSGD_REQUIRE(!(st->flags & BSGD_STATE_BLOCK_SELECT) || st->nrhs == 1,
               "block-select states use the block store");
  BSGD_REQUIRE(st->vt == BSGD_VAL_F32 || fused_has_f16(fused),
               "the store has no FP16 values (plan without BSGD_PLAN_F16)");
  FusedPartials fp;
  const size_t need = fused_partials(fused, st->nrhs, &fp, partials);
  if (partials_bytes < need) {
    set_error("partials workspace has %zu bytes, needs %zu", partials_bytes, need);
    return BSGD_ERR_WORKSPACE;
  }
  st->fz = fused;
  st->fzp = fp;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_state_set_launch(bsgd_state* st, int pass_waves, int prox_split) {
  clear_error();
  BSGD_REQUIRE(st != nullptr, "state is NULL");
  BSGD_REQUIRE(pass_waves == 0 || pass_waves == 2 || pass_waves == 4 || pass_waves == 8 ||
                   pass_waves == 16,
               "pass_waves must be 0, 2, 4, 8 or 16");
  BSGD_REQUIRE(pass_waves != 16 || st->nrhs > 1, "16 wavefronts: several-RHS passes only");
  BSGD_REQUIRE(st->nrhs == 1 || pass_waves == 0 || pass_waves >= 8,
               "several-RHS passes run 8 or 16 wavefronts");
  BSGD_REQUIRE(prox_split >= 0, "prox_split must be >= 0");
  st->pass_waves = pass_waves;
  st->prox_split = prox_split;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_state_launch(const bsgd_state* st, int* pass_waves, int* prox_split) {
  clear_error();
  BSGD_REQUIRE(st && pass_waves && prox_split, "NULL argument");
  *pass_waves = st->pass_waves;
  *prox_split = st->prox_split;
  return BSGD_OK;
}

// Time `reps` epochs (after one untimed) of the state on zero data; seconds.
static bsgd_status time_epochs(bsgd_state* st, float mu, float lam, int prox_iters, int reps,
                               hipStream_t stream, hipEvent_t e0, hipEvent_t e1, double* ms) {
  bsgd_status r = bsgd_run_epochs(st, mu, lam, 1, prox_iters, stream);
  if (r != BSGD_OK) return r;
  BSGD_HIP(hipEventRecord(e0, stream));
  r = bsgd_run_epochs(st, mu, lam, reps, prox_iters, stream);
  if (r != BSGD_OK) return r;
  BSGD_HIP(hipEventRecord(e1, stream));
  BSGD_HIP(hipEventSynchronize(e1));
  float t = 0.f;
  BSGD_HIP(hipEventElapsedTime(&t, e0, e1));
  *ms = t;
  return BSGD_OK;
}

static bsgd_status zero_state(bsgd_state* st, hipStream_t stream) {
  const bsgd_plan* p = st->plan;
  const size_t rb = sizeof(float) * p->L.r_int * st->nrhs, cb = sizeof(float) * p->L.c_int * st->nrhs;
  BSGD_HIP(hipMemsetAsync(st->y, 0, rb, stream));
  BSGD_HIP(hipMemsetAsync(st->r[0], 0, rb, stream));
  BSGD_HIP(hipMemsetAsync(st->r[1], 0, rb, stream));
  BSGD_HIP(hipMemsetAsync(st->x[0], 0, cb, stream));
  BSGD_HIP(hipMemsetAsync(st->x[1], 0, cb, stream));
  BSGD_HIP(hipMemsetAsync(st->lam, 0, sizeof(float) * st->nrhs, stream));
  st->cur = 0;
  st->epochs_done = 0;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_state_autotune(bsgd_state* st, float mu, float lam, int prox_iters,
                                           int reps, hipStream_t stream, int* choice) {
  clear_error();
  BSGD_REQUIRE(st != nullptr, "state is NULL");
  BSGD_REQUIRE(!st->initialised, "autotune runs before bsgd_state_init (it overwrites the state)");
  BSGD_REQUIRE(std::isfinite(mu) && mu > 0.f, "mu must be finite and > 0");
  BSGD_REQUIRE(std::isfinite(lam) && lam >= 0.f, "lam must be finite and >= 0");
  BSGD_REQUIRE(lam == 0.f || prox_iters >= 1, "prox_iters must be >= 1 when lam != 0");
  BSGD_REQUIRE(reps >= 1 && reps <= 1000, "reps must be in [1, 1000]");
  bsgd_status r = zero_state(st, stream);
  if (r != BSGD_OK) return r;
  st->initialised = true;
  const int t_cap = st->t_cap;
  st->t_cap = 0;  // no kernel timers while tuning
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto done = [&](bsgd_status s) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    st->t_cap = t_cap;
    st->initialised = false;
    const bsgd_status z = zero_state(st, stream);
    (void)hipStreamSynchronize(stream);
    return s != BSGD_OK ? s : z;
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("event creation failed");
    return done(BSGD_ERR_HIP);
  }
  const bool volume = (st->flags & BSGD_STATE_VOLUME) != 0;
  // the pass: wavefronts per workgroup (one RHS: the store's 4 or 8; several: 8 or 16)
  int best_w = 0;
  if (st->fz && st->method == BSGD_METHOD_BSGD) {
    const int one[2] = {4, 8}, many[2] = {8, 16};
    const int* cand = st->nrhs == 1 ? one : many;
    double best = 1e300;
    for (int i = 0; i < 2; ++i) {
      st->pass_waves = cand[i];
      double ms = 0.0;
      r = time_epochs(st, mu, 0.f, 0, reps, stream, e0, e1, &ms);
      if (r != BSGD_OK) return done(r);
      if (ms < best) {
        best = ms;
        best_w = cand[i];
      }
    }
  }
  st->pass_waves = best_w;
  // the prox: most FGP iterations per launch (2-D: 5, 7 or 10; volumes: 1, 2 or 3)
  int best_s = 0;
  if (lam > 0.f && st->prox_schedule != kFgpPerIteration) {
    const int two[3] = {5, 7, 10}, three[3] = {1, 2, 3};
    const int* cand = volume ? three : two;
    const int nc = 3;
    double best = 1e300;
    for (int i = 0; i < nc; ++i) {
      st->prox_split = cand[i];
      double ms = 0.0;
      r = time_epochs(st, mu, lam, prox_iters, reps, stream, e0, e1, &ms);
      if (r != BSGD_OK) return done(r);
      if (ms < best) {
        best = ms;
        best_s = cand[i];
      }
    }
  }
  st->prox_split = best_s;
  if (choice) {
    choice[0] = best_w;
    choice[1] = best_s;
  }
  return done(BSGD_OK);
}

extern "C" bsgd_status bsgd_state_set_prox_schedule(bsgd_state* st, int schedule) {
  clear_error();
  BSGD_REQUIRE(st != nullptr, "state is NULL");
  BSGD_REQUIRE(schedule == kFgpFused || schedule == kFgpPerIteration ||
                   schedule == kFgpFusedLds,
               "prox schedule must be 0, 1 or 2");
  st->prox_schedule = schedule;
  return BSGD_OK;
}

// ---------------------------------------------------------------------------
// Batches of independent reconstructions: per-slot set-up, lambdas, results
// ---------------------------------------------------------------------------
extern "C" bsgd_status bsgd_state_set_rhs(bsgd_state* st, int k, const float* y, const float* x0,
                                          hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(st != nullptr, "state is NULL");
  BSGD_REQUIRE(st->initialised, "state_init must be called first");
  BSGD_REQUIRE(k >= 0 && k < st->nrhs, "slot %d out of range", k);
  const bsgd_plan* p = st->plan;
  if (y && x0) BSGD_NEED_FWD(p, "bsgd_state_set_rhs with x0");
  const Layout& L = p->L;
  const int S = st->nrhs, c = st->cur;
  // y == NULL empties the slot (all its vectors zero: it stays zero)
  BSGD_HIP(scatter_column(L, kRays, y, st->y, S, k, stream));
  BSGD_HIP(scatter_column(L, kPixels, x0, st->x[c], S, k, stream));
  BSGD_HIP(scatter_column(L, kPixels, nullptr, st->x[1 - c], S, k, stream));
  BSGD_HIP(scatter_column(L, kPixels, nullptr, st->xhat, S, k, stream));
  BSGD_HIP(scatter_column(L, kRays, nullptr, st->r[1 - c], S, k, stream));
  if (y && x0) {
    // r = y - A x0 for this slot only (one-RHS product in internal order,
    // in place over the permuted y, then into the slot's column)
    BSGD_HIP(permute_in(L, kPixels, x0, st->tmp_c, stream));
    BSGD_HIP(permute_in(L, kRays, y, st->tmp_r, stream));
    BSGD_HIP(launch_rows(p->fwd, st->vt, kResidual, st->tmp_c, st->tmp_r, nullptr, 1.0f,
                         st->tmp_r, stream));
    BSGD_HIP(set_column(st->tmp_r, st->r[c], L.r_int, S, k, stream));
  } else {
    BSGD_HIP(scatter_column(L, kRays, y, st->r[c], S, k, stream));
  }
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_state_set_lambda(bsgd_state* st, const float* lam, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(st && lam, "NULL argument");
  for (int j = 0; j < st->nrhs; ++j)
    BSGD_REQUIRE(std::isfinite(lam[j]) && lam[j] >= 0.f, "lam[%d] must be finite and >= 0", j);
  BSGD_HIP(hipMemcpyAsync(st->lam, lam, sizeof(float) * st->nrhs, hipMemcpyHostToDevice, stream));
  BSGD_HIP(hipStreamSynchronize(stream));
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_get_x_rhs(const bsgd_state* st, int k, float* x, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(st && x, "NULL argument");
  BSGD_REQUIRE(k >= 0 && k < st->nrhs, "slot %d out of range", k);
  BSGD_HIP(gather_column(st->plan->L, kPixels, st->x[st->cur], x, st->nrhs, k, stream));
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_get_stats_rhs(const bsgd_state* st, hipStream_t stream,
                                          double* res_norm2) {
  clear_error();
  BSGD_REQUIRE(st && res_norm2, "NULL argument");
  const int S = st->nrhs;
  double* out = st->partial + (size_t)kColBlocks * S;
  BSGD_HIP(launch_colsumsq(st->r[st->cur], st->plan->L.r_int, S, st->partial, out, stream));
  BSGD_HIP(hipMemcpyAsync(res_norm2, out, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
  BSGD_HIP(hipStreamSynchronize(stream));
  for (int j = 0; j < S; ++j)
    if (!std::isfinite(res_norm2[j])) {
      set_error("residual norm of slot %d is not finite", j);
      return BSGD_ERR_DIVERGED;
    }
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_get_res_change_rhs(const bsgd_state* st, hipStream_t stream,
                                               double* now, double* prev) {
  clear_error();
  BSGD_REQUIRE(st && now && prev, "NULL argument");
  const int S = st->nrhs;
  double* out = st->partial + (size_t)kColBlocks * S;
  // stream order keeps each copy ahead of the next reduction into `out`
  BSGD_HIP(launch_colsumsq(st->r[st->cur], st->plan->L.r_int, S, st->partial, out, stream));
  BSGD_HIP(hipMemcpyAsync(now, out, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
  BSGD_HIP(launch_colsumsq(st->r[1 - st->cur], st->plan->L.r_int, S, st->partial, out, stream));
  BSGD_HIP(hipMemcpyAsync(prev, out, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
  BSGD_HIP(hipStreamSynchronize(stream));
  for (int j = 0; j < S; ++j)
    if (!std::isfinite(now[j]) || !std::isfinite(prev[j])) {
      set_error("residual norm of slot %d is not finite", j);
      return BSGD_ERR_DIVERGED;
    }
  return BSGD_OK;
}

// ---------------------------------------------------------------------------
// HIP graph of a fixed number of epochs
// ---------------------------------------------------------------------------
// What a captured graph has baked into its kernels' arguments: the iterate
// and residual buffers of the state's current parity, the attached
// single-pass store and its partial sums, the update rule and the kernel
// choices of the epoch schedule.  A replay is valid only while all of them
// are unchanged.
struct GraphKey {
  int cur = 0, method = 0, overlap = 0, schedule = 0, pass_waves = 0, prox_split = 0;
  const bsgd_fused* fz = nullptr;
  const float* zp = nullptr;
  const float* gp = nullptr;
  const unsigned* rmax = nullptr;
  int lanes_fwd = 0, lanes_bwd = 0, staged_fwd = 0, staged_bwd = 0;
  bool operator==(const GraphKey& o) const {
    return cur == o.cur && method == o.method && overlap == o.overlap &&
           schedule == o.schedule && pass_waves == o.pass_waves &&
           prox_split == o.prox_split && fz == o.fz && zp == o.zp && gp == o.gp && rmax == o.rmax &&
           lanes_fwd == o.lanes_fwd && lanes_bwd == o.lanes_bwd && staged_fwd == o.staged_fwd &&
           staged_bwd == o.staged_bwd;
  }
};

static GraphKey graph_key(const bsgd_state* st) {
  GraphKey k;
  k.cur = st->cur;
  k.method = st->method;
  k.overlap = st->overlap;
  k.schedule = st->prox_schedule;
  k.pass_waves = st->pass_waves;
  k.prox_split = st->prox_split;
  k.fz = st->fz;
  k.zp = st->fzp.zp;
  k.gp = st->fzp.gp;
  k.rmax = st->fzp.rmax;
  k.lanes_fwd = st->plan->fwd.lanes_per_row;
  k.lanes_bwd = st->plan->bwd.lanes_per_row;
  k.staged_fwd = st->plan->sfwd.lanes;
  k.staged_bwd = st->plan->sbwd.lanes;
  return k;
}

struct bsgd_graph {
  bsgd_state* st = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int epochs = 0;
  GraphKey key;  // the state's configuration at capture
};

extern "C" bsgd_status bsgd_graph_create(bsgd_state* st, float mu, float lam, int epochs,
                                         int prox_iters, hipStream_t stream, bsgd_graph** out) {
  clear_error();
  BSGD_REQUIRE(st && out, "NULL argument");
  BSGD_REQUIRE(epochs >= 2 && epochs % 2 == 0,
               "a graph holds an even number of epochs (the iterate buffers alternate)");
  BSGD_REQUIRE(stream != nullptr, "capture needs a non-default stream");
  const int t_cap = st->t_cap, t_used = st->t_used;
  st->t_cap = 0;  // no timing events inside the graph
  const int64_t done = st->epochs_done;
  const int cur = st->cur;
  const GraphKey key = graph_key(st);
  BSGD_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  bsgd_status s = bsgd_run_epochs(st, mu, lam, epochs, prox_iters, stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(stream, &g);
  st->t_cap = t_cap;
  st->t_used = t_used;
  st->epochs_done = done;
  st->cur = cur;
  if (s != BSGD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) {
    set_error("graph capture failed: %s", hipGetErrorString(e));
    return BSGD_ERR_HIP;
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    set_error("graph instantiation failed: %s", hipGetErrorString(e));
    return BSGD_ERR_HIP;
  }
  bsgd_graph* gr = new bsgd_graph();
  gr->st = st;
  gr->graph = g;
  gr->exec = ex;
  gr->epochs = epochs;
  gr->key = key;
  *out = gr;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_graph_launch(bsgd_graph* gr, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(gr != nullptr, "graph is NULL");
  const GraphKey now = graph_key(gr->st);
  BSGD_REQUIRE(now.cur == gr->key.cur,
               "the state's iterate buffers changed parity since capture (an odd number of "
               "epochs ran outside the graph); recapture");
  BSGD_REQUIRE(now == gr->key,
               "the state's configuration (single-pass store, partials, update rule, epoch "
               "schedule or kernel choice) changed since capture; recapture");
  BSGD_HIP(hipGraphLaunch(gr->exec, stream));
  gr->st->epochs_done += gr->epochs;
  return BSGD_OK;
}

extern "C" void bsgd_graph_destroy(bsgd_graph* gr) {
  if (!gr) return;
  if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
  if (gr->graph) (void)hipGraphDestroy(gr->graph);
  delete gr;
}

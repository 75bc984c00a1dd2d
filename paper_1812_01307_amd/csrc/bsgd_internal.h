// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <vector>

#include "bsgd.h"

namespace bsgd {

// Every stored row (of A and of A^T) is padded with zero-valued entries to a
// multiple of kPad entries, so that 16-byte vector loads of columns and
// values are aligned and never straddle two rows.
constexpr int kPad = 8;
constexpr size_t kAlign = 256;
constexpr int kViewTile = 8;  // views interleaved in the internal ray order
constexpr int kPixTile = 8;   // 8 x 8 pixel tiles in the internal pixel order

void set_error(const char* fmt, ...);
void clear_error();

#define BSGD_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::bsgd::set_error("%s failed: %s", #call, hipGetErrorString(e_));                \
      return BSGD_ERR_HIP;                                                             \
    }                                                                                  \
  } while (0)

#define BSGD_REQUIRE(cond, ...)                                                        \
  do {                                                                                 \
    if (!(cond)) {                                                                     \
      ::bsgd::set_error(__VA_ARGS__);                                                  \
      return BSGD_ERR_INVALID;                                                         \
    }                                                                                  \
  } while (0)

// The call needs the block store of A, which a BSGD_PLAN_SINGLE_PASS_ONLY plan
// lacks.
#define BSGD_NEED_FWD(plan, what)                                                      \
  do {                                                                                 \
    if ((plan)->flags & BSGD_PLAN_SINGLE_PASS_ONLY) {                                  \
      ::bsgd::set_error("%s needs the block store of A (a SINGLE_PASS_ONLY plan)", what); \
      return BSGD_ERR_UNSUPPORTED;                                                     \
    }                                                                                  \
  } while (0)

// The call needs the block store of A^T, which a BSGD_PLAN_FWD_ONLY plan lacks.
#define BSGD_NEED_BWD(plan, what)                                                      \
  do {                                                                                 \
    if ((plan)->flags & BSGD_PLAN_FWD_ONLY) {                                          \
      ::bsgd::set_error("%s needs the A^T block store (a FWD_ONLY plan)", what);     \
      return BSGD_ERR_UNSUPPORTED;                                                     \
    }                                                                                  \
  } while (0)

#define BSGD_LAUNCH_CHECK()                                                            \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess) {                                                            \
      ::bsgd::set_error("kernel launch failed: %s", hipGetErrorString(e_));            \
      return BSGD_ERR_HIP;                                                             \
    }                                                                                  \
  } while (0)

inline size_t align_up(size_t n, size_t a) { return (n + a - 1) / a * a; }

// Hands out aligned sub-buffers of a caller workspace.  With base == nullptr it
// only measures.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, kAlign);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Internal vector orders.  The sparse products gather x (by pixel) and r (by
// ray); in the natural orders a steep ray touches a new cache line per pixel
// and a pixel's rays are one view (view_len floats) apart.  Internally:
//   pixels: 8 x 8 tiles of each slice, row-major inside a tile
//           (a ray crossing a tile reads one 256-byte block);
//   rays:   groups of kViewTile consecutive views interleaved bin by bin
//           (the rays through one pixel over 8 views lie within a few lines).
// Internal vectors have holes (ragged tiles / a last partial view group);
// holes hold 0 and no stored entry refers to them.
struct Layout {
  int64_t nrows = 0, nviews = 0, view_len = 0, r_int = 0;
  int H = 1, W = 1, D = 1, Ht = 1, Wt = 1;
  int64_t c_int = 0;

  __host__ __device__ int64_t ray_in(int64_t rho) const {
    if (view_len == 0) return rho;
    const int64_t a = rho / view_len, b = rho - a * view_len;
    return (a / kViewTile) * (kViewTile * view_len) + b * kViewTile + (a % kViewTile);
  }
  __host__ __device__ int64_t ray_out(int64_t k) const {  // -1 for a hole
    if (view_len == 0) return k < nrows ? k : -1;
    const int64_t g = k / (kViewTile * view_len), rem = k - g * (kViewTile * view_len);
    const int64_t a = g * kViewTile + rem % kViewTile, b = rem / kViewTile;
    return a < nviews ? a * view_len + b : -1;
  }
  __host__ __device__ int64_t pix_st(int d, int s, int t) const {
    return (int64_t)d * ((int64_t)Ht * Wt * 64) + ((int64_t)((s >> 3) * Wt + (t >> 3)) << 6) +
           ((s & 7) << 3) + (t & 7);
  }
  __host__ __device__ int64_t pix_in(int64_t p) const {
    const int64_t hw = (int64_t)H * W;
    const int d = (int)(p / hw);
    const int64_t rem = p - d * hw;
    const int s = (int)(rem / W), t = (int)(rem - (int64_t)s * W);
    return pix_st(d, s, t);
  }
  __host__ __device__ int64_t pix_out(int64_t k) const {  // -1 for a hole
    const int64_t sl = (int64_t)Ht * Wt * 64;
    const int d = (int)(k / sl);
    const int64_t rem = k - d * sl;
    const int tile = (int)(rem >> 6), w = (int)(rem & 63);
    const int s = (tile / Wt) * 8 + (w >> 3), t = (tile % Wt) * 8 + (w & 7);
    return (s < H && t < W) ? (int64_t)d * H * W + (int64_t)s * W + t : -1;
  }
};

Layout make_layout(int64_t nrows, int64_t view_len, int H, int W, int D);

// One direction of the block store: rows of A (rays, segments = column
// blocks) or rows of A^T (pixels, segments = row blocks), rows in internal
// order.  Row `row` holds its entries in [ptr[row], ptr[row] + seg[row*(nseg+1)
// + nseg]) followed by zero padding up to ptr[row+1]; segment k is the
// relative range [seg[.. + k], seg[.. + k + 1]) and holds the entries whose
// natural column lies in [seg_off[k], seg_off[k+1]).  Entries keep the
// natural column order; their stored indices are internal (pixel or ray)
// indices.
struct Store {
  int64_t nrows = 0, ncols = 0, nnz = 0, cap = 0;
  int nseg = 0;
  int64_t* ptr = nullptr;
  int32_t* seg = nullptr;
  int32_t* col = nullptr;
  float* val = nullptr;
  __half* val16 = nullptr;
  std::vector<int64_t> seg_off;   // host copy, nseg + 1 entries
  int lanes_per_row = 8;          // launch choice for the fused row kernels
  bool nontemporal = false;       // non-temporal loads of the matrix streams
};

// Staged form of one direction (optional, BSGD_PLAN_STAGED).  The internal
// column space is cut into P stages of SW columns; rows (internal order) are
// grouped into chunks of RW.  For chunk w and stage s the rows' entries whose
// column lies in the stage are stored back to back (row by row, each row's
// segment padded with zero entries to a multiple of kStageVec), with 16-bit
// stage-local column indices:
//   wbase[w]                    int64, first entry of chunk w;
//   segp[(w*P + s)*(RW+1) + k]  int32, offset (from wbase[w]) of row k's
//                               segment for stage s; k = RW gives the end;
//   col[e] uint16, val[e] FP32 (optional FP16 copy).
// A product runs one workgroup per (chunk, stage): the stage's slice of the
// vector is copied to LDS once and every gather is an LDS read; the per-stage
// row sums go to a partial buffer that a second pass adds in stage order.
constexpr int kStageVec = 8;
constexpr int kStageRows = 2048;
constexpr int kStageSmall = 19456;  // LDS floats: two workgroups per CU
constexpr int kStageLarge = 32768;  // LDS floats: one workgroup per CU
struct Staged {
  bool built = false;
  int lanes = 0;        // 0: the epoch uses the row kernel; 4 or 8: staged, lanes per row
  int SW = 0, P = 0, RW = kStageRows;
  int64_t nW = 0, nrows = 0, cap = 0, total = 0;
  int64_t* wbase = nullptr;
  int32_t* segp = nullptr;
  uint16_t* col = nullptr;
  float* val = nullptr;
  __half* val16 = nullptr;
  std::vector<int64_t> bnd;  // P + 1 natural column bounds of the stages
};

}  // namespace bsgd

// Result of the single-pass store's segment count pass for one chunk count
// and column width; while valid, scratch64 holds the rays' segment offsets
// it produced (every other writer of scratch64 clears it).
struct FusedCountCache {
  bool valid = false;
  int Q = 0;
  bool wide = false;
  bool narrow = true;
  int64_t pairs = 0, slices = 0, bound = 0;
  int maxrank = 0, maxlen = 0, maxstep = 0;
};

struct bsgd_plan {
  int M = 0, N = 0, H = 0, W = 0, D = 0;
  unsigned flags = 0;
  bsgd::Layout L;
  bsgd::Store fwd;   // A   (rows: internal ray order; columns: internal pixel indices)
  bsgd::Store bwd;   // A^T (rows: internal pixel order; columns: internal ray indices)
  bsgd::Staged sfwd, sbwd;        // staged forms (BSGD_PLAN_STAGED)
  int64_t* stage_cnt = nullptr;   // segment counts / offsets while building
  float* stage_z = nullptr;       // stage partials for the autotuner
  std::vector<int64_t> row_off, col_off;
  int64_t* scratch64 = nullptr;   // max(r_int, c_int) + 1 entries (build, export)
  mutable FusedCountCache fz_count;  // lets bsgd_fused_create reuse the count of
                                     // bsgd_fused_workspace_size
  int64_t* scan_tmp = nullptr;    // block sums for scans
  int* err = nullptr;             // validation flags
  unsigned long long* colmax = nullptr;  // 2 words: column-sum / max |a| bits while building
  // A's CSR as given (BSGD_PLAN_SINGLE_PASS_ONLY: the caller's arrays, natural order)
  const int64_t* src_ptr = nullptr;
  const int32_t* src_col = nullptr;
  const float* src_val = nullptr;
  int64_t src_nnz = 0;
  double smax = 0.0;              // largest column sum of |A| (FP64)
  double amax = 0.0;              // largest |a|
  int64_t* seg_dev = nullptr;     // segment bounds staged for the fill kernel
  float* vin = nullptr;           // max(r_int, c_int): permuted inputs of step-level calls
  float* vaux = nullptr;          // max(r_int, c_int): second permuted input
  float* vout = nullptr;          // max(r_int, c_int): outputs before un-permuting
};

namespace bsgd {

// Kernels and launchers implemented in the .hip files.
hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp,
                              hipStream_t s);
size_t scan_tmp_count(int64_t n);

// Fused row products over a whole store (all blocks), internal orders:
//   mode kPlain:    out = scale * (row . v)
//   mode kResidual: out = y - row . v
//   mode kStep:     out = xadd + scale * (row . v)
enum RowMode { kPlain = 0, kResidual = 1, kStep = 2 };
hipError_t launch_rows(const Store& st, bsgd_valtype vt, RowMode mode, const float* v,
                       const float* y, const float* xadd, float scale, float* out,
                       hipStream_t s, int lanes = 0, int nt = -1);

// Staged products (Staged::lanes must be 4 or 8); zpart holds P * nrows floats.
hipError_t launch_staged(const Staged& st, bsgd_valtype vt, RowMode mode, const float* v,
                         int64_t nv, const float* y, const float* xadd, float scale, float* out,
                         float* zpart, hipStream_t s);
// Stage geometry of one direction (false if the direction cannot be staged).
bool stage_geometry(const Layout& L, bool fwd, Staged& st);
size_t stage_cnt_count(const Layout& L);
template <bool FWD>
bsgd_status build_staged(Staged& st, const bsgd_csr& src, const Layout& L, int64_t* scratch,
                         hipStream_t s);

// Single-pass products over the tile-sliced store (bsgd_fused): one pass
// writes the per-segment partials of A x (zp) and the per-chunk partials of
// A^T r (gp), with a fixed-point scale set from max |r| (*rmax_in); the
// reduce adds them: out_r = y - A x (A x when y is NULL) and out_x = xadd +
// scale * A^T r (scale * A^T r when xadd is NULL), and gathers max |out_r|
// into *rmax_out (zeroed by the pass through rmax_zero) for the next pass.
// All vectors in internal order.
struct FusedPartials {
  float* zp = nullptr;
  float* gp = nullptr;
  unsigned* rmax = nullptr;  // 2 words: max |r| of the two residual buffers
};
// zp: maxrank x r_int x S floats (one RHS: also at least one per slot), gp:
// Q x c_int x S, rmax: 2 x S words
size_t fused_partials(const bsgd_fused* F, int S, FusedPartials* fp, void* ws);
// several RHS (S a multiple of 4, vectors [rows][S]): per-RHS max |v|, the
// pass (both products, rmax_in: S words) and the reduce
hipError_t launch_fused_absmax_mr(const float* v, int64_t n, int S, unsigned* out,
                                  hipStream_t s);
hipError_t launch_fused_zero(unsigned* p, int n, hipStream_t s);
// waves: wavefronts per workgroup (8 or 16; 0: 16)
hipError_t launch_fused_pass_mr(const bsgd_fused* F, bsgd_valtype vt, int S, const float* x,
                                const float* r, const unsigned* rmax_in, float* zp, float* gp,
                                hipStream_t s, int waves = 0);
hipError_t launch_fused_reduce_mr(const bsgd_fused* F, int S, const float* zp, const float* gp,
                                  const float* y, float* out_r, unsigned* rmax_out,
                                  const float* xadd, float scale, float* out_x, hipStream_t s,
                                  int parts);
hipError_t launch_fused_absmax(const float* v, int64_t n, unsigned* out, hipStream_t s);
// mode kPassBoth: both products; kPassA: only the A x partials (no r,
// rmax_in may be NULL); kPassAt: only the A^T r partials (x unused).
enum { kPassBoth = 0, kPassA = 1, kPassAt = 2 };
hipError_t launch_fused_pass(const bsgd_fused* F, bsgd_valtype vt, const float* x,
                             const float* r, const unsigned* rmax_in, unsigned* rmax_zero,
                             float* zp, float* gp, hipStream_t s, int mode = kPassBoth,
                             int waves = 0,        // waves 0: the store's
                             bool slotz = false);  // one row-sum partial per slot (kPassBoth)
// parts: kReduceRays (out_r, *rmax_out), kReducePixels (out_x), or both.
enum { kReduceRays = 1, kReducePixels = 2, kReduceAll = 3 };
hipError_t launch_fused_reduce(const bsgd_fused* F, const float* zp, const float* gp,
                               const float* y, float* out_r, unsigned* rmax_out,
                               const float* xadd, float scale, float* out_x, hipStream_t s,
                               int parts = kReduceAll, bool slotz = false);
// Whether one-RHS epochs whose ray reduce overlaps the prox keep the row-sum
// partials in slot order (see the definition).
bool fused_slot_partials(const bsgd_fused* F);
bool fused_has_f16(const bsgd_fused* F);
const bsgd_plan* fused_plan(const bsgd_fused* F);

// Same products for S right-hand sides ([rows][S] and [cols][S] matrices, the
// RHS index fastest; S a multiple of 4).
hipError_t launch_spmm(const Store& st, bsgd_valtype vt, RowMode mode, const float* V,
                       const float* Y, const float* XADD, float scale, float* OUT, int S,
                       hipStream_t s);

// Products of one segment (one block) of a store, natural orders in and out.
hipError_t launch_segment_rows(const bsgd_plan* p, bool fwd, bsgd_valtype vt, int64_t nat_row0,
                               int64_t nrows, int segk, int64_t col_base, const float* v,
                               float scale, float* out, hipStream_t s);

// Iterations over drawn block subsets (bit masks of at most kMaxSelBlocks
// row and column blocks).  blk_r / blk_c: block of each internal ray /
// pixel (0xFF for holes).  Forward: for rays of drawn row blocks, Z[j *
// r_int + ray] = segment-j product for drawn j, r_out = y - sum_j Z[j]
// (ascending j, all blocks); other rays copy r_in.  Backward: for pixels of
// drawn column blocks, out = xadd + scale * (sum of the drawn row blocks'
// segments . r); other pixels copy xadd.  Both read the block-major copies.
constexpr int kMaxSelBlocks = 64;
// Block-major copy of a store direction: segment j of row k at off[j * nrows
// + k] (nrows * nseg + 1 offsets), padded to multiples of 4 entries.
struct BlockMajor {
  int64_t nrows = 0;
  int nseg = 0;
  int64_t* off = nullptr;
  int32_t* col = nullptr;
  float* val = nullptr;
  __half* val16 = nullptr;
};
size_t block_major_entries(const Store& st);  // capacity of col / val
hipError_t build_block_major(const Store& st, BlockMajor& bm, int64_t* scan_tmp, hipStream_t s);
hipError_t launch_block_ids(const bsgd_plan* p, uint8_t* blk_r, uint8_t* blk_c, hipStream_t s);
hipError_t launch_sel_forward(const Store& st, const BlockMajor& bm, bsgd_valtype vt,
                              const uint8_t* blk, uint64_t rows, uint64_t cols, const float* x,
                              const float* y, const float* r_in, float* r_out, float* Z,
                              hipStream_t s);
hipError_t launch_sel_backward(const Store& st, const BlockMajor& bm, bsgd_valtype vt,
                               const uint8_t* blk, uint64_t rows, uint64_t cols, const float* r,
                               const float* xadd, float scale, float* out, hipStream_t s);

// Natural <-> internal vector orders (holes are written as 0).  With S > 1
// the vectors are [rows][S] matrices (RHS fastest) and whole rows move.
enum VecKind { kPixels = 0, kRays = 1 };
hipError_t permute_in(const Layout& L, VecKind kind, const float* nat, float* internal,
                      hipStream_t s, int S = 1);
hipError_t permute_out(const Layout& L, VecKind kind, const float* internal, float* nat,
                       hipStream_t s, int S = 1);
// Column j of an internal [n_int][S] matrix from / to a natural vector
// (nat == nullptr writes zeros).
hipError_t scatter_column(const Layout& L, VecKind kind, const float* nat, float* internal,
                          int S, int j, hipStream_t s);
hipError_t gather_column(const Layout& L, VecKind kind, const float* internal, float* nat, int S,
                         int j, hipStream_t s);
// mat[k * S + j] = v[k] for k < n (both internal order)
hipError_t set_column(const float* v, float* mat, int64_t n, int S, int j, hipStream_t s);
// Per-column sums of squares of an [n][S] matrix, FP64, fixed order:
// partial must hold kColBlocks * S doubles, out S doubles.
constexpr int kColBlocks = 64;
hipError_t launch_colsumsq(const float* X, int64_t n, int S, double* partial, double* out,
                           hipStream_t s);
// v = 1 on every pixel, 0 on holes (internal order)
hipError_t fill_pixels_one(const Layout& L, float* v, hipStream_t s);

// Deterministic sum of squares in FP64 (fixed grid, fixed order).
constexpr int kReduceBlocks = 512;
hipError_t launch_sumsq(const float* x, int64_t n, double* partial, double* out, hipStream_t s);

hipError_t fill_f32(float* x, int64_t n, float v, hipStream_t s);

// FGP TV prox.  tiled = false: natural row-major image (H*W*D floats);
// tiled = true: the internal pixel order of L (c_int floats).  ws must hold
// tv_ws_floats(n) floats with n the vector length.
size_t tv_ws_floats(int64_t n, int D);
enum FgpSchedule { kFgpFused = 0, kFgpPerIteration = 1, kFgpFusedLds = 2 };
// split: most FGP iterations per launch of the chunked schedules (2-D: 1 to
// 10, volumes: 1 to 3; 0 or larger: the most)
hipError_t tv_prox_run(const Layout& L, bool tiled, const float* b, float theta, int iters,
                       float* out, float* ws, hipStream_t s, int schedule, int split = 0);
// S images in the internal 2-D pixel order, [c_int][S] (image index fastest),
// each with its own theta_j = mu * lam[j] (lam: device array of S floats, or
// nullptr for theta_j = mu * lam0 for all j).  ws: tv_ws_floats(c_int * S, 1).
hipError_t tv_prox_batch(const Layout& L, int S, const float* b, float mu, const float* lam,
                         float lam0, int iters, float* out, float* ws, hipStream_t s,
                         int schedule, int split = 0);
// One volume of S slices in the internal order [c_int][S] (slice index
// fastest), 3-D TV.  ws: tv_ws_floats(c_int * S, 2).
// schedule kFgpPerIteration: one launch per iteration (k_fgp_iter3v);
// otherwise launches of up to three iterations (k_fgp_tb3).  Same results.
hipError_t tv_prox_volume(const Layout& L, int S, const float* b, float theta, int iters,
                          float* out, float* ws, hipStream_t s, int schedule, int split = 0);

}  // namespace bsgd

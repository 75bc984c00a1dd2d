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

// One direction of the block store: rows of A (rays, segments = column
// blocks) or rows of A^T (pixels, segments = row blocks).  Row `row` holds
// its entries in [ptr[row], ptr[row] + seg[row*(nseg+1) + nseg]) followed by
// zero padding up to ptr[row+1]; segment k is the relative range
// [seg[.. + k], seg[.. + k + 1]) and holds the columns in
// [seg_off[k], seg_off[k+1]).
struct Store {
  int64_t nrows = 0, ncols = 0, nnz = 0, cap = 0;
  int nseg = 0;
  int64_t* ptr = nullptr;
  int32_t* seg = nullptr;
  int32_t* col = nullptr;
  float* val = nullptr;
  __half* val16 = nullptr;
  std::vector<int64_t> seg_off;   // host copy, nseg + 1 entries
  int lanes_per_row = 64;         // launch choice for the fused row kernels
};

}  // namespace bsgd

struct bsgd_plan {
  int M = 0, N = 0, H = 0, W = 0, D = 0;
  unsigned flags = 0;
  bsgd::Store fwd;   // A
  bsgd::Store bwd;   // A^T
  std::vector<int64_t> row_off, col_off;
  int64_t* scratch64 = nullptr;   // max(nrows, ncols) + 1 entries (tile export)
  int64_t* scan_tmp = nullptr;    // block sums for scans
  int* err = nullptr;             // validation flags
  int64_t* seg_dev = nullptr;     // segment bounds staged for the fill kernel
};

namespace bsgd {

// Kernels and launchers implemented in the .hip files.
hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp,
                              hipStream_t s);
size_t scan_tmp_count(int64_t n);

// Fused row products over a whole store (all blocks):
//   mode kPlain:    out = scale * (row . v)
//   mode kResidual: out = y - row . v
//   mode kStep:     out = xadd + scale * (row . v)
enum RowMode { kPlain = 0, kResidual = 1, kStep = 2 };
hipError_t launch_rows(const Store& st, bsgd_valtype vt, RowMode mode, const float* v,
                       const float* y, const float* xadd, float scale, float* out,
                       hipStream_t s);

// Products of one segment (one block) of a store.
hipError_t launch_segment_rows(const Store& st, bsgd_valtype vt, int64_t row0, int64_t nrows,
                               int segk, int64_t col_base, const float* v, float scale,
                               float* out, hipStream_t s);

// Deterministic sum of squares in FP64 (fixed grid, fixed order).
constexpr int kReduceBlocks = 512;
hipError_t launch_sumsq(const float* x, int64_t n, double* partial, double* out, hipStream_t s);

hipError_t fill_f32(float* x, int64_t n, float v, hipStream_t s);

// FGP TV prox on device buffers; ws must hold tv_ws_floats(H, W, D) floats.
size_t tv_ws_floats(int H, int W, int D);
hipError_t tv_prox_run(int H, int W, int D, const float* b, float theta, int iters, float* out,
                       float* ws, hipStream_t s);

}  // namespace bsgd

// Single-pass epoch products (the block products, block sums and gradient step of Algorithm 1, with the delay of Eq. 3).
//
// The block backprojection of an epoch uses the residual r_k of the previous epoch and the block forward projection
// the current iterate x_k.  Both are known when the epoch starts, so one
// pass over the stored entries a = A[rho, p] can produce both sums:
//     z[rho] += a * x_k[p]      (the block forward projection; summed over the column blocks: the residual update)
//     g[p]   += a * r_k[rho]    (the block backprojection; summed over the row blocks:    the gradient sum)
// which reads the matrix once per epoch instead of once as A and once as A^T.
//
// Tile-sliced store.  Pixels are grouped into 64 x 64 tiles (8 x 8 of the
// internal 8 x 8 tiles, across slices for volumes); rays into Q chunks of
// whole ray groups (8 interleaved views, see bsgd::Layout).  A segment is
// the part of one ray inside one tile.  Unit u = (tile, chunk) holds the
// segments of the chunk's rays in the tile, sorted longest first, ties by
// (view, bin parity, bin), 64 per slice, one per lane (neighbouring lanes
// then follow parallel rays two bins apart, which never cross the same pixel:
// a pixel's shadow on the detector is at most sqrt(2) bins wide).  A slice
// stores its entries
// lane-interleaved in groups of 4:
//     entry j of lane l at soff[s] + (j / 4) * 256 + l * 4 + j % 4
// as a column and an FP32 value (optional FP16 copy).  The column is the
// pixel's address in the tile's LDS image (row stride 65); entries of a
// segment are in ascending address order, and when every step from one
// entry to the next is below 256 (for rays: about one row stride) the store
// keeps 8-bit steps with a 16-bit start address per lane (5 bytes per entry
// with FP32 values, 3 with FP16), else 16-bit addresses.  Lanes shorter than
// the slice's longest are padded with zero values on an address they
// already use (a zero step).
//
// Pass.  One workgroup per unit copies the tile of x_k to LDS.  Each of its W
// wavefronts takes every W-th slice of the unit, gathers x from LDS for the
// row sums (one partial per segment, stored at [rank][ray], rank = the
// segment's place among the ray's segments) and adds a * r[rho] into the
// tile's g in LDS.  Those adds are 32-bit integer LDS atomics on fixed-point
// terms (see term32): exact and order-free, so the lanes and wavefronts
// that meet on a pixel need no ordering (FP32 LDS atomics measured about 4x
// slower than the whole pass on gfx950).  The unit's partial of g is
// converted back to FP32 once.  A second kernel adds each ray's segment
// partials in the order the ray enters the tiles (r = y - sum) and each
// pixel's Q chunk partials in chunk order (x^ = x + mu * 2 sum).  No global
// atomics: results are bitwise reproducible for a given store.
//
// The store is built on the device from the plan's forward store: one
// wavefront per ray finds its segments (first-appearance rank and length),
// a stable radix sort orders them by (unit, length), and the entries are
// scattered into their slices.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "bsgd_internal.h"

namespace bsgd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

constexpr int kFT = 64;              // tile side in pixels
constexpr int kFTS = kFT + 1;        // LDS row stride (rows and columns hit distinct banks)
constexpr int kFTA = kFT * kFTS;     // LDS floats per tile image
constexpr int kKeyLen = 8192;        // key >> 32 = unit * 8192 + (8191 - segment length)
constexpr int kMaxSeg = kFT * kFT;   // a segment holds at most one entry per pixel
// One-RHS epochs keep the row sums in slot order up to this many slots
// (measured on gfx950: 3.8 M slots at 512^2, epochs 1.5% faster; 30 M at
// 1024^2, 3.5% slower: the ray reduce's gathers leave the caches and slow
// the pixel half and the prox beside it).
constexpr int64_t kSlotPartialsMax = int64_t{1} << 23;

struct TileGeom {
  int Ht = 1, Wt = 1;        // 8 x 8 tiles per image column / row
  float rWt = 1.f;           // 1 / Wt rounded to FP32 (division by Wt in the build)
  int FTh = 1, FTw = 1;      // 64 x 64 tiles per image column / row
  int D = 1;
  int Q = 1;                 // ray chunks
  int64_t slice_px = 0;      // internal pixels per slice (Ht * Wt * 64)
  int64_t group_len = 64;    // internal rays per ray group
  int64_t ngroups = 1;
  int64_t view_len = 0;      // rays per view (0: rows without view structure)
  int W = 1;                 // image width (natural pixel p = d H W + s W + t)
  float rW = 1.f;            // 1 / W rounded to FP32
  int64_t hw = 1;            // H W
  int64_t ncols = 0;         // D H W
  int64_t tiles() const { return (int64_t)D * FTh * FTw; }
  int64_t units() const { return tiles() * Q; }
};

}  // namespace bsgd

struct bsgd_fused {
  const bsgd_plan* plan = nullptr;
  bsgd::TileGeom g;
  int waves = 8;             // wavefronts per unit workgroup (2, 4 or 8)
  bool slotz = false;        // per launch: one-RHS row-sum partials in slot order
  int64_t pairs = 0, slices = 0, entries = 0, cap = 0;
  int maxrank = 0;           // most segments of one ray
  double smax = 0.0;         // largest column sum of |A| (bounds the sums of A^T r)
  double amax = 0.0;         // largest |a| (bounds one term of A^T r)
  int32_t* sbeg = nullptr;   // units + 1: first slice of each unit
  int32_t* uorder = nullptr; // units: launch order (most slices first)
  int32_t* sng = nullptr;    // slices: 4-entry groups per lane
  int64_t* soff = nullptr;   // slices + 1: first entry of each slice
  int32_t* sray = nullptr;   // slices * 64: internal ray of each lane (-1: none)
  int32_t* poff = nullptr;   // r_int + 1: first segment of each ray
  int32_t* pslot = nullptr;  // pairs: slot of each segment (ray order: poff[ray] + rank)
  uint16_t* srank = nullptr; // slices * 64: the lane's segment's rank within its ray
  bool narrow = true;        // 8-bit address steps (col8, sbase) or 16-bit addresses (col)
  uint8_t* col8 = nullptr;   // cap
  uint16_t* sbase = nullptr; // slices * 64: first address of each lane (narrow)
  uint16_t* col = nullptr;   // cap (wide)
  float* val = nullptr;      // cap
  __half* val16 = nullptr;   // cap (plans with BSGD_PLAN_F16)
  // internal-order operands of bsgd_fused_apply
  float *xin = nullptr, *xadd = nullptr, *rin = nullptr, *yin = nullptr, *zo = nullptr,
        *go = nullptr;
};

namespace bsgd {

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
static TileGeom tile_geom(const Layout& L, int chunks) {
  TileGeom g;
  g.Ht = L.Ht;
  g.Wt = L.Wt;
  g.rWt = 1.0f / (float)L.Wt;
  g.W = L.W;
  g.rW = 1.0f / (float)L.W;
  g.hw = (int64_t)L.H * L.W;
  g.ncols = (int64_t)L.D * L.H * L.W;
  g.FTh = (L.Ht + 7) / 8;
  g.FTw = (L.Wt + 7) / 8;
  g.D = L.D;
  g.slice_px = (int64_t)L.Ht * L.Wt * 64;
  g.view_len = L.view_len;
  if (L.view_len > 0) {
    g.group_len = (int64_t)kViewTile * L.view_len;
    g.ngroups = L.r_int / g.group_len;
  } else {
    g.group_len = 64;
    g.ngroups = (L.r_int + 63) / 64;
  }
  if (chunks > 0) {
    g.Q = chunks;
  } else {
    // at least about 1024 unit workgroups, and chunks of at most 128 K rays
    // (512 KB of r, so that a unit's residual gathers stay in L2; measured
    // on gfx950: 16 chunks at 512^2 and at 1024^2, within 1% of the best
    // of 8 to 32 at both), no more chunks than ray groups
    const int64_t want = std::max<int64_t>((1024 + g.tiles() - 1) / g.tiles(),
                                           (L.r_int + 131071) / 131072);
    g.Q = (int)std::max<int64_t>(1, std::min<int64_t>(want, g.ngroups));
  }
  return g;
}

__device__ __forceinline__ int chunk_of(const TileGeom& g, int64_t k) {
  return (int)((k / g.group_len) * g.Q / g.ngroups);
}

// Internal pixel index -> row-band key G (slice, tile row), tile column f and
// address in the tile's LDS image.
__device__ __forceinline__ void decode_pixel(const TileGeom& g, int64_t cp, int& G, int& f,
                                             int& a) {
  const int64_t d = g.D == 1 ? 0 : cp / g.slice_px;
  const int64_t rem = cp - d * g.slice_px;
  const int t8 = (int)(rem >> 6), w = (int)(rem & 63);
  // t8 / Wt from the FP32 reciprocal: t8 < 2^24 is exact in FP32 and the
  // product is within 1 of the quotient, so one correction step makes it exact
  int tr8 = (int)((float)t8 * g.rWt);
  int tc8 = t8 - tr8 * g.Wt;
  if (tc8 < 0) {
    --tr8;
    tc8 += g.Wt;
  } else if (tc8 >= g.Wt) {
    ++tr8;
    tc8 -= g.Wt;
  }
  G = (int)d * g.FTh + (tr8 >> 3);
  f = tc8 >> 3;
  a = (((tr8 & 7) << 3) + (w >> 3)) * kFTS + ((tc8 & 7) << 3) + (w & 7);
}

// The same for a natural pixel index (d H W + s W + t: the columns of A as
// given), s = rem / W from the FP32 reciprocal as above (rem < H W <= 2^24).
__device__ __forceinline__ void decode_nat(const TileGeom& g, int64_t cp, int& G, int& f,
                                           int& a) {
  const int64_t d = g.D == 1 ? 0 : cp / g.hw;
  const int rem = (int)(cp - d * g.hw);
  int s = (int)((float)rem * g.rW);
  int t = rem - s * g.W;
  if (t < 0) {
    --s;
    t += g.W;
  } else if (t >= g.W) {
    ++s;
    t -= g.W;
  }
  G = (int)d * g.FTh + (s >> 6);
  f = t >> 6;
  a = (s & 63) * kFTS + (t & 63);
}

// Walk one ray's entries (one wavefront; the entries are in ascending natural
// pixel order, so the band key G never decreases along the row).  Lane f
// keeps, for the current band, the rank and running length of the segment
// in tile column f.  Segments are ranked in the order the ray enters them.
//   vis.prefetch(e, ok) / vis.advance()  per-entry data of the next batch
//                                      (entry e of this lane) / make it current
//   vis.group(rank)                     before the entries of one segment in
//                                      a batch (called by the whole wavefront)
//   vis.entry(rank, j, lds_addr, e, prev)  entry e is the j-th of segment
//                                      `rank`; prev = the segment's previous
//                                      address (-1 for j = 0)
//   vis.close(G, f, len, rank, first)  called by every lane f when band G ends
//                                      (rank < 0: no segment in column f;
//                                      first = the segment's first address)
//   vis.finish(nseg)
// NAT: the columns are natural pixel indices (A as given) rather than the
// block store's internal ones.  CHECK: also returns whether every column is
// in range and the columns strictly ascend.
template <bool NAT, bool CHECK, class V>
__device__ bool walk_ray(const TileGeom& g, const int32_t* __restrict__ col, int64_t beg,
                         int64_t len, V& vis) {
  const int lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1ull;
  int Gcur = -1, cnt = 0, rank = -1, nseen = 0, first = 0, last = 0;
  bool ok = true;
  int32_t lastc = 0;  // the previous batch's last column (CHECK)
  int32_t cnext = lane < len ? col[beg + lane] : 0;
  vis.prefetch(beg + lane, lane < len);
  for (int64_t c0 = 0; c0 < len; c0 += 64) {
    const int64_t e = c0 + lane;
    const bool valid = e < len;
    const int32_t cp = cnext;
    vis.advance();
    // the next batch's columns (and the visitor's data) load while this one
    // is walked
    if (e + 64 < len) cnext = col[beg + e + 64];
    vis.prefetch(beg + e + 64, e + 64 < len);
    if constexpr (CHECK) {
      const int32_t up = __shfl_up(cp, 1);
      const int32_t prev = lane == 0 ? lastc : up;
      if (valid && (cp < 0 || cp >= g.ncols || (e > 0 && cp <= prev))) ok = false;
      lastc = __shfl(cp, 63);
    }
    int G = 0x7fffffff, f = 0, a = 0;
    if (valid) {
      if constexpr (NAT)
        decode_nat(g, cp, G, f, a);
      else
        decode_pixel(g, cp, G, f, a);
    }
    bool done = !valid;
    uint64_t live;
    while ((live = __ballot(!done)) != 0ull) {
      const int leader = __builtin_ctzll(live);
      const int Gl = __shfl(G, leader);
      if (Gl != Gcur) {
        if (Gcur >= 0) vis.close(Gcur, lane, cnt, rank, first);
        cnt = 0;
        rank = -1;
        Gcur = Gl;
      }
      const bool inG = !done && G == Gl;
      uint64_t todo = __ballot(inG);
      while (todo) {
        const int l2 = __builtin_ctzll(todo);
        const int fl = __shfl(f, l2);
        const uint64_t mm = __ballot(inG && f == fl);
        int rk = __shfl(rank, fl);
        const int base = __shfl(cnt, fl);
        const int lastf = __shfl(last, fl);
        // previous entry of the segment: the batch lane before this one, or
        // the segment's last entry from an earlier batch
        const uint64_t pm = mm & below;
        const int plane = pm ? 63 - __builtin_clzll(pm) : lane;
        const int pa = __shfl(a, plane);
        const int prev = pm ? pa : (base > 0 ? lastf : -1);
        const int alast = __shfl(a, 63 - __builtin_clzll(mm));
        const int afirst = __shfl(a, l2);
        if (rk < 0) rk = nseen++;
        vis.group(rk);  // rk is the same in every lane
        if (lane == fl) {
          if (base == 0) first = afirst;
          rank = rk;
          cnt = base + __popcll(mm);
          last = alast;
        }
        if (inG && f == fl) vis.entry(rk, base + __popcll(mm & below), a, beg + e, prev);
        todo &= ~mm;
      }
      done = done || inG;
    }
  }
  if (Gcur >= 0) vis.close(Gcur, lane, cnt, rank, first);
  vis.finish(nseen);
  return __ballot(!ok) == 0ull;
}

// Raise *word to v (one word shared by the whole grid: read first, so that
// only the few values that raise it take an atomic).
__device__ __forceinline__ void raise_to(int32_t* word, int32_t v) {
  if (v > __atomic_load_n(word, __ATOMIC_RELAXED)) atomicMax(word, v);
}

// Segments per ray, and the grid-wide maxima of segments per ray (maxc),
// entries per segment (maxlen) and address step inside a segment (maxstep).
struct VisCount {
  int64_t k;
  int64_t* ncross;
  int32_t *maxc, *maxlen, *maxstep;
  int mlen = 0, mstep = 0;
  __device__ void prefetch(int64_t, bool) {}
  __device__ void advance() {}
  __device__ void group(int) {}
  __device__ void entry(int, int, int a, int64_t, int prev) {
    if (prev >= 0) mstep = max(mstep, a - prev);
  }
  __device__ void close(int, int, int len, int rank, int) {
    if (rank >= 0) mlen = max(mlen, len);
  }
  __device__ void finish(int n) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      mlen = max(mlen, __shfl_xor(mlen, off));
      mstep = max(mstep, __shfl_xor(mstep, off));
    }
    if ((threadIdx.x & 63) == 0) {
      ncross[k] = n;
      raise_to(maxc, n);
      raise_to(maxlen, mlen);
      raise_to(maxstep, mstep);
    }
  }
};

// Tie order inside a length class: view, bin parity, bin (rays of the
// internal order k = group * 8 * bins + bin * 8 + view-in-group); the ray
// order when the rows have no view structure.
__device__ __forceinline__ uint32_t tie_of(const TileGeom& g, int64_t k) {
  if (g.view_len == 0) return (uint32_t)k;
  const int64_t G = k / g.group_len, rem = k - G * g.group_len;
  const int64_t b = rem / kViewTile, v = rem % kViewTile;
  const int64_t half = (g.view_len + 1) / 2;
  return (uint32_t)(((v * g.ngroups + G) * 2 + (b & 1)) * half + (b >> 1));
}

struct VisPairs {
  TileGeom g;
  int64_t k;
  int q;
  int64_t pk;  // the ray's first segment index
  uint64_t* key;
  int32_t* idx;
  int32_t* pray;
  uint16_t* pbase;
  __device__ void prefetch(int64_t, bool) {}
  __device__ void advance() {}
  __device__ void group(int) {}
  __device__ void entry(int, int, int, int64_t, int) {}
  __device__ void close(int G, int f, int len, int rank, int first) {
    if (rank < 0) return;
    const int64_t p = pk + rank;
    const int64_t u = ((int64_t)G * g.FTw + f) * g.Q + q;
    key[p] = ((uint64_t)(u * kKeyLen + (kKeyLen - 1 - len)) << 32) | tie_of(g, k);
    idx[p] = (int32_t)p;
    pray[p] = (int32_t)k;
    pbase[p] = (uint16_t)first;
  }
  __device__ void finish(int) {}
};

// Entry j of the ray's segment `rank` goes to dst + (j / 4) * 256 + j % 4,
// dst and the slice's group count from the segment's packed destination.
// Lane i holds the packed destination of the ray's segment i (loaded once
// per ray); a batch's segment takes it from that lane's register.
constexpr int kDstShift = 11;  // a segment has at most 4096 entries: ng <= 1024

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

struct VisFill {
  int64_t pk;    // the ray's first segment index
  int64_t dpre;  // this lane's segment's packed destination (lane < segments)
  int64_t d;     // the current segment's
  const int64_t* pdst;
  const float* vsrc;
  const __half* v16src;
  uint16_t* col;
  uint8_t* col8;
  float* val;
  __half* val16;
  int* err;
  float vnext = 0.f, vcur = 0.f;  // this lane's entry of the next / current batch
  __half hnext = 0.f, hcur = 0.f; // its FP16 copy (plans with one)
  __device__ void prefetch(int64_t e, bool ok) {
    if (!ok) return;
    vnext = vsrc[e];
    if (v16src) hnext = v16src[e];
  }
  __device__ void advance() {
    vcur = vnext;
    hcur = hnext;
  }
  __device__ void group(int rk) { d = rk < 64 ? readlane64(dpre, rk) : pdst[pk + rk]; }
  __device__ void entry(int, int j, int a, int64_t, int prev) {
    if (j >= 4 * (int)(d & ((1 << kDstShift) - 1))) {
      atomicOr(err, 1);
      return;
    }
    const int64_t addr = (d >> kDstShift) + (int64_t)(j >> 2) * 256 + (j & 3);
    if (col8)
      col8[addr] = (uint8_t)(j == 0 ? 0 : a - prev);
    else
      col[addr] = (uint16_t)a;
    val[addr] = vcur;
    if (val16) val16[addr] = v16src ? hcur : __float2half_rn(vcur);
  }
  __device__ void close(int, int, int, int, int) {}
  __device__ void finish(int) {}
};

// MODE 0: count, 1: segments, 2: fill.  One wavefront per internal ray.  The
// rows come from the block store of A (ptr, seg: internal order and columns)
// or, NAT, from A as given (ptr = row_ptr of the natural rows, internal ray
// k being natural row L.ray_out(k)); the NAT count also checks the columns
// and sets *err on a bad one.
template <int MODE, bool NAT>
__global__ __launch_bounds__(256) void k_fz_walk(
    TileGeom g, Layout L, const int64_t* __restrict__ ptr, const int32_t* __restrict__ seg,
    int nseg,
    const int32_t* __restrict__ col, const float* __restrict__ vsrc,
    const __half* __restrict__ v16src, int64_t r_int, int64_t* ncross, int32_t* maxc,
    int32_t* maxlen, int32_t* maxstep, const int64_t* poff, uint64_t* key, int32_t* idx,
    int32_t* pray, uint16_t* pbase, const int64_t* pdst, uint16_t* ocol, uint8_t* ocol8,
    float* oval, __half* oval16, int* err) {
  int64_t b = blockIdx.x;
  if constexpr (MODE == 2) {
    // workgroups are dealt to the 8 XCDs in turn; the fill gives each XCD a
    // contiguous range of rays instead (the grid is a multiple of 8), so the
    // few rays whose segments share a line of the store (neighbouring bins
    // of one view) write it through one L2, which merges their partial writes
    const int64_t per = gridDim.x / 8;
    b = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  }
  const int64_t k = (b * 256 + threadIdx.x) >> 6;
  if (k >= r_int) return;  // uniform per wavefront
  int64_t beg = 0, len = 0;
  if constexpr (NAT) {
    const int64_t n = L.ray_out(k);  // -1: a hole of the internal order (no entries)
    if (n >= 0) {
      beg = ptr[n];
      len = ptr[n + 1] - beg;
    }
  } else {
    beg = ptr[k];
    len = seg[k * (nseg + 1) + nseg];
  }
  const int q = chunk_of(g, k);
  if constexpr (MODE == 0) {
    VisCount v{k, ncross, maxc, maxlen, maxstep};
    const bool ok = walk_ray<NAT, NAT>(g, col, beg, len, v);
    if (NAT && !ok && (threadIdx.x & 63) == 0) atomicOr(err, 1);
  } else if constexpr (MODE == 1) {
    VisPairs v{g, k, q, poff[k], key, idx, pray, pbase};
    walk_ray<NAT, false>(g, col, beg, len, v);
  } else {
    const int64_t pk = poff[k], nr = poff[k + 1] - pk;
    const int lane = threadIdx.x & 63;
    const int64_t dpre = lane < nr ? pdst[pk + lane] : 0;
    VisFill v{pk, dpre, 0, pdst, vsrc, v16src, ocol, ocol8, oval, oval16, err};
    walk_ray<NAT, false>(g, col, beg, len, v);
  }
}

// A's rows for the walks: the block store of A, or A as given
// (BSGD_PLAN_SINGLE_PASS_ONLY).
struct WalkSrc {
  bool nat = false;
  const int64_t* ptr = nullptr;
  const int32_t* seg = nullptr;
  int nseg = 0;
  const int32_t* col = nullptr;
  const float* val = nullptr;
  const __half* val16 = nullptr;
  int64_t nnz = 0;
};

static WalkSrc walk_src(const bsgd_plan* p) {
  WalkSrc w;
  if (p->flags & BSGD_PLAN_SINGLE_PASS_ONLY) {
    w.nat = true;
    w.ptr = p->src_ptr;
    w.col = p->src_col;
    w.val = p->src_val;
    w.nnz = p->src_nnz;
  } else {
    w.ptr = p->fwd.ptr;
    w.seg = p->fwd.seg;
    w.nseg = p->fwd.nseg;
    w.col = p->fwd.col;
    w.val = p->fwd.val;
    w.val16 = p->fwd.val16;
    w.nnz = p->fwd.nnz;
  }
  return w;
}

template <int MODE, typename... Args>
static void launch_walk(const WalkSrc& w, const TileGeom& g, const Layout& L, unsigned blocks,
                        hipStream_t s, Args... args) {
  if (w.nat)
    k_fz_walk<MODE, true><<<blocks, 256, 0, s>>>(g, L, w.ptr, w.seg, w.nseg, w.col, args...);
  else
    k_fz_walk<MODE, false><<<blocks, 256, 0, s>>>(g, L, w.ptr, w.seg, w.nseg, w.col, args...);
}

// First and last sorted position of each unit (keys sorted by unit first);
// empty units keep first = 0, last = -1.
__global__ void k_fz_unit_bounds(const uint64_t* __restrict__ keys, int64_t n,
                                 int64_t* __restrict__ first, int64_t* __restrict__ last) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t u = (uint32_t)(keys[i] >> 32) / kKeyLen;
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) / kKeyLen != u) first[u] = i;
    if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) / kKeyLen != u) last[u] = i;
  }
}

__global__ void k_fz_unit_init(int64_t* __restrict__ first, int64_t* __restrict__ last,
                               int64_t units) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units;
       u += (int64_t)gridDim.x * blockDim.x) {
    first[u] = 0;
    last[u] = -1;
  }
}

// Sorted segment i -> its slot; lane 0 of a slice holds its longest segment.
__global__ void k_fz_place(const uint64_t* __restrict__ keys, const int32_t* __restrict__ idx,
                           const int32_t* __restrict__ pray, const int64_t* __restrict__ poff,
                           int64_t npairs, const int64_t* __restrict__ ubeg,
                           const int32_t* __restrict__ sbeg, int64_t nslots,
                           const uint16_t* __restrict__ pbase, int32_t* __restrict__ pos,
                           int32_t* __restrict__ sray, uint16_t* __restrict__ srank,
                           uint16_t* __restrict__ sbase, int32_t* __restrict__ slen,
                           int32_t* __restrict__ sng, int64_t* __restrict__ sng256,
                           int* __restrict__ err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npairs;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t key = (uint32_t)(keys[i] >> 32);
    const int64_t u = key / kKeyLen;
    const int len = kKeyLen - 1 - (int)(key % kKeyLen);
    const int64_t m = i - ubeg[u];
    const int64_t s = sbeg[u] + m / 64;
    const int l = (int)(m % 64);
    const int64_t P = s * 64 + l;
    if (m < 0 || P >= nslots) {
      atomicOr(err, 2);
      continue;
    }
    const int32_t p = idx[i];
    pos[p] = (int32_t)P;
    sray[P] = pray[p];
    srank[P] = (uint16_t)(p - poff[pray[p]]);
    if (sbase) sbase[P] = pbase[p];
    slen[P] = len;
    if (l == 0) {
      sng[s] = (len + 3) / 4;
      sng256[s] = (int64_t)((len + 3) / 4) * 256;
    }
  }
}

// Packed destination of each segment once the slice offsets are known: the
// first word of its lane, shifted, or-ed with the slice's group count.
__global__ void k_fz_dst(const int32_t* __restrict__ pos, int64_t npairs,
                         const int64_t* __restrict__ soff, const int32_t* __restrict__ sng,
                         int64_t* __restrict__ pdst) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t P = pos[p];
    const int64_t s = P >> 6;
    pdst[p] = ((soff[s] + (P & 63) * 4) << kDstShift) | sng[s];
  }
}

__global__ void k_fz_init_slots(int32_t* __restrict__ sray, int32_t* __restrict__ slen,
                                uint16_t* __restrict__ sbase, int64_t nslots) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (int64_t)gridDim.x * blockDim.x) {
    sray[i] = -1;
    slen[i] = 0;
    if (sbase) sbase[i] = (uint16_t)(i & 63);  // empty lanes: distinct addresses
  }
}

// Zero-valued padding of every lane up to its slice's group count; the
// column repeats the lane's last real entry (an empty lane uses its own
// lane number, so padded lanes do not meet on one LDS address).
__global__ void k_fz_pad(const int32_t* __restrict__ slen, const int32_t* __restrict__ sng,
                         const int64_t* __restrict__ soff, int64_t nslots,
                         uint16_t* __restrict__ col, uint8_t* __restrict__ col8,
                         float* __restrict__ val, __half* __restrict__ val16) {
  for (int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; P < nslots;
       P += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = P >> 6;
    const int l = (int)(P & 63);
    const int len = slen[P], ng = sng[s];
    const int64_t base = soff[s] + l * 4;
    const uint16_t c = col8 || len == 0
                           ? (uint16_t)l
                           : col[base + (int64_t)((len - 1) >> 2) * 256 + ((len - 1) & 3)];
    for (int j = len; j < 4 * ng; ++j) {
      const int64_t a = base + (int64_t)(j >> 2) * 256 + (j & 3);
      if (col8)
        col8[a] = 0;  // a zero step: the lane's last address (its start when empty)
      else
        col[a] = c;
      val[a] = 0.f;
      if (val16) val16[a] = __float2half_rn(0.f);
    }
  }
}

__global__ void k_i64_to_i32(const int64_t* __restrict__ in, int32_t* __restrict__ out,
                             int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)in[i];
}

__global__ void k_fill_i32(int32_t* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0;
}

static unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
}

// ---------------------------------------------------------------------------
// The pass
// ---------------------------------------------------------------------------
// Fixed-point terms for the LDS sums of A^T r.  A term t = rint(a r 2^e) is
// added as a 32-bit integer; the scale 2^e comes from the largest |r| (rmax,
// gathered by the kernel that wrote r), the largest column sum of |A|
// (smax) and the largest |a| (amax): every sum of a pixel stays below 2^30 in
// magnitude and every term below 2^21.  The latter lets one FP32 FMA round a
// term: f = a (r 2^e) + 1.5 * 2^23 is rounded once, and its bit pattern minus
// that of 1.5 * 2^23 is t.  Integer addition is exact and associative, so the
// order of the atomics does not change the result; the rounding of a term is
// below 2^-31 of the largest possible sum.
constexpr float kMagic32 = 12582912.0f;  // 1.5 * 2^23
constexpr int kMagic32Bits = 0x4B400000;
constexpr unsigned long long kMagicPair = 0x4B4000004B400000ull;  // the magic in both words

__device__ __forceinline__ int fixed_exponent32(double smax, double amax, float rmax) {
  const double b = smax * (double)rmax, t = amax * (double)rmax;
  if (!(b > 0.0) || !isfinite(b)) return 0;
  int Es, Et;
  (void)frexp(b, &Es);  // b < 2^Es
  (void)frexp(t, &Et);
  return min(max(min(30 - Es, 21 - Et), -200), 200);
}

__device__ __forceinline__ int term32(float a, float rs) {
  return __float_as_int(fmaf(a, rs, kMagic32)) - kMagic32Bits;
}

struct SliceMeta {
  int rho, rk, ng, a0;
  int64_t base;
};

__device__ __forceinline__ SliceMeta slice_meta(const int32_t* __restrict__ sray,
                                                const uint16_t* __restrict__ srank,
                                                const uint16_t* __restrict__ sbase,
                                                const int32_t* __restrict__ sng,
                                                const int64_t* __restrict__ soff, int s, int s1,
                                                int lane) {
  SliceMeta m{-1, 0, 0, 0, 0};
  if (s < s1) {
    m.rho = sray[(int64_t)s * 64 + lane];
    m.rk = srank[(int64_t)s * 64 + lane];
    m.a0 = sbase ? sbase[(int64_t)s * 64 + lane] : 0;
    m.ng = sng[s];
    m.base = soff[s] + lane * 4;
  }
  return m;
}

// Matrix streams are read once per pass: non-temporal loads keep them from
// evicting the gathered r, the partial sums and the tables from the caches.
template <typename T>
__device__ __forceinline__ T ld_nt(const T* p) {
  return __builtin_nontemporal_load(p);
}

// Column data of one group of 4 entries of a lane: 4 addresses (wide) or 4
// 8-bit steps in one word (narrow).
template <bool NARROW>
using ColRaw = typename std::conditional<NARROW, uint32_t, u16x4>::type;

template <typename VT, bool NARROW>
__device__ __forceinline__ void load_group(const void* __restrict__ col,
                                           const VT* __restrict__ val, int64_t i,
                                           ColRaw<NARROW>& c, float (&a)[4]) {
  if constexpr (NARROW)
    c = ld_nt(reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(col) + i));
  else
    c = ld_nt(reinterpret_cast<const u16x4*>(static_cast<const uint16_t*>(col) + i));
  if constexpr (sizeof(VT) == 4) {
    const f32x4 v = ld_nt(reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(val) + i));
    a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
  } else {
    const f16x4 v = ld_nt(reinterpret_cast<const f16x4*>(reinterpret_cast<const _Float16*>(val) + i));
    a[0] = (float)v[0]; a[1] = (float)v[1]; a[2] = (float)v[2]; a[3] = (float)v[3];
  }
}

// z += a . x[c] (LDS gathers) and g[c] += a * r (fixed-point LDS atomics);
// narrow columns are decoded from the lane's running address ap (groups of
// a lane are decoded in order).  MERGED: x[c] and g[c] share one 64-bit LDS
// cell (x's bits low, the fixed-point sum high), and one 64-bit atomic add of
// the term shifted into the high word returns x with the old value: one LDS
// instruction per entry instead of two.  The high word wraps like a 32-bit
// add and the low word never changes, so the results are the same bits.
template <bool NARROW, int MODE, bool MERGED>
__device__ __forceinline__ void group_step(const float* xs, int* gs, unsigned long long* xg,
                                           const ColRaw<NARROW>& raw, const float (&a)[4],
                                           float rs, float& z, int& ap) {
  int c[4];
  if constexpr (NARROW) {
    c[0] = ap + (int)(raw & 255u);
    c[1] = c[0] + (int)((raw >> 8) & 255u);
    c[2] = c[1] + (int)((raw >> 16) & 255u);
    c[3] = c[2] + (int)(raw >> 24);
    ap = c[3];
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) c[t] = raw[t];
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if constexpr (MERGED) {
      const unsigned long long old =
          atomicAdd(&xg[c[t]], (unsigned long long)(unsigned)term32(a[t], rs) << 32);
      z = fmaf(a[t], __uint_as_float((unsigned)old), z);
    } else {
      if constexpr (MODE != kPassAt) z = fmaf(a[t], xs[c[t]], z);
      if constexpr (MODE != kPassA) atomicAdd(&gs[c[t]], term32(a[t], rs));
    }
  }
}

// Slice of wavefront wv in round k of a unit's slices (longest first): even
// rounds in wavefront order, odd rounds reversed, so that the wavefronts of a
// workgroup get nearly equal shares of a sorted list.
template <int W>
__device__ __forceinline__ int snake(int s0, int k, int wv) {
  return s0 + k * W + ((k & 1) ? (W - 1 - wv) : wv);
}

// FP16 values: at most 64 VGPRs (eight wavefronts per SIMD), so that with
// 33 KB of LDS four 8-wavefront workgroups share a CU and all 1024 units of a
// 512^2 pass run at once (left to itself the compiler takes 80-88 VGPRs,
// which holds a CU to two workgroups); 2% faster at 512^2 and 1024^2, where
// the LDS work bounds the pass.  With FP32 values the cap left the 512^2
// pass unchanged and made the 1024^2 one 4% slower, so they keep the
// compiler's choice.
template <typename VT>
constexpr int kFusedWavesPerSimd = sizeof(VT) == 2 ? 8 : 1;

template <typename VT, bool NARROW, int W, int MODE>
__global__ __launch_bounds__(64 * W, kFusedWavesPerSimd<VT>) void k_fused(
    TileGeom g, const int32_t* __restrict__ uorder, const int32_t* __restrict__ sbeg,
    const int32_t* __restrict__ sng, const int64_t* __restrict__ soff,
    const int32_t* __restrict__ sray, const uint16_t* __restrict__ srank,
    const uint16_t* __restrict__ sbase, const void* __restrict__ col,
    const VT* __restrict__ val, const float* __restrict__ x,
    const float* __restrict__ r, const unsigned* __restrict__ rmax_in, unsigned* rmax_zero,
    float* __restrict__ zp, float* __restrict__ gp, int64_t r_int, int64_t c_int, double smax,
    double amax, bool slotz) {
  // the tile of x and the fixed-point A^T r image: two arrays, or (FP16
  // values, both products: there the LDS work bounds the pass, and halving
  // its instructions took it from 0.1825 to 0.175 ms at 512^2; with FP32
  // values it made the pass slower, 0.233 to 0.238 ms) one array of 64-bit
  // cells
  constexpr bool MERGED = MODE == kPassBoth && sizeof(VT) == 2;
  __shared__ unsigned long long lds[kFTA];
  float* xs = reinterpret_cast<float*>(lds);
  int* gs = reinterpret_cast<int*>(lds) + kFTA;
  unsigned long long* xg = lds;
  constexpr int NT = 64 * W;
  const int u = uorder[blockIdx.x];  // largest units first
  const int tile = u / g.Q, q = u - tile * g.Q;
  const int per = g.FTh * g.FTw;
  const int d = tile / per;
  const int tt = tile - d * per;
  const int ftr = tt / g.FTw, ftc = tt - ftr * g.FTw;
  const int64_t xbase = (int64_t)d * g.slice_px;
  const int tid = threadIdx.x;
  const int wv = tid >> 6, lane = tid & 63;
  const int s0 = sbeg[u], s1 = sbeg[u + 1];
  // the next kernel of the epoch gathers the next residual's |r| maximum here
  if (rmax_zero && blockIdx.x == 0 && tid == 0) *rmax_zero = 0u;
  for (int i = tid; i < kFTA; i += NT) {
    if constexpr (MERGED) {
      xg[i] = 0ull;
    } else {
      if constexpr (MODE != kPassAt) xs[i] = 0.f;
      if constexpr (MODE != kPassA) gs[i] = 0;
    }
  }
  __syncthreads();
  if constexpr (MODE != kPassAt)
    for (int i = tid; i < kFT * kFT; i += NT) {
      const int b = i >> 6, w = i & 63;
      const int tr8 = ftr * 8 + (b >> 3), tc8 = ftc * 8 + (b & 7);
      if (tr8 < g.Ht && tc8 < g.Wt) {
        const float xv = x[xbase + ((int64_t)(tr8 * g.Wt + tc8) << 6) + w];
        const int ai = (((b >> 3) << 3) + (w >> 3)) * kFTS + ((b & 7) << 3) + (w & 7);
        if constexpr (MERGED)
          xg[ai] = (unsigned long long)__float_as_uint(xv);
        else
          xs[ai] = xv;
      }
    }
  const float rmax = MODE == kPassA ? 0.f : __uint_as_float(*rmax_in);
  const int e = fixed_exponent32(smax, amax, rmax);
  // a residual with an infinite or NaN entry has no fixed-point scale: its
  // terms are left out and the partials carry a NaN instead, so the
  // divergence reaches x and the next residual
  const bool rbad = !(rmax <= 3.40282347e38f);
  __syncthreads();
  // the next slice's table entries and its r value load while a slice streams
  int k = 0, s = snake<W>(s0, 0, wv);
  SliceMeta cur = slice_meta(sray, srank, sbase, sng, soff, s, s1, lane);
  float rcur = (MODE != kPassA && cur.rho >= 0) ? r[cur.rho] : 0.f;
  while (s < s1) {
    const int sn = snake<W>(s0, k + 1, wv);
    const SliceMeta nxt = slice_meta(sray, srank, sbase, sng, soff, sn, s1, lane);
    const float rs = rbad ? 0.f : ldexpf(rcur, e);
    const int64_t base = cur.base;
    const int ng = cur.ng;
    float z0 = 0.f, z1 = 0.f;
    float rnext = 0.f;
    int ap = cur.a0;
    bool fetched = false;
    int j = 0;
    for (; j + 3 < ng; j += 4) {
      ColRaw<NARROW> c0, c1, c2, c3;
      float a0[4], a1[4], a2[4], a3[4];
      load_group<VT, NARROW>(col, val, base + (int64_t)j * 256, c0, a0);
      load_group<VT, NARROW>(col, val, base + (int64_t)(j + 1) * 256, c1, a1);
      load_group<VT, NARROW>(col, val, base + (int64_t)(j + 2) * 256, c2, a2);
      load_group<VT, NARROW>(col, val, base + (int64_t)(j + 3) * 256, c3, a3);
      if (!fetched) {
        fetched = true;
        if (MODE != kPassA && nxt.rho >= 0) rnext = r[nxt.rho];
      }
      group_step<NARROW, MODE, MERGED>(xs, gs, xg, c0, a0, rs, z0, ap);
      group_step<NARROW, MODE, MERGED>(xs, gs, xg, c1, a1, rs, z1, ap);
      group_step<NARROW, MODE, MERGED>(xs, gs, xg, c2, a2, rs, z0, ap);
      group_step<NARROW, MODE, MERGED>(xs, gs, xg, c3, a3, rs, z1, ap);
    }
    for (; j + 1 < ng; j += 2) {
      ColRaw<NARROW> c0, c1;
      float a0[4], a1[4];
      load_group<VT, NARROW>(col, val, base + (int64_t)j * 256, c0, a0);
      load_group<VT, NARROW>(col, val, base + (int64_t)(j + 1) * 256, c1, a1);
      if (!fetched) {
        fetched = true;
        if (MODE != kPassA && nxt.rho >= 0) rnext = r[nxt.rho];
      }
      group_step<NARROW, MODE, MERGED>(xs, gs, xg, c0, a0, rs, z0, ap);
      group_step<NARROW, MODE, MERGED>(xs, gs, xg, c1, a1, rs, z1, ap);
    }
    if (j < ng) {
      ColRaw<NARROW> c0;
      float a0[4];
      load_group<VT, NARROW>(col, val, base + (int64_t)j * 256, c0, a0);
      group_step<NARROW, MODE, MERGED>(xs, gs, xg, c0, a0, rs, z0, ap);
    }
    if (MODE != kPassA && !fetched && nxt.rho >= 0) rnext = r[nxt.rho];
    // row sum of the lane's segment: at its slot (one 256-byte store per
    // slice; the reduce gathers a ray's segments through pslot) or at
    // [rank][ray] (the reduce reads rank planes with unit stride)
    if constexpr (MODE != kPassAt) {
      if (slotz)
        zp[(int64_t)s * 64 + lane] = z0 + z1;
      else if (cur.rho >= 0)
        zp[(int64_t)cur.rk * r_int + cur.rho] = z0 + z1;
    }
    ++k;
    s = sn;
    cur = nxt;
    rcur = rnext;
  }
  __syncthreads();
  if constexpr (MODE == kPassA) return;
  for (int i = tid; i < kFT * kFT; i += NT) {
    const int b = i >> 6, w = i & 63;
    const int tr8 = ftr * 8 + (b >> 3), tc8 = ftc * 8 + (b & 7);
    if (tr8 < g.Ht && tc8 < g.Wt) {
      const int a = (((b >> 3) << 3) + (w >> 3)) * kFTS + ((b & 7) << 3) + (w & 7);
      gp[(int64_t)q * c_int + xbase + ((int64_t)(tr8 * g.Wt + tc8) << 6) + w] =
          rbad ? __uint_as_float(0x7fc00000u)
               : ldexpf((float)(MERGED ? (int)(xg[a] >> 32) : gs[a]), -e);
    }
  }
}

// ---------------------------------------------------------------------------
// Several right-hand sides (batches of images and the slices of a volume,
// vectors [rows][S] with the RHS index fastest, S a multiple of 4).  The same
// store and units; a workgroup takes one unit for one column of kMrC = 4
// consecutive RHS.  The unit's tile of x for those RHS goes to LDS as
// 4-vectors.  Each slice's 64 segments are taken a half at a time, two lanes
// per segment (two RHS each): a lane forms its segment's row sums for its two
// RHS in registers and adds its terms a * r_k of A^T r into the tile in LDS as
// 32-bit fixed-point integers, the pair packed into one 64-bit integer atomic
// (the high word absorbs the low word's borrow, so the two sums separate
// exactly at the end).  Scale 2^e_k from max |r_k|, the largest column sum of
// |A| and the largest |a|: every sum stays below 2^30 in magnitude and every
// term below 2^21, so one FMA with 1.5 * 2^23 rounds a term to an integer (a
// term's rounding is below 2^-31 of the largest possible sum; integer
// additions make the result independent of the order of the atomics).  Launch slots are mapped so that the columns of one unit run side
// by side on one XCD (workgroups are dealt to the 8 XCDs in turn): the unit's
// stored entries are read from HBM once per pass and from that XCD's L2 by
// its other columns.  Partials: A x per (segment, RHS) at [rank][ray][S],
// A^T r per (chunk, pixel, RHS) at [chunk][pixel][S].
// ---------------------------------------------------------------------------
constexpr int kMrC = 4;      // RHS per workgroup
constexpr int kXcds = 8;     // workgroups are dealt to the XCDs round robin

template <typename VT, bool NARROW, int W>
__global__ __launch_bounds__(64 * W) void k_fused_mr(
    TileGeom g, const int32_t* __restrict__ uorder, const int32_t* __restrict__ sbeg,
    const int32_t* __restrict__ sng, const int64_t* __restrict__ soff,
    const int32_t* __restrict__ sray, const uint16_t* __restrict__ srank,
    const uint16_t* __restrict__ sbase, const void* __restrict__ col,
    const VT* __restrict__ val, const float* __restrict__ x, const float* __restrict__ r,
    const unsigned* __restrict__ rmax_in, float* __restrict__ zp, float* __restrict__ gp,
    int64_t r_int, int64_t c_int, int S, int64_t units, double smax, double amax) {
  // tile of x as [cell][4 RHS] and the A^T r sums as [cell][2 pairs] of
  // packed 64-bit integers (low word: the pair's first RHS, high word: the
  // second plus the first's borrow): lane pairs of a segment address 16
  // consecutive bytes of one cell
  __shared__ f32x4 xs[kFTA];
  __shared__ unsigned long long gs[kFTA * 2];
  constexpr int NT = 64 * W;
  const int RC = S / kMrC;
  const int64_t nwg = units * RC;
  const int64_t per_xcd = (nwg + kXcds - 1) / kXcds;
  const int64_t slot = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  if (slot >= nwg) return;  // padding of the grid to a multiple of the XCD count
  const int u = uorder[slot / RC];  // largest units first
  const int cc = (int)(slot % RC);  // RHS column: RHS cc * 4 .. cc * 4 + 3
  const int tile = u / g.Q, q = u - tile * g.Q;
  const int per = g.FTh * g.FTw;
  const int d = tile / per;
  const int tt = tile - d * per;
  const int ftr = tt / g.FTw, ftc = tt - ftr * g.FTw;
  const int64_t xbase = (int64_t)d * g.slice_px;
  const int tid = threadIdx.x;
  const int wv = tid >> 6, lane = tid & 63;
  const int hp = lane & 1, sg = lane >> 1;  // this lane's RHS pair and segment of a half
  const int s0 = sbeg[u], s1 = sbeg[u + 1];
  for (int i = tid; i < kFTA; i += NT) {
    xs[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    gs[2 * i] = 0ull;
    gs[2 * i + 1] = 0ull;
  }
  __syncthreads();
  for (int i = tid; i < kFT * kFT; i += NT) {
    const int b = i >> 6, w = i & 63;
    const int tr8 = ftr * 8 + (b >> 3), tc8 = ftc * 8 + (b & 7);
    if (tr8 < g.Ht && tc8 < g.Wt)
      xs[(((b >> 3) << 3) + (w >> 3)) * kFTS + ((b & 7) << 3) + (w & 7)] =
          *reinterpret_cast<const f32x4*>(
              x + (xbase + ((int64_t)(tr8 * g.Wt + tc8) << 6) + w) * S + cc * kMrC);
  }
  const int rhs0 = cc * kMrC + 2 * hp;  // this lane's RHS: rhs0, rhs0 + 1
  const float rm0 = __uint_as_float(rmax_in[rhs0]), rm1 = __uint_as_float(rmax_in[rhs0 + 1]);
  const int e0 = fixed_exponent32(smax, amax, rm0);
  const int e1 = fixed_exponent32(smax, amax, rm1);
  // a residual with a non-finite entry has no scale: its terms are left out
  // (they would spill into the other word of the pair) and its partials carry
  // a NaN
  const bool bad0 = !(rm0 <= 3.40282347e38f), bad1 = !(rm1 <= 3.40282347e38f);
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const f32x2* xsp = reinterpret_cast<const f32x2*>(xs) + hp;
  unsigned long long* gsp = gs + hp;
  __syncthreads();
  // work item = (slice, half): the half's 32 segments, 2 lanes each; the next
  // item's table entries and r load while an item streams
  auto meta = [&](int s, int hf) {
    SliceMeta m{-1, 0, 0, 0, 0};
    if (s < s1) {
      const int L = hf * 32 + sg;
      m.rho = sray[(int64_t)s * 64 + L];
      m.rk = srank[(int64_t)s * 64 + L];
      m.a0 = sbase ? sbase[(int64_t)s * 64 + L] : 0;
      m.ng = sng[s];
      m.base = soff[s] + L * 4;
    }
    return m;
  };
  auto rpair = [&](int rho) {
    return rho >= 0 ? *reinterpret_cast<const f32x2*>(r + (int64_t)rho * S + rhs0)
                    : f32x2{0.f, 0.f};
  };
  int kk = 0, hf = 0, s = snake<W>(s0, 0, wv);
  SliceMeta cur = meta(s, 0);
  f32x2 rcur = rpair(cur.rho);
  while (s < s1) {
    const int hn = hf ^ 1;
    const int sn = hn == 0 ? snake<W>(s0, kk + 1, wv) : s;
    const SliceMeta nxt = meta(sn, hn);
    const f32x2 rnext = rpair(nxt.rho);
    const float rs0 = bad0 ? 0.f : ldexpf(rcur[0], e0), rs1 = bad1 ? 0.f : ldexpf(rcur[1], e1);
    const int64_t base = cur.base;
    const int ng = cur.ng;
    float za = 0.f, zb = 0.f, zc = 0.f, zd = 0.f;
    int ap = cur.a0;
    auto step = [&](const ColRaw<NARROW>& raw, const float (&a)[4], float& z0, float& z1) {
      int c[4];
      if constexpr (NARROW) {
        c[0] = ap + (int)(raw & 255u);
        c[1] = c[0] + (int)((raw >> 8) & 255u);
        c[2] = c[1] + (int)((raw >> 16) & 255u);
        c[3] = c[2] + (int)(raw >> 24);
        ap = c[3];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) c[e] = raw[e];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const f32x2 xv = xsp[c[e] * 2];
        z0 = fmaf(a[e], xv[0], z0);
        z1 = fmaf(a[e], xv[1], z1);
        // the two rounded terms' bit patterns side by side, minus the magic
        // constant in each word: a 64-bit subtraction leaves t0 + 2^32 t1 in
        // two's complement (the high word takes the low word's borrow)
        const unsigned b0 = __float_as_uint(fmaf(a[e], rs0, kMagic32));
        const unsigned b1 = __float_as_uint(fmaf(a[e], rs1, kMagic32));
        const unsigned long long pk = (((unsigned long long)b1 << 32) | b0) - kMagicPair;
        atomicAdd(gsp + c[e] * 2, pk);
      }
    };
    int j = 0;
    for (; j + 1 < ng; j += 2) {
      ColRaw<NARROW> c0, c1;
      float a0[4], a1[4];
      load_group<VT, NARROW>(col, val, base + (int64_t)j * 256, c0, a0);
      load_group<VT, NARROW>(col, val, base + (int64_t)(j + 1) * 256, c1, a1);
      step(c0, a0, za, zb);
      step(c1, a1, zc, zd);
    }
    if (j < ng) {
      ColRaw<NARROW> c0;
      float a0[4];
      load_group<VT, NARROW>(col, val, base + (int64_t)j * 256, c0, a0);
      step(c0, a0, za, zb);
    }
    if (cur.rho >= 0)
      *reinterpret_cast<f32x2*>(zp + ((int64_t)cur.rk * r_int + cur.rho) * S + rhs0) =
          f32x2{za + zc, zb + zd};
    if (hn == 0) ++kk;
    hf = hn;
    s = sn;
    cur = nxt;
    rcur = rnext;
  }
  __syncthreads();
  // NT is even, so every thread flushes its own pair hp
  for (int i = tid; i < kFT * kFT * 2; i += NT) {
    const int px = i >> 1;
    const int b = px >> 6, w = px & 63;
    const int tr8 = ftr * 8 + (b >> 3), tc8 = ftc * 8 + (b & 7);
    if (tr8 < g.Ht && tc8 < g.Wt) {
      const int a = (((b >> 3) << 3) + (w >> 3)) * kFTS + ((b & 7) << 3) + (w & 7);
      const unsigned long long tot = gsp[a * 2];
      const int lo = (int)(unsigned)(tot & 0xffffffffull);
      const int hi = (int)(unsigned)((tot - (unsigned long long)(long long)lo) >> 32);
      const f32x2 o{bad0 ? __uint_as_float(0x7fc00000u) : ldexpf((float)lo, -e0),
                    bad1 ? __uint_as_float(0x7fc00000u) : ldexpf((float)hi, -e1)};
      *reinterpret_cast<f32x2*>(
          gp + ((int64_t)q * c_int + xbase + ((int64_t)(tr8 * g.Wt + tc8) << 6) + w) * S +
          rhs0) = o;
    }
  }
}

// Maximum of v over a 256-thread block into *out: one atomic per block at
// most, and only while it raises the stored value (every block of a launch
// reading and updating one word serialises on one L2 channel otherwise).
__device__ __forceinline__ void block_max_to(unsigned v, unsigned* out) {
  __shared__ unsigned wmax[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, off));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    v = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    if (v > __atomic_load_n(out, __ATOMIC_RELAXED)) atomicMax(out, v);
  }
}

// Rays: out_r = y - sum of the ray's segment partials zp[rank][ray] in rank
// order, or the sum when y is NULL; max |out_r| is gathered in *rmax_out (as
// the bit pattern of a non-negative float, which orders like the value).  Pixels: out_x = xadd + scale * (sum of the Q chunk
// partials, in chunk order), or scale * sum when xadd is NULL.
__global__ __launch_bounds__(256) void k_fz_reduce(
    const int32_t* __restrict__ poff, const int32_t* __restrict__ pslot,
    const float* __restrict__ zp, const float* __restrict__ y, float* __restrict__ out_r,
    unsigned* rmax_out, int64_t r_int, const float* __restrict__ gp, int Q,
    const float* __restrict__ xadd, float scale, float* __restrict__ out_x, int64_t c_int,
    int64_t lo, int64_t hi) {
  float m = 0.f;
  bool bad = false;  // a NaN residual (fmaxf would drop it)
  for (int64_t i = lo + (int64_t)blockIdx.x * 256 + threadIdx.x; i < hi;
       i += (int64_t)gridDim.x * 256) {
    if (i < r_int) {
      const int b = poff[i], n = poff[i + 1] - b;
      float a = 0.f;
      int k = 0;
      if (pslot) {
        // the segments' row sums at their slots, gathered in rank order
        const int32_t* ps = pslot + b;
        for (; k + 3 < n; k += 4) {
          const float v0 = zp[ps[k]], v1 = zp[ps[k + 1]], v2 = zp[ps[k + 2]], v3 = zp[ps[k + 3]];
          a += v0;
          a += v1;
          a += v2;
          a += v3;
        }
        for (; k < n; ++k) a += zp[ps[k]];
      } else {
        const float* z = zp + i;
        for (; k + 3 < n; k += 4) {
          const float v0 = z[(int64_t)k * r_int], v1 = z[(int64_t)(k + 1) * r_int];
          const float v2 = z[(int64_t)(k + 2) * r_int], v3 = z[(int64_t)(k + 3) * r_int];
          a += v0;
          a += v1;
          a += v2;
          a += v3;
        }
        for (; k < n; ++k) a += z[(int64_t)k * r_int];
      }
      const float o = y ? y[i] - a : a;
      out_r[i] = o;
      m = fmaxf(m, fabsf(o));
      bad = bad || (o != o);
    } else {
      const int64_t p = i - r_int;
      // chunk order, 8 loads in flight (a loop of dependent single loads
      // left this half of the reduce latency-bound)
      const float* g = gp + p;
      float a = 0.f;
      int k = 0;
      for (; k + 7 < Q; k += 8) {
        float v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = g[(int64_t)(k + t) * c_int];
#pragma unroll
        for (int t = 0; t < 8; ++t) a += v[t];
      }
      for (; k < Q; ++k) a += g[(int64_t)k * c_int];
      out_x[p] = xadd ? fmaf(scale, a, xadd[p]) : scale * a;
    }
  }
  if (rmax_out && lo < r_int)
    block_max_to(bad ? 0x7fc00000u : __float_as_uint(m), rmax_out);  // NaN > +inf
}

// Several RHS ([rows][S], RHS fastest): rays out_r = y - sum of the segment
// partials zp[rank][ray][k] in rank order, per-RHS max |out_r| into
// rmax_out[k]; pixels out_x = xadd + scale * sum over chunks of
// gp[q][pixel][k].  Index space [0, r_int S) rays then [r_int S, (r_int +
// c_int) S) pixels; the grid stride is a multiple of S, so a thread keeps one
// RHS k throughout.
__global__ __launch_bounds__(256) void k_fz_reduce_mr(
    const int32_t* __restrict__ poff, const float* __restrict__ zp,
    const float* __restrict__ y, float* __restrict__ out_r, unsigned* rmax_out,
    int64_t r_int, const float* __restrict__ gp, int Q, const float* __restrict__ xadd,
    float scale, float* __restrict__ out_x, int64_t c_int, int S, int64_t lo, int64_t hi) {
  __shared__ unsigned smx[256];
  float m = 0.f;
  bool bad = false;
  const int64_t rS = r_int * S, cS = c_int * S;
  const int64_t i0 = lo + (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t i = i0; i < hi; i += (int64_t)gridDim.x * 256) {
    if (i < rS) {
      const int64_t ray = i / S;
      const int n = poff[ray + 1] - poff[ray];
      const float* z = zp + i;
      float a = 0.f;
      int k = 0;
      for (; k + 3 < n; k += 4) {
        const float v0 = z[(int64_t)k * rS], v1 = z[(int64_t)(k + 1) * rS];
        const float v2 = z[(int64_t)(k + 2) * rS], v3 = z[(int64_t)(k + 3) * rS];
        a += v0;
        a += v1;
        a += v2;
        a += v3;
      }
      for (; k < n; ++k) a += z[(int64_t)k * rS];
      const float o = y ? y[i] - a : a;
      out_r[i] = o;
      m = fmaxf(m, fabsf(o));
      bad = bad || (o != o);
    } else {
      const int64_t pk = i - rS;
      const float* g = gp + pk;
      float a = 0.f;
      int k = 0;
      for (; k + 7 < Q; k += 8) {
        float v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = g[(int64_t)(k + t) * cS];
#pragma unroll
        for (int t = 0; t < 8; ++t) a += v[t];
      }
      for (; k < Q; ++k) a += g[(int64_t)k * cS];
      out_x[pk] = xadd ? fmaf(scale, a, xadd[pk]) : scale * a;
    }
  }
  if (!rmax_out || lo >= rS) return;
  const unsigned bits = bad ? 0x7fc00000u : __float_as_uint(m);  // NaN > +inf
  const int kr = (int)(i0 % S);
  if (S <= 256) {
    // threads of the block with the same RHS meet in LDS first
    smx[threadIdx.x] = 0u;
    __syncthreads();
    if (i0 < rS) atomicMax(&smx[kr], bits);
    __syncthreads();
    if ((int)threadIdx.x < S && smx[threadIdx.x] > __atomic_load_n(rmax_out + threadIdx.x,
                                                                  __ATOMIC_RELAXED))
      atomicMax(rmax_out + threadIdx.x, smx[threadIdx.x]);
  } else if (i0 < rS && bits > __atomic_load_n(rmax_out + kr, __ATOMIC_RELAXED)) {
    atomicMax(rmax_out + kr, bits);
  }
}

__global__ void k_fz_zero_n(unsigned* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// per-RHS max |v| of a [rows][S] array into out[S] (zeroed by the preceding launch)
__global__ __launch_bounds__(256) void k_fz_absmax_mr(const float* __restrict__ v, int64_t n,
                                                      int S, unsigned* out) {
  __shared__ unsigned smx[256];
  float m = 0.f;
  bool bad = false;
  const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t i = i0; i < n * S; i += (int64_t)gridDim.x * 256) {
    const float o = v[i];
    m = fmaxf(m, fabsf(o));
    bad = bad || (o != o);
  }
  const unsigned bits = bad ? 0x7fc00000u : __float_as_uint(m);
  const int kr = (int)(i0 % S);
  if (S <= 256) {
    smx[threadIdx.x] = 0u;
    __syncthreads();
    atomicMax(&smx[kr], bits);
    __syncthreads();
    if ((int)threadIdx.x < S && smx[threadIdx.x] > __atomic_load_n(out + threadIdx.x,
                                                                  __ATOMIC_RELAXED))
      atomicMax(out + threadIdx.x, smx[threadIdx.x]);
  } else if (bits > __atomic_load_n(out + kr, __ATOMIC_RELAXED)) {
    atomicMax(out + kr, bits);
  }
}

__global__ void k_fz_zero_u32(unsigned* p) { *p = 0u; }

// max |v| over n floats into *out (zeroed by the preceding launch)
__global__ __launch_bounds__(256) void k_fz_absmax(const float* __restrict__ v, int64_t n,
                                                   unsigned* out) {
  float m = 0.f;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const float o = v[i];
    m = fmaxf(m, fabsf(o));
    bad = bad || (o != o);
  }
  block_max_to(bad ? 0x7fc00000u : __float_as_uint(m), out);
}

template <typename VT, int W, int MODE>
static void launch_fused_m(const bsgd_fused& F, const VT* val, const float* x, const float* r,
                           const unsigned* rmax_in, unsigned* rmax_zero, float* zp, float* gp,
                           hipStream_t s) {
  if (F.narrow)
    k_fused<VT, true, W, MODE><<<(unsigned)F.g.units(), 64 * W, 0, s>>>(
        F.g, F.uorder, F.sbeg, F.sng, F.soff, F.sray, F.srank, F.sbase, F.col8, val, x, r,
        rmax_in, rmax_zero, zp, gp, F.plan->L.r_int, F.plan->L.c_int, F.smax, F.amax, F.slotz);
  else
    k_fused<VT, false, W, MODE><<<(unsigned)F.g.units(), 64 * W, 0, s>>>(
        F.g, F.uorder, F.sbeg, F.sng, F.soff, F.sray, F.srank, nullptr, F.col, val, x, r,
        rmax_in, rmax_zero, zp, gp, F.plan->L.r_int, F.plan->L.c_int, F.smax, F.amax, F.slotz);
}

template <typename VT, int W>
static void launch_fused_w(const bsgd_fused& F, int mode, const VT* val, const float* x,
                           const float* r, const unsigned* rmax_in, unsigned* rmax_zero,
                           float* zp, float* gp, hipStream_t s) {
  switch (mode) {
    case kPassA: launch_fused_m<VT, W, kPassA>(F, val, x, r, rmax_in, rmax_zero, zp, gp, s); break;
    case kPassAt: launch_fused_m<VT, W, kPassAt>(F, val, x, r, rmax_in, rmax_zero, zp, gp, s); break;
    default: launch_fused_m<VT, W, kPassBoth>(F, val, x, r, rmax_in, rmax_zero, zp, gp, s); break;
  }
}

template <typename VT>
static void launch_fused_vt(const bsgd_fused& F, int mode, const VT* val, const float* x,
                            const float* r, const unsigned* rmax_in, unsigned* rmax_zero,
                            float* zp, float* gp, hipStream_t s) {
  switch (F.waves) {
    case 2: launch_fused_w<VT, 2>(F, mode, val, x, r, rmax_in, rmax_zero, zp, gp, s); break;
    case 4: launch_fused_w<VT, 4>(F, mode, val, x, r, rmax_in, rmax_zero, zp, gp, s); break;
    default: launch_fused_w<VT, 8>(F, mode, val, x, r, rmax_in, rmax_zero, zp, gp, s); break;
  }
}

bool fused_has_f16(const bsgd_fused* F) { return F->val16 != nullptr; }

// Slot-order row sums save the pass its scattered per-segment stores (one
// coalesced store per slice instead of 64 lines touched), and cost the ray
// reduce one gather per segment; that reduce runs beside the pixel half and
// the prox, which hide it while the partials stay cache-sized.
bool fused_slot_partials(const bsgd_fused* F) { return F->slices * 64 <= kSlotPartialsMax; }
const bsgd_plan* fused_plan(const bsgd_fused* F) { return F->plan; }

size_t fused_partials(const bsgd_fused* F, int S, FusedPartials* fp, void* ws) {
  Carver cv(ws);
  // row-sum partials: [rank][ray] planes, or (one RHS) one per slot
  size_t za = (size_t)std::max(F->maxrank, 1) * F->plan->L.r_int * S;
  if (S == 1) za = std::max<size_t>(za, (size_t)std::max<int64_t>(F->slices, 1) * 64);
  float* a = cv.take<float>(za);
  float* b = cv.take<float>((size_t)F->g.Q * F->plan->L.c_int * S);
  unsigned* m = cv.take<unsigned>(2 * (size_t)S);
  if (fp) {
    fp->zp = a;
    fp->gp = b;
    fp->rmax = m;
  }
  return align_up(cv.off, kAlign);
}

hipError_t launch_fused_absmax(const float* v, int64_t n, unsigned* out, hipStream_t s) {
  k_fz_zero_u32<<<1, 1, 0, s>>>(out);
  k_fz_absmax<<<std::min<unsigned>(grid_for(n), 1024), 256, 0, s>>>(v, n, out);
  return hipGetLastError();
}

hipError_t launch_fused_pass(const bsgd_fused* F, bsgd_valtype vt, const float* x,
                             const float* r, const unsigned* rmax_in, unsigned* rmax_zero,
                             float* zp, float* gp, hipStream_t s, int mode, int waves,
                             bool slotz) {
  bsgd_fused G = *F;  // the launch's wave count: the caller's, else the store's
  G.waves = waves > 0 ? waves : F->waves;
  G.slotz = slotz;
  if (vt == BSGD_VAL_F16)
    launch_fused_vt<__half>(G, mode, F->val16, x, r, rmax_in, rmax_zero, zp, gp, s);
  else
    launch_fused_vt<float>(G, mode, F->val, x, r, rmax_in, rmax_zero, zp, gp, s);
  return hipGetLastError();
}

// grid for the several-RHS reduce kernels: a multiple of S / 256 blocks, so that
// the grid stride (blocks * 256) is a multiple of S
static unsigned grid_mr(int64_t n, int S) {
  const unsigned mult = (unsigned)std::max(1, S / 256);
  unsigned b = std::min<unsigned>(grid_for(n), 1024);
  return (b + mult - 1) / mult * mult;
}

hipError_t launch_fused_zero(unsigned* p, int n, hipStream_t s) {
  k_fz_zero_n<<<1, 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_fused_absmax_mr(const float* v, int64_t n, int S, unsigned* out,
                                  hipStream_t s) {
  k_fz_zero_n<<<1, 256, 0, s>>>(out, S);
  k_fz_absmax_mr<<<grid_mr(n * S, S), 256, 0, s>>>(v, n, S, out);
  return hipGetLastError();
}

template <typename VT, int W>
static void launch_mr_w(const bsgd_fused& F, const VT* val, const float* x, const float* r,
                        const unsigned* rmax_in, float* zp, float* gp, int64_t ri, int64_t ci,
                        int S, int64_t units, unsigned grid, hipStream_t s) {
  if (F.narrow)
    k_fused_mr<VT, true, W><<<grid, 64 * W, 0, s>>>(F.g, F.uorder, F.sbeg, F.sng, F.soff, F.sray,
                                                    F.srank, F.sbase, F.col8, val, x, r, rmax_in,
                                                    zp, gp, ri, ci, S, units, F.smax, F.amax);
  else
    k_fused_mr<VT, false, W><<<grid, 64 * W, 0, s>>>(F.g, F.uorder, F.sbeg, F.sng, F.soff,
                                                     F.sray, F.srank, nullptr, F.col, val, x, r,
                                                     rmax_in, zp, gp, ri, ci, S, units, F.smax,
                                                     F.amax);
}

hipError_t launch_fused_pass_mr(const bsgd_fused* F, bsgd_valtype vt, int S, const float* x,
                                const float* r, const unsigned* rmax_in, float* zp, float* gp,
                                hipStream_t s, int waves) {
  const int64_t units = F->g.units();
  const int64_t nwg = units * (S / kMrC);
  const unsigned grid = (unsigned)((nwg + kXcds - 1) / kXcds * kXcds);
  const int64_t ri = F->plan->L.r_int, ci = F->plan->L.c_int;
  // one workgroup per CU (its LDS): 16 wavefronts unless 8 are asked for
  const bool w16 = waves != 8;
  if (vt == BSGD_VAL_F16) {
    if (w16)
      launch_mr_w<__half, 16>(*F, F->val16, x, r, rmax_in, zp, gp, ri, ci, S, units, grid, s);
    else
      launch_mr_w<__half, 8>(*F, F->val16, x, r, rmax_in, zp, gp, ri, ci, S, units, grid, s);
  } else {
    if (w16)
      launch_mr_w<float, 16>(*F, F->val, x, r, rmax_in, zp, gp, ri, ci, S, units, grid, s);
    else
      launch_mr_w<float, 8>(*F, F->val, x, r, rmax_in, zp, gp, ri, ci, S, units, grid, s);
  }
  return hipGetLastError();
}

hipError_t launch_fused_reduce_mr(const bsgd_fused* F, int S, const float* zp, const float* gp,
                                  const float* y, float* out_r, unsigned* rmax_out,
                                  const float* xadd, float scale, float* out_x, hipStream_t s,
                                  int parts) {
  const Layout& L = F->plan->L;
  const int64_t rS = L.r_int * S, cS = L.c_int * S;
  const int64_t lo = (parts & kReduceRays) ? 0 : rS;
  const int64_t hi = (parts & kReducePixels) ? rS + cS : rS;
  if (hi <= lo) return hipSuccess;
  k_fz_reduce_mr<<<grid_mr(hi - lo, S), 256, 0, s>>>(F->poff, zp, y, out_r, rmax_out, L.r_int,
                                                     gp, F->g.Q, xadd, scale, out_x, L.c_int, S,
                                                     lo, hi);
  return hipGetLastError();
}

hipError_t launch_fused_reduce(const bsgd_fused* F, const float* zp, const float* gp,
                               const float* y, float* out_r, unsigned* rmax_out,
                               const float* xadd, float scale, float* out_x, hipStream_t s,
                               int parts, bool slotz) {
  const Layout& L = F->plan->L;
  const int64_t lo = (parts & kReduceRays) ? 0 : L.r_int;
  const int64_t hi = (parts & kReducePixels) ? L.r_int + L.c_int : L.r_int;
  if (hi <= lo) return hipSuccess;
  const unsigned blocks = std::min<unsigned>(grid_for(hi - lo), 1024);
  k_fz_reduce<<<blocks, 256, 0, s>>>(F->poff, slotz ? F->pslot : nullptr, zp, y, out_r,
                                     rmax_out, L.r_int, gp, F->g.Q, xadd, scale, out_x, L.c_int,
                                     lo, hi);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Build
// ---------------------------------------------------------------------------
struct FusedCounts {
  bool narrow = true;  // 8-bit address steps
  int64_t pairs = 0;
  int64_t slices = 0;  // upper bound until the build has sorted the segments
  int64_t bound = 0;   // upper bound of the stored entries
  int maxrank = 0, maxlen = 0, maxstep = 0;
};

// Count pass: segments per ray (into plan->scratch64, then scanned in place:
// the rays' segment offsets), most segments of a ray and longest segment.
// Bounds for the workspace: a unit with n segments has ceil(n / 64) slices,
// so there are at most pairs / 64 + units; slices are sorted longest first,
// so slice k >= 1 of a unit is no longer than the shortest segment of the
// full slice k - 1 and stores at most that slice's entries, plus up to 3
// padding entries per lane (groups of 4) -- entries <= nnz + units *
// 64 * (maxlen + 3) + 192 * slices.  Synchronises.
static bsgd_status fused_count(const bsgd_plan* p, const TileGeom& g, bool wide, hipStream_t s,
                               FusedCounts& fc) {
  FusedCountCache& cc = p->fz_count;
  if (cc.valid && cc.Q == g.Q && cc.wide == wide) {
    // bsgd_fused_workspace_size counted this geometry and synchronised;
    // scratch64 still holds the offsets
    fc.narrow = cc.narrow;
    fc.pairs = cc.pairs;
    fc.slices = cc.slices;
    fc.bound = cc.bound;
    fc.maxrank = cc.maxrank;
    fc.maxlen = cc.maxlen;
    fc.maxstep = cc.maxstep;
    return BSGD_OK;
  }
  cc.valid = false;
  const Layout& L = p->L;
  const int64_t units = g.units();
  int32_t* words = reinterpret_cast<int32_t*>(p->vin);  // maxc, maxlen, maxstep
  int* err = reinterpret_cast<int*>(words + 4);
  k_fill_i32<<<1, 256, 0, s>>>(words, 5);
  BSGD_LAUNCH_CHECK();
  const unsigned blocks = (unsigned)((L.r_int * 64 + 255) / 256);
  const WalkSrc w = walk_src(p);
  launch_walk<0>(w, g, L, blocks, s, nullptr, nullptr, L.r_int, p->scratch64, words, words + 1,
                 words + 2, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                 nullptr, nullptr, nullptr, err);
  BSGD_LAUNCH_CHECK();
  BSGD_HIP(exclusive_scan_i64(p->scratch64, p->scratch64, L.r_int, p->scan_tmp, s));
  int32_t hw[5] = {0, 0, 0, 0, 0};
  BSGD_HIP(hipMemcpyAsync(&fc.pairs, p->scratch64 + L.r_int, sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
  BSGD_HIP(hipMemcpyAsync(hw, words, sizeof(hw), hipMemcpyDeviceToHost, s));
  BSGD_HIP(hipStreamSynchronize(s));
  if (hw[4] != 0) {
    set_error("A's column indices are out of range or not ascending within a row");
    return BSGD_ERR_INVALID;
  }
  fc.maxrank = hw[0];
  fc.maxlen = hw[1];
  fc.maxstep = hw[2];
  fc.narrow = !wide && fc.maxstep < 256;
  BSGD_REQUIRE(fc.maxrank < 65536, "a ray crosses %d tiles (at most 65535)", fc.maxrank);
  fc.slices = (fc.pairs + 63) / 64 + units;
  fc.bound = w.nnz + units * 64 * ((int64_t)fc.maxlen + 3) + 192 * fc.slices;
  BSGD_REQUIRE(fc.slices * 64 < ((int64_t)1 << 31), "too many slices (%lld)",
               (long long)fc.slices);
  cc.Q = g.Q;
  cc.wide = wide;
  cc.narrow = fc.narrow;
  cc.pairs = fc.pairs;
  cc.slices = fc.slices;
  cc.bound = fc.bound;
  cc.maxrank = fc.maxrank;
  cc.maxlen = fc.maxlen;
  cc.maxstep = fc.maxstep;
  cc.valid = true;
  return BSGD_OK;
}

struct FusedTemps {
  uint64_t *key = nullptr, *key2 = nullptr;
  int32_t *idx = nullptr, *idx2 = nullptr, *pray = nullptr, *slen = nullptr, *pos = nullptr;
  uint16_t* pbase = nullptr;
  int64_t *first = nullptr, *last = nullptr, *sng256 = nullptr, *scan_tmp = nullptr;
  int64_t* pdst = nullptr;
  int* err = nullptr;
  void* cub = nullptr;
  size_t cub_bytes = 0;
};

static int key_bits(int64_t units) {
  int b = 1;
  while (((int64_t)1 << b) < units * kKeyLen) ++b;
  return b;
}

static size_t fused_layout(const bsgd_plan* p, const TileGeom& g, const FusedCounts& fc,
                           void* ws, bsgd_fused* F, FusedTemps* T) {
  Carver cv(ws);
  const Layout& L = p->L;
  const int64_t units = g.units();
  const int64_t nslots = std::max<int64_t>(fc.slices, 1) * 64;
  const int64_t np = std::max<int64_t>(fc.pairs, 1);
  const bool f16 = (p->flags & BSGD_PLAN_F16) != 0;
  F->sbeg = cv.take<int32_t>(units + 1);
  F->uorder = cv.take<int32_t>(units);
  F->sng = cv.take<int32_t>(std::max<int64_t>(fc.slices, 1));
  F->soff = cv.take<int64_t>(fc.slices + 1);
  F->sray = cv.take<int32_t>(nslots);
  F->poff = cv.take<int32_t>(L.r_int + 1);
  F->pslot = cv.take<int32_t>(np);
  T->pos = F->pslot;  // the build's placement fills it
  F->srank = cv.take<uint16_t>(nslots);
  F->narrow = fc.narrow;
  if (fc.narrow) {
    F->col8 = cv.take<uint8_t>(std::max<int64_t>(fc.bound, 4));
    F->sbase = cv.take<uint16_t>(nslots);
  } else {
    F->col = cv.take<uint16_t>(std::max<int64_t>(fc.bound, 4));
  }
  F->val = cv.take<float>(std::max<int64_t>(fc.bound, 4));
  F->val16 = f16 ? cv.take<__half>(std::max<int64_t>(fc.bound, 4)) : nullptr;
  F->xin = cv.take<float>(L.c_int);
  F->xadd = cv.take<float>(L.c_int);
  F->go = cv.take<float>(L.c_int);
  F->rin = cv.take<float>(L.r_int);
  F->yin = cv.take<float>(L.r_int);
  F->zo = cv.take<float>(L.r_int);
  // build-only temporaries
  T->key = cv.take<uint64_t>(np);
  T->key2 = cv.take<uint64_t>(np);
  T->pdst = cv.take<int64_t>(np);
  T->idx = cv.take<int32_t>(np);
  T->idx2 = cv.take<int32_t>(np);
  T->pray = cv.take<int32_t>(np);
  T->pbase = cv.take<uint16_t>(np);
  T->slen = cv.take<int32_t>(nslots);
  T->first = cv.take<int64_t>(units);
  T->last = cv.take<int64_t>(units);
  T->sng256 = cv.take<int64_t>(fc.slices + 1);
  T->scan_tmp = cv.take<int64_t>(scan_tmp_count(fc.slices) + 1);
  T->err = cv.take<int>(64);
  size_t cub_bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, cub_bytes, (const uint64_t*)nullptr,
                                           (uint64_t*)nullptr, (const int32_t*)nullptr,
                                           (int32_t*)nullptr, (int)np, 0, 32 + key_bits(units));
  T->cub_bytes = std::max<size_t>(cub_bytes, 1);
  T->cub = cv.take<char>(T->cub_bytes);
  return align_up(cv.off, kAlign);
}

static bsgd_status fused_check(const bsgd_plan* p, int chunks, unsigned flags, TileGeom* g) {
  BSGD_REQUIRE(p != nullptr, "plan is NULL");
  BSGD_REQUIRE((flags & ~BSGD_FUSED_WIDE) == 0, "unknown single-pass flags 0x%x", flags);
  BSGD_REQUIRE(chunks >= 0, "chunks must be >= 0 (0: automatic)");
  const Layout& L = p->L;
  if ((L.Wt + 7) / 8 > 64) {
    set_error("the single-pass form supports images up to 4096 pixels wide");
    return BSGD_ERR_UNSUPPORTED;
  }
  *g = tile_geom(L, chunks);
  BSGD_REQUIRE(g->Q <= g->ngroups, "chunks (%d) exceeds the number of ray groups (%lld)", g->Q,
               (long long)g->ngroups);
  BSGD_REQUIRE(g->units() * kKeyLen < ((int64_t)1 << 32) &&
                   g->units() < std::max(L.r_int, L.c_int),
               "too many tiles x chunks (%lld)", (long long)g->units());
  BSGD_REQUIRE(walk_src(p).nnz < ((int64_t)1 << 31), "too many entries");
  if ((p->flags & BSGD_PLAN_SINGLE_PASS_ONLY) && (int64_t)L.H * L.W > ((int64_t)1 << 24)) {
    // A's natural columns are split into (row, column) with an FP32 reciprocal
    set_error("a plan without a block store supports slices of at most 2^24 pixels");
    return BSGD_ERR_UNSUPPORTED;
  }
  return BSGD_OK;
}

}  // namespace bsgd

using namespace bsgd;

extern "C" bsgd_status bsgd_fused_workspace_size(const bsgd_plan* plan, int chunks,
                                                 unsigned flags, hipStream_t stream,
                                                 size_t* bytes) {
  clear_error();
  BSGD_REQUIRE(bytes != nullptr, "bytes is NULL");
  TileGeom g;
  bsgd_status st = fused_check(plan, chunks, flags, &g);
  if (st != BSGD_OK) return st;
  FusedCounts fc;
  st = fused_count(plan, g, (flags & BSGD_FUSED_WIDE) != 0, stream, fc);
  if (st != BSGD_OK) return st;
  bsgd_fused tmp;
  FusedTemps T;
  *bytes = fused_layout(plan, g, fc, nullptr, &tmp, &T);
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_fused_create(const bsgd_plan* plan, int chunks, unsigned flags,
                                         void* workspace, size_t workspace_bytes,
                                         hipStream_t stream, bsgd_fused** out) {
  clear_error();
  BSGD_REQUIRE(workspace && out, "NULL argument");
  BSGD_REQUIRE(((uintptr_t)workspace % kAlign) == 0, "workspace must be 256-byte aligned");
  TileGeom g;
  bsgd_status st = fused_check(plan, chunks, flags, &g);
  if (st != BSGD_OK) return st;
  FusedCounts fc;
  st = fused_count(plan, g, (flags & BSGD_FUSED_WIDE) != 0, stream, fc);
  if (st != BSGD_OK) return st;
  bsgd_fused* F = new bsgd_fused();
  F->plan = plan;
  F->g = g;
  FusedTemps T;
  const size_t need = fused_layout(plan, g, fc, workspace, F, &T);
  if (workspace_bytes < need) {
    delete F;
    set_error("single-pass workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return BSGD_ERR_WORKSPACE;
  }
  const Layout& L = plan->L;
  const WalkSrc A = walk_src(plan);
  const int64_t units = g.units();
  const unsigned wblocks = (unsigned)((L.r_int * 64 + 255) / 256);
  auto fail = [&](bsgd_status s) {
    delete F;
    return s;
  };
  auto hip_fail = [&](hipError_t e, const char* what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    delete F;
    return BSGD_ERR_HIP;
  };
  hipError_t e;
  e = hipMemsetAsync(T.err, 0, sizeof(int), stream);
  if (e != hipSuccess) return hip_fail(e, "single-pass build set-up");
  // per-ray segment offsets (plan->scratch64 holds their exclusive scan)
  k_i64_to_i32<<<grid_for(L.r_int + 1), 256, 0, stream>>>(plan->scratch64, F->poff, L.r_int + 1);
  k_fz_unit_init<<<grid_for(units), 256, 0, stream>>>(T.first, T.last, units);
  if (fc.pairs > 0) {
    launch_walk<1>(A, g, L, wblocks, stream, nullptr, nullptr, L.r_int, nullptr, nullptr,
                   nullptr, nullptr, plan->scratch64, T.key, T.idx, T.pray, T.pbase, nullptr,
                   nullptr, nullptr, nullptr, nullptr, nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "segment pass");
    size_t cb = T.cub_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(T.cub, cb, T.key, T.key2, T.idx, T.idx2, (int)fc.pairs,
                                           0, 32 + key_bits(units), stream);
    if (e != hipSuccess) return hip_fail(e, "segment sort");
    k_fz_unit_bounds<<<grid_for(fc.pairs), 256, 0, stream>>>(T.key2, fc.pairs, T.first, T.last);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "unit bounds");
  }
  // slices per unit, launch order (most slices first) and slice offsets on the host
  std::vector<int64_t> hf(units), hl(units);
  e = hipMemcpyAsync(hf.data(), T.first, sizeof(int64_t) * units, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hl.data(), T.last, sizeof(int64_t) * units, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "unit bounds");
  std::vector<int32_t> sbeg(units + 1, 0), uorder(units);
  int64_t nsl = 0, npl = 0;
  for (int64_t u = 0; u < units; ++u) {
    const int64_t n = hl[u] - hf[u] + 1;
    sbeg[u] = (int32_t)nsl;
    nsl += (n + 63) / 64;
    npl += n;
    uorder[u] = (int32_t)u;
  }
  sbeg[units] = (int32_t)nsl;
  if (npl != fc.pairs || nsl > fc.slices) {
    set_error("single-pass build: %lld sorted segments in %lld slices (expected %lld, <= %lld)",
              (long long)npl, (long long)nsl, (long long)fc.pairs, (long long)fc.slices);
    return fail(BSGD_ERR_INVALID);
  }
  std::stable_sort(uorder.begin(), uorder.end(), [&](int32_t a, int32_t b) {
    return sbeg[a + 1] - sbeg[a] > sbeg[b + 1] - sbeg[b];
  });
  fc.slices = nsl;
  const int64_t nslots = nsl * 64;
  e = hipMemcpyAsync(F->sbeg, sbeg.data(), sizeof(int32_t) * (units + 1), hipMemcpyHostToDevice,
                     stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(F->uorder, uorder.data(), sizeof(int32_t) * units, hipMemcpyHostToDevice,
                       stream);
  if (e != hipSuccess) return hip_fail(e, "single-pass build upload");
  if (fc.pairs > 0) {
    k_fz_init_slots<<<grid_for(nslots), 256, 0, stream>>>(F->sray, T.slen, F->sbase, nslots);
    k_fz_place<<<grid_for(fc.pairs), 256, 0, stream>>>(T.key2, T.idx2, T.pray, plan->scratch64,
                                                       fc.pairs, T.first, F->sbeg, nslots,
                                                       T.pbase, T.pos, F->sray, F->srank,
                                                       F->sbase, T.slen, F->sng, T.sng256,
                                                       T.err);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "slot placement");
  }
  e = exclusive_scan_i64(T.sng256, F->soff, fc.slices, T.scan_tmp, stream);
  if (e != hipSuccess) return hip_fail(e, "slice offsets");
  int64_t total = 0;
  int h_err = 0;
  e = hipMemcpyAsync(&total, F->soff + fc.slices, sizeof(int64_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&h_err, T.err, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "slice offsets");
  if (h_err) {  // a segment without a slot: stop before any entry is scattered
    set_error("single-pass build found inconsistent slots (code %d)", h_err);
    return fail(BSGD_ERR_INVALID);
  }
  if (total > fc.bound) {
    set_error("single-pass store needs %lld entries, bound %lld", (long long)total,
              (long long)fc.bound);
    return fail(BSGD_ERR_INVALID);
  }
  if (fc.pairs > 0) {
    k_fz_dst<<<grid_for(fc.pairs), 256, 0, stream>>>(T.pos, fc.pairs, F->soff, F->sng, T.pdst);
    launch_walk<2>(A, g, L, (wblocks + 7) / 8 * 8, stream, A.val, A.val16, L.r_int, nullptr,
                   nullptr, nullptr, nullptr, plan->scratch64, nullptr, nullptr, nullptr,
                   nullptr, T.pdst, F->col, F->col8, F->val, F->val16, T.err);
    k_fz_pad<<<grid_for(nslots), 256, 0, stream>>>(T.slen, F->sng, F->soff, nslots, F->col,
                                                   F->col8, F->val, F->val16);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "entry fill");
  }
  e = hipMemcpyAsync(&h_err, T.err, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "single-pass build");
  if (h_err) {
    set_error("single-pass build found inconsistent slots (code %d)", h_err);
    return fail(BSGD_ERR_INVALID);
  }
  F->pairs = fc.pairs;
  F->maxrank = fc.maxrank;
  // the plan's FP64 column sums of |A| and max |a|.  FP16 values round |a|
  // up by at most 2^-11 relative: sums stay below 2^30 (1 + 2^-11) < 2^31
  // and terms below 2^21 (1 + 2^-11) < 2^22, where the FMA rounding of a
  // term still holds
  F->smax = plan->smax;
  F->amax = plan->amax;
  F->slices = fc.slices;
  F->entries = total;
  F->cap = fc.bound;
  *out = F;
  return BSGD_OK;
}

extern "C" void bsgd_fused_destroy(bsgd_fused* F) { delete F; }

extern "C" bsgd_status bsgd_fused_shape(const bsgd_fused* F, int* tiles, int* chunks,
                                        int64_t* segments, int64_t* slices, int64_t* entries,
                                        int* col_bytes) {
  clear_error();
  BSGD_REQUIRE(F && tiles && chunks && segments && slices && entries && col_bytes,
               "NULL argument");
  *col_bytes = F->narrow ? 1 : 2;
  *tiles = (int)F->g.tiles();
  *chunks = F->g.Q;
  *segments = F->pairs;
  *slices = F->slices;
  *entries = F->entries;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_fused_set_waves(bsgd_fused* F, int waves) {
  clear_error();
  BSGD_REQUIRE(F != nullptr, "fused store is NULL");
  BSGD_REQUIRE(waves == 2 || waves == 4 || waves == 8, "waves must be 2, 4 or 8");
  F->waves = waves;
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_fused_partials_size(const bsgd_fused* F, size_t* bytes) {
  clear_error();
  BSGD_REQUIRE(F && bytes, "NULL argument");
  *bytes = fused_partials(F, 1, nullptr, nullptr);
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_fused_partials_size_rhs(const bsgd_fused* F, int nrhs,
                                                    size_t* bytes) {
  clear_error();
  BSGD_REQUIRE(F && bytes, "NULL argument");
  BSGD_REQUIRE(nrhs == 1 || (nrhs >= kMrC && nrhs % kMrC == 0),
               "nrhs must be 1 or a multiple of %d", kMrC);
  *bytes = fused_partials(F, nrhs, nullptr, nullptr);
  return BSGD_OK;
}

extern "C" bsgd_status bsgd_fused_apply(const bsgd_fused* F, bsgd_valtype vt, const float* x,
                                        const float* y, const float* r, const float* xadd,
                                        float mu, float* out_r, float* out_x, void* partials,
                                        size_t partials_bytes, hipStream_t stream) {
  clear_error();
  BSGD_REQUIRE(F && x && r && out_r && out_x && partials, "NULL argument");
  BSGD_REQUIRE(vt == BSGD_VAL_F32 || (vt == BSGD_VAL_F16 && F->val16),
               "value type not available in this store");
  BSGD_REQUIRE(std::isfinite(mu), "mu must be finite");
  FusedPartials fp;
  const size_t need = fused_partials(F, 1, &fp, partials);
  if (partials_bytes < need) {
    set_error("partials workspace has %zu bytes, needs %zu", partials_bytes, need);
    return BSGD_ERR_WORKSPACE;
  }
  const Layout& L = F->plan->L;
  BSGD_HIP(permute_in(L, kPixels, x, F->xin, stream));
  BSGD_HIP(permute_in(L, kRays, r, F->rin, stream));
  if (y) BSGD_HIP(permute_in(L, kRays, y, F->yin, stream));
  if (xadd) BSGD_HIP(permute_in(L, kPixels, xadd, F->xadd, stream));
  BSGD_HIP(launch_fused_absmax(F->rin, L.r_int, fp.rmax, stream));
  BSGD_HIP(launch_fused_pass(F, vt, F->xin, F->rin, fp.rmax, nullptr, fp.zp, fp.gp, stream));
  BSGD_HIP(launch_fused_reduce(F, fp.zp, fp.gp, y ? F->yin : nullptr, F->zo, nullptr,
                               xadd ? F->xadd : nullptr, xadd ? 2.0f * mu : 2.0f, F->go, stream));
  BSGD_HIP(permute_out(L, kRays, F->zo, out_r, stream));
  BSGD_HIP(permute_out(L, kPixels, F->go, out_x, stream));
  return BSGD_OK;
}

// Render-path kernels for gfx950: clear, render, resolve.
//
// Method: Schuetz, Kerbl & Wimmer, "Software Rasterization of 2 Billion Points
// in Real Time", Sec. 3.2 (one workgroup per batch, batch frustum culling,
// point rasterization with a 64-bit depth|index atomic minimum and an
// early-depth test) and Sec. 3.3 (adaptive 10/20/30-bit coordinates, Eq. 1,
// visibility-buffer resolve).
//
// Arithmetic contract (bit for bit; compiled with -ffp-contract=off):
//  * per-batch decisions in binary64, plain + - * /, left to right, never fused;
//  * per point: X = (float)F (RNE), hx/hy/hw = three fmaf chains in a fixed
//    order, pixel = exact floor of hx/hw, key = bits(hw) << 32 | index.
//
// Two kernels per view.  The classify kernel runs the per-batch prologue of
// Sec. 3.2 / 3.3 for every batch at once (one thread per batch): it projects
// the 8 box corners, culls, picks the precision level, folds the decode into
// the batch matrix, and appends the surviving batches to a compact list with
// a wave ballot.  The persistent render kernel then hands the live batches to
// its workgroups (four waves each) through an atomic work queue.  Classes:
//  CULLED  : some frustum plane has all corners outside by a margin that
//            exceeds every rounding of the per-point evaluation;
//  INSIDE  : all corners strictly inside every plane by that margin and w in
//            [2^-60, 2^60]: every point passes the visibility tests, which are
//            therefore skipped;
//  PARTIAL : w in [2^-60, 2^60] for every point: per-point tests, fast exact
//            floor from a reciprocal;
//  SLOW    : anything else (box reaching w <= 0 or absurd scales): per-point
//            tests, floor of a correctly rounded binary64 quotient.
// All classes give the same result for every point; they differ only in
// which tests are provably redundant.
//
// Combining keys.  If the batch lies in front of the eye and its projected
// box (plus one pixel of margin) covers at most TILE_MAX pixels, the points
// are first combined by minimum in an LDS tile over that box (behind an
// early-depth read of the tile entry); afterwards each covered tile pixel
// goes into the global atomic minimum once.  The minimum is associative and commutative, so this
// equals combining every point globally; it replaces one global round trip
// per point by one per covered pixel.  Larger batches (close to the eye,
// few points per pixel) combine every point globally.
#include "internal.h"

namespace ptr {
namespace {

constexpr int CLS_INSIDE = 0, CLS_PARTIAL = 1, CLS_SLOW = 2;
constexpr int WAVES = 4;
constexpr int THREADS = 64 * WAVES;
constexpr uint32_t TILE_MAX = 4096;  // 32 KiB of 64-bit keys
// Point loads in flight per wave (groups of 256 points); 10,240-point batches
// give each of the four waves exactly ten groups.
#ifndef PREFETCH
#define PREFETCH 5
#endif

// ------------------------------------------------------------------ clear
// Fills the visibility buffer with all-ones (PR_EMPTY), resets the frame's
// work-queue counters and optionally the frame counters.
__global__ void __launch_bounds__(256) k_clear(uint4* __restrict__ vb4, uint64_t n4, uint64_t* __restrict__ vb,
                                               uint64_t npix, DevBlock* __restrict__ dev,
                                               FrameHeader* __restrict__ hdr, int reset_stats) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u);
  for (uint64_t i = tid; i < n4; i += stride) vb4[i] = ones;
  if (tid == 0 && (npix & 1)) vb[npix - 1] = ~0ull;
  if (blockIdx.x == 0) {
    if (hdr && threadIdx.x == 0) hdr->live_count = 0;
    if (hdr && threadIdx.x < RENDER_QUEUES) hdr->queue[threadIdx.x][0] = 0;
    if (reset_stats && threadIdx.x < 16) dev->stats[threadIdx.x] = 0;
  }
}

// ------------------------------------------------------------------ render
template <int K>
__device__ __forceinline__ void decode(uint32_t lw, uint32_t mw, uint32_t hw, float& X, float& Y, float& Z) {
  if constexpr (K == 10) {
    X = (float)(lw & 1023u);
    Y = (float)((lw >> 10) & 1023u);
    Z = (float)((lw >> 20) & 1023u);
  } else if constexpr (K == 20) {
    X = (float)(((lw & 1023u) << 10) | (mw & 1023u));
    Y = (float)((((lw >> 10) & 1023u) << 10) | ((mw >> 10) & 1023u));
    Z = (float)((((lw >> 20) & 1023u) << 10) | ((mw >> 20) & 1023u));
  } else {
    X = (float)(((lw & 1023u) << 20) | ((mw & 1023u) << 10) | (hw & 1023u));
    Y = (float)((((lw >> 10) & 1023u) << 20) | (((mw >> 10) & 1023u) << 10) | ((hw >> 10) & 1023u));
    Z = (float)((((lw >> 20) & 1023u) << 20) | (((mw >> 20) & 1023u) << 10) | ((hw >> 20) & 1023u));
  }
}

// Frame-wide and batch-wide values of the point loop (uniform: SGPRs).
struct Loop {
  float P[3][3], t[3];
  uint32_t W, H;
  uint32_t cx, cy;  // 0x4B000000 + tile origin (x0, y0), in VGPRs: pixel_fast yields tile coordinates
  uint32_t tw, th;  // tile rectangle size (tiled batches)
  uint32_t tw8;     // tile row pitch in bytes
  uint64_t* vb;
  // high-quality shading pass only
  float window;     // depth window factor
  uint64_t* acc;    // global sums, two words per pixel
  float* thr;       // LDS tile of thresholds fl32(closest depth * window)
};

// Projection of one decoded point (the three fmaf chains, fixed order).
struct Proj {
  float hx, hy, hw;
};
__device__ __forceinline__ Proj project(const Loop& L, float X, float Y, float Z) {
  Proj p;
  p.hx = __builtin_fmaf(L.P[0][2], Z, __builtin_fmaf(L.P[0][1], Y, __builtin_fmaf(L.P[0][0], X, L.t[0])));
  p.hy = __builtin_fmaf(L.P[1][2], Z, __builtin_fmaf(L.P[1][1], Y, __builtin_fmaf(L.P[1][0], X, L.t[1])));
  p.hw = __builtin_fmaf(L.P[2][2], Z, __builtin_fmaf(L.P[2][1], Y, __builtin_fmaf(L.P[2][0], X, L.t[2])));
  return p;
}

// hw > 0, 0 <= hx < W hw, 0 <= hy < H hw, exactly: the fma residuals carry the
// exact sign of hx - W hw (denormals are kept, so nothing underflows to 0).
__device__ __forceinline__ bool visible(const Loop& L, const Proj& p) {
  return (p.hw > 0.0f) & (p.hx >= 0.0f) & (__builtin_fmaf(-(float)L.W, p.hw, p.hx) < 0.0f) & (p.hy >= 0.0f) &
         (__builtin_fmaf(-(float)L.H, p.hw, p.hy) < 0.0f);
}

// floor(hx / hw) - x0 and floor(hy / hw) - y0 for quotients in [0, 2^13), hw
// in [2^-60, 2^60]: fma(hx, rcp(hw), 2^23) rounds the exact product to an
// integer n (the spacing of floats in [2^23, 2^24) is 1) with
// |n - hx/hw| < 1/2 + 2^-9; the exactly signed residual hx - n hw picks n or
// n - 1.  The integer is read from the float's bits (cx = 0x4B000000 + x0),
// the correction is the borrow of the same subtraction.
__device__ __forceinline__ void pixel_fast(const Proj& p, uint32_t cx, uint32_t cy, uint32_t& px, uint32_t& py) {
  const float r = __builtin_amdgcn_rcpf(p.hw);
  const float tx = __builtin_fmaf(p.hx, r, 0x1p23f);
  const float ty = __builtin_fmaf(p.hy, r, 0x1p23f);
  const float ex = __builtin_fmaf(-(tx - 0x1p23f), p.hw, p.hx);
  const float ey = __builtin_fmaf(-(ty - 0x1p23f), p.hw, p.hy);
  unsigned int bo;
  px = __builtin_subc(__float_as_uint(tx), cx, (unsigned int)(ex < 0.0f), &bo);
  py = __builtin_subc(__float_as_uint(ty), cy, (unsigned int)(ey < 0.0f), &bo);
}

// Exact floor of the real quotient for any class: the binary64 quotient of two
// binary32 values below 2^13 never crosses an integer.
__device__ __forceinline__ void pixel_exact(const Proj& p, uint32_t& px, uint32_t& py) {
  px = (uint32_t)floor((double)p.hx / (double)p.hw);
  py = (uint32_t)floor((double)p.hy / (double)p.hw);
}

__device__ __forceinline__ uint64_t make_key(float hw, uint32_t idx) {
  return ((uint64_t)__float_as_uint(hw) << 32) | (uint64_t)idx;
}

struct Words {
  uint4 l, m, h;
  uint4 c;  // colours (shading pass)
};

// Shading sums of one colour: R + G << 32 and B + 1 << 32 (four 32-bit fields
// in two 64-bit words, Sec. 3.6).
__device__ __forceinline__ uint64_t sum_rg(uint32_t c) {
  return (uint64_t)(c & 255u) | ((uint64_t)((c >> 8) & 255u) << 32);
}
__device__ __forceinline__ uint64_t sum_bn(uint32_t c) { return (uint64_t)((c >> 16) & 255u) | (1ull << 32); }

// Shading pass, four consecutive points of one lane: a drawn point joins its
// pixel's sums iff hw <= fl32(closest depth * window).  Tiled batches add into
// the LDS sums (tile) behind the LDS threshold tile; others read the closest
// depth from the visibility buffer and add into the global sums.
template <int K, int CLS, bool TILED>
__device__ __forceinline__ void four_points_acc(const Loop& L, uint64_t* tile, const Words& w, uint32_t nvalid) {
  const uint32_t Lw[4] = {w.l.x, w.l.y, w.l.z, w.l.w};
  const uint32_t Mw[4] = {w.m.x, w.m.y, w.m.z, w.m.w};
  const uint32_t Hw[4] = {w.h.x, w.h.y, w.h.z, w.h.w};
  const uint32_t Cw[4] = {w.c.x, w.c.y, w.c.z, w.c.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float X, Y, Z;
    decode<K>(Lw[j], Mw[j], Hw[j], X, Y, Z);
    const Proj p = project(L, X, Y, Z);
    bool ok = (uint32_t)j < nvalid;
    if constexpr (CLS != CLS_INSIDE) ok = ok && visible(L, p);
    uint32_t px, py;
    if constexpr (CLS == CLS_SLOW)
      pixel_exact(p, px, py);
    else
      pixel_fast(p, L.cx, L.cy, px, py);
    if constexpr (TILED) {
      const uint32_t e = __umul24(py, L.tw) + px;
      if (ok && p.hw <= L.thr[e]) {
        __hip_atomic_fetch_add(&tile[2 * e], sum_rg(Cw[j]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&tile[2 * e + 1], sum_bn(Cw[j]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    } else {
      ok = ok && (px < L.W) && (py < L.H);
      const uint32_t off = __umul24(py, L.W) + px;
      if (ok) {
        const uint64_t k = __hip_atomic_load(L.vb + off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p.hw <= __uint_as_float((uint32_t)(k >> 32)) * L.window) {
          __hip_atomic_fetch_add(L.acc + 2 * (uint64_t)off, sum_rg(Cw[j]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_add(L.acc + 2 * (uint64_t)off + 1, sum_bn(Cw[j]), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
}

// Four consecutive points of one lane.
template <int K, int CLS, bool TILED, bool ACC = false>
__device__ __forceinline__ void four_points(const Loop& L, uint64_t* tile, const Words& w, uint32_t i0,
                                            uint32_t nvalid, uint32_t& natom) {
  if constexpr (ACC) {
    four_points_acc<K, CLS, TILED>(L, tile, w, nvalid);
    return;
  }
  const uint32_t Lw[4] = {w.l.x, w.l.y, w.l.z, w.l.w};
  const uint32_t Mw[4] = {w.m.x, w.m.y, w.m.z, w.m.w};
  const uint32_t Hw[4] = {w.h.x, w.h.y, w.h.z, w.h.w};
  if constexpr (TILED) {
    // Tile coordinates straight from the pixel computation.  The classify
    // kernel tiles a batch only when it has proved that the pixel of every
    // point of the batch box lies inside the tile rectangle.
    // Early depth in LDS: the tile entry is read first and the 64-bit LDS
    // atomic is issued only by a key that beats it (a stale read only costs
    // an extra atomic: entries never increase).  Most points of a densely
    // covered pixel lose this test, which removes most of the atomics and
    // their same-address serialisation.
    uint8_t* const tb = reinterpret_cast<uint8_t*>(tile);
    uint32_t ad[4];
    uint64_t key[4], old[4];
    bool ok[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float X, Y, Z;
      decode<K>(Lw[j], Mw[j], Hw[j], X, Y, Z);
      const Proj p = project(L, X, Y, Z);
      ok[j] = (uint32_t)j < nvalid;
      if constexpr (CLS != CLS_INSIDE) ok[j] = ok[j] && visible(L, p);
      uint32_t lx, ly;
      pixel_fast(p, L.cx, L.cy, lx, ly);
      key[j] = make_key(p.hw, i0 + j);
      ad[j] = __umul24(ly, L.tw8) + (lx << 3);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (CLS == CLS_INSIDE) {
        // Every point of an INSIDE batch box (padding lanes decode to points
        // of the box too) maps into the tile: the read needs no guard.
        old[j] = __hip_atomic_load(reinterpret_cast<uint64_t*>(tb + ad[j]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        old[j] = 0;
        if (ok[j])
          old[j] = __hip_atomic_load(reinterpret_cast<uint64_t*>(tb + ad[j]), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (ok[j] && key[j] < old[j])
        __hip_atomic_fetch_min(reinterpret_cast<uint64_t*>(tb + ad[j]), key[j], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    uint32_t off[4];
    uint64_t key[4], old[4];
    bool ok[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float X, Y, Z;
      decode<K>(Lw[j], Mw[j], Hw[j], X, Y, Z);
      const Proj p = project(L, X, Y, Z);
      ok[j] = (uint32_t)j < nvalid;
      if constexpr (CLS != CLS_INSIDE) ok[j] = ok[j] && visible(L, p);
      uint32_t px, py;
      if constexpr (CLS == CLS_SLOW)
        pixel_exact(p, px, py);
      else
        pixel_fast(p, L.cx, L.cy, px, py);
      // Never address outside the image, whatever the class proofs say.
      ok[j] = ok[j] && (px < L.W) && (py < L.H);
      off[j] = __umul24(py, L.W) + px;
      key[j] = make_key(p.hw, i0 + j);
    }
    // all early-depth reads first, then the atomics
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      old[j] = 0;
      if (ok[j]) old[j] = __hip_atomic_load(L.vb + off[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (ok[j] && key[j] < old[j]) {
        __hip_atomic_fetch_min(L.vb + off[j], key[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        natom++;
      }
    }
  }
}

// The coordinate streams of the cloud (low, medium, high words).
struct Streams {
  const uint32_t* low;
  const uint32_t* med;
  const uint32_t* high;
  const uint32_t* colors;  // shading pass only
};

template <int K, bool ACC = false>
__device__ __forceinline__ Words load_group(const Streams& a, uint32_t first, uint32_t g, uint32_t lane) {
  const uint32_t q = first / 4 + g * 64 + lane;  // first is a multiple of 4
  Words w;
  w.l = reinterpret_cast<const uint4*>(a.low)[q];
  if constexpr (K >= 20) w.m = reinterpret_cast<const uint4*>(a.med)[q];
  else w.m = make_uint4(0, 0, 0, 0);
  if constexpr (K == 30) w.h = reinterpret_cast<const uint4*>(a.high)[q];
  else w.h = make_uint4(0, 0, 0, 0);
  if constexpr (ACC) w.c = reinterpret_cast<const uint4*>(a.colors)[q];
  else w.c = make_uint4(0, 0, 0, 0);
  return w;
}

// The points of one batch, split over the workgroup's waves: wave w takes the
// groups of 256 points w, w + WAVES, ... (4 consecutive points per lane, one
// 16-byte load per word).  Wave 0 also takes the ragged tail.
template <int K, int CLS, bool TILED, bool ACC = false>
__device__ void raster_points(const Loop& L, const Streams& a, uint64_t* tile, uint32_t first, uint32_t count,
                              uint32_t wave, uint32_t lane, uint32_t& natom) {
  const uint32_t ngrp = count >> 8;
  const uint32_t nj = wave < ngrp ? (ngrp - wave + WAVES - 1) / WAVES : 0;  // this wave's groups
  if (nj > 0) {
    // PREFETCH register sets rotate through the wave's groups; each is
    // reloaded in place right after use, so every load is issued PREFETCH
    // groups ahead of its use.  The body is branch-free: reloads are
    // unconditional and clamped to the wave's last group, and a group
    // index past the end repeats the last group with no valid points.
    // Every wait then counts exactly the loads in flight.
    const uint32_t glast = wave + (nj - 1) * WAVES;
    Words R[PREFETCH];
    uint32_t gi[PREFETCH];
#pragma unroll
    for (int d = 0; d < PREFETCH; ++d) {
      gi[d] = wave + d * WAVES;
      R[d] = load_group<K, ACC>(a, first, min(gi[d], glast), lane);
      // keep the initial loads in the order of their use, the order the
      // loop reissues them in: the loop's waits then count PREFETCH - 1
      // younger loads on every path
      __builtin_amdgcn_sched_barrier(0);
    }
    for (uint32_t j = 0; j < nj; j += PREFETCH) {
#pragma unroll
      for (int d = 0; d < PREFETCH; ++d) {
        const uint32_t g = gi[d];
        four_points<K, CLS, TILED, ACC>(L, tile, R[d], first + min(g, glast) * 256 + lane * 4,
                                        g <= glast ? 4u : 0u, natom);
        gi[d] = g + PREFETCH * WAVES;
        R[d] = load_group<K, ACC>(a, first, min(gi[d], glast), lane);
      }
    }
  }
  const uint32_t rem = count & 255u;
  if (rem && wave == 0) {  // ragged tail of the batch: scalar loads, per-point bounds
    const uint32_t j0 = ngrp * 256 + lane * 4;
    const uint32_t nv = j0 < count ? min(4u, count - j0) : 0u;
    uint32_t l[4] = {0, 0, 0, 0}, m[4] = {0, 0, 0, 0}, h[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if ((uint32_t)j < nv) {
        l[j] = a.low[first + j0 + j];
        if constexpr (K >= 20) m[j] = a.med[first + j0 + j];
        if constexpr (K == 30) h[j] = a.high[first + j0 + j];
        if constexpr (ACC) c[j] = a.colors[first + j0 + j];
      }
    }
    Words t;
    t.l = make_uint4(l[0], l[1], l[2], l[3]);
    t.m = make_uint4(m[0], m[1], m[2], m[3]);
    t.h = make_uint4(h[0], h[1], h[2], h[3]);
    t.c = make_uint4(c[0], c[1], c[2], c[3]);
    four_points<K, CLS, TILED, ACC>(L, tile, t, first + j0, nv, natom);
  }
}

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// A uniform value as a VGPR operand (the pixel subtraction takes its carry
// from an SGPR and may read only one scalar operand).
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x) {
  uint32_t v;
  asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
  return v;
}

// ---------------------------------------------------------------- classify
// The per-batch prologue (Sec. 3.2 culling, Sec. 3.3 precision choice) for one
// batch per thread, in binary64 without contraction:
//  corners  h_r(c) = ((Pm[r][0] cx + Pm[r][1] cy) + Pm[r][2] cz) + Pm[r][3]
//  margin   M_r = 2^-16 max_c (|Pm[r][0] cx| + |Pm[r][1] cy| + |Pm[r][2] cz| + |Pm[r][3]|),
//           which exceeds every rounding of the binary32 per-point evaluation
//           (below 2^-20 of that sum);
//  cull     all corners outside one plane by the margin;
//  level    E = larger side of the projected corners' box (+inf if a corner
//           has w <= 0); 10 bits if E < t10, 20 if E < t20, else 30;
//  fold     P[r][j] = fp32(Pm[r][j] (size_j 2^-k)),
//           t[r] = fp32(((Pm[r][0] min_x + Pm[r][1] min_y) + Pm[r][2] min_z) + Pm[r][3]).
// decide_batch applies it to one batch and one view: returns whether the
// batch is live; out receives its render record, li its level index.
// Projected extent of the cube of a LOD node (8 corners, binary64, left to
// right): +inf if a corner has w <= 0, else the larger side of the screen box
// of the projected corners.
__device__ __forceinline__ double cube_extent(const double (&Pm)[3][4], const LodNode& nd) {
  double umin = __builtin_inf(), umax = -__builtin_inf(), vmin = __builtin_inf(), vmax = -__builtin_inf();
  for (int c = 0; c < 8; ++c) {
    const double cx = (c & 1) ? nd.origin[0] + nd.edge : nd.origin[0];
    const double cy = (c & 2) ? nd.origin[1] + nd.edge : nd.origin[1];
    const double cz = (c & 4) ? nd.origin[2] + nd.edge : nd.origin[2];
    const double hx = ((Pm[0][0] * cx + Pm[0][1] * cy) + Pm[0][2] * cz) + Pm[0][3];
    const double hy = ((Pm[1][0] * cx + Pm[1][1] * cy) + Pm[1][2] * cz) + Pm[1][3];
    const double hw = ((Pm[2][0] * cx + Pm[2][1] * cy) + Pm[2][2] * cz) + Pm[2][3];
    if (!(hw > 0.0)) return __builtin_inf();
    const double u = hx / hw, v = hy / hw;
    umin = fmin(umin, u);
    umax = fmax(umax, u);
    vmin = fmin(vmin, v);
    vmax = fmax(vmax, v);
  }
  const double ex = umax - umin, ey = vmax - vmin;
  return ex > ey ? ex : ey;
}

// node: the batch's LOD node or nullptr.  LOD culling (Sec. 3.5): with
// lod_px > 0, a batch of a node below the root is culled iff its node's cube
// projects to less than lod_px pixels.
__device__ __forceinline__ bool decide_batch(const BatchRec& rec, const double (&Pm)[3][4], uint32_t W, uint32_t Hh,
                                             int32_t precision, int32_t cull, float t10, float t20,
                                             const LodNode* node, float lod_px, LiveBatch& out, bool& culled,
                                             int& li) {
  bool live = false;
  double H[3][8], M[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double amax = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double cx = (double)((c & 1) ? rec.mx[0] : rec.mn[0]);
      const double cy = (double)((c & 2) ? rec.mx[1] : rec.mn[1]);
      const double cz = (double)((c & 4) ? rec.mx[2] : rec.mn[2]);
      H[r][c] = ((Pm[r][0] * cx + Pm[r][1] * cy) + Pm[r][2] * cz) + Pm[r][3];
      const double ar = ((fabs(Pm[r][0] * cx) + fabs(Pm[r][1] * cy)) + fabs(Pm[r][2] * cz)) + fabs(Pm[r][3]);
      if (ar > amax) amax = ar;
    }
    M[r] = 0x1p-16 * amax;
  }
  const double Wd = (double)W, Hd = (double)Hh;
  bool behind = true, left = true, right = true, bottom = true, top = true, front = true;
  bool safe = true, ins = true;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    behind = behind && (H[2][c] < -M[2]);
    left = left && (H[0][c] < -M[0]);
    right = right && (H[0][c] - Wd * H[2][c] > M[0] + Wd * M[2]);
    bottom = bottom && (H[1][c] < -M[1]);
    top = top && (H[1][c] - Hd * H[2][c] > M[1] + Hd * M[2]);
    front = front && (H[2][c] > 0.0);
    const bool sc = (H[2][c] - M[2] >= 0x1p-60) && (H[2][c] + M[2] <= 0x1p60);
    safe = safe && sc;
    ins = ins && sc && (H[0][c] > M[0]) && (H[0][c] - Wd * H[2][c] < -(M[0] + Wd * M[2])) && (H[1][c] > M[1]) &&
          (H[1][c] - Hd * H[2][c] < -(M[1] + Hd * M[2]));
  }
  culled = cull && (behind || left || right || bottom || top);
  if (!culled && lod_px > 0.0f && node && node->level > 0) culled = cube_extent(Pm, *node) < (double)lod_px;
  if (!culled) {
    double umin = __builtin_inf(), umax = -__builtin_inf(), vmin = __builtin_inf(), vmax = -__builtin_inf();
    if (front) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const double u = H[0][c] / H[2][c], v = H[1][c] / H[2][c];
        if (u < umin) umin = u;
        if (u > umax) umax = u;
        if (v < vmin) vmin = v;
        if (v > vmax) vmax = v;
      }
    }
    int k;
    if (precision == 10 || precision == 20 || precision == 30) {
      k = precision;
    } else {
      double E = __builtin_inf();
      if (front) {
        const double ex = umax - umin, ey = vmax - vmin;
        E = ex > ey ? ex : ey;
      }
      k = E < (double)t10 ? 10 : (E < (double)t20 ? 20 : 30);
    }
    const int cls = ins ? CLS_INSIDE : (safe ? CLS_PARTIAL : CLS_SLOW);
    // Tile rectangle: the projected corners' box, one pixel wider on each
    // side, clipped to the image (front batches only).  Every point's pixel
    // lies inside it when the binary32 evaluation (hx, hw off by at most
    // M/16 each) moves its quotient by less than half a pixel:
    //   (Mx + max|u| Mw) / 16 / (min_c hw - Mw) < 1/2, and likewise for y.
    uint32_t tiled = 0, x0 = 0, y0 = 0, tw = 0, th = 0;
    double hwmin = H[2][0];
#pragma unroll
    for (int c = 1; c < 8; ++c) hwmin = fmin(hwmin, H[2][c]);
    const double hwlo = hwmin - M[2];
    const bool tight = front && hwlo > 0.0 &&
                       M[0] + fmax(fabs(umin), fabs(umax)) * M[2] < 8.0 * hwlo &&
                       M[1] + fmax(fabs(vmin), fabs(vmax)) * M[2] < 8.0 * hwlo;
    if (tight && cls != CLS_SLOW) {
      const double fx0 = fmax(floor(fmax(umin, -4.0)) - 1.0, 0.0);
      const double fx1 = fmin(floor(fmin(umax, Wd + 4.0)) + 1.0, Wd - 1.0);
      const double fy0 = fmax(floor(fmax(vmin, -4.0)) - 1.0, 0.0);
      const double fy1 = fmin(floor(fmin(vmax, Hd + 4.0)) + 1.0, Hd - 1.0);
      if (fx1 >= fx0 && fy1 >= fy0 && (fx1 - fx0 + 1.0) * (fy1 - fy0 + 1.0) <= (double)TILE_MAX) {
        tiled = 1;
        x0 = (uint32_t)fx0;
        y0 = (uint32_t)fy0;
        tw = (uint32_t)(fx1 - fx0) + 1u;
        th = (uint32_t)(fy1 - fy0) + 1u;
      }
    }
    const double scale = k == 10 ? 0x1p-10 : (k == 20 ? 0x1p-20 : 0x1p-30);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int j = 0; j < 3; ++j) out.P[r][j] = (float)(Pm[r][j] * (((double)rec.mx[j] - (double)rec.mn[j]) * scale));
      out.t[r] = (float)(((Pm[r][0] * (double)rec.mn[0] + Pm[r][1] * (double)rec.mn[1]) +
                          Pm[r][2] * (double)rec.mn[2]) +
                         Pm[r][3]);
    }
    out.first = rec.first;
    out.count = rec.count;
    out.mode = (uint32_t)k | ((uint32_t)cls << 8) | (tiled << 16);
    out.rect_xy = x0 | (y0 << 16);
    out.rect_wh = tw | (th << 16);
    out.pad[0] = out.pad[1] = out.pad[2] = 0;
    live = true;
    li = k / 10 - 1;
  }
  return live;
}

// One batch per thread; live batches are appended to a compact list (wave
// ballot + one atomic per wave).
template <bool CNT>
__global__ void __launch_bounds__(256) k_classify(RenderArgs a) {
  const uint32_t b = blockIdx.x * 256u + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63;
  const bool valid = b < a.nb;
  bool live = false;
  LiveBatch out;
  uint32_t count = 0;
  int li = 0;
  bool culled = false;
  if (valid) {
    const BatchRec rec = a.batches[b];
    count = rec.count;
    live = decide_batch(rec, a.Pm, a.W, a.H, a.precision, a.cull, a.t10, a.t20, a.nodes ? a.nodes + b : nullptr,
                        a.lod_px, out, culled, li);
  }
  if constexpr (CNT) {
    const uint64_t mv = __ballot(valid), mc = __ballot(valid && culled);
    uint64_t pts = live ? count : 0, lp[3] = {0, 0, 0}, lb[3] = {0, 0, 0};
    if (live) {
      lp[li] = count;
      lb[li] = 1;
    }
    for (int o = 32; o > 0; o >>= 1) {
      pts += __shfl_xor(pts, o);
      for (int q = 0; q < 3; ++q) {
        lp[q] += __shfl_xor(lp[q], o);
        lb[q] += __shfl_xor(lb[q], o);
      }
    }
    if (lane == 0 && mv) {
      atomicAdd((unsigned long long*)&a.stats[ST_BATCHES], (unsigned long long)__popcll(mv));
      if (mc) atomicAdd((unsigned long long*)&a.stats[ST_CULLED], (unsigned long long)__popcll(mc));
      if (pts) atomicAdd((unsigned long long*)&a.stats[ST_POINTS], (unsigned long long)pts);
      for (int q = 0; q < 3; ++q) {
        if (lb[q]) atomicAdd((unsigned long long*)&a.stats[ST_LB0 + q], (unsigned long long)lb[q]);
        if (lp[q]) atomicAdd((unsigned long long*)&a.stats[ST_LP0 + q], (unsigned long long)lp[q]);
      }
    }
  }
  const uint64_t m = __ballot(live);
  uint32_t base = 0;
  if (lane == 0 && m) base = atomicAdd(&a.hdr->live_count, (uint32_t)__popcll(m));
  base = __shfl(base, 0);
  if (live) {
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    a.live[base + (uint32_t)__popcll(m & lt)] = out;
  }
}

// Several views: one thread per batch runs the prologue for each view of
// this launch; the records go to fixed slots (batch, view), the batch's live
// views to one run record (wave ballot + one atomic per wave).
template <bool CNT>
__global__ void __launch_bounds__(256) k_classify_views(ClassifyViewsArgs a) {
  const uint32_t b = blockIdx.x * 256u + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63;
  const bool valid = b < a.nb;
  uint64_t mask = 0;
  uint64_t nculled = 0, pts = 0, lp[3] = {0, 0, 0}, lb[3] = {0, 0, 0};
  if (valid) {
    const BatchRec rec = a.batches[b];
    for (uint32_t v = 0; v < a.nchunk; ++v) {
      LiveBatch out;
      bool culled = false;
      int li = 0;
      if (decide_batch(rec, a.v[v].Pm, a.v[v].W, a.v[v].H, a.precision, a.cull, a.t10, a.t20,
                       a.nodes ? a.nodes + b : nullptr, a.lod_px, out, culled, li)) {
        a.sub[(uint64_t)b * a.nviews + a.view0 + v] = out;
        mask |= 1ull << v;
        if constexpr (CNT) {
          pts += rec.count;
          lp[li] += rec.count;
          lb[li] += 1;
        }
      }
      if constexpr (CNT) nculled += culled ? 1u : 0u;
    }
  }
  if constexpr (CNT) {
    uint64_t nbv = valid ? a.nchunk : 0u;
    for (int o = 32; o > 0; o >>= 1) {
      nbv += __shfl_xor(nbv, o);
      nculled += __shfl_xor(nculled, o);
      pts += __shfl_xor(pts, o);
      for (int q = 0; q < 3; ++q) {
        lp[q] += __shfl_xor(lp[q], o);
        lb[q] += __shfl_xor(lb[q], o);
      }
    }
    if (lane == 0 && nbv) {
      atomicAdd((unsigned long long*)&a.stats[ST_BATCHES], (unsigned long long)nbv);
      if (nculled) atomicAdd((unsigned long long*)&a.stats[ST_CULLED], (unsigned long long)nculled);
      if (pts) atomicAdd((unsigned long long*)&a.stats[ST_POINTS], (unsigned long long)pts);
      for (int q = 0; q < 3; ++q) {
        if (lb[q]) atomicAdd((unsigned long long*)&a.stats[ST_LB0 + q], (unsigned long long)lb[q]);
        if (lp[q]) atomicAdd((unsigned long long*)&a.stats[ST_LP0 + q], (unsigned long long)lp[q]);
      }
    }
  }
  const bool live = mask != 0;
  const uint64_t m = __ballot(live);
  uint32_t base = 0;
  if (lane == 0 && m) base = atomicAdd(&a.hdr->live_count, (uint32_t)__popcll(m));
  base = __shfl(base, 0);
  if (live) {
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    Run r;
    r.batch = b;
    r.view0 = a.view0;
    r.mask = mask;
    a.runs[base + (uint32_t)__popcll(m & lt)] = r;
  }
}

// Clears every view's visibility buffer (blockIdx.y = view) unless
// accumulating, and resets the frame's work queue and counters.
__global__ void __launch_bounds__(256) k_clear_views(ClearViewsArgs a) {
  const ViewOut& v = a.v[blockIdx.y];
  if (a.clear) {
    const uint64_t npix = (uint64_t)v.W * v.H, n4 = npix / 2;
    uint4* const vb4 = reinterpret_cast<uint4*>(v.vb);
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint64_t i = tid; i < n4; i += stride) vb4[i] = ones;
    if (tid == 0 && (npix & 1)) v.vb[npix - 1] = ~0ull;
  }
  if (blockIdx.x == 0 && blockIdx.y == 0) {
    if (threadIdx.x == 0) a.hdr->live_count = 0;
    if (threadIdx.x < RENDER_QUEUES) a.hdr->queue[threadIdx.x][0] = 0;
    if (a.reset_stats && threadIdx.x < 16) a.stats[threadIdx.x] = 0;
  }
}

// ------------------------------------------------------------------ render
template <int K, bool TILED, bool ACC = false>
__device__ __forceinline__ void raster_by_class(int cls, const Loop& L, const Streams& a, uint64_t* tile,
                                                uint32_t first, uint32_t count, uint32_t wave, uint32_t lane,
                                                uint32_t& natom) {
  if (cls == CLS_INSIDE)
    raster_points<K, CLS_INSIDE, TILED, ACC>(L, a, tile, first, count, wave, lane, natom);
  else if (cls == CLS_PARTIAL)
    raster_points<K, CLS_PARTIAL, TILED, ACC>(L, a, tile, first, count, wave, lane, natom);
  else if constexpr (!TILED)
    raster_points<K, CLS_SLOW, false, ACC>(L, a, tile, first, count, wave, lane, natom);
}

// One live batch of one view by the whole workgroup: its points into the LDS
// tile (or straight into the global buffer), then the tile flush.  The LDS
// tile is all PR_EMPTY between batches (the flush resets what it reads), so a
// batch needs two barriers: one after its points, one after its flush.
// publish: thread 0 stores next into s_next between the barriers (the
// workgroup reads it after the second one).
__device__ __forceinline__ void render_batch(const LiveBatch& rec, uint32_t W, uint32_t H, uint64_t* vb,
                                             const Streams& st, uint64_t* tile, uint32_t tid, uint32_t wave,
                                             uint32_t lane, bool publish, uint32_t next, uint32_t* s_next,
                                             uint32_t& natom) {
  Loop L;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int j = 0; j < 3; ++j) L.P[r][j] = rec.P[r][j];
    L.t[r] = rec.t[r];
  }
  L.W = W;
  L.H = H;
  L.vb = vb;
  const uint32_t mode = rec.mode, rxy = rec.rect_xy, rwh = rec.rect_wh;
  const uint32_t first = rec.first, count = rec.count;
  const uint32_t x0 = rxy & 0xFFFFu, y0 = rxy >> 16;
  L.tw = rwh & 0xFFFFu;
  L.th = rwh >> 16;
  L.tw8 = L.tw * 8u;
  const int k = (int)(mode & 0xFFu), cls = (int)((mode >> 8) & 0xFFu);
  const bool tiled = (mode >> 16) & 1u;
  L.cx = in_vgpr(uni(0x4B000000u + (tiled ? x0 : 0u)));
  L.cy = in_vgpr(uni(0x4B000000u + (tiled ? y0 : 0u)));
  if (tiled) {
    if (k == 10) raster_by_class<10, true>(cls, L, st, tile, first, count, wave, lane, natom);
    else if (k == 20) raster_by_class<20, true>(cls, L, st, tile, first, count, wave, lane, natom);
    else raster_by_class<30, true>(cls, L, st, tile, first, count, wave, lane, natom);
  } else {
    if (k == 10) raster_by_class<10, false>(cls, L, st, tile, first, count, wave, lane, natom);
    else if (k == 20) raster_by_class<20, false>(cls, L, st, tile, first, count, wave, lane, natom);
    else raster_by_class<30, false>(cls, L, st, tile, first, count, wave, lane, natom);
  }
  __syncthreads();  // the batch's points are all in the tile; s_next has been read
  if (publish && tid == 0) *s_next = next;
  if (tiled) {
    // Flush: every covered tile pixel once into the global buffer, leaving
    // the entry PR_EMPTY for the next batch.  Most covered pixels improve
    // the global minimum, so the atomic is issued without a prior read
    // (no round trip on this path).
    const uint32_t n = L.tw * L.th;
    for (uint32_t e = tid; e < n; e += THREADS) {
      const uint64_t v = tile[e];
      if (v != ~0ull) {
        tile[e] = ~0ull;
        const uint32_t ly = e / L.tw, lx = e - ly * L.tw;
        __hip_atomic_fetch_min(L.vb + ((y0 + ly) * L.W + (x0 + lx)), v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        natom++;
      }
    }
  }
  __syncthreads();  // tile clean again; s_next visible
}

__device__ __forceinline__ void fill_tile(uint64_t* tile, uint32_t tid) {
  const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u);
  for (uint32_t e = tid; e < TILE_MAX / 2; e += THREADS) reinterpret_cast<uint4*>(tile)[e] = ones;
}

template <bool CNT>
__device__ __forceinline__ void add_atomics(uint64_t* stats, uint32_t natom, uint32_t lane) {
  if constexpr (CNT) {
    for (int o = 32; o > 0; o >>= 1) natom += __shfl_xor(natom, o);
    if (lane == 0 && natom) atomicAdd((unsigned long long*)&stats[ST_ATOMICS], (unsigned long long)natom);
  }
}

// Persistent: each workgroup takes live batches from its work queue until it
// is empty.  The next batch is requested while the current one renders.
template <bool CNT>
__global__ void __launch_bounds__(THREADS) k_render(RenderArgs a) {
  __shared__ uint64_t tile[TILE_MAX];
  __shared__ uint32_t s_next;
  const uint32_t tid = threadIdx.x, wave = uni(tid >> 6), lane = tid & 63;
  fill_tile(tile, tid);
  // this workgroup's queue: workgroups are spread over the queues round-robin
  const uint32_t q = blockIdx.x % RENDER_QUEUES;
  uint32_t* const qc = &a.hdr->queue[q][0];
  if (tid == 0) s_next = atomicAdd(qc, 1u) * RENDER_QUEUES + q;
  const uint32_t nlive = a.hdr->live_count;
  const Streams st = {a.low, a.med, a.high, nullptr};
  __syncthreads();
  uint32_t i = uni(s_next);
  uint32_t natom = 0;
  while (i < nlive) {
    // Take the next batch now; the atomic's latency hides behind this batch.
    uint32_t grab = 0;
    if (tid == 0) grab = atomicAdd(qc, 1u) * RENDER_QUEUES + q;
    render_batch(a.live[i], a.W, a.H, a.vb, st, tile, tid, wave, lane, true, grab, &s_next, natom);
    i = uni(s_next);
  }
  add_atomics<CNT>(a.stats, natom, lane);
}

// Several views in one launch: the work items are runs (a batch and its live
// views); the workgroup renders the batch once per view, so its coordinate
// words come from HBM once and from the caches for the further views.
template <bool CNT>
__global__ void __launch_bounds__(THREADS) k_render_views(RenderViewsArgs a) {
  __shared__ uint64_t tile[TILE_MAX];
  __shared__ uint32_t s_next;
  const uint32_t tid = threadIdx.x, wave = uni(tid >> 6), lane = tid & 63;
  fill_tile(tile, tid);
  const uint32_t q = blockIdx.x % RENDER_QUEUES;
  uint32_t* const qc = &a.hdr->queue[q][0];
  if (tid == 0) s_next = atomicAdd(qc, 1u) * RENDER_QUEUES + q;
  const uint32_t nruns = a.hdr->live_count;
  const Streams st = {a.low, a.med, a.high, nullptr};
  __syncthreads();
  uint32_t i = uni(s_next);
  uint32_t natom = 0;
  while (i < nruns) {
    uint32_t grab = 0;
    if (tid == 0) grab = atomicAdd(qc, 1u) * RENDER_QUEUES + q;
    const Run run = a.runs[i];
    uint64_t mask = run.mask;
    bool publish = true;
    while (mask) {
      const uint32_t v = run.view0 + (uint32_t)(__ffsll((unsigned long long)mask) - 1);
      mask &= mask - 1;
      const ViewOut& vo = a.v[v];
      render_batch(a.sub[(uint64_t)run.batch * a.nviews + v], vo.W, vo.H, vo.vb, st, tile, tid, wave, lane, publish,
                   grab, &s_next, natom);
      publish = false;
    }
    i = uni(s_next);
  }
  add_atomics<CNT>(a.stats, natom, lane);
}

// ------------------------------------------------------------------ shading
// High-quality shading (Sec. 3.6), second pass over the live batches of the
// frame's render: every drawn point within the depth window of its pixel
// adds its colour and a count.  Tiled batches whose rectangle fits HQS_TILE
// pixels stage the thresholds of the rectangle in LDS, add into LDS sums and
// flush each covered pixel with two global additions; the others read the
// visibility buffer and add globally per point.  Integer sums: the result
// does not depend on the order of the additions.
constexpr uint32_t HQS_TILE = 1536;  // 6 KiB of thresholds + 24 KiB of sums

__global__ void __launch_bounds__(THREADS) k_accum(RenderArgs a) {
  __shared__ float thr[HQS_TILE];
  __shared__ uint64_t sums[2 * HQS_TILE];
  __shared__ uint32_t s_next;
  const uint32_t tid = threadIdx.x, wave = uni(tid >> 6), lane = tid & 63;
  const uint32_t q = blockIdx.x % RENDER_QUEUES;
  uint32_t* const qc = &a.hdr->queue[q][0];
  if (tid == 0) s_next = atomicAdd(qc, 1u) * RENDER_QUEUES + q;
  const uint32_t nlive = a.hdr->live_count;
  const Streams st = {a.low, a.med, a.high, a.colors};
  __syncthreads();
  uint32_t i = uni(s_next);
  uint32_t natom = 0;
  while (i < nlive) {
    uint32_t grab = 0;
    if (tid == 0) grab = atomicAdd(qc, 1u) * RENDER_QUEUES + q;
    const LiveBatch& rec = a.live[i];
    Loop L;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int j = 0; j < 3; ++j) L.P[r][j] = rec.P[r][j];
      L.t[r] = rec.t[r];
    }
    L.W = a.W;
    L.H = a.H;
    L.vb = a.vb;
    L.window = a.window;
    L.acc = a.accum;
    L.thr = thr;
    const uint32_t mode = rec.mode, rxy = rec.rect_xy, rwh = rec.rect_wh;
    const uint32_t first = rec.first, count = rec.count;
    const uint32_t x0 = rxy & 0xFFFFu, y0 = rxy >> 16;
    L.tw = rwh & 0xFFFFu;
    L.th = rwh >> 16;
    L.tw8 = L.tw * 8u;
    const int k = (int)(mode & 0xFFu), cls = (int)((mode >> 8) & 0xFFu);
    const uint32_t n = L.tw * L.th;
    const bool tiled = ((mode >> 16) & 1u) && n <= HQS_TILE;
    L.cx = in_vgpr(uni(0x4B000000u + (tiled ? x0 : 0u)));
    L.cy = in_vgpr(uni(0x4B000000u + (tiled ? y0 : 0u)));
    if (tiled) {
      for (uint32_t e = tid; e < n; e += THREADS) {
        const uint32_t ly = e / L.tw, lx = e - ly * L.tw;
        const uint64_t key = a.vb[(y0 + ly) * a.W + (x0 + lx)];
        thr[e] = __uint_as_float((uint32_t)(key >> 32)) * a.window;
        sums[2 * e] = 0;
        sums[2 * e + 1] = 0;
      }
      __syncthreads();
      if (k == 10) raster_by_class<10, true, true>(cls, L, st, sums, first, count, wave, lane, natom);
      else if (k == 20) raster_by_class<20, true, true>(cls, L, st, sums, first, count, wave, lane, natom);
      else raster_by_class<30, true, true>(cls, L, st, sums, first, count, wave, lane, natom);
    } else {
      if (k == 10) raster_by_class<10, false, true>(cls, L, st, sums, first, count, wave, lane, natom);
      else if (k == 20) raster_by_class<20, false, true>(cls, L, st, sums, first, count, wave, lane, natom);
      else raster_by_class<30, false, true>(cls, L, st, sums, first, count, wave, lane, natom);
    }
    __syncthreads();  // the batch's sums are complete; s_next has been read
    if (tid == 0) s_next = grab;
    if (tiled) {
      for (uint32_t e = tid; e < n; e += THREADS) {
        const uint64_t bn = sums[2 * e + 1];
        if (bn >> 32) {
          const uint32_t ly = e / L.tw, lx = e - ly * L.tw;
          uint64_t* const g = a.accum + 2 * (uint64_t)((y0 + ly) * a.W + (x0 + lx));
          __hip_atomic_fetch_add(g, sums[2 * e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_add(g + 1, bn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __syncthreads();  // tile free for the next batch; s_next visible
    i = uni(s_next);
  }
}

__global__ void __launch_bounds__(64) k_reset_queues(FrameHeader* hdr) {
  if (threadIdx.x < RENDER_QUEUES) hdr->queue[threadIdx.x][0] = 0;
}

__global__ void __launch_bounds__(256) k_zero64(uint64_t* p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

// The average of the sums: each channel (sum + n / 2) / n, alpha 255; the
// clear colour where no point joined.
__global__ void __launch_bounds__(256) k_resolve_hqs(const uint64_t* __restrict__ acc, uint64_t npix,
                                                     uint32_t clear_rgba, uint32_t* __restrict__ fb) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const uint64_t rg = acc[2 * p], bn = acc[2 * p + 1];
  const uint64_t n = bn >> 32;
  if (n == 0) {
    fb[p] = clear_rgba;
    return;
  }
  const uint64_t r = ((rg & 0xFFFFFFFFull) + n / 2) / n, g = ((rg >> 32) + n / 2) / n;
  const uint64_t b = ((bn & 0xFFFFFFFFull) + n / 2) / n;
  fb[p] = (uint32_t)r | ((uint32_t)g << 8) | ((uint32_t)b << 16) | (255u << 24);
}

// ------------------------------------------------------------------ resolve
// An index outside the cloud (a visibility buffer of some other cloud) resolves
// to the clear colour instead of reading out of bounds.
__global__ void __launch_bounds__(256) k_resolve(const uint64_t* __restrict__ vb, uint64_t npix,
                                                 const uint32_t* __restrict__ colors, uint64_t ncolors,
                                                 uint32_t clear_rgba, uint32_t* __restrict__ fb) {
  const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i + 4 <= npix) {
    const uint4 a = *reinterpret_cast<const uint4*>(vb + i);
    const uint4 b = *reinterpret_cast<const uint4*>(vb + i + 2);
    const uint64_t k[4] = {(uint64_t)a.x | ((uint64_t)a.y << 32), (uint64_t)a.z | ((uint64_t)a.w << 32),
                           (uint64_t)b.x | ((uint64_t)b.y << 32), (uint64_t)b.z | ((uint64_t)b.w << 32)};
    uint32_t o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t idx = (uint32_t)k[j];
      o[j] = (k[j] == ~0ull || idx >= ncolors) ? clear_rgba : colors[idx];
    }
    *reinterpret_cast<uint4*>(fb + i) = make_uint4(o[0], o[1], o[2], o[3]);
  } else {
    for (uint64_t p = i; p < npix; ++p) {
      const uint64_t k = vb[p];
      const uint32_t idx = (uint32_t)k;
      fb[p] = (k == ~0ull || idx >= ncolors) ? clear_rgba : colors[idx];
    }
  }
}

}  // namespace

hipError_t launch_clear(uint64_t* vb, uint64_t npix, DevBlock* dev, FrameHeader* hdr, int reset_stats, hipStream_t s) {
  const uint64_t n4 = npix / 2;
  uint64_t blocks = (n4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_clear, dim3((uint32_t)blocks), dim3(256), 0, s, reinterpret_cast<uint4*>(vb), n4, vb, npix,
                     dev, hdr, reset_stats);
  return hipGetLastError();
}

uint32_t render_grid(int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_render<false>, THREADS, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  return (uint32_t)(per_cu * cus);
}

hipError_t launch_render(const RenderArgs& a, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  const uint32_t cblocks = (a.nb + 255) / 256;
  const uint32_t rblocks = a.grid < a.nb ? a.grid : a.nb;
  if (a.counters) {
    hipLaunchKernelGGL(k_classify<true>, dim3(cblocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_render<true>, dim3(rblocks), dim3(THREADS), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_classify<false>, dim3(cblocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_render<false>, dim3(rblocks), dim3(THREADS), 0, s, a);
  }
  return hipGetLastError();
}

uint32_t render_views_grid(int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_render_views<false>, THREADS, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  return (uint32_t)(per_cu * cus);
}

hipError_t launch_clear_views(const ClearViewsArgs& a, hipStream_t s) {
  uint64_t maxpix = 0;
  for (uint32_t v = 0; v < a.nviews; ++v) {
    const uint64_t p = (uint64_t)a.v[v].W * a.v[v].H;
    if (p > maxpix) maxpix = p;
  }
  uint64_t blocks = a.clear ? (maxpix / 2 + 255) / 256 : 1;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_clear_views, dim3((uint32_t)blocks, a.nviews), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_classify_views(const ClassifyViewsArgs& a, int counters, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  const uint32_t blocks = (a.nb + 255) / 256;
  if (counters)
    hipLaunchKernelGGL(k_classify_views<true>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_classify_views<false>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_render_views(const RenderViewsArgs& a, uint64_t max_runs, int counters, hipStream_t s) {
  if (max_runs == 0) return hipSuccess;
  const uint32_t blocks = a.grid < max_runs ? a.grid : (uint32_t)max_runs;
  if (counters)
    hipLaunchKernelGGL(k_render_views<true>, dim3(blocks), dim3(THREADS), 0, s, a);
  else
    hipLaunchKernelGGL(k_render_views<false>, dim3(blocks), dim3(THREADS), 0, s, a);
  return hipGetLastError();
}

uint32_t accum_grid(int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_accum, THREADS, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  return (uint32_t)(per_cu * cus);
}

hipError_t launch_accumulate(const RenderArgs& a, hipStream_t s) {
  const uint64_t n = 2ull * a.W * a.H;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero64, dim3((uint32_t)blocks), dim3(256), 0, s, a.accum, n);
  if (a.nb == 0) return hipGetLastError();
  // the shading pass walks the render's live list with fresh work-queue counters
  hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(64), 0, s, a.hdr);
  const uint32_t blocks_r = a.grid < a.nb ? a.grid : a.nb;
  hipLaunchKernelGGL(k_accum, dim3(blocks_r), dim3(THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_resolve_hqs(const uint64_t* accum, uint64_t npix, uint32_t clear_rgba, uint32_t* fb,
                              hipStream_t s) {
  const uint64_t blocks = (npix + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_resolve_hqs, dim3((uint32_t)blocks), dim3(256), 0, s, accum, npix, clear_rgba, fb);
  return hipGetLastError();
}

hipError_t launch_resolve(const uint64_t* vb, uint64_t npix, const uint32_t* colors, uint64_t ncolors,
                          uint32_t clear_rgba, uint32_t* fb, hipStream_t s) {
  const uint64_t threads = (npix + 3) / 4;
  const uint64_t blocks = (threads + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_resolve, dim3((uint32_t)blocks), dim3(256), 0, s, vb, npix, colors, ncolors, clear_rgba, fb);
  return hipGetLastError();
}

}  // namespace ptr

// Point-raster core shared by every render-path translation unit: decode,
// projection, exact floor, the per-point loops of the visibility pass and of
// the shading pass, and the persistent render kernels.
//
// The workgroup shape is fixed per translation unit by three macros, so that
// the library can carry several compiled shapes of the same kernels and pick
// one at run time (every shape computes the same result):
//   PR_WAVES  waves per workgroup (64 lanes each)                  [4]
//   PR_DEPTH  groups of 256 points in flight per wave (prefetch)   [5]
//   PR_TILE   pixels of the workgroup's LDS tile (8 bytes each)    [4992]
#ifndef PR_RASTER_CORE_H
#define PR_RASTER_CORE_H

#include "internal.h"

#ifndef PR_WAVES
#define PR_WAVES 4
#endif
#ifndef PR_DEPTH
#define PR_DEPTH 5
#endif
#ifndef PR_TILE
#define PR_TILE 4992
#endif

namespace ptr {
namespace {

constexpr int CLS_INSIDE = 0, CLS_PARTIAL = 1, CLS_SLOW = 2;
constexpr int WAVES = PR_WAVES;
constexpr int THREADS = 64 * WAVES;
constexpr uint32_t TILE_MAX = PR_TILE;  // LDS tile of 64-bit keys
constexpr int PREFETCH = PR_DEPTH;      // groups of 256 points in flight per wave
static_assert(WAVES >= 1 && WAVES <= 16 && PREFETCH >= 1 && PREFETCH <= 8, "workgroup shape");
static_assert(TILE_MAX >= 256 && TILE_MAX % (2 * 64) == 0 && TILE_MAX * 8 <= 131072, "LDS tile (160 KiB per CU)");

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
  uint32_t base8;   // byte offset of this view's sub-tile in the LDS tile (two-view passes)
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
template <int K, int CLS, bool TILED, bool BAND = false>
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
      if constexpr (BAND) ok = ok && (py < L.th);  // rows of this band only
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
// BAND (tiled path only): the tile covers one band of rows of the batch's
// rectangle (L.th rows from the band origin); points of other rows are
// skipped (their tile row, taken as unsigned, is >= L.th).
template <int K, int CLS, bool TILED, bool ACC = false, bool BAND = false>
__device__ __forceinline__ void four_points(const Loop& L, uint64_t* tile, const Words& w, uint32_t i0,
                                            uint32_t nvalid, uint32_t& natom) {
  if constexpr (ACC) {
    four_points_acc<K, CLS, TILED, BAND>(L, tile, w, nvalid);
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
      if constexpr (BAND) ok[j] = ok[j] && (ly < L.th);
      key[j] = make_key(p.hw, i0 + j);
      ad[j] = __umul24(ly, L.tw8) + (lx << 3);
      asm volatile("" : "+v"(ad[j]));  // kept for the atomic, not recomputed
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (CLS == CLS_INSIDE && !BAND) {
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

// Two views in one pass (multi-view frames): four consecutive 10-bit points
// of one lane, decoded once, projected into view A and view B and combined in
// each view's LDS sub-tile exactly as four_points does for one view.  Both
// views' batch records are tiled, unbanded and INSIDE (CA/CB = CLS_INSIDE) or
// PARTIAL.
template <int CA, int CB>
__device__ __forceinline__ void four_points_pair(const Loop& A, const Loop& B, uint64_t* tile, const Words& w,
                                                 uint32_t i0, uint32_t nvalid) {
  const uint32_t Lw[4] = {w.l.x, w.l.y, w.l.z, w.l.w};
  uint8_t* const tb = reinterpret_cast<uint8_t*>(tile);
  uint32_t ad[8];
  uint64_t key[8], old[8];
  bool ok[8];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float X, Y, Z;
    decode<10>(Lw[j], 0u, 0u, X, Y, Z);
    const uint32_t idx = i0 + j;
    {
      const Proj p = project(A, X, Y, Z);
      ok[j] = (uint32_t)j < nvalid;
      if constexpr (CA != CLS_INSIDE) ok[j] = ok[j] && visible(A, p);
      uint32_t lx, ly;
      pixel_fast(p, A.cx, A.cy, lx, ly);
      key[j] = make_key(p.hw, idx);
      ad[j] = __umul24(ly, A.tw8) + (lx << 3);
      asm volatile("" : "+v"(ad[j]));
    }
    {
      const Proj p = project(B, X, Y, Z);
      ok[4 + j] = (uint32_t)j < nvalid;
      if constexpr (CB != CLS_INSIDE) ok[4 + j] = ok[4 + j] && visible(B, p);
      uint32_t lx, ly;
      pixel_fast(p, B.cx, B.cy, lx, ly);
      key[4 + j] = make_key(p.hw, idx);
      ad[4 + j] = __umul24(ly, B.tw8) + ((lx << 3) + B.base8);
      asm volatile("" : "+v"(ad[4 + j]));
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const bool inside = j < 4 ? CA == CLS_INSIDE : CB == CLS_INSIDE;
    if (inside) {
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
  for (int j = 0; j < 8; ++j)
    if (ok[j] && key[j] < old[j])
      __hip_atomic_fetch_min(reinterpret_cast<uint64_t*>(tb + ad[j]), key[j], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Two views whose y and w projection rows are bit-equal (a stereo pair whose
// eyes differ by a shift along the camera's x axis): the y and w chains, the
// reciprocal, the y floor and the key are computed once; only the x chain and
// x floor are per view.  Every value equals what four_points_pair computes.
template <int CA, int CB>
__device__ __forceinline__ void four_points_pair_shared(const Loop& A, const Loop& B, uint64_t* tile, const Words& w,
                                                        uint32_t i0, uint32_t nvalid) {
  const uint32_t Lw[4] = {w.l.x, w.l.y, w.l.z, w.l.w};
  uint8_t* const tb = reinterpret_cast<uint8_t*>(tile);
  uint32_t ad[8];
  uint64_t key[4], old[8];
  bool ok[8];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float X, Y, Z;
    decode<10>(Lw[j], 0u, 0u, X, Y, Z);
    const Proj pa = project(A, X, Y, Z);
    Proj pb = pa;
    pb.hx = __builtin_fmaf(B.P[0][2], Z, __builtin_fmaf(B.P[0][1], Y, __builtin_fmaf(B.P[0][0], X, B.t[0])));
    ok[j] = (uint32_t)j < nvalid;
    ok[4 + j] = ok[j];
    if constexpr (CA != CLS_INSIDE) ok[j] = ok[j] && visible(A, pa);
    if constexpr (CB != CLS_INSIDE) ok[4 + j] = ok[4 + j] && visible(B, pb);
    const float r = __builtin_amdgcn_rcpf(pa.hw);
    const float ty = __builtin_fmaf(pa.hy, r, 0x1p23f);
    const float ey = __builtin_fmaf(-(ty - 0x1p23f), pa.hw, pa.hy);
    const float txa = __builtin_fmaf(pa.hx, r, 0x1p23f);
    const float exa = __builtin_fmaf(-(txa - 0x1p23f), pa.hw, pa.hx);
    const float txb = __builtin_fmaf(pb.hx, r, 0x1p23f);
    const float exb = __builtin_fmaf(-(txb - 0x1p23f), pa.hw, pb.hx);
    const unsigned int by = (unsigned int)(ey < 0.0f);
    unsigned int bo;
    const uint32_t lxa = __builtin_subc(__float_as_uint(txa), A.cx, (unsigned int)(exa < 0.0f), &bo);
    const uint32_t lya = __builtin_subc(__float_as_uint(ty), A.cy, by, &bo);
    const uint32_t lxb = __builtin_subc(__float_as_uint(txb), B.cx, (unsigned int)(exb < 0.0f), &bo);
    const uint32_t lyb = __builtin_subc(__float_as_uint(ty), B.cy, by, &bo);
    key[j] = make_key(pa.hw, i0 + j);
    ad[j] = __umul24(lya, A.tw8) + (lxa << 3);
    asm volatile("" : "+v"(ad[j]));
    ad[4 + j] = __umul24(lyb, B.tw8) + ((lxb << 3) + B.base8);
    asm volatile("" : "+v"(ad[4 + j]));
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const bool inside = j < 4 ? CA == CLS_INSIDE : CB == CLS_INSIDE;
    if (inside) {
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
  for (int j = 0; j < 8; ++j)
    if (ok[j] && key[j & 3] < old[j])
      __hip_atomic_fetch_min(reinterpret_cast<uint64_t*>(tb + ad[j]), key[j & 3], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The coordinate streams of the cloud (low, medium, high words).
struct Streams {
  const uint32_t* low;
  const uint32_t* med;
  const uint32_t* high;
  const uint32_t* colors;  // shading pass only
};

// The streams of one batch as buffer resources based at its first point: a
// group's 16-byte word of a lane is then at the lane's constant offset
// lane * 16 plus the group's uniform offset g * 1024, so loads need no vector
// address arithmetic.  A batch of up to 2^22 groups (2^30 points) fits the
// 32-bit offsets; raster_points cuts longer batches into such chunks.
struct BatchStreams {
  __amdgpu_buffer_rsrc_t l, m, h, c;
};
constexpr uint32_t RSRC_WORD3 = 0x00020000;  // raw 32-bit buffer (gfx9 family)
constexpr uint32_t CHUNK_POINTS = 1u << 30;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t stream_rsrc(const uint32_t* s, uint32_t first) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)(s + first), (short)0, -1, RSRC_WORD3);
}
template <int K, bool ACC>
__device__ __forceinline__ BatchStreams batch_streams(const Streams& a, uint32_t first) {
  BatchStreams b;
  b.l = stream_rsrc(a.low, first);
  if constexpr (K >= 20) b.m = stream_rsrc(a.med, first);
  if constexpr (K == 30) b.h = stream_rsrc(a.high, first);
  if constexpr (ACC) b.c = stream_rsrc(a.colors, first);
  return b;
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 buf16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  return make_uint4(v.x, v.y, v.z, v.w);
}

template <int K, bool ACC = false>
__device__ __forceinline__ Words load_group(const BatchStreams& b, uint32_t g, uint32_t lane16) {
  const uint32_t go = g * 1024u;
  Words w;
  w.l = buf16(b.l, lane16, go);
  if constexpr (K >= 20) w.m = buf16(b.m, lane16, go);
  else w.m = make_uint4(0, 0, 0, 0);
  if constexpr (K == 30) w.h = buf16(b.h, lane16, go);
  else w.h = make_uint4(0, 0, 0, 0);
  if constexpr (ACC) w.c = buf16(b.c, lane16, go);
  else w.c = make_uint4(0, 0, 0, 0);
  return w;
}

// The points of one batch, split over the workgroup's waves: wave w takes the
// groups of 256 points w, w + WAVES, ... (4 consecutive points per lane, one
// 16-byte load per word) and hands each lane's four points to
// fn(words, index of the first, number valid).  The ragged tail goes to wave
// ngrp mod WAVES, the next in that rotation (one of the waves with the fewest
// groups).  PF groups are in flight per wave.
template <int K, bool ACC, int PF, typename Fn>
__device__ __forceinline__ void stream_chunk(const Streams& a, uint32_t first, uint32_t count, uint32_t wave,
                                             uint32_t lane, Fn&& fn) {
  const BatchStreams bs = batch_streams<K, ACC>(a, first);
  const uint32_t lane16 = lane * 16u;
  const uint32_t ngrp = count >> 8;
  const uint32_t nj = wave < ngrp ? (ngrp - wave + WAVES - 1) / WAVES : 0;  // this wave's groups
  if (nj > 0) {
    // PF register sets rotate through the wave's groups; each is
    // reloaded in place right after use, so every load is issued PF
    // groups ahead of its use.  The rounds are branch-free: reloads are
    // unconditional and clamped to the wave's last group, so every wait
    // counts exactly the loads in flight.  Only whole rounds run this way;
    // the last nj mod PF groups are then already loaded in the first
    // register sets and are processed without reloads (no empty slots).
    const uint32_t glast = wave + (nj - 1) * WAVES;
    Words R[PF];
    uint32_t gi[PF];
#pragma unroll
    for (int d = 0; d < PF; ++d) {
      gi[d] = wave + d * WAVES;
      R[d] = load_group<K, ACC>(bs, min(gi[d], glast), lane16);
      // keep the initial loads in the order of their use, the order the
      // loop reissues them in: the loop's waits then count PF - 1
      // younger loads on every path
      __builtin_amdgcn_sched_barrier(0);
    }
    const uint32_t whole = nj - nj % PF;
    for (uint32_t j = 0; j < whole; j += PF) {
#pragma unroll
      for (int d = 0; d < PF; ++d) {
        const uint32_t g = gi[d];  // <= glast in every whole round
        fn(R[d], first + g * 256 + lane * 4, 4u);
        gi[d] = g + PF * WAVES;
        R[d] = load_group<K, ACC>(bs, min(gi[d], glast), lane16);
      }
    }
    const uint32_t rest = nj - whole;  // groups gi[0 .. rest - 1], loaded in R[0 .. rest - 1]
#pragma unroll
    for (int d = 0; d < PF; ++d)
      if ((uint32_t)d < rest) fn(R[d], first + gi[d] * 256 + lane * 4, 4u);
  }
  const uint32_t rem = count & 255u;
  if (rem && wave == ngrp % WAVES) {  // ragged tail of the batch: scalar loads, per-point bounds
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
    fn(t, first + j0, nv);
  }
}

// The points of one batch into one view (tile or visibility buffer).
template <int K, int CLS, bool TILED, bool ACC = false, bool BAND = false>
__device__ __forceinline__ void raster_chunk(const Loop& L, const Streams& a, uint64_t* tile, uint32_t first,
                                             uint32_t count, uint32_t wave, uint32_t lane, uint32_t& natom) {
  // The rare SLOW class (binary64 floor) keeps one group in flight and the
  // rare 20- and 30-bit batches (two and three words per point) at most
  // three: deeper prefetch there would set the register count of the whole
  // kernel, which the 10-bit loops (almost every point) then pay for.
  constexpr int PF = CLS == CLS_SLOW ? 1 : (K == 10 ? PREFETCH : (PREFETCH < 3 ? PREFETCH : 3));
  stream_chunk<K, ACC, PF>(a, first, count, wave, lane, [&](const Words& w, uint32_t i0, uint32_t nv) {
    four_points<K, CLS, TILED, ACC, BAND>(L, tile, w, i0, nv, natom);
  });
}

// A batch, in chunks of at most CHUNK_POINTS points (one chunk for every
// batch of a regular build).
template <int K, int CLS, bool TILED, bool ACC = false, bool BAND = false>
__device__ __forceinline__ void raster_points(const Loop& L, const Streams& a, uint64_t* tile, uint32_t first,
                                              uint32_t count, uint32_t wave, uint32_t lane, uint32_t& natom) {
  for (uint32_t c0 = 0; c0 < count; c0 += CHUNK_POINTS) {
    const uint32_t n = count - c0 < CHUNK_POINTS ? count - c0 : CHUNK_POINTS;
    raster_chunk<K, CLS, TILED, ACC, BAND>(L, a, tile, first + c0, n, wave, lane, natom);
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


// ------------------------------------------------------------------ render
template <int K, bool TILED, bool ACC = false, bool BAND = false>
__device__ __forceinline__ void raster_by_class(int cls, const Loop& L, const Streams& a, uint64_t* tile,
                                                uint32_t first, uint32_t count, uint32_t wave, uint32_t lane,
                                                uint32_t& natom) {
  if (cls == CLS_INSIDE)
    raster_points<K, CLS_INSIDE, TILED, ACC, BAND>(L, a, tile, first, count, wave, lane, natom);
  else if (cls == CLS_PARTIAL)
    raster_points<K, CLS_PARTIAL, TILED, ACC, BAND>(L, a, tile, first, count, wave, lane, natom);
  else if constexpr (!TILED)
    raster_points<K, CLS_SLOW, false, ACC>(L, a, tile, first, count, wave, lane, natom);
}

// Flush of a tile rectangle (tw x th pixels at x0, y0): every covered tile
// pixel once into the global buffer, leaving the entry PR_EMPTY for the next
// batch.  Most covered pixels improve the global minimum, so the atomic is
// issued without a prior read (no round trip on this path).
// The entry's row and column are stepped with the loop instead of divided
// out per entry: floor((tid + 1/2) * rcp(tw)) is exactly floor(tid / tw) in
// binary32 (the reciprocal within an ulp moves the product by less than the
// distance 1/(2 tw) of the half-integer numerator's quotient to an integer,
// for numerators below 2^20), and one carry per step keeps lx below tw.
__device__ __forceinline__ void flush_tile(uint64_t* tile, uint32_t tid, uint64_t* vb, uint32_t W, uint32_t x0,
                                           uint32_t y0, uint32_t tw, uint32_t th, uint32_t& natom) {
  const uint32_t n = tw * th;
  const float rtw = __builtin_amdgcn_rcpf((float)tw);
  const uint32_t dy = (uint32_t)(((float)THREADS + 0.5f) * rtw), dx = THREADS - dy * tw;
  uint32_t ly = (uint32_t)(((float)tid + 0.5f) * rtw), lx = tid - ly * tw;
  uint64_t* const base = vb + ((uint64_t)y0 * W + x0);
  for (uint32_t e = tid; e < n; e += THREADS) {
    const uint64_t v = tile[e];
    if (v != ~0ull) {
      tile[e] = ~0ull;
      __hip_atomic_fetch_min(base + (__umul24(ly, W) + lx), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      natom++;
    }
    lx += dx;
    ly += dy;
    if (lx >= tw) {
      lx -= tw;
      ly += 1u;
    }
  }
}

// One live batch of one view by the whole workgroup: its points into the LDS
// tile (or straight into the global buffer), then the tile flush.  The LDS
// tile is all PR_EMPTY between batches (the flush resets what it reads), so a
// batch needs two barriers: one after its points, one after its flush.  A
// banded batch (rectangle up to a few tiles, at most one tile wide) streams its
// points once per band of rows that fits the tile, with the same two barriers
// per band.  publish: thread 0 stores next into s_next after the first
// barrier (the workgroup reads it after the last one).
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
  if ((mode >> 17) & 1u) {
    const uint32_t th = L.th, bh = TILE_MAX / L.tw;  // rows per band (the rectangle is at most one tile wide)
    L.cx = in_vgpr(uni(0x4B000000u + x0));
    for (uint32_t by = 0; by < th; by += bh) {
      L.th = min(bh, th - by);
      L.cy = in_vgpr(uni(0x4B000000u + y0 + by));
      // classify bands 10-bit batches only (more levels here would raise the kernel's register count)
      raster_by_class<10, true, false, true>(cls, L, st, tile, first, count, wave, lane, natom);
      __syncthreads();  // the band's points are all in the tile; s_next has been read
      if (by == 0 && publish && tid == 0) *s_next = next;
      flush_tile(tile, tid, L.vb, L.W, x0, y0 + by, L.tw, L.th, natom);
      __syncthreads();  // tile clean again
    }
    return;
  }
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
  if (tiled) flush_tile(tile, tid, L.vb, L.W, x0, y0, L.tw, L.th, natom);
  __syncthreads();  // tile clean again; s_next visible
}

// A batch record's Loop values for the tiled point loops.
__device__ __forceinline__ Loop tiled_loop(const LiveBatch& rec, uint32_t W, uint32_t H, uint64_t* vb) {
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
  const uint32_t rwh = uni(rec.rect_wh), rxy = uni(rec.rect_xy);
  L.tw = rwh & 0xFFFFu;
  L.th = rwh >> 16;
  L.tw8 = L.tw * 8u;
  L.base8 = 0;
  L.cx = in_vgpr(uni(0x4B000000u + (rxy & 0xFFFFu)));
  L.cy = in_vgpr(uni(0x4B000000u + (rxy >> 16)));
  return L;
}

// Whether a view's record of a batch can share a two-view pass: 10 bits,
// tiled, not banded, INSIDE or PARTIAL.
__device__ __forceinline__ bool pairable(const LiveBatch& rec) {
  const uint32_t m = rec.mode;
  return (m & 0xFFu) == 10u && ((m >> 16) & 3u) == 1u && ((m >> 8) & 0xFFu) != (uint32_t)CLS_SLOW;
}
__device__ __forceinline__ uint32_t rect_area(const LiveBatch& rec) {
  return (rec.rect_wh & 0xFFFFu) * (rec.rect_wh >> 16);
}

// Groups in flight per wave in a two-view pass: each group carries twice the
// work of a one-view group, so fewer cover the same memory latency.
constexpr int PAIR_PF = PREFETCH < 3 ? PREFETCH : 3;

// One batch into two views in one pass over its points: view A's sub-tile
// first in the LDS tile, view B's right after it (the two rectangles fit the
// tile together), one barrier after the points, both flushes, one barrier.
__device__ __forceinline__ void render_pair(const LiveBatch& ra, const ViewOut& va, const LiveBatch& rb,
                                            const ViewOut& vb, const Streams& st, uint64_t* tile, uint32_t tid,
                                            uint32_t wave, uint32_t lane, bool publish, uint32_t next,
                                            uint32_t* s_next, uint32_t& natom) {
  const Loop A = tiled_loop(ra, va.W, va.H, va.vb);
  Loop B = tiled_loop(rb, vb.W, vb.H, vb.vb);
  const uint32_t na = uni(rect_area(ra));
  B.base8 = na * 8u;
  // uniform by construction (one record per workgroup); said so for the compiler
  const uint32_t first = uni(ra.first), count = uni(ra.count);
  const int ca = (int)((uni(ra.mode) >> 8) & 0xFFu), cb = (int)((uni(rb.mode) >> 8) & 0xFFu);
  // y and w rows bit-equal in both records: shared chains
  bool shared = true;
#pragma unroll
  for (int r = 1; r < 3; ++r) {
#pragma unroll
    for (int j = 0; j < 3; ++j) shared = shared && __float_as_uint(A.P[r][j]) == __float_as_uint(B.P[r][j]);
    shared = shared && __float_as_uint(A.t[r]) == __float_as_uint(B.t[r]);
  }
  for (uint32_t c0 = 0; c0 < count; c0 += CHUNK_POINTS) {
    const uint32_t n = count - c0 < CHUNK_POINTS ? count - c0 : CHUNK_POINTS;
    if (shared) {
      if (ca == CLS_INSIDE && cb == CLS_INSIDE)
        stream_chunk<10, false, PAIR_PF>(st, first + c0, n, wave, lane, [&](const Words& w, uint32_t i0, uint32_t nv) {
          four_points_pair_shared<CLS_INSIDE, CLS_INSIDE>(A, B, tile, w, i0, nv);
        });
      else if (ca == CLS_INSIDE)
        stream_chunk<10, false, PAIR_PF>(st, first + c0, n, wave, lane, [&](const Words& w, uint32_t i0, uint32_t nv) {
          four_points_pair_shared<CLS_INSIDE, CLS_PARTIAL>(A, B, tile, w, i0, nv);
        });
      else if (cb == CLS_INSIDE)
        stream_chunk<10, false, PAIR_PF>(st, first + c0, n, wave, lane, [&](const Words& w, uint32_t i0, uint32_t nv) {
          four_points_pair_shared<CLS_PARTIAL, CLS_INSIDE>(A, B, tile, w, i0, nv);
        });
      else
        stream_chunk<10, false, PAIR_PF>(st, first + c0, n, wave, lane, [&](const Words& w, uint32_t i0, uint32_t nv) {
          four_points_pair_shared<CLS_PARTIAL, CLS_PARTIAL>(A, B, tile, w, i0, nv);
        });
    } else if (ca == CLS_INSIDE && cb == CLS_INSIDE)
      stream_chunk<10, false, PAIR_PF>(st, first + c0, n, wave, lane, [&](const Words& w, uint32_t i0, uint32_t nv) {
        four_points_pair<CLS_INSIDE, CLS_INSIDE>(A, B, tile, w, i0, nv);
      });
    else if (ca == CLS_INSIDE)
      stream_chunk<10, false, PAIR_PF>(st, first + c0, n, wave, lane, [&](const Words& w, uint32_t i0, uint32_t nv) {
        four_points_pair<CLS_INSIDE, CLS_PARTIAL>(A, B, tile, w, i0, nv);
      });
    else if (cb == CLS_INSIDE)
      stream_chunk<10, false, PAIR_PF>(st, first + c0, n, wave, lane, [&](const Words& w, uint32_t i0, uint32_t nv) {
        four_points_pair<CLS_PARTIAL, CLS_INSIDE>(A, B, tile, w, i0, nv);
      });
    else
      stream_chunk<10, false, PAIR_PF>(st, first + c0, n, wave, lane, [&](const Words& w, uint32_t i0, uint32_t nv) {
        four_points_pair<CLS_PARTIAL, CLS_PARTIAL>(A, B, tile, w, i0, nv);
      });
  }
  __syncthreads();  // both views' points are in their sub-tiles; s_next has been read
  if (publish && tid == 0) *s_next = next;
  flush_tile(tile, tid, va.vb, va.W, ra.rect_xy & 0xFFFFu, ra.rect_xy >> 16, A.tw, A.th, natom);
  flush_tile(tile + na, tid, vb.vb, vb.W, rb.rect_xy & 0xFFFFu, rb.rect_xy >> 16, B.tw, B.th, natom);
  __syncthreads();  // tile clean again; s_next visible
}

// The live list (or run list) of nb slots holds nt tiled entries from the
// front and nd entries with untiled batches from the back (slots nb - 1,
// nb - 2, ...).  Queue position p of n = nt + nd takes an untiled one iff
// floor((p + 1) nd / n) > floor(p nd / n), which spreads the untiled batches
// (and their global atomics) evenly over the frame.  Returns ~0u past the end.
// One division: with k = floor(p nd / n) and r = p nd - k n, the next
// quotient is k + floor((r + nd) / n), and r + nd < 2n, so it exceeds k iff
// r >= n - nd = nt.
__device__ __forceinline__ uint32_t live_slot(uint32_t p, uint32_t nt, uint32_t nd, uint32_t nb) {
  const uint32_t n = nt + nd;
  if (p >= n) return ~0u;
  if (nd == 0) return p;
  const uint64_t num = (uint64_t)p * nd;
  const uint32_t k = (uint32_t)(num / n), r = (uint32_t)(num - (uint64_t)k * n);
  return r >= nt ? nb - 1u - k : p - k;
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
// The shape (SW waves, SD groups in flight, ST tile pixels) is among the
// render kernels' template arguments only so that profiles name the shape
// that ran; it must equal the translation unit's shape.
template <bool CNT, int SW, int SD, int ST>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_render(RenderArgs a) {
  static_assert(SW == WAVES && SD == PREFETCH && ST == (int)TILE_MAX, "shape tag");
  __shared__ uint64_t tile[TILE_MAX];
  __shared__ uint32_t s_next;
  const uint32_t tid = threadIdx.x, wave = uni(tid >> 6), lane = tid & 63;
  fill_tile(tile, tid);
  // this workgroup's queue: workgroups are spread over the queues round-robin
  const uint32_t q = blockIdx.x % RENDER_QUEUES;
  uint32_t* const qc = &a.hdr->queue[q][0];
  const uint32_t nt = a.hdr->live_count, nd = a.hdr->direct_count;
  if (tid == 0) s_next = live_slot(atomicAdd(qc, 1u) * RENDER_QUEUES + q, nt, nd, a.nb);
  const Streams st = {a.low, a.med, a.high, nullptr};
  __syncthreads();
  uint32_t i = uni(s_next);
  uint32_t natom = 0;
  while (i != ~0u) {
    // Take the next batch now; the atomic's latency hides behind this batch.
    uint32_t grab = 0;
    if (tid == 0) grab = live_slot(atomicAdd(qc, 1u) * RENDER_QUEUES + q, nt, nd, a.nb);
    render_batch(a.live[i], a.W, a.H, a.vb, st, tile, tid, wave, lane, true, grab, &s_next, natom);
    i = uni(s_next);
  }
  add_atomics<CNT>(a.stats, natom, lane);
}

// Several views in one launch: the work items are runs (a batch and its live
// views); the workgroup renders the batch once per view, so its coordinate
// words come from HBM once and from the caches for the further views.
template <bool CNT, int SW, int SD, int ST>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_render_views(RenderViewsArgs a) {
  static_assert(SW == WAVES && SD == PREFETCH && ST == (int)TILE_MAX, "shape tag");
  __shared__ uint64_t tile[TILE_MAX];
  __shared__ uint32_t s_next;
  const uint32_t tid = threadIdx.x, wave = uni(tid >> 6), lane = tid & 63;
  fill_tile(tile, tid);
  const uint32_t q = blockIdx.x % RENDER_QUEUES;
  uint32_t* const qc = &a.hdr->queue[q][0];
  const uint32_t nt = a.hdr->live_count, nd = a.hdr->direct_count;
  if (tid == 0) s_next = live_slot(atomicAdd(qc, 1u) * RENDER_QUEUES + q, nt, nd, a.cap);
  const Streams st = {a.low, a.med, a.high, nullptr};
  __syncthreads();
  uint32_t i = uni(s_next);
  uint32_t natom = 0;
  while (i != ~0u) {
    uint32_t grab = 0;
    if (tid == 0) grab = live_slot(atomicAdd(qc, 1u) * RENDER_QUEUES + q, nt, nd, a.cap);
    const Run run = a.runs[i];
    uint64_t mask = run.mask;
    bool publish = true;
    const LiveBatch* const recs = a.sub + (uint64_t)run.batch * a.nviews;
    while (mask) {
      const uint32_t v = run.view0 + (uint32_t)(__ffsll((unsigned long long)mask) - 1);
      mask &= mask - 1;
      const LiveBatch& rec = recs[v];
      // the next live view shares the pass when both records allow it and
      // their rectangles fit the tile together
      if (mask && pairable(rec)) {
        const uint32_t v2 = run.view0 + (uint32_t)(__ffsll((unsigned long long)mask) - 1);
        const LiveBatch& rec2 = recs[v2];
        if (pairable(rec2) && rect_area(rec) + rect_area(rec2) <= TILE_MAX) {
          mask &= mask - 1;
          render_pair(rec, a.v[v], rec2, a.v[v2], st, tile, tid, wave, lane, publish, grab, &s_next, natom);
          publish = false;
          continue;
        }
      }
      const ViewOut& vo = a.v[v];
      render_batch(rec, vo.W, vo.H, vo.vb, st, tile, tid, wave, lane, publish, grab, &s_next, natom);
      publish = false;
    }
    i = uni(s_next);
  }
  add_atomics<CNT>(a.stats, natom, lane);
}

}  // namespace
}  // namespace ptr

#endif  // PR_RASTER_CORE_H

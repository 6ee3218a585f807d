// Render-path kernels for gfx950: clear (+ per-frame constants), render, resolve.
//
// Method: Schuetz, Kerbl & Wimmer, "Software Rasterization of 2 Billion Points
// in Real Time", Sec. 3.2 (one workgroup per batch, batch frustum culling,
// point rasterization with a 64-bit depth|index atomic minimum and an
// early-depth test) and Sec. 3.3 (adaptive 10/20/30-bit coordinates, Eq. 1,
// visibility-buffer resolve).
//
// Arithmetic contract (must hold bit for bit; compiled with -ffp-contract=off):
//  * frame matrix and per-batch decisions in binary64, plain + - * /, left to
//    right, never fused;
//  * per point: X = (float)F (RNE), hx/hy/hw = three fmaf chains in a fixed
//    order, pixel = exact floor of hx/hw, key = bits(hw) << 32 | index.
//
// Each batch is processed by one wave64.  Its prologue projects the 8 box
// corners (one corner per lane, replicated 8 times), and classifies the batch
// with wave ballots:
//  CULLED  : some frustum plane has all corners outside by a margin that
//            exceeds every rounding of the per-point evaluation;
//  INSIDE  : all corners strictly inside every plane by that margin and w in
//            [2^-60, 2^60]: every point passes the visibility tests, which are
//            therefore skipped;
//  PARTIAL : w in [2^-60, 2^60] for every point: per-point tests, fast exact
//            floor from a reciprocal;
//  SLOW    : anything else (box reaching w <= 0 or absurd scales): per-point
//            tests, floor of a correctly rounded binary64 quotient.
// All three rendering classes give the same result for every point; they only
// differ in which tests are provably redundant.
#include "internal.h"

namespace ptr {
namespace {

constexpr int CLS_INSIDE = 0, CLS_PARTIAL = 1, CLS_SLOW = 2;

// ------------------------------------------------------------------ clear
// Fills the visibility buffer with all-ones (PR_EMPTY), computes the frame's
// pixel-space matrix, and resets the counters.
__global__ void __launch_bounds__(256) k_clear(uint4* __restrict__ vb4, uint64_t n4, uint64_t* __restrict__ vb,
                                               uint64_t npix, ViewArgs v, uint32_t W, uint32_t H,
                                               DevBlock* __restrict__ dev, int reset_stats) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u);
  for (uint64_t i = tid; i < n4; i += stride) vb4[i] = ones;
  if (tid == 0 && (npix & 1)) vb[npix - 1] = ~0ull;
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      // C = proj * view for rows 0, 1, 3 (row-major storage, column vectors)
      double C[3][4];
      const int rows[3] = {0, 1, 3};
      for (int q = 0; q < 3; ++q) {
        const int i = rows[q];
        for (int j = 0; j < 4; ++j)
          C[q][j] = (((double)v.proj[4 * i + 0] * (double)v.view[0 + j] +
                      (double)v.proj[4 * i + 1] * (double)v.view[4 + j]) +
                     (double)v.proj[4 * i + 2] * (double)v.view[8 + j]) +
                    (double)v.proj[4 * i + 3] * (double)v.view[12 + j];
      }
      for (int j = 0; j < 4; ++j) {
        dev->fc.Pm[0][j] = (0.5 * (double)W) * (C[0][j] + C[2][j]);
        dev->fc.Pm[1][j] = (0.5 * (double)H) * (C[1][j] + C[2][j]);
        dev->fc.Pm[2][j] = C[2][j];
      }
    }
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

struct Folded {
  float P[3][3];
  float t[3];
};

// One point: returns true and fills (off, key) if it lands inside the image.
template <int CLS>
__device__ __forceinline__ bool project(const Folded& f, float X, float Y, float Z, uint32_t idx, uint32_t W,
                                        uint32_t H, uint32_t& off, uint64_t& key) {
  const float hx = __builtin_fmaf(f.P[0][2], Z, __builtin_fmaf(f.P[0][1], Y, __builtin_fmaf(f.P[0][0], X, f.t[0])));
  const float hy = __builtin_fmaf(f.P[1][2], Z, __builtin_fmaf(f.P[1][1], Y, __builtin_fmaf(f.P[1][0], X, f.t[1])));
  const float hw = __builtin_fmaf(f.P[2][2], Z, __builtin_fmaf(f.P[2][1], Y, __builtin_fmaf(f.P[2][0], X, f.t[2])));
  bool ok = true;
  if constexpr (CLS != CLS_INSIDE) {
    // hw > 0, 0 <= hx < W hw, 0 <= hy < H hw; the fma residuals carry the
    // exact sign of hx - W hw (denormals are kept, so nothing underflows to 0).
    ok = (hw > 0.0f) & (hx >= 0.0f) & (__builtin_fmaf(-(float)W, hw, hx) < 0.0f) & (hy >= 0.0f) &
         (__builtin_fmaf(-(float)H, hw, hy) < 0.0f);
  }
  uint32_t px, py;
  if constexpr (CLS == CLS_SLOW) {
    // Exact floor of the real quotient: the binary64 quotient of two binary32
    // values below 2^13 never crosses an integer.
    px = (uint32_t)floor((double)hx / (double)hw);
    py = (uint32_t)floor((double)hy / (double)hw);
  } else {
    // n = nearest integer to hx * rcp(hw) is within 1 of the quotient q
    // (|q - hx rcp(hw)| < 2^-9 for q < 2^13); the sign of the exactly
    // signed residual hx - n hw decides between n and n - 1.
    const float r = __builtin_amdgcn_rcpf(hw);
    const float nx = __builtin_rintf(hx * r);
    const float ny = __builtin_rintf(hy * r);
    const float ex = __builtin_fmaf(-nx, hw, hx);
    const float ey = __builtin_fmaf(-ny, hw, hy);
    px = (uint32_t)nx - (ex < 0.0f ? 1u : 0u);
    py = (uint32_t)ny - (ey < 0.0f ? 1u : 0u);
  }
  // Never address outside the image, whatever the class proofs say.
  ok = ok & (px < W) & (py < H);
  off = py * W + px;
  key = ((uint64_t)__float_as_uint(hw) << 32) | (uint64_t)idx;
  return ok;
}

// Four consecutive points of one lane: project all, issue all early-depth
// reads, then the atomic minimum where the key beats the value read.
template <int K, int CLS, bool CNT>
__device__ __forceinline__ void four_points(const Folded& f, uint64_t* __restrict__ vb, uint4 lw, uint4 mw, uint4 hw,
                                            uint32_t i0, uint32_t nvalid, uint32_t W, uint32_t H,
                                            uint32_t& natom) {
  const uint32_t L[4] = {lw.x, lw.y, lw.z, lw.w};
  const uint32_t M[4] = {mw.x, mw.y, mw.z, mw.w};
  const uint32_t Hh[4] = {hw.x, hw.y, hw.z, hw.w};
  uint32_t off[4];
  uint64_t key[4], old[4];
  bool ok[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float X, Y, Z;
    decode<K>(L[j], M[j], Hh[j], X, Y, Z);
    ok[j] = project<CLS>(f, X, Y, Z, i0 + j, W, H, off[j], key[j]) && ((uint32_t)j < nvalid);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    old[j] = 0;
    if (ok[j]) old[j] = __hip_atomic_load(vb + off[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (ok[j] && key[j] < old[j]) {
      __hip_atomic_fetch_min(vb + off[j], key[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if constexpr (CNT) natom++;
    }
  }
}

template <int K, int CLS, bool CNT>
__device__ void raster_batch(const RenderArgs& a, const Folded& f, uint32_t first, uint32_t count, uint32_t lane) {
  const uint4* __restrict__ L4 = reinterpret_cast<const uint4*>(a.low + first);
  const uint4* __restrict__ M4 = reinterpret_cast<const uint4*>(a.med + first);
  const uint4* __restrict__ H4 = reinterpret_cast<const uint4*>(a.high + first);
  const uint4 zero4 = make_uint4(0, 0, 0, 0);
  const uint32_t ngrp = count >> 8;  // full groups of 256 points (4 per lane)
  uint32_t natom = 0;
  uint4 cl = zero4, cm = zero4, ch = zero4;
  if (ngrp > 0) {
    cl = L4[lane];
    if constexpr (K >= 20) cm = M4[lane];
    if constexpr (K == 30) ch = H4[lane];
  }
  for (uint32_t g = 0; g < ngrp; ++g) {
    uint4 nl = zero4, nm = zero4, nh = zero4;
    if (g + 1 < ngrp) {  // software prefetch of the next group
      const uint32_t q = (g + 1) * 64 + lane;
      nl = L4[q];
      if constexpr (K >= 20) nm = M4[q];
      if constexpr (K == 30) nh = H4[q];
    }
    four_points<K, CLS, CNT>(f, a.vb, cl, cm, ch, first + g * 256 + lane * 4, 4, a.W, a.H, natom);
    cl = nl;
    cm = nm;
    ch = nh;
  }
  const uint32_t rem = count & 255u;
  if (rem) {  // ragged tail of the batch: scalar loads, per-point bounds
    const uint32_t j0 = ngrp * 256 + lane * 4;
    const uint32_t nv = j0 < count ? min(4u, count - j0) : 0u;
    uint32_t l[4] = {0, 0, 0, 0}, m[4] = {0, 0, 0, 0}, h[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if ((uint32_t)j < nv) {
        l[j] = a.low[first + j0 + j];
        if constexpr (K >= 20) m[j] = a.med[first + j0 + j];
        if constexpr (K == 30) h[j] = a.high[first + j0 + j];
      }
    }
    four_points<K, CLS, CNT>(f, a.vb, make_uint4(l[0], l[1], l[2], l[3]), make_uint4(m[0], m[1], m[2], m[3]),
                             make_uint4(h[0], h[1], h[2], h[3]), first + j0, nv, a.W, a.H, natom);
  }
  if constexpr (CNT) {
    for (int o = 32; o > 0; o >>= 1) natom += __shfl_xor(natom, o);
    if (lane == 0 && natom) atomicAdd((unsigned long long*)&a.stats[ST_ATOMICS], (unsigned long long)natom);
  }
}

__device__ __forceinline__ double max8(double v) {
  v = fmax(v, __shfl_xor(v, 1));
  v = fmax(v, __shfl_xor(v, 2));
  v = fmax(v, __shfl_xor(v, 4));
  return v;
}
__device__ __forceinline__ double min8(double v) {
  v = fmin(v, __shfl_xor(v, 1));
  v = fmin(v, __shfl_xor(v, 2));
  v = fmin(v, __shfl_xor(v, 4));
  return v;
}
__device__ __forceinline__ float uniform_f(float x) {
  return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x)));
}

template <bool CNT>
__device__ void render_one_batch(const RenderArgs& a, uint32_t b, uint32_t lane) {
  const BatchRec rec = a.batches[b];
  double Pm[3][4];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int j = 0; j < 4; ++j) Pm[r][j] = a.dev->fc.Pm[r][j];

  // ---- corners: lane c (mod 8) takes corner c of [min, max]
  const int c = lane & 7;
  const double cx = (double)((c & 1) ? rec.mx[0] : rec.mn[0]);
  const double cy = (double)((c & 2) ? rec.mx[1] : rec.mn[1]);
  const double cz = (double)((c & 4) ? rec.mx[2] : rec.mn[2]);
  double Hc[3], M[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    Hc[r] = ((Pm[r][0] * cx + Pm[r][1] * cy) + Pm[r][2] * cz) + Pm[r][3];
    const double ar = ((fabs(Pm[r][0] * cx) + fabs(Pm[r][1] * cy)) + fabs(Pm[r][2] * cz)) + fabs(Pm[r][3]);
    M[r] = 0x1p-16 * max8(ar);
  }
  const double Wd = (double)a.W, Hd = (double)a.H;
  const uint64_t full = __ballot(1);
  const bool behind = __ballot(Hc[2] < -M[2]) == full;
  const bool left = __ballot(Hc[0] < -M[0]) == full;
  const bool right = __ballot(Hc[0] - Wd * Hc[2] > M[0] + Wd * M[2]) == full;
  const bool bottom = __ballot(Hc[1] < -M[1]) == full;
  const bool top = __ballot(Hc[1] - Hd * Hc[2] > M[1] + Hd * M[2]) == full;
  const bool culled = a.cull && (behind | left | right | bottom | top);

  if constexpr (CNT) {
    if (lane == 0) {
      atomicAdd((unsigned long long*)&a.stats[ST_BATCHES], 1ull);
      if (culled) atomicAdd((unsigned long long*)&a.stats[ST_CULLED], 1ull);
    }
  }
  if (culled) return;

  // ---- precision level (Sec. 3.3: < 500 px -> 10 bits)
  int k;
  if (a.precision == 10 || a.precision == 20 || a.precision == 30) {
    k = a.precision;
  } else {
    const bool front = __ballot(Hc[2] > 0.0) == full;
    double E = __builtin_inf();
    if (front) {
      const double u = Hc[0] / Hc[2], v = Hc[1] / Hc[2];
      const double ex = max8(u) - min8(u), ey = max8(v) - min8(v);
      E = ex > ey ? ex : ey;
    }
    k = E < (double)a.t10 ? 10 : (E < (double)a.t20 ? 20 : 30);
  }

  // ---- class of the per-point tests
  const bool safe = (Hc[2] - M[2] >= 0x1p-60) && (Hc[2] + M[2] <= 0x1p60);
  const bool ins = safe && (Hc[0] > M[0]) && (Hc[0] - Wd * Hc[2] < -(M[0] + Wd * M[2])) && (Hc[1] > M[1]) &&
                   (Hc[1] - Hd * Hc[2] < -(M[1] + Hd * M[2]));
  const int cls = (__ballot(ins) == full) ? CLS_INSIDE : ((__ballot(safe) == full) ? CLS_PARTIAL : CLS_SLOW);

  // ---- fold decode into the matrix: P[r][j] = fp32(Pm[r][j] (size_j 2^-k)),
  //      t[r] = fp32(Pm[r] . min + Pm[r][3])  (lower-corner decode)
  const double scale = k == 10 ? 0x1p-10 : (k == 20 ? 0x1p-20 : 0x1p-30);
  const double s[3] = {(double)rec.mx[0] - (double)rec.mn[0], (double)rec.mx[1] - (double)rec.mn[1],
                       (double)rec.mx[2] - (double)rec.mn[2]};
  Folded f;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int j = 0; j < 3; ++j) f.P[r][j] = uniform_f((float)(Pm[r][j] * (s[j] * scale)));
    f.t[r] = uniform_f((float)(((Pm[r][0] * (double)rec.mn[0] + Pm[r][1] * (double)rec.mn[1]) +
                                Pm[r][2] * (double)rec.mn[2]) +
                               Pm[r][3]));
  }

  if constexpr (CNT) {
    if (lane == 0) {
      const int li = k / 10 - 1;
      atomicAdd((unsigned long long*)&a.stats[ST_POINTS], (unsigned long long)rec.count);
      atomicAdd((unsigned long long*)&a.stats[ST_LB0 + li], 1ull);
      atomicAdd((unsigned long long*)&a.stats[ST_LP0 + li], (unsigned long long)rec.count);
    }
  }

  const uint32_t first = rec.first, count = rec.count;
  if (k == 10) {
    if (cls == CLS_INSIDE) raster_batch<10, CLS_INSIDE, CNT>(a, f, first, count, lane);
    else if (cls == CLS_PARTIAL) raster_batch<10, CLS_PARTIAL, CNT>(a, f, first, count, lane);
    else raster_batch<10, CLS_SLOW, CNT>(a, f, first, count, lane);
  } else if (k == 20) {
    if (cls == CLS_INSIDE) raster_batch<20, CLS_INSIDE, CNT>(a, f, first, count, lane);
    else if (cls == CLS_PARTIAL) raster_batch<20, CLS_PARTIAL, CNT>(a, f, first, count, lane);
    else raster_batch<20, CLS_SLOW, CNT>(a, f, first, count, lane);
  } else {
    if (cls == CLS_INSIDE) raster_batch<30, CLS_INSIDE, CNT>(a, f, first, count, lane);
    else if (cls == CLS_PARTIAL) raster_batch<30, CLS_PARTIAL, CNT>(a, f, first, count, lane);
    else raster_batch<30, CLS_SLOW, CNT>(a, f, first, count, lane);
  }
}

// One wave64 workgroup per batch (Sec. 3.2: one workgroup per batch).
template <bool CNT>
__global__ void __launch_bounds__(64) k_render(RenderArgs a) {
  const uint32_t b = blockIdx.x;
  if (b >= a.nb) return;
  render_one_batch<CNT>(a, b, threadIdx.x);
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

hipError_t launch_clear(uint64_t* vb, uint64_t npix, const ViewArgs& v, uint32_t W, uint32_t H, DevBlock* dev,
                        int reset_stats, hipStream_t s) {
  const uint64_t n4 = npix / 2;
  uint64_t blocks = (n4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_clear, dim3((uint32_t)blocks), dim3(256), 0, s, reinterpret_cast<uint4*>(vb), n4, vb, npix, v,
                     W, H, dev, reset_stats);
  return hipGetLastError();
}

hipError_t launch_render(const RenderArgs& a, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  if (a.counters)
    hipLaunchKernelGGL(k_render<true>, dim3(a.nb), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(k_render<false>, dim3(a.nb), dim3(64), 0, s, a);
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

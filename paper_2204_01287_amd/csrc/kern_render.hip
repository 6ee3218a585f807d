// Render-path kernels for gfx950: clear, classify, resolve.  The
// point loops and the persistent render kernels are in raster_core.h, compiled
// once per workgroup shape (kern_raster.hip).
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
// a wave ballot (tiled batches from its front, untiled ones from its back).
// The persistent render kernel then hands the live batches to its workgroups
// through atomic work queues, the untiled ones (whose points go to the global
// atomic minimum one by one) spread evenly over the frame: concentrated, their
// atomics contend and the frame is slower.  Classes:
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
// box (plus one pixel of margin) covers at most tile_max pixels (no more than
// the LDS tile of the render kernel that follows), the points
// are first combined by minimum in an LDS tile over that box (behind an
// early-depth read of the tile entry); afterwards each covered tile pixel
// goes into the global atomic minimum once.  The minimum is associative and commutative, so this
// equals combining every point globally; it replaces one global round trip
// per point by one per covered pixel.  Larger batches (close to the eye,
// few points per pixel) combine every point globally.
#include "raster_core.h"

namespace ptr {
namespace {

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
    if (hdr && threadIdx.x == 0) {
      hdr->live_count = 0;
      hdr->direct_count = 0;
    }
    if (hdr && threadIdx.x < RENDER_QUEUES) hdr->queue[threadIdx.x][0] = 0;
    if (reset_stats && threadIdx.x < 16) dev->stats[threadIdx.x] = 0;
  }
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
// projects to less than lod_px pixels.  max_bands: see below.  tile_max: the most pixels a tiled
// batch's rectangle may cover (the render kernel's LDS tile or less).
__device__ __forceinline__ bool decide_batch(const BatchRec& rec, const double (&Pm)[3][4], uint32_t W, uint32_t Hh,
                                             int32_t precision, int32_t cull, float t10, float t20,
                                             const LodNode* node, float lod_px, uint32_t tile_max,
                                             uint32_t max_bands, LiveBatch& out,
                                             bool& culled, int& li) {
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
    uint32_t tiled = 0, banded = 0, x0 = 0, y0 = 0, tw = 0, th = 0;
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
      const double rw = fx1 - fx0 + 1.0, area = rw * (fy1 - fy0 + 1.0);
      if (fx1 >= fx0 && fy1 >= fy0 && area <= (double)tile_max) tiled = 1;
      // larger, but at most max_bands tiles and one tile wide, at 10 bits: rendered band by band
      else if (k == 10 && max_bands > 1 && fx1 >= fx0 && fy1 >= fy0 && rw <= (double)tile_max &&
               area <= (double)max_bands * (double)tile_max)
        banded = 1;
      if (tiled || banded) {
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
    out.mode = (uint32_t)k | ((uint32_t)cls << 8) | (tiled << 16) | (banded << 17);
    out.rect_xy = x0 | (y0 << 16);
    out.rect_wh = tw | (th << 16);
    out.pad[0] = out.pad[1] = out.pad[2] = 0;
    live = true;
    li = k / 10 - 1;
  }
  return live;
}

// One batch per thread; live batches are appended to a compact list (wave
// ballot + one atomic per wave).  With clear_vb the launch also fills the
// visibility buffer with PR_EMPTY (grid-stride 16-byte stores, overlapping the
// prologue's arithmetic); the grid then has at least enough threads for that.
template <bool CNT>
__global__ void __launch_bounds__(256) k_classify(RenderArgs a) {
  const uint32_t b = blockIdx.x * 256u + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63;
  if (a.clear_vb) {
    const uint64_t npix = (uint64_t)a.W * a.H, n4 = npix / 2;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint4* const vb4 = reinterpret_cast<uint4*>(a.vb);
    const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint64_t i = b; i < n4; i += stride) vb4[i] = ones;
    if (b == 0 && (npix & 1)) a.vb[npix - 1] = ~0ull;
  }
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
                        a.lod_px, a.tile_max, a.max_bands, out, culled, li);
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
      const unsigned long long words = 4ull * lp[0] + 8ull * lp[1] + 12ull * lp[2];
      if (words) atomicAdd((unsigned long long*)&a.stats[ST_WORDS], words);
    }
  }
  // tiled batches from the front of the list, untiled ones from the back, and
  // every live batch's slot into the batch-order index (for the shading
  // pass): the wave's prefix there is the sum of its two list prefixes
  const bool tiled = live && ((out.mode >> 16) & 1u);
  const uint64_t mt = __ballot(tiled), md = __ballot(live && !tiled);
  uint64_t pre = 0;
  if (lane == 0 && (mt | md))
    pre = atomicAdd(reinterpret_cast<unsigned long long*>(&a.hdr->live_count),
                    (unsigned long long)__popcll(mt) | ((unsigned long long)__popcll(md) << 32));
  pre = __shfl(pre, 0);
  const uint32_t bt = (uint32_t)pre, bd = (uint32_t)(pre >> 32);
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  if (live) {
    const uint32_t slot = tiled ? bt + (uint32_t)__popcll(mt & lt) : a.nb - 1u - (bd + (uint32_t)__popcll(md & lt));
    a.live[slot] = out;
    a.order[bt + bd + (uint32_t)__popcll((mt | md) & lt)] = slot;
  }
}

// Several views: one thread per batch runs the prologue for each view of
// this launch; the records go to fixed slots (batch, view), the batch's live
// views to one run record (wave ballot + one atomic per wave): from the back
// of the run list if no live view is tiled, else from its front.
template <bool CNT>
__global__ void __launch_bounds__(256) k_classify_views(ClassifyViewsArgs a) {
  const uint32_t b = blockIdx.x * 256u + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63;
  const bool valid = b < a.nb;
  uint64_t mask = 0;
  bool tiled_any = false;
  int lmax = -1;  // highest level index among the live views (the words the run streams)
  uint64_t nculled = 0, pts = 0, lp[3] = {0, 0, 0}, lb[3] = {0, 0, 0}, words = 0;
  if (valid) {
    const BatchRec rec = a.batches[b];
    for (uint32_t v = 0; v < a.nchunk; ++v) {
      LiveBatch out;
      bool culled = false;
      int li = 0;
      if (decide_batch(rec, a.v[v].Pm, a.v[v].W, a.v[v].H, a.precision, a.cull, a.t10, a.t20,
                       a.nodes ? a.nodes + b : nullptr, a.lod_px, a.tile_max, a.max_bands, out, culled, li)) {
        a.sub[(uint64_t)b * a.nviews + a.view0 + v] = out;
        mask |= 1ull << v;
        tiled_any = tiled_any || ((out.mode >> 16) & 1u);
        lmax = li > lmax ? li : lmax;
        if constexpr (CNT) {
          pts += rec.count;
          lp[li] += rec.count;
          lb[li] += 1;
        }
      }
      if constexpr (CNT) nculled += culled ? 1u : 0u;
    }
    if (lmax >= 0) words = 4ull * (uint64_t)(lmax + 1) * rec.count;
  }
  if constexpr (CNT) {
    uint64_t nbv = valid ? a.nchunk : 0u;
    for (int o = 32; o > 0; o >>= 1) {
      nbv += __shfl_xor(nbv, o);
      nculled += __shfl_xor(nculled, o);
      pts += __shfl_xor(pts, o);
      words += __shfl_xor(words, o);
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
      if (words) atomicAdd((unsigned long long*)&a.stats[ST_WORDS], (unsigned long long)words);
    }
  }
  const bool live = mask != 0, direct = live && !tiled_any;
  const uint64_t mt = __ballot(live && !direct), md = __ballot(direct);
  uint64_t pre = 0;
  if (lane == 0 && (mt | md))
    pre = atomicAdd(reinterpret_cast<unsigned long long*>(&a.hdr->live_count),
                    (unsigned long long)__popcll(mt) | ((unsigned long long)__popcll(md) << 32));
  pre = __shfl(pre, 0);
  const uint32_t bt = (uint32_t)pre, bd = (uint32_t)(pre >> 32);
  if (live) {
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    Run r;
    r.batch = b;
    r.view0 = a.view0;
    r.mask = mask;
    if (direct) a.runs[a.cap - 1u - (bd + (uint32_t)__popcll(md & lt))] = r;
    else a.runs[bt + (uint32_t)__popcll(mt & lt)] = r;
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
    if (threadIdx.x == 0) {
      a.hdr->live_count = 0;
      a.hdr->direct_count = 0;
    }
    if (threadIdx.x < RENDER_QUEUES) a.hdr->queue[threadIdx.x][0] = 0;
    if (a.reset_stats && threadIdx.x < 16) a.stats[threadIdx.x] = 0;
  }
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

hipError_t launch_classify(const RenderArgs& a, hipStream_t s) {
  uint64_t blocks = ((uint64_t)a.nb + 255) / 256;
  if (a.clear_vb) {
    uint64_t cb = ((uint64_t)a.W * a.H / 2 + 255) / 256;
    if (cb > 4096) cb = 4096;
    if (cb < 1) cb = 1;
    if (cb > blocks) blocks = cb;
  }
  if (blocks == 0) return hipSuccess;
  if (a.counters)
    hipLaunchKernelGGL(k_classify<true>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_classify<false>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
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

hipError_t launch_resolve(const uint64_t* vb, uint64_t npix, const uint32_t* colors, uint64_t ncolors,
                          uint32_t clear_rgba, uint32_t* fb, hipStream_t s) {
  const uint64_t threads = (npix + 3) / 4;
  const uint64_t blocks = (threads + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_resolve, dim3((uint32_t)blocks), dim3(256), 0, s, vb, npix, colors, ncolors, clear_rgba, fb);
  return hipGetLastError();
}

}  // namespace ptr

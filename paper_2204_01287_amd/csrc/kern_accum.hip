// High-quality shading pass (Sec. 3.6) for gfx950: the sums of the colours of
// the points near each pixel's closest depth, and their average.
//
// Its own translation unit: the pass runs eight-wave workgroups (two per CU,
// each with an 80 KiB LDS tile of thresholds and sums) over the point loops
// of raster_core.h.
#define PR_WAVES 8
#include "raster_core.h"

namespace ptr {
namespace {

// ------------------------------------------------------------------ shading
// High-quality shading (Sec. 3.6), second pass over the live batches of the
// frame's render: every drawn point within the depth window of its pixel
// adds its colour and a count.  Tiled batches whose rectangle fits HQS_TILE
// pixels stage the thresholds of the rectangle in LDS, add into LDS sums and
// flush each covered pixel with two global additions; the others read the
// visibility buffer and add globally per point.  Integer sums: the result
// does not depend on the order of the additions.
// 4064 pixels: 16 KiB of thresholds + 64 KiB of sums (+ s_next), two workgroups in 160 KiB of LDS
constexpr uint32_t HQS_TILE = 4064;

// Thresholds fl32(closest depth * window) of a tw x th rectangle at (x0, y0)
// into the LDS tile, and its sums zeroed.
__device__ __forceinline__ void stage_band(const RenderArgs& a, float* thr, uint64_t* sums, uint32_t tid, uint32_t x0,
                                           uint32_t y0, uint32_t tw, uint32_t th) {
  const uint32_t n = tw * th;
  for (uint32_t e = tid; e < n; e += THREADS) {
    const uint32_t ly = e / tw, lx = e - ly * tw;
    const uint64_t key = a.vb[(y0 + ly) * a.W + (x0 + lx)];
    thr[e] = __uint_as_float((uint32_t)(key >> 32)) * a.window;
    sums[2 * e] = 0;
    sums[2 * e + 1] = 0;
  }
}

// Every pixel of the rectangle with a point in its sums: two global additions.
__device__ __forceinline__ void flush_band(const RenderArgs& a, const uint64_t* sums, uint32_t tid, uint32_t x0,
                                           uint32_t y0, uint32_t tw, uint32_t th) {
  const uint32_t n = tw * th;
  for (uint32_t e = tid; e < n; e += THREADS) {
    const uint64_t bn = sums[2 * e + 1];
    if (bn >> 32) {
      const uint32_t ly = e / tw, lx = e - ly * tw;
      uint64_t* const g = a.accum + 2 * (uint64_t)((y0 + ly) * a.W + (x0 + lx));
      __hip_atomic_fetch_add(g, sums[2 * e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(g + 1, bn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void __launch_bounds__(THREADS) k_accum(RenderArgs a) {
  __shared__ float thr[HQS_TILE];
  __shared__ uint64_t sums[2 * HQS_TILE];
  __shared__ uint32_t s_next;
  const uint32_t tid = threadIdx.x, wave = uni(tid >> 6), lane = tid & 63;
  const uint32_t q = blockIdx.x % RENDER_QUEUES;
  uint32_t* const qc = &a.hdr->queue[q][0];
  // batch order (Morton order for sorted clouds): the sums' lines of neighbouring
  // batches stay in the caches; measured faster than the render's order here
  const uint32_t nlive = a.hdr->live_count + a.hdr->direct_count;
  if (tid == 0) {
    const uint32_t p = atomicAdd(qc, 1u) * RENDER_QUEUES + q;
    s_next = p < nlive ? a.order[p] : ~0u;
  }
  const Streams st = {a.low, a.med, a.high, a.colors};
  __syncthreads();
  uint32_t i = uni(s_next);
  uint32_t natom = 0;
  while (i != ~0u) {
    uint32_t grab = 0;
    if (tid == 0) {
      const uint32_t p = atomicAdd(qc, 1u) * RENDER_QUEUES + q;
      grab = p < nlive ? a.order[p] : ~0u;
    }
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
    // 10-bit batches with a proven rectangle too large for the tile but at most
    // one tile wide: band by band (stage the band's thresholds, add, flush)
    const bool banded = !tiled && k == 10 && ((mode >> 16) & 3u) && L.tw <= HQS_TILE;
    if (banded) {
      const uint32_t th = L.th, bh = HQS_TILE / L.tw;
      L.cx = in_vgpr(uni(0x4B000000u + x0));
      for (uint32_t by = 0; by < th; by += bh) {
        L.th = min(bh, th - by);
        L.cy = in_vgpr(uni(0x4B000000u + y0 + by));
        stage_band(a, thr, sums, tid, x0, y0 + by, L.tw, L.th);
        __syncthreads();
        raster_by_class<10, true, true, true>(cls, L, st, sums, first, count, wave, lane, natom);
        __syncthreads();  // the band's sums are complete; s_next has been read
        if (by == 0 && tid == 0) s_next = grab;
        flush_band(a, sums, tid, x0, y0 + by, L.tw, L.th);
        __syncthreads();  // tile free again
      }
      i = uni(s_next);
      continue;
    }
    L.cx = in_vgpr(uni(0x4B000000u + (tiled ? x0 : 0u)));
    L.cy = in_vgpr(uni(0x4B000000u + (tiled ? y0 : 0u)));
    if (tiled) {
      stage_band(a, thr, sums, tid, x0, y0, L.tw, L.th);
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
    if (tiled) flush_band(a, sums, tid, x0, y0, L.tw, L.th);
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

}  // namespace

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

}  // namespace ptr

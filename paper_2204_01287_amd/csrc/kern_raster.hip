// One compiled workgroup shape of the persistent render kernels in
// raster_core.h.  The build compiles this file once per entry of
// PR_RASTER_SHAPES (internal.h), with PR_WAVES, PR_DEPTH and PR_TILE set, and
// each copy exports its launchers as one RasterShape record.
#include "raster_core.h"

namespace ptr {
namespace {

constexpr int SW = WAVES, SD = PREFETCH, ST = (int)TILE_MAX;

hipError_t render(const RenderArgs& a, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  const uint32_t blocks = a.grid < a.nb ? a.grid : a.nb;
  if (a.counters)
    hipLaunchKernelGGL((k_render<true, SW, SD, ST>), dim3(blocks), dim3(THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((k_render<false, SW, SD, ST>), dim3(blocks), dim3(THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t render_views(const RenderViewsArgs& a, uint64_t max_runs, int counters, hipStream_t s) {
  if (max_runs == 0) return hipSuccess;
  const uint32_t blocks = a.grid < max_runs ? a.grid : (uint32_t)max_runs;
  if (counters)
    hipLaunchKernelGGL((k_render_views<true, SW, SD, ST>), dim3(blocks), dim3(THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((k_render_views<false, SW, SD, ST>), dim3(blocks), dim3(THREADS), 0, s, a);
  return hipGetLastError();
}

int per_cu(int views) {
  int n = 0;
  const hipError_t e =
      views ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_render_views<false, SW, SD, ST>, THREADS, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_render<false, SW, SD, ST>, THREADS, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

// A host function (not a variable holding host pointers), so that the device
// pass of this file references none of them.
const RasterShape* PR_SHAPE_NAME(PR_WAVES, PR_DEPTH, PR_TILE)() {
  static const RasterShape shape = {PR_WAVES, PR_DEPTH, PR_TILE, render, render_views, per_cu};
  return &shape;
}

}  // namespace ptr

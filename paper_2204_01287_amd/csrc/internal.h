// Internal declarations shared by the host runtime and the kernel files of
// libptraster.so.  Not part of the ABI (see include/ptraster.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ptr {

struct BatchRec {  // identical layout to pr_batch
  uint32_t first, count;
  float mn[3], mx[3];
};
static_assert(sizeof(BatchRec) == 32, "batch record is 32 bytes");

// Octree node of a batch in a level-of-detail layout (identical layout to pr_lod_node).
struct LodNode {
  double origin[3], edge;
  uint32_t level, pad[3];
};
static_assert(sizeof(LodNode) == 48, "LOD node record is 48 bytes");

// Device-side context block (one per pr_ctx), 4 KiB.
struct DevBlock {
  uint64_t stats[16];     // batches, culled, points, lvl_b[3], lvl_p[3], atomics, words bytes
  uint32_t flags[16];     // [0] non-finite coordinate seen
  uint64_t sink;          // streaming read probe
};
enum { ST_BATCHES = 0, ST_CULLED, ST_POINTS, ST_LB0, ST_LB1, ST_LB2, ST_LP0, ST_LP1, ST_LP2, ST_ATOMICS, ST_WORDS };

// A batch that survived culling, with everything its workgroup needs
// (written by the classify kernel, read with scalar loads by the render kernel).
struct LiveBatch {
  uint32_t first, count;
  uint32_t mode;     // level (10, 20, 30) | class << 8 | tiled << 16 | banded << 17
  uint32_t rect_xy;  // tile rectangle origin: x0 | y0 << 16
  uint32_t rect_wh;  // tile rectangle size: tw | th << 16
  float P[3][3];     // folded per-batch matrix (binary32)
  float t[3];
  uint32_t pad[3];
};
static_assert(sizeof(LiveBatch) == 80, "live batch record is 80 bytes");

// Per-frame counters of the render path (in the cloud's scratch area).  The
// live batches are handed out through RENDER_QUEUES work queues (queue q
// owns queue positions q, q + RENDER_QUEUES, ...), each counter on its own
// 128-byte line: one shared counter serialises every workgroup's request.
// A position maps to a live-list slot with the untiled batches spread evenly
// among the tiled ones (live_slot in raster_core.h).
constexpr uint32_t RENDER_QUEUES = 8;
// A 10-bit batch whose tile rectangle exceeds the tile but is at most one
// tile wide and max_bands tiles large is rendered in bands of rows that fit
// the tile (max_bands: a tuning; 1 = no bands).
constexpr uint32_t DEFAULT_BANDS = 4, MAX_BANDS = 64;
struct FrameHeader {
  // One 64-bit counter (classify adds tiled | untiled << 32 with one atomic
  // per wave, so the two prefixes it returns come from one order):
  uint32_t live_count;    // tiled live batches / runs with a tiled view, stored from the front of the list
  uint32_t direct_count;  // untiled live batches / runs with no tiled view, stored from the back
  uint32_t pad[30];
  uint32_t queue[RENDER_QUEUES][32];  // queue[q][0]: next position of queue q
};
static_assert(sizeof(FrameHeader) == 128 * (1 + RENDER_QUEUES), "frame header layout");
static_assert(offsetof(FrameHeader, direct_count) == offsetof(FrameHeader, live_count) + 4, "64-bit counter pair");

// header, live list (nb records), batch-order index of the live list (nb slots)
inline uint64_t frame_area_bytes(uint64_t nb) { return sizeof(FrameHeader) + (sizeof(LiveBatch) + 4) * nb; }

struct RenderArgs {
  const uint32_t* low;
  const uint32_t* med;
  const uint32_t* high;
  const BatchRec* batches;
  LiveBatch* live;
  uint32_t* order;  // live-list slots in batch order (read by the shading pass)
  FrameHeader* hdr;
  uint64_t* vb;
  uint64_t* stats;
  double Pm[3][4];  // pixel-space matrix rows (hx, hy, hw), binary64
  uint32_t nb, W, H;
  int32_t precision, cull, counters;
  float t10, t20;
  uint32_t grid;    // persistent render workgroups
  uint32_t tile_max;     // classify: largest rectangle (pixels) a tiled batch may cover
  uint32_t max_bands;    // classify: largest rectangle of a banded batch, in tiles
  const LodNode* nodes;  // LOD layouts: node per batch (else nullptr)
  float lod_px;          // > 0: cull nodes below the root whose cube projects below lod_px pixels
  uint32_t clear_vb;     // classify: also fill vb (W x H) with PR_EMPTY
  // high-quality shading pass only
  const uint32_t* colors;
  uint64_t* accum;  // two words per pixel
  float window;
};

// ---- several views in one launch
// A live batch of a multi-view frame: the batch and the mask of its live
// views among views view0 .. view0 + 63.  Its render records sit at
// sub[batch * nviews + view].
constexpr uint32_t MAX_VIEWS = 64;
constexpr uint32_t VIEW_CHUNK = 16;  // views per classify launch (kernel-argument size)
struct Run {
  uint32_t batch, view0;
  uint64_t mask;
};
static_assert(sizeof(Run) == 16, "run record is 16 bytes");
struct ViewIn {  // what the prologue needs of one view
  double Pm[3][4];
  uint32_t W, H;
};
struct ViewOut {  // what the point loop needs of one view
  uint64_t* vb;
  uint32_t W, H;
};
struct ClassifyViewsArgs {
  const BatchRec* batches;
  LiveBatch* sub;
  Run* runs;
  FrameHeader* hdr;
  uint64_t* stats;
  uint32_t nb, nviews, view0, nchunk;  // all views, first view of this launch, views in it
  int32_t precision, cull;
  float t10, t20;
  const LodNode* nodes;
  float lod_px;
  uint32_t tile_max, max_bands;
  uint32_t cap;  // run slots (one per batch and classify launch)
  ViewIn v[VIEW_CHUNK];
};
struct RenderViewsArgs {
  const uint32_t* low;
  const uint32_t* med;
  const uint32_t* high;
  const LiveBatch* sub;
  const Run* runs;
  FrameHeader* hdr;
  uint64_t* stats;
  uint32_t nviews, grid, cap;
  ViewOut v[MAX_VIEWS];
};
struct ClearViewsArgs {
  FrameHeader* hdr;
  uint64_t* stats;
  uint32_t nviews, clear, reset_stats;
  ViewOut v[MAX_VIEWS];
};
// header, runs (one per batch and launch of classify), records (one per batch and view)
inline uint64_t views_work_bytes(uint64_t nb, uint32_t nviews) {
  const uint64_t chunks = (nviews + VIEW_CHUNK - 1) / VIEW_CHUNK;
  return sizeof(FrameHeader) + sizeof(Run) * nb * chunks + sizeof(LiveBatch) * nb * nviews;
}

// ---- render path (kern_render.hip)
hipError_t launch_clear(uint64_t* vb, uint64_t npix, DevBlock* dev, FrameHeader* hdr, int reset_stats, hipStream_t s);
// classify: cull, level, fold, compaction into the live list (a.tile_max bounds the tiles)
hipError_t launch_classify(const RenderArgs& a, hipStream_t s);
// several views: clear, classify per chunk of VIEW_CHUNK views, then one persistent render launch
hipError_t launch_clear_views(const ClearViewsArgs& a, hipStream_t s);
hipError_t launch_classify_views(const ClassifyViewsArgs& a, int counters, hipStream_t s);

// ---- persistent render kernels, one compiled workgroup shape each (kern_raster.hip)
// Every shape computes the same result; they differ in speed only.  The
// classify launch before a render must bound its tiles by the shape's tile.
struct RasterShape {
  uint32_t waves;  // waves of 64 lanes per workgroup
  uint32_t depth;  // groups of 256 points in flight per wave
  uint32_t tile;   // pixels of the LDS tile
  // the live list of the last launch_classify (a.grid workgroups at most)
  hipError_t (*render)(const RenderArgs& a, hipStream_t s);
  // the runs of the last classify_views launches
  hipError_t (*render_views)(const RenderViewsArgs& a, uint64_t max_runs, int counters, hipStream_t s);
  // workgroups per CU that fit at once (views = 0: single-view kernel, 1: multi-view kernel)
  int (*per_cu)(int views);
};
// The compiled shapes: X(waves, depth, tile).  The first is the default: four
// workgroups of 4 waves fill a CU's 16 wave slots at 128 VGPRs, and a tile of
// 4992 pixels (39 KiB) is the largest that still lets four of them share the
// CU's 160 KiB of LDS; the larger tile leaves fewer batches to bands and to
// the global path than 4096 pixels do.
#define PR_RASTER_SHAPES(X)                                                                                  \
  X(4, 5, 4992) X(4, 3, 4992) X(4, 4, 4992) X(4, 6, 4992) X(4, 5, 2048) X(2, 5, 2048) X(2, 5, 4096)        \
  X(8, 5, 8192) X(1, 5, 1024) X(16, 5, 16384) X(16, 4, 16384) X(8, 5, 16384) X(4, 1, 4992) X(4, 5, 4096)
#define PR_SHAPE_NAME_(W_, D_, T_) raster_shape_w##W_##_d##D_##_t##T_
#define PR_SHAPE_NAME(W_, D_, T_) PR_SHAPE_NAME_(W_, D_, T_)
#define PR_DECLARE_SHAPE(W_, D_, T_) const RasterShape* PR_SHAPE_NAME_(W_, D_, T_)();
PR_RASTER_SHAPES(PR_DECLARE_SHAPE)
#undef PR_DECLARE_SHAPE

hipError_t launch_resolve(const uint64_t* vb, uint64_t npix, const uint32_t* colors, uint64_t ncolors,
                          uint32_t clear_rgba, uint32_t* fb, hipStream_t s);
// high-quality shading (kern_accum.hip): zero the sums, the shading pass over
// the live batches of the last classify + render, the averaging resolve
hipError_t launch_accumulate(const RenderArgs& a, hipStream_t s);
uint32_t accum_grid(int device);
hipError_t launch_resolve_hqs(const uint64_t* accum, uint64_t npix, uint32_t clear_rgba, uint32_t* fb, hipStream_t s);

// ---- HBM streaming probes (kern_stream.hip): copy src -> dst, or (dst null) only read src (sink: a marker
// store that keeps the loads)
hipError_t launch_stream(const void* src, void* dst, uint64_t bytes, uint64_t* sink, uint32_t blocks, hipStream_t s);

// ---- load-time build (kern_build.hip)
struct SortScratch {
  uint64_t* keys0;
  uint64_t* keys1;
  uint32_t* vals1;  // vals0 is the caller's perm buffer
  uint32_t* hist;   // 256 * nblk
  uint32_t* part;   // scan partial sums
  uint32_t* aabb;   // 6 ordered keys: min x,y,z then max x,y,z
  uint64_t nblk, npart;
};
// Scratch layout for n points (a Morton order); returns total bytes.
uint64_t sort_scratch_layout(uint64_t n, uint8_t* base, SortScratch* out);
uint64_t small_scratch_bytes();

hipError_t launch_finite_check(const float* xyz, uint64_t n, uint32_t* flag, hipStream_t s);
hipError_t launch_iota(uint32_t* p, uint64_t n, hipStream_t s);
// cloud box (with the finite check: flag) and Morton codes
hipError_t launch_morton_codes(const float* xyz, uint64_t n, uint32_t* aabb, uint64_t* keys, uint32_t* vals,
                               uint32_t* flag, hipStream_t s);
hipError_t radix_sort_pairs(const SortScratch& sc, uint32_t* vals0, uint64_t n, hipStream_t s);
// positions and colours in sorted order (perm[sorted] = original), through
// 16-byte records in the key buffers (xyz_out may be xyz: the gather reads
// the records)
// spread: every batch of batch_size points (the last one shorter) in the spread
// order (position r <- Morton rank (r * m) mod c, m = spread_step(c)); perm is
// then rewritten in that order
hipError_t launch_gather(const SortScratch& sc, const float* xyz, const uint32_t* rgba, uint32_t* perm,
                         uint64_t n, uint32_t batch_size, bool spread, float* xyz_out, uint32_t* colors,
                         hipStream_t s);
// the first integer >= floor(c / 4) + 1 coprime with c
uint64_t spread_step(uint64_t c);
hipError_t launch_batch_bbox(const float* xyz, uint64_t n, uint32_t S, uint64_t nb, BatchRec* out, hipStream_t s);
// variable-size batches: recs[b].first / .count are set, the boxes are filled in
hipError_t launch_batch_bbox_spans(const float* xyz, uint64_t nb, BatchRec* recs, hipStream_t s);
hipError_t launch_quantize_spans(const float* xyz, uint64_t nb, const BatchRec* recs, uint32_t* low, uint32_t* med,
                                 uint32_t* high, hipStream_t s);
hipError_t launch_quantize(const float* xyz, uint64_t n, uint32_t S, const BatchRec* batches, uint32_t* low,
                           uint32_t* med, uint32_t* high, hipStream_t s);

}  // namespace ptr

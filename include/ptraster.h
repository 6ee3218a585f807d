/* ptraster.h -- C ABI of the MI355X (gfx950) point rasterizer.
 *
 * Method: Schuetz, Kerbl & Wimmer, "Software Rasterization of 2 Billion
 * Points in Real Time" (HPG 2022).  One-pixel points are grouped into batches
 * of consecutive points with a bounding box (Sec. 3.1); each GPU workgroup
 * frustum-culls its batch and chooses 10-, 20- or 30-bit coordinates relative
 * to the batch box (Sec. 3.2, 3.3, Eq. 1); every visible point is written with
 * a 64-bit atomic minimum of (depth bits << 32 | point index) into a
 * visibility buffer (Sec. 3.2 rasterization listing), and a resolve pass maps
 * indices to colours (Sec. 3.3, visibility buffer).
 *
 * Conventions for every call:
 *   - Every call returns pr_status (0 = PR_OK, negative = error) and never
 *     throws; pr_last_error() gives a message for the calling thread.
 *   - Device work is enqueued on the context's HIP stream and is asynchronous
 *     unless stated.  Argument errors are reported at once; faults and
 *     non-finite input found on the device are reported by the next call
 *     that synchronises (pr_build_batches, pr_get_stats, pr_sync).
 *   - Ownership: the caller allocates and owns every device buffer (cloud
 *     buffers sized by pr_cloud_sizes, visibility buffers, framebuffers).
 *     The library allocates device memory only in pr_create (a few hundred
 *     bytes of frame constants and counters); never on the render path.
 *   - Layouts: visibility buffer (VB) = uint64_t[h*w], framebuffer (FB) =
 *     uint32_t[h*w], both row-major with row 0 at the bottom (NDC y = -1):
 *     pixel (px, py) is element py*w + px.  Colours are opaque 32-bit words
 *     (RGBA8, R in the low byte).  view and proj are float[16], row-major
 *     storage, column vectors: clip = proj * view * (x, y, z, 1)^T in OpenGL
 *     clip space (w_clip = -z_eye for a perspective projection).
 *   - Keys: VB[p] = (bits of the point's w_clip as float) << 32 | point index,
 *     where the index is the point's position in render order (after the
 *     optional Morton sort; perm[] maps it back to input order).  Empty
 *     pixels hold PR_EMPTY.  Keys compare as unsigned 64-bit integers.
 *   - Limits: n < 2^32; 1 <= w, h <= 8192; batch sizes are multiples of 4.
 *   - Contexts and streams: a built cloud may be rendered and resolved through
 *     any context on its device; pr_build_batches uses the context that
 *     loaded it.  With one context per HIP stream, pr_render_views frames
 *     (each with a work buffer of its own) and resolves may overlap;
 *     pr_render and pr_render_hqs keep their frame in the cloud's scratch
 *     buffer, so those calls on one cloud must not overlap.
 */
#ifndef PTRASTER_H
#define PTRASTER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PR_OK = 0,
  PR_EINVAL = -1,     /* null pointer, undersized buffer, bad option, wrong cloud state */
  PR_ENOMEM = -2,     /* host allocation failed */
  PR_EDEVICE = -3,    /* no usable GPU, or a HIP call / kernel failed */
  PR_ESTATE = -4,     /* call out of order (e.g. render before build) */
  PR_ENONFINITE = -5, /* NaN or Inf in coordinates or matrices */
  PR_ERANGE = -6      /* size outside the limits above */
} pr_status;

#define PR_EMPTY 0xFFFFFFFFFFFFFFFFull

enum { PR_ADAPTIVE = 0, PR_FORCE10 = 10, PR_FORCE20 = 20, PR_FORCE30 = 30 };

typedef struct pr_ctx pr_ctx;     /* device ordinal, HIP stream, frame constants, counters */
typedef struct pr_cloud pr_cloud; /* host handle with non-owning device pointers */

/* Batch record (Sec. 3.1: first point, number of points, bounding box). 32 bytes. */
typedef struct {
  uint32_t first, count;
  float min[3], max[3];
} pr_batch;

/* Octree node of a batch in a level-of-detail layout (Sec. 3.5): the node's
 * cube (origin and edge, binary64) and its level (0 = root).  48 bytes. */
typedef struct {
  double origin[3], edge;
  uint32_t level, pad[3];
} pr_lod_node;

/* Byte sizes of the cloud buffers; see pr_cloud_bufs. */
typedef struct {
  uint64_t xyz, rgba, low, med, high, colors, perm, batches, scratch, nodes;
} pr_sizes;

/* Caller-allocated device buffers of one cloud (each 256-byte aligned).
 *   xyz     float[n][3]   positions (AoS), filled by pr_load_points; after a
 *                         Morton build they are in render order
 *   rgba    uint32[n]     input colours, filled by pr_load_points
 *   low     uint32[n]     Eq. 1 bits 29..20 per axis, packed x | y<<10 | z<<20
 *   med     uint32[n]     bits 19..10, same packing
 *   high    uint32[n]     bits 9..0, same packing
 *   colors  uint32[n]     colours in render order
 *   perm    uint32[n]     perm[render index] = input index
 *   batches pr_batch[nb]  nb = ceil(n / batch_size)
 *   scratch               load-time working memory (Morton sort) and the
 *                         frame work area of pr_render
 *   nodes   pr_lod_node[nb] LOD layouts only (pr_build_batches_spans); may
 *                         be NULL otherwise
 * capacity must hold the sizes the caller allocated (normally the output of
 * pr_cloud_sizes); pr_build_batches checks it and fails with PR_EINVAL if a
 * buffer is too small for (n, batch_size, morton). */
typedef struct {
  void *xyz, *rgba, *low, *med, *high, *colors, *perm, *batches, *scratch, *nodes;
  pr_sizes capacity;
} pr_cloud_bufs;

/* Per-frame options; NULL means the defaults in brackets. */
typedef struct {
  int32_t precision; /* PR_ADAPTIVE [default] or PR_FORCE10/20/30 (Sec. 3.3)          */
  int32_t cull;      /* 1 [default]: skip batches whose box misses the view (Sec. 3.2)  */
  float t10;         /* adaptive: 10 bits if the projected box is < t10 px [500]         */
  float t20;         /* adaptive: 20 bits if < t20 px [512000 = 500 * 2^10], else 30    */
  int32_t counters;  /* 1: accumulate pr_stats for this frame (extra atomics) [0]       */
  int32_t accumulate;/* 1: do not clear visbuf first; points combine with its content by
                        minimum, so a sequence of renders into one buffer equals the
                        elementwise minimum of the separate results [0]               */
  float lod_px;      /* LOD layouts (Sec. 3.5): > 0 culls every batch of a node below the
                        root whose cube projects to less than lod_px pixels (the larger
                        side of the screen box of its 8 corners; a cube reaching w <= 0 is
                        kept) [0 = no LOD culling; the paper suggests 100]             */
} pr_render_opts;

/* Frame counters (Table 2 definitions): processed batches = every batch,
 * processed points = points in batches that were not culled; atomics = number
 * of 64-bit atomic minimum calls issued, which depends on timing and is
 * reported, never compared.  words_bytes = bytes of coordinate words the
 * frame must stream (4, 8 or 12 per point of a live batch at 10, 20 or 30
 * bits; in a pr_render_views frame once per batch and classify launch, at the
 * highest level among the batch's live views there), the algorithmic HBM
 * bytes of the point loop. */
typedef struct {
  uint64_t batches, culled, points;
  uint64_t level_batches[3], level_points[3]; /* index 0, 1, 2 = 10, 20, 30 bits */
  uint64_t atomics;
  uint64_t words_bytes;
} pr_stats;

/* Message of the last failed call on this thread (never NULL). */
const char* pr_last_error(void);

/* Create a context on HIP device `device`, enqueuing on `hip_stream` (a
 * hipStream_t; NULL = the null stream).  Allocates 4 KiB of device memory for
 * frame constants and counters.  PR_EDEVICE if no GPU is usable. */
pr_status pr_create(int device, void* hip_stream, pr_ctx** out);
void pr_destroy(pr_ctx* ctx);

/* Byte sizes of the cloud buffers for n points in batches of batch_size
 * (multiple of 4), with or without the Morton sort (Sec. 3.1).  Pure host
 * arithmetic; needs no GPU. */
pr_status pr_cloud_sizes(uint64_t n, uint32_t batch_size, int morton, pr_sizes* out);

/* Byte sizes for a cloud of n point slots in nb variable-size batches
 * (pr_build_batches_spans): no Morton scratch, a nodes buffer. */
pr_status pr_cloud_sizes_spans(uint64_t n, uint64_t nb, pr_sizes* out);

/* Copy n positions (float[n][3]) and colours (uint32[n]) into bufs->xyz and
 * bufs->rgba (skipped where source and destination coincide), from host
 * memory (src_on_device = 0) or device memory (1).  Creates a host handle
 * that keeps `bufs` (not owning it).  Sec. 3.1: the data structure is built
 * while the data set is loaded. */
pr_status pr_load_points(pr_ctx* ctx, const float* xyz, const uint32_t* rgba, uint64_t n,
                         int src_on_device, const pr_cloud_bufs* bufs, pr_cloud** out);

/* Point orders of pr_build_batches. */
enum {
  PR_ORDER_INPUT = 0,          /* the order of the xyz buffer */
  PR_ORDER_MORTON = 1,         /* stable Morton order (Sec. 3.1) */
  PR_ORDER_MORTON_SPREAD = 2   /* the batches of PR_ORDER_MORTON, each stored in the spread order below */
};

/* Load-time build (Sec. 3.1, 3.3): checks every coordinate is finite;
 * orders the points (morton: one of PR_ORDER_*; nonzero needs the sort
 * scratch of pr_cloud_sizes): PR_ORDER_MORTON sorts them by 63-bit Morton
 * code (21 bits per axis over the cloud box, x in the lowest bit; stable);
 * groups batch_size consecutive points into batches with their fp32 bounding
 * boxes; quantises every coordinate by Eq. 1 relative to its batch box and
 * splits the 30 bits into low / med / high words.  PR_ORDER_MORTON_SPREAD
 * (an option of this library; the paper fixes no order inside a batch) keeps
 * the same batches but stores a batch of c points so that position r holds
 * its Morton rank (r * m) mod c, m the first integer >= floor(c / 4) + 1
 * coprime with c: the four points a lane loads with one 16-byte word then lie
 * in four different quarters of the batch, while each of its four point
 * loops over a wave still walks Morton neighbours.  Back-to-back LDS reads
 * and atomics of one wave then rarely hit the same tile entries, which
 * shortens the queues on them (the render and two-view passes are faster;
 * pr_resolve's colour gather is a little less coherent).  perm and colors
 * follow the stored order.  Synchronises the
 * stream once.  PR_ENONFINITE if any coordinate is NaN or Inf, PR_EINVAL for
 * an unknown order. */
pr_status pr_build_batches(pr_ctx* ctx, pr_cloud* cloud, uint32_t batch_size, int morton);

/* One view of a multi-view render: matrices and image size as for
 * pr_render, and the view's visibility buffer (uint64[h*w], device, 16-byte
 * aligned). */
#define PR_MAX_VIEWS 64
typedef struct {
  float view[16], proj[16];
  uint32_t w, h;
  uint64_t* visbuf;
} pr_view;

/* Bytes of device workspace pr_render_views needs for this (built) cloud and
 * nviews views (1 <= nviews <= PR_MAX_VIEWS). */
pr_status pr_views_work_bytes(const pr_cloud* cloud, uint32_t nviews, uint64_t* out);

/* Render nviews views (stereo pairs, camera arrays) of one cloud with one
 * persistent render launch (Sec. 3.7: both eyes of a VR frame in one pass).
 * The per-batch prologue (culling, precision level, tile) runs for every
 * (batch, view) pair exactly as in pr_render; each workgroup then renders a
 * batch for all of its live views in turn, so the batch's coordinate words
 * are streamed from HBM once per frame instead of once per view.  Every
 * view's visibility buffer equals pr_render of that view with the same opts,
 * bit for bit.  opts apply to every view (accumulate: no view is cleared;
 * counters: pr_stats sums over all (batch, view) pairs).  work: caller-owned
 * device memory of at least pr_views_work_bytes bytes, 256-byte aligned; it
 * must not be used by another call in flight.  Asynchronous.  PR_ERANGE for
 * nviews or image sizes outside the limits, PR_ENONFINITE for non-finite
 * matrices, PR_ESTATE before pr_build_batches. */
pr_status pr_render_views(pr_ctx* ctx, const pr_cloud* cloud, const pr_view* views, uint32_t nviews,
                          const pr_render_opts* opts, void* work, uint64_t work_bytes);

/* For callers that cannot allocate device memory on the frame path (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): pr_render_views with its work area in a device array of
 * PR_STATIC_WORK_BYTES that the library holds on each device it runs on
 * (from pr_create on that device until the process ends), so the caller
 * passes no work buffer.  Same frame, same results and the same errors as
 * pr_render_views; this call allocates nothing.  Every call on one GPU shares
 * that GPU's array: calls whose frames overlap on one GPU (several streams or
 * threads) race and must be serialised by the caller (the frame resets
 * what it reads of the array, so the contents a previous call left are
 * harmless).  PR_ERANGE when the frame needs more than PR_STATIC_WORK_BYTES,
 * i.e. when pr_views_work_bytes(cloud, nviews) exceeds it (for example
 * 64 views of a 5e8-point cloud in 10,240-point batches). */
#define PR_STATIC_WORK_BYTES (64ull << 20)
pr_status pr_render_views_static(pr_ctx* ctx, const pr_cloud* cloud, const pr_view* views, uint32_t nviews,
                                 const pr_render_opts* opts);

/* Load-time build of a level-of-detail layout (Sec. 3.5): the points are
 * already in render order (a layered point cloud: octree nodes level by
 * level) and grouped into nb variable-size batches given on the host as
 * spans[2b] = first point, spans[2b + 1] = number of points (first a multiple
 * of 4, spans ascending and disjoint, inside the cloud; slots between batches
 * are padding and never read).  nodes (host, may be NULL): the octree node of
 * each batch, copied to bufs->nodes for LOD culling at render time.  Checks
 * every coordinate is finite, computes each batch's fp32 box and the Eq. 1
 * words.  Synchronises once.  PR_EINVAL for bad spans or small buffers,
 * PR_ENONFINITE for NaN / Inf coordinates. */
pr_status pr_build_batches_spans(pr_ctx* ctx, pr_cloud* cloud, const uint32_t* spans, const pr_lod_node* nodes,
                                 uint64_t nb);

/* Fill visbuf (uint64[h*w], device, 16-byte aligned) with PR_EMPTY (the
 * frame clear of Sec. 4.3).  Asynchronous. */
pr_status pr_clear(pr_ctx* ctx, uint64_t* visbuf, uint32_t w, uint32_t h);

/* Render one view (Sec. 3.2, 3.3): clears visbuf (uint64[h*w], device) to
 * PR_EMPTY (unless opts->accumulate), then every batch is culled or rendered
 * at its precision level and every visible point is combined into visbuf by
 * 64-bit atomic minimum.  visbuf must be 16-byte aligned (PR_EINVAL
 * otherwise).  The frame's work area lives in the cloud's scratch buffer, so
 * pr_render calls on one cloud must not overlap (keep them on one stream;
 * overlapping frames use pr_render_views with work buffers of their own).
 * Asynchronous.  PR_ENONFINITE for non-finite matrices, PR_ESTATE before
 * pr_build_batches or after pr_cloud_drop_load_buffers. */
pr_status pr_render(pr_ctx* ctx, const pr_cloud* cloud, const float view[16], const float proj[16],
                    uint32_t w, uint32_t h, const pr_render_opts* opts, uint64_t* visbuf);

/* High-quality shading of one view (Sec. 3.6): renders the view into visbuf
 * exactly as pr_render (the closest depth per pixel), then every drawn point
 * whose w is within the depth window of its pixel's closest point,
 *   hw <= fl32(w_closest * window)   (binary32 product; window >= 1, e.g.
 *                                     1.01 lets points up to one percent farther
 *                                     than the pixel's closest point join),
 * adds its colour and a count to accum (uint64[2*h*w], device, 16-byte
 * aligned, zeroed by this call): accum[2p] += R + G * 2^32, accum[2p+1] +=
 * B + 2^32, with R, G, B the low three bytes of the colour (additions wrap
 * mod 2^64, exact while a pixel's sums stay below 2^32).  Finally
 * rgba_out[p] (uint32[h*w], 16-byte aligned) = the rounded average
 * (sum + n/2) / n per channel with alpha 255, or clear_rgba where no point
 * landed.  opts->accumulate must be 0.  Asynchronous; uses the cloud's
 * scratch like pr_render.  PR_EINVAL for a window below 1 or not finite. */
pr_status pr_render_hqs(pr_ctx* ctx, const pr_cloud* cloud, const float view[16], const float proj[16],
                        uint32_t w, uint32_t h, const pr_render_opts* opts, float window, uint64_t* visbuf,
                        uint64_t* accum, uint32_t clear_rgba, uint32_t* rgba_out);

/* Resolve (Sec. 3.3): rgba_out[p] = colors[VB[p] & 0xFFFFFFFF], or
 * clear_rgba where VB[p] == PR_EMPTY (or holds an index >= n, which a buffer
 * rendered from this cloud never does).  visbuf and rgba_out (uint32[h*w])
 * are device memory, 16-byte aligned (PR_EINVAL otherwise).  Asynchronous. */
pr_status pr_resolve(pr_ctx* ctx, const pr_cloud* cloud, const uint64_t* visbuf, uint32_t w,
                     uint32_t h, uint32_t clear_rgba, uint32_t* rgba_out);

/* Counters of the last pr_render that had counters = 1.  Synchronises. */
pr_status pr_get_stats(pr_ctx* ctx, pr_stats* out);

/* Wait for the context's stream; reports device-side failures. */
pr_status pr_sync(pr_ctx* ctx);

/* Measurement of the render kernel alone (the roofline of Sec. 4.1's
 * throughput figures needs the kernel's own duration, without the classify
 * launch and the header reset that pr_render enqueues before it).  With
 * n > 0 the next n render-kernel launches (the k_render launch of pr_render
 * and pr_render_hqs, the k_render_views launch of pr_render_views) each
 * record a pair of HIP events around that launch on the context's stream;
 * later launches record nothing (a launch enqueued under HIP graph capture
 * records its pair at every replay of the graph).  Creates the 2n events (host allocations,
 * never device memory) and drops any earlier ones; n = 0 only drops them.
 * PR_EINVAL for n > PR_MAX_TIMED_LAUNCHES. */
#define PR_MAX_TIMED_LAUNCHES 4096
pr_status pr_time_kernels(pr_ctx* ctx, uint32_t n);

/* Durations of the launches recorded since pr_time_kernels, in ms, in launch
 * order: ms_out[i] for i < *count (ms_out holds at least capacity floats;
 * *count = number recorded, at most capacity).  Synchronises on the last
 * recorded launch. */
pr_status pr_kernel_times(pr_ctx* ctx, float* ms_out, uint32_t capacity, uint32_t* count);

/* Cloud facts: point count, batch count, batch size (0 before a build). */
pr_status pr_cloud_info(const pr_cloud* cloud, uint64_t* n, uint64_t* nbatches, uint32_t* batch_size);

/* After pr_build_batches: the cloud no longer uses its xyz, rgba, perm and
 * scratch buffers, which the caller may then free; what stays is what
 * rendering reads (low, med, high, colors, batches: 16 bytes per point plus
 * 32 per batch).  Afterwards pr_render_views and pr_resolve work as before;
 * pr_render (whose work area is the scratch buffer) and pr_build_batches
 * fail with PR_ESTATE.  For many resident clouds (served mode). */
pr_status pr_cloud_drop_load_buffers(pr_cloud* cloud);

/* Free the host handle only; device buffers stay the caller's. */
void pr_cloud_free(pr_cloud* cloud);

/* ---- workgroup shapes and autotuning (Sec. 3.2 fixes one workgroup size and
 * number of points per thread for its GPU and reports a sweep of the latter)
 *
 * The library carries several compiled shapes of its persistent render
 * kernel.  A context renders with one shape and two run-time settings, its
 * tuning.  Every shape and every tuning gives the same visibility buffers and
 * counters, bit for bit (the combination is a minimum): they change the speed
 * only.  The batch size S, the third parameter of the paper's sweep, is fixed
 * when the cloud is built (pr_build_batches); points per thread follow as
 * S / (64 * waves). */
typedef struct {
  uint32_t waves;         /* waves of 64 lanes per workgroup                     */
  uint32_t depth;         /* groups of 256 points (4 per lane) in flight per wave */
  uint32_t tile_px;       /* pixels of the workgroup's LDS tile (8 bytes each)   */
  uint32_t max_wg_per_cu; /* single-view workgroups that fit on one CU at once   */
} pr_raster_shape;

typedef struct {
  uint32_t shape;     /* index into the shapes of pr_raster_shapes [0]                      */
  uint32_t tile_px;   /* largest batch rectangle combined in LDS, at most the shape's tile;
                         0 = the shape's tile [0]                                           */
  uint32_t wg_per_cu; /* persistent workgroups per CU, at most what fits; 0 = all that fit [0] */
  uint32_t max_bands; /* a 10-bit batch larger than the tile bound, at most one tile wide and
                         at most max_bands tiles large, renders in bands of rows through
                         the LDS tile (1 = never, at most 64); 0 = 4 [0]                    */
} pr_tuning;

/* The compiled shapes in index order (shape 0 is the default): writes
 * min(cap, count) records to out (host, may be NULL when cap is 0) and the
 * count to *count. */
pr_status pr_raster_shapes(const pr_ctx* ctx, pr_raster_shape* out, uint32_t cap, uint32_t* count);

/* Set the context's tuning (NULL: the default {0, 0, 0, 0}); later frames on
 * this context use it.  Not for a context with frames being enqueued from
 * another thread.  PR_EINVAL for an unknown shape, tile_px above the
 * shape's tile, wg_per_cu above what fits, or max_bands above 64. */
pr_status pr_set_tuning(pr_ctx* ctx, const pr_tuning* tuning);
pr_status pr_get_tuning(const pr_ctx* ctx, pr_tuning* out);

/* One candidate of pr_autotune and its mean frame time. */
typedef struct {
  pr_tuning tuning;
  float ms;           /* one pr_render_views frame (all views), HIP events on the context's stream */
  uint32_t reserved;
} pr_tune_trial;

/* Autotuner: times pr_render_views(ctx, cloud, views, nviews, opts, work,
 * work_bytes) under each candidate tuning, one untimed frame then reps timed
 * frames each (reps 0 = 3), and sets the context's tuning to the fastest (the
 * first of equal times).  Candidates: every shape with its full and half tile
 * bound and all or half of the workgroups that fit (band limit 4); then the
 * winner with band limits 1, 2, 8 and 16.  The trials go to trials (host,
 * first min(cap, total) in candidate order; may be NULL when cap is 0), their
 * number to *ntrials, the winner to *best (may be NULL).  Afterwards every
 * view's visibility buffer holds the frame.  Synchronises.
 * opts->accumulate and opts->counters must be 0 (PR_EINVAL); other errors as
 * pr_render_views.  On an error the context's tuning is left unchanged. */
pr_status pr_autotune(pr_ctx* ctx, const pr_cloud* cloud, const pr_view* views, uint32_t nviews,
                      const pr_render_opts* opts, void* work, uint64_t work_bytes, uint32_t reps,
                      pr_tune_trial* trials, uint32_t cap, uint32_t* ntrials, pr_tuning* best);

/* ---- HBM streaming reference (not part of the method) ----
 * A plain vectorised grid-stride kernel over bytes bytes of device memory
 * (bytes a multiple of 16, pointers 16-byte aligned): copies src to dst, or,
 * with dst NULL, only reads src.  Its measured rate is the streaming ceiling
 * the render kernel's HBM roofline is reported beside, and the copy is a
 * kernel of known traffic for calibrating HBM byte counters.  Asynchronous on
 * the context's stream.  PR_EINVAL for NULL src, a size that is not a
 * multiple of 16 or misaligned pointers. */
pr_status pr_stream_probe(pr_ctx* ctx, const void* src, void* dst, uint64_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* PTRASTER_H */

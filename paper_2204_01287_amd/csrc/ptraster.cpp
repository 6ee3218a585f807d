// Host runtime of libptraster.so: the C ABI declared in include/ptraster.h.
// Validates arguments, lays out caller-provided memory, and enqueues the
// build / render / resolve kernels on the context's HIP stream.
#include "../../include/ptraster.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace ptr {
// render_static.hip: the library-held work area of pr_render_views_static
hipError_t static_work_init(int device);
void* static_work_addr(int device);
}  // namespace ptr

static_assert(sizeof(pr_lod_node) == sizeof(ptr::LodNode), "LOD node layout");
static_assert(sizeof(pr_batch) == sizeof(ptr::BatchRec), "batch record layout");

namespace {
// The compiled workgroup shapes of the persistent render kernels; index 0 is the default.
const ptr::RasterShape* (*const kShapeOf[])() = {
#define PR_SHAPE_REF(W_, D_, T_) &ptr::PR_SHAPE_NAME_(W_, D_, T_),
    PR_RASTER_SHAPES(PR_SHAPE_REF)
#undef PR_SHAPE_REF
};
constexpr uint32_t kNumShapes = sizeof(kShapeOf) / sizeof(kShapeOf[0]);
const ptr::RasterShape& shape_at(uint32_t i) { return *kShapeOf[i](); }
}  // namespace

struct pr_ctx {
  int device;
  hipStream_t stream;
  ptr::DevBlock* dev;  // counters and flags (device memory)
  uint32_t cus;                     // compute units of the device
  uint32_t per_cu[kNumShapes][2];   // workgroups per CU that fit at once: single-view, multi-view kernel
  uint32_t accum_grid;              // persistent workgroups of the shading pass
  pr_tuning tuning;                 // render shape, tile bound and grid of this context's frames
  std::vector<hipEvent_t> tev;      // pr_time_kernels: 2 events per armed render launch
  uint32_t t_used = 0;              // launches recorded so far
};

struct pr_cloud {
  pr_ctx* ctx;
  uint64_t n;
  uint64_t nb;
  uint32_t batch_size;
  int morton;
  int built;
  int load_dropped;  // xyz, rgba, perm and scratch released by the caller: pr_render_views / pr_resolve only
  int lod;           // built from spans with LOD nodes
  pr_cloud_bufs bufs;
};

namespace {

thread_local std::string g_err = "no error";

pr_status fail(pr_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pr_status fail(pr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

pr_status hip_fail(hipError_t e, const char* what) {
  return fail(PR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)               \
  do {                                    \
    hipError_t e_ = (expr);               \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr uint64_t kMaxPoints = 0xFFFFFFFFull;  // n < 2^32: the key holds a 32-bit index
constexpr uint32_t kMaxDim = 8192;

uint64_t a256(uint64_t x) { return (x + 255) & ~255ull; }

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

pr_status check_dims(uint32_t w, uint32_t h) {
  if (w < 1 || h < 1 || w > kMaxDim || h > kMaxDim)
    return fail(PR_ERANGE, "image size %ux%u outside 1..%u", w, h, kMaxDim);
  return PR_OK;
}

pr_status set_device(const pr_ctx* ctx) {
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  return PR_OK;
}

// A frame reads the context's tuning once: its render shape, the tile bound of
// its classify launches (never more than the shape's LDS tile) and its
// persistent grid.
const ptr::RasterShape& shape_of(const pr_tuning& t) { return shape_at(t.shape); }
uint32_t shape_tile(const pr_tuning& t) {
  const uint32_t full = shape_of(t).tile;
  return t.tile_px && t.tile_px < full ? t.tile_px : full;
}
uint32_t tune_bands(const pr_tuning& t) { return t.max_bands ? t.max_bands : ptr::DEFAULT_BANDS; }
uint32_t shape_grid(const pr_ctx* ctx, const pr_tuning& t, int views) {
  uint32_t per = ctx->per_cu[t.shape][views];
  if (t.wg_per_cu && t.wg_per_cu < per) per = t.wg_per_cu;
  return per * ctx->cus;
}

// Pixel-space matrix (Sec. 3.2 projection; the paper leaves toPixelID open):
// C = proj * view (row-major storage, column vectors); window x =
// (x_clip / w_clip + 1) W / 2, so the rows are hx = (W/2)(C0 + C3),
// hy = (H/2)(C1 + C3), hw = C3.  binary64, sums left to right, no fused
// multiply-add (this file is compiled with -ffp-contract=off).
void frame_matrix(const float* view, const float* proj, uint32_t w, uint32_t h, double Pm[3][4]) {
  double C[3][4];
  const int rows[3] = {0, 1, 3};
  for (int q = 0; q < 3; ++q) {
    const int i = rows[q];
    for (int j = 0; j < 4; ++j)
      C[q][j] = (((double)proj[4 * i + 0] * (double)view[0 + j] + (double)proj[4 * i + 1] * (double)view[4 + j]) +
                 (double)proj[4 * i + 2] * (double)view[8 + j]) +
                (double)proj[4 * i + 3] * (double)view[12 + j];
  }
  for (int j = 0; j < 4; ++j) {
    Pm[0][j] = (0.5 * (double)w) * (C[0][j] + C[2][j]);
    Pm[1][j] = (0.5 * (double)h) * (C[1][j] + C[2][j]);
    Pm[2][j] = C[2][j];
  }
}

pr_status sizes_for(uint64_t n, uint32_t batch_size, int morton, pr_sizes* s) {
  if (batch_size == 0 || (batch_size & 3u)) return fail(PR_EINVAL, "batch_size %u must be a positive multiple of 4", batch_size);
  if (n > kMaxPoints - 1) return fail(PR_ERANGE, "n = %llu points: at most 2^32 - 1", (unsigned long long)n);
  const uint64_t nb = (n + batch_size - 1) / batch_size;
  s->xyz = a256(12 * n);
  s->rgba = a256(4 * n);
  s->low = s->med = s->high = s->colors = s->perm = a256(4 * n);
  s->batches = a256(32 * nb);
  // Load-time sort area and per-frame area (live batch list) share the space.
  const uint64_t sort = morton ? ptr::sort_scratch_layout(n, nullptr, nullptr) : 0;
  const uint64_t frame = ptr::frame_area_bytes(nb);
  s->scratch = a256(ptr::small_scratch_bytes() + (sort > frame ? sort : frame));
  s->nodes = 0;
  return PR_OK;
}

pr_status sizes_spans(uint64_t n, uint64_t nb, pr_sizes* s) {
  if (n > kMaxPoints - 1) return fail(PR_ERANGE, "n = %llu point slots: at most 2^32 - 1", (unsigned long long)n);
  if (nb > n) return fail(PR_EINVAL, "%llu batches for %llu point slots", (unsigned long long)nb, (unsigned long long)n);
  s->xyz = a256(12 * n);
  s->rgba = a256(4 * n);
  s->low = s->med = s->high = s->colors = s->perm = a256(4 * n);
  s->batches = a256(32 * nb);
  s->scratch = a256(ptr::small_scratch_bytes() + ptr::frame_area_bytes(nb));
  s->nodes = a256(sizeof(ptr::LodNode) * nb);
  return PR_OK;
}

// The event pair of the next render launch, if pr_time_kernels armed one (else nullptr).
hipEvent_t* timed_pair(pr_ctx* ctx) {
  return 2u * ctx->t_used < ctx->tev.size() ? &ctx->tev[2u * ctx->t_used] : nullptr;
}

// A render launch between its timing events (when armed).
template <typename Launch>
hipError_t timed_launch(pr_ctx* ctx, Launch&& launch) {
  hipEvent_t* ev = timed_pair(ctx);
  if (ev) {
    const hipError_t e = hipEventRecord(ev[0], ctx->stream);
    if (e != hipSuccess) return e;
  }
  const hipError_t e = launch();
  if (e != hipSuccess || !ev) return e;
  ctx->t_used++;
  return hipEventRecord(ev[1], ctx->stream);
}

}  // namespace

extern "C" {

const char* pr_last_error(void) { return g_err.c_str(); }

pr_status pr_create(int device, void* hip_stream, pr_ctx** out) {
  if (!out) return fail(PR_EINVAL, "pr_create: out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) return fail(PR_EDEVICE, "no HIP device available (%s)", hipGetErrorString(e));
  if (device < 0 || device >= count) return fail(PR_EDEVICE, "device %d outside 0..%d", device, count - 1);
  HIP_TRY(hipSetDevice(device), "hipSetDevice");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(PR_EDEVICE, "device %d is %s; this library is built for gfx950 only", device, prop.gcnArchName);
  pr_ctx* c = new (std::nothrow) pr_ctx;
  if (!c) return fail(PR_ENOMEM, "pr_create: host allocation");
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->dev = nullptr;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  c->cus = (uint32_t)cus;
  for (uint32_t i = 0; i < kNumShapes; ++i)
    for (int v = 0; v < 2; ++v) c->per_cu[i][v] = (uint32_t)shape_at(i).per_cu(v);
  c->accum_grid = ptr::accum_grid(device);
  c->tuning = {0, 0, 0, 0};
  e = ptr::static_work_init(device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "static work area of pr_render_views_static (hipGetSymbolAddress)");
  }
  e = hipMalloc(reinterpret_cast<void**>(&c->dev), 4096);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipMalloc(context block)");
  }
  e = hipMemsetAsync(c->dev, 0, 4096, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    (void)hipFree(c->dev);
    delete c;
    return hip_fail(e, "context block init");
  }
  *out = c;
  return PR_OK;
}

void pr_destroy(pr_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t e : ctx->tev) (void)hipEventDestroy(e);
  (void)hipFree(ctx->dev);
  delete ctx;
}

pr_status pr_cloud_sizes(uint64_t n, uint32_t batch_size, int morton, pr_sizes* out) {
  if (!out) return fail(PR_EINVAL, "pr_cloud_sizes: out is NULL");
  return sizes_for(n, batch_size, morton, out);
}

pr_status pr_load_points(pr_ctx* ctx, const float* xyz, const uint32_t* rgba, uint64_t n, int src_on_device,
                         const pr_cloud_bufs* bufs, pr_cloud** out) {
  if (!ctx || !bufs || !out) return fail(PR_EINVAL, "pr_load_points: NULL argument");
  *out = nullptr;
  if (n > kMaxPoints - 1) return fail(PR_ERANGE, "n = %llu points: at most 2^32 - 1", (unsigned long long)n);
  if (n > 0 && (!xyz || !rgba || !bufs->xyz || !bufs->rgba)) return fail(PR_EINVAL, "pr_load_points: NULL buffer");
  if (bufs->capacity.xyz < 12 * n || bufs->capacity.rgba < 4 * n)
    return fail(PR_EINVAL, "pr_load_points: xyz/rgba buffers hold fewer than n points");
  if (pr_status s = set_device(ctx)) return s;
  const hipMemcpyKind kind = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (n > 0 && static_cast<const void*>(xyz) != bufs->xyz)
    HIP_TRY(hipMemcpyAsync(bufs->xyz, xyz, 12 * n, kind, ctx->stream), "copy positions");
  if (n > 0 && static_cast<const void*>(rgba) != bufs->rgba)
    HIP_TRY(hipMemcpyAsync(bufs->rgba, rgba, 4 * n, kind, ctx->stream), "copy colours");
  pr_cloud* c = new (std::nothrow) pr_cloud;
  if (!c) return fail(PR_ENOMEM, "pr_load_points: host allocation");
  c->ctx = ctx;
  c->n = n;
  c->nb = 0;
  c->batch_size = 0;
  c->morton = 0;
  c->built = 0;
  c->load_dropped = 0;
  c->lod = 0;
  c->bufs = *bufs;
  *out = c;
  return PR_OK;
}

pr_status pr_cloud_sizes_spans(uint64_t n, uint64_t nb, pr_sizes* out) {
  if (!out) return fail(PR_EINVAL, "pr_cloud_sizes_spans: out is NULL");
  return sizes_spans(n, nb, out);
}

pr_status pr_build_batches_spans(pr_ctx* ctx, pr_cloud* cloud, const uint32_t* spans, const pr_lod_node* nodes,
                                 uint64_t nb) {
  if (!ctx || !cloud || (nb && !spans)) return fail(PR_EINVAL, "pr_build_batches_spans: NULL argument");
  if (cloud->ctx != ctx) return fail(PR_EINVAL, "pr_build_batches_spans: cloud belongs to another context");
  if (cloud->load_dropped) return fail(PR_ESTATE, "pr_build_batches_spans: the cloud's load buffers were released");
  const uint64_t n = cloud->n;
  pr_sizes need;
  if (pr_status s = sizes_spans(n, nb, &need)) return s;
  uint64_t end = 0;
  for (uint64_t b = 0; b < nb; ++b) {
    const uint64_t f = spans[2 * b], c = spans[2 * b + 1];
    if ((f & 3u) || f < end || c == 0 || f + c > n)
      return fail(PR_EINVAL, "pr_build_batches_spans: span %llu (first %llu, count %llu) must start at a multiple "
                  "of 4 after the previous span, hold at least one point and lie inside the %llu slots",
                  (unsigned long long)b, (unsigned long long)f, (unsigned long long)c, (unsigned long long)n);
    end = f + c;
  }
  const pr_cloud_bufs& B = cloud->bufs;
  const pr_sizes& cap = B.capacity;
  if (cap.low < need.low || cap.med < need.med || cap.high < need.high || cap.colors < need.colors ||
      cap.perm < need.perm || cap.batches < need.batches || cap.scratch < need.scratch ||
      (nodes && cap.nodes < need.nodes))
    return fail(PR_EINVAL, "pr_build_batches_spans: a cloud buffer is smaller than pr_cloud_sizes_spans requires");
  if (n > 0) {
    const void* ptrs[] = {B.xyz, B.rgba, B.low, B.med, B.high, B.colors, B.perm, B.batches, B.scratch};
    for (const void* p : ptrs)
      if (!p || !aligned256(p)) return fail(PR_EINVAL, "pr_build_batches_spans: NULL or unaligned cloud buffer");
  }
  if (nodes && nb && (!B.nodes || !aligned256(B.nodes)))
    return fail(PR_EINVAL, "pr_build_batches_spans: NULL or unaligned nodes buffer");
  if (pr_status s = set_device(ctx)) return s;
  hipStream_t st = ctx->stream;
  cloud->built = 0;
  std::vector<ptr::BatchRec> recs(nb);
  for (uint64_t b = 0; b < nb; ++b) {
    std::memset(&recs[b], 0, sizeof recs[b]);
    recs[b].first = spans[2 * b];
    recs[b].count = spans[2 * b + 1];
  }
  uint32_t* flag = &ctx->dev->flags[0];
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(uint32_t), st), "clear flag");
  if (n > 0) {
    const float* xyz = static_cast<const float*>(B.xyz);
    HIP_TRY(ptr::launch_finite_check(xyz, n, flag, st), "finite check");
    HIP_TRY(ptr::launch_iota(static_cast<uint32_t*>(B.perm), n, st), "iota");
    HIP_TRY(hipMemcpyAsync(B.colors, B.rgba, 4 * n, hipMemcpyDeviceToDevice, st), "copy colours");
    ptr::BatchRec* dbat = static_cast<ptr::BatchRec*>(B.batches);
    if (nb) {
      HIP_TRY(hipMemcpyAsync(dbat, recs.data(), sizeof(ptr::BatchRec) * nb, hipMemcpyHostToDevice, st), "spans");
      HIP_TRY(ptr::launch_batch_bbox_spans(xyz, nb, dbat, st), "batch boxes");
      HIP_TRY(ptr::launch_quantize_spans(xyz, nb, dbat, static_cast<uint32_t*>(B.low), static_cast<uint32_t*>(B.med),
                                         static_cast<uint32_t*>(B.high), st),
              "quantise");
      if (nodes)
        HIP_TRY(hipMemcpyAsync(B.nodes, nodes, sizeof(pr_lod_node) * nb, hipMemcpyHostToDevice, st), "nodes");
    }
  }
  uint32_t h_flag = 0;
  HIP_TRY(hipMemcpyAsync(&h_flag, flag, sizeof h_flag, hipMemcpyDeviceToHost, st), "read flag");
  HIP_TRY(hipStreamSynchronize(st), "build");
  if (h_flag) return fail(PR_ENONFINITE, "pr_build_batches_spans: a coordinate is NaN or Inf");
  cloud->nb = nb;
  cloud->batch_size = 0;
  cloud->morton = 0;
  cloud->lod = nodes ? 1 : 0;
  cloud->built = 1;
  return PR_OK;
}

pr_status pr_build_batches(pr_ctx* ctx, pr_cloud* cloud, uint32_t batch_size, int morton) {
  if (!ctx || !cloud) return fail(PR_EINVAL, "pr_build_batches: NULL argument");
  if (morton < PR_ORDER_INPUT || morton > PR_ORDER_MORTON_SPREAD)
    return fail(PR_EINVAL, "pr_build_batches: order %d is not PR_ORDER_INPUT, PR_ORDER_MORTON or PR_ORDER_MORTON_SPREAD",
                morton);
  if (cloud->ctx != ctx) return fail(PR_EINVAL, "pr_build_batches: cloud belongs to another context");
  if (cloud->load_dropped) return fail(PR_ESTATE, "pr_build_batches: the cloud's load buffers were released");
  pr_sizes need;
  if (pr_status s = sizes_for(cloud->n, batch_size, morton, &need)) return s;
  const pr_cloud_bufs& B = cloud->bufs;
  const pr_sizes& cap = B.capacity;
  if (cap.low < need.low || cap.med < need.med || cap.high < need.high || cap.colors < need.colors ||
      cap.perm < need.perm || cap.batches < need.batches || cap.scratch < need.scratch)
    return fail(PR_EINVAL, "pr_build_batches: a cloud buffer is smaller than pr_cloud_sizes requires");
  const uint64_t n = cloud->n;
  if (n > 0) {
    const void* ptrs[] = {B.xyz, B.rgba, B.low, B.med, B.high, B.colors, B.perm, B.batches, B.scratch};
    for (const void* p : ptrs)
      if (!p) return fail(PR_EINVAL, "pr_build_batches: NULL cloud buffer");
    for (const void* p : ptrs)
      if (!aligned256(p)) return fail(PR_EINVAL, "pr_build_batches: cloud buffers must be 256-byte aligned");
  }
  if (pr_status s = set_device(ctx)) return s;
  hipStream_t st = ctx->stream;
  const uint64_t nb = (n + batch_size - 1) / batch_size;
  cloud->built = 0;
  uint32_t* flag = &ctx->dev->flags[0];
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(uint32_t), st), "clear flag");
  if (n > 0) {
    const float* xyz = static_cast<const float*>(B.xyz);
    const uint32_t* rgba = static_cast<const uint32_t*>(B.rgba);
    uint32_t* perm = static_cast<uint32_t*>(B.perm);
    uint32_t* colors = static_cast<uint32_t*>(B.colors);
    if (morton) {
      ptr::SortScratch sc;
      uint8_t* base = static_cast<uint8_t*>(B.scratch) + ptr::small_scratch_bytes();
      ptr::sort_scratch_layout(n, base, &sc);
      HIP_TRY(ptr::launch_morton_codes(xyz, n, sc.aabb, sc.keys0, perm, flag, st), "morton codes");
      HIP_TRY(ptr::radix_sort_pairs(sc, perm, n, st), "radix sort");
      // sorted positions straight into the caller's xyz buffer (the gather reads copies of the inputs)
      HIP_TRY(ptr::launch_gather(sc, xyz, rgba, perm, n, batch_size, morton == PR_ORDER_MORTON_SPREAD,
                                 static_cast<float*>(B.xyz), colors, st),
              "gather");
    } else {
      HIP_TRY(ptr::launch_finite_check(xyz, n, flag, st), "finite check");
      HIP_TRY(ptr::launch_iota(perm, n, st), "iota");
      HIP_TRY(hipMemcpyAsync(colors, rgba, 4 * n, hipMemcpyDeviceToDevice, st), "copy colours");
    }
    ptr::BatchRec* batches = static_cast<ptr::BatchRec*>(B.batches);
    HIP_TRY(ptr::launch_batch_bbox(xyz, n, batch_size, nb, batches, st), "batch boxes");
    HIP_TRY(ptr::launch_quantize(xyz, n, batch_size, batches, static_cast<uint32_t*>(B.low),
                                 static_cast<uint32_t*>(B.med), static_cast<uint32_t*>(B.high), st),
            "quantise");
  }
  uint32_t h_flag = 0;
  HIP_TRY(hipMemcpyAsync(&h_flag, flag, sizeof h_flag, hipMemcpyDeviceToHost, st), "read flag");
  HIP_TRY(hipStreamSynchronize(st), "build");
  if (h_flag) return fail(PR_ENONFINITE, "pr_build_batches: a coordinate is NaN or Inf");
  cloud->nb = nb;
  cloud->batch_size = batch_size;
  cloud->morton = morton;
  cloud->lod = 0;
  cloud->built = 1;
  return PR_OK;
}

namespace {

// Argument checks shared by pr_render and pr_render_hqs.
pr_status check_render(const char* fn, pr_ctx* ctx, const pr_cloud* cloud, const float* view, const float* proj,
                       uint32_t w, uint32_t h, const pr_render_opts* opts, uint64_t* visbuf, pr_render_opts* o) {
  if (!ctx || !cloud || !view || !proj || !visbuf) return fail(PR_EINVAL, "%s: NULL argument", fn);
  if (cloud->ctx->device != ctx->device) return fail(PR_EINVAL, "%s: cloud lives on another device", fn);
  if (!cloud->built) return fail(PR_ESTATE, "%s: cloud is not built (call pr_build_batches)", fn);
  if (cloud->load_dropped)
    return fail(PR_ESTATE, "%s: the cloud's scratch was released (pr_cloud_drop_load_buffers); use pr_render_views",
                fn);
  if (pr_status s = check_dims(w, h)) return s;
  if (reinterpret_cast<uintptr_t>(visbuf) & 15u) return fail(PR_EINVAL, "%s: visbuf must be 16-byte aligned", fn);
  *o = {PR_ADAPTIVE, 1, 500.0f, 512000.0f, 0, 0, 0.0f};
  if (opts) *o = *opts;
  if (o->precision != PR_ADAPTIVE && o->precision != PR_FORCE10 && o->precision != PR_FORCE20 &&
      o->precision != PR_FORCE30)
    return fail(PR_EINVAL, "%s: precision %d is not 0, 10, 20 or 30", fn, o->precision);
  if (std::isnan(o->t10) || std::isnan(o->t20) || !(o->lod_px >= 0.0f) || !std::isfinite(o->lod_px))
    return fail(PR_EINVAL, "%s: NaN threshold or lod_px not finite and >= 0", fn);
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(view[i]) || !std::isfinite(proj[i])) return fail(PR_ENONFINITE, "%s: non-finite matrix", fn);
  return set_device(ctx);
}

// Reset the frame's work queues (and counters), classify (which also clears
// the visibility buffer unless accumulating) and render one view; a receives
// the frame's arguments.
pr_status render_frame(pr_ctx* ctx, const pr_cloud* cloud, const float view[16], const float proj[16], uint32_t w,
                       uint32_t h, const pr_render_opts& o, uint64_t* visbuf, ptr::RenderArgs& a) {
  ptr::FrameHeader* hdr =
      reinterpret_cast<ptr::FrameHeader*>(static_cast<uint8_t*>(cloud->bufs.scratch) + ptr::small_scratch_bytes());
  // the frame header (and counters) here; the visibility buffer is filled by the classify launch
  HIP_TRY(ptr::launch_clear(visbuf, 0, ctx->dev, hdr, o.counters ? 1 : 0, ctx->stream), "clear");
  std::memset(&a, 0, sizeof a);
  a.clear_vb = o.accumulate ? 0u : 1u;
  a.low = static_cast<const uint32_t*>(cloud->bufs.low);
  a.med = static_cast<const uint32_t*>(cloud->bufs.med);
  a.high = static_cast<const uint32_t*>(cloud->bufs.high);
  a.batches = static_cast<const ptr::BatchRec*>(cloud->bufs.batches);
  a.hdr = hdr;
  a.live = reinterpret_cast<ptr::LiveBatch*>(hdr + 1);
  a.order = reinterpret_cast<uint32_t*>(a.live + cloud->nb);
  const pr_tuning tune = ctx->tuning;
  a.grid = shape_grid(ctx, tune, 0);
  a.tile_max = shape_tile(tune);
  a.max_bands = tune_bands(tune);
  a.vb = visbuf;
  a.stats = ctx->dev->stats;
  frame_matrix(view, proj, w, h, a.Pm);
  a.nb = (uint32_t)cloud->nb;
  a.W = w;
  a.H = h;
  a.precision = o.precision;
  a.cull = o.cull ? 1 : 0;
  a.counters = o.counters ? 1 : 0;
  a.t10 = o.t10;
  a.t20 = o.t20;
  a.nodes = cloud->lod ? static_cast<const ptr::LodNode*>(cloud->bufs.nodes) : nullptr;
  a.lod_px = o.lod_px;
  HIP_TRY(ptr::launch_classify(a, ctx->stream), "classify");
  HIP_TRY(timed_launch(ctx, [&] { return shape_of(tune).render(a, ctx->stream); }), "render");
  return PR_OK;
}

}  // namespace

pr_status pr_render(pr_ctx* ctx, const pr_cloud* cloud, const float view[16], const float proj[16], uint32_t w,
                    uint32_t h, const pr_render_opts* opts, uint64_t* visbuf) {
  pr_render_opts o;
  if (pr_status s = check_render("pr_render", ctx, cloud, view, proj, w, h, opts, visbuf, &o)) return s;
  ptr::RenderArgs a;
  return render_frame(ctx, cloud, view, proj, w, h, o, visbuf, a);
}

pr_status pr_render_hqs(pr_ctx* ctx, const pr_cloud* cloud, const float view[16], const float proj[16], uint32_t w,
                        uint32_t h, const pr_render_opts* opts, float window, uint64_t* visbuf, uint64_t* accum,
                        uint32_t clear_rgba, uint32_t* rgba_out) {
  pr_render_opts o;
  if (pr_status s = check_render("pr_render_hqs", ctx, cloud, view, proj, w, h, opts, visbuf, &o)) return s;
  if (!accum || !rgba_out) return fail(PR_EINVAL, "pr_render_hqs: NULL argument");
  if ((reinterpret_cast<uintptr_t>(accum) & 15u) || (reinterpret_cast<uintptr_t>(rgba_out) & 15u))
    return fail(PR_EINVAL, "pr_render_hqs: accum and rgba_out must be 16-byte aligned");
  if (o.accumulate) return fail(PR_EINVAL, "pr_render_hqs: accumulate is not supported (the depth pass is a frame)");
  if (!(window >= 1.0f) || !std::isfinite(window)) return fail(PR_EINVAL, "pr_render_hqs: window must be finite and >= 1");
  ptr::RenderArgs a;
  if (pr_status s = render_frame(ctx, cloud, view, proj, w, h, o, visbuf, a)) return s;
  a.colors = static_cast<const uint32_t*>(cloud->bufs.colors);
  a.accum = accum;
  a.window = window;
  a.grid = ctx->accum_grid;
  HIP_TRY(ptr::launch_accumulate(a, ctx->stream), "shading pass");
  HIP_TRY(ptr::launch_resolve_hqs(accum, (uint64_t)w * h, clear_rgba, rgba_out, ctx->stream), "shading resolve");
  return PR_OK;
}

pr_status pr_cloud_drop_load_buffers(pr_cloud* cloud) {
  if (!cloud) return fail(PR_EINVAL, "pr_cloud_drop_load_buffers: NULL argument");
  if (!cloud->built) return fail(PR_ESTATE, "pr_cloud_drop_load_buffers: cloud is not built");
  cloud->load_dropped = 1;
  cloud->bufs.xyz = cloud->bufs.rgba = cloud->bufs.perm = cloud->bufs.scratch = nullptr;
  return PR_OK;
}

pr_status pr_views_work_bytes(const pr_cloud* cloud, uint32_t nviews, uint64_t* out) {
  if (!cloud || !out) return fail(PR_EINVAL, "pr_views_work_bytes: NULL argument");
  if (nviews < 1 || nviews > PR_MAX_VIEWS) return fail(PR_ERANGE, "pr_views_work_bytes: nviews %u not in 1..%d", nviews, PR_MAX_VIEWS);
  if (!cloud->built) return fail(PR_ESTATE, "pr_views_work_bytes: cloud is not built");
  *out = a256(ptr::views_work_bytes(cloud->nb, nviews));
  return PR_OK;
}

namespace {

// pr_render_views and pr_render_views_static: every step of the frame, with
// the work area at work (work_bytes of device memory).
pr_status render_views(pr_ctx* ctx, const pr_cloud* cloud, const pr_view* views, uint32_t nviews,
                       const pr_render_opts* opts, void* work, uint64_t work_bytes) {
  if (cloud->ctx->device != ctx->device) return fail(PR_EINVAL, "pr_render_views: cloud lives on another device");
  if (!cloud->built) return fail(PR_ESTATE, "pr_render_views: cloud is not built (call pr_build_batches)");
  if (nviews < 1 || nviews > PR_MAX_VIEWS) return fail(PR_ERANGE, "pr_render_views: nviews %u not in 1..%d", nviews, PR_MAX_VIEWS);
  if (reinterpret_cast<uintptr_t>(work) & 255u) return fail(PR_EINVAL, "pr_render_views: work must be 256-byte aligned");
  if (work_bytes < ptr::views_work_bytes(cloud->nb, nviews))
    return fail(PR_EINVAL, "pr_render_views: work holds %llu bytes, %llu needed", (unsigned long long)work_bytes,
                (unsigned long long)ptr::views_work_bytes(cloud->nb, nviews));
  pr_render_opts o = {PR_ADAPTIVE, 1, 500.0f, 512000.0f, 0, 0, 0.0f};
  if (opts) o = *opts;
  if (o.precision != PR_ADAPTIVE && o.precision != PR_FORCE10 && o.precision != PR_FORCE20 &&
      o.precision != PR_FORCE30)
    return fail(PR_EINVAL, "pr_render_views: precision %d is not 0, 10, 20 or 30", o.precision);
  if (std::isnan(o.t10) || std::isnan(o.t20) || !(o.lod_px >= 0.0f) || !std::isfinite(o.lod_px))
    return fail(PR_EINVAL, "pr_render_views: NaN threshold or lod_px not finite and >= 0");
  for (uint32_t v = 0; v < nviews; ++v) {
    const pr_view& pv = views[v];
    if (!pv.visbuf) return fail(PR_EINVAL, "pr_render_views: view %u has no visbuf", v);
    if (pr_status s = check_dims(pv.w, pv.h)) return s;
    if (reinterpret_cast<uintptr_t>(pv.visbuf) & 15u)
      return fail(PR_EINVAL, "pr_render_views: visbuf of view %u must be 16-byte aligned", v);
    for (int i = 0; i < 16; ++i)
      if (!std::isfinite(pv.view[i]) || !std::isfinite(pv.proj[i]))
        return fail(PR_ENONFINITE, "pr_render_views: non-finite matrix in view %u", v);
  }
  if (pr_status s = set_device(ctx)) return s;
  const pr_tuning tune = ctx->tuning;
  const uint64_t nb = cloud->nb;
  const uint32_t nchunks = (nviews + ptr::VIEW_CHUNK - 1) / ptr::VIEW_CHUNK;
  if (nb * nchunks > 0xFFFFFFFFull)
    return fail(PR_ERANGE, "pr_render_views: %llu batches x %u classify launches exceed 2^32 run slots",
                (unsigned long long)nb, nchunks);
  ptr::FrameHeader* hdr = static_cast<ptr::FrameHeader*>(work);
  ptr::Run* runs = reinterpret_cast<ptr::Run*>(hdr + 1);
  ptr::LiveBatch* sub = reinterpret_cast<ptr::LiveBatch*>(runs + nb * nchunks);

  ptr::ClearViewsArgs ca;
  std::memset(&ca, 0, sizeof ca);
  ca.hdr = hdr;
  ca.stats = ctx->dev->stats;
  ca.nviews = nviews;
  ca.clear = o.accumulate ? 0u : 1u;
  ca.reset_stats = o.counters ? 1u : 0u;
  for (uint32_t v = 0; v < nviews; ++v) ca.v[v] = {views[v].visbuf, views[v].w, views[v].h};
  HIP_TRY(ptr::launch_clear_views(ca, ctx->stream), "clear views");

  for (uint32_t c = 0; c < nchunks; ++c) {
    ptr::ClassifyViewsArgs k;
    std::memset(&k, 0, sizeof k);
    k.batches = static_cast<const ptr::BatchRec*>(cloud->bufs.batches);
    k.sub = sub;
    k.runs = runs;
    k.hdr = hdr;
    k.stats = ctx->dev->stats;
    k.nb = (uint32_t)nb;
    k.nviews = nviews;
    k.view0 = c * ptr::VIEW_CHUNK;
    k.nchunk = nviews - k.view0 < ptr::VIEW_CHUNK ? nviews - k.view0 : ptr::VIEW_CHUNK;
    k.precision = o.precision;
    k.cull = o.cull ? 1 : 0;
    k.t10 = o.t10;
    k.t20 = o.t20;
    k.nodes = cloud->lod ? static_cast<const ptr::LodNode*>(cloud->bufs.nodes) : nullptr;
    k.lod_px = o.lod_px;
    k.tile_max = shape_tile(tune);
    k.max_bands = tune_bands(tune);
    k.cap = (uint32_t)(nb * nchunks);
    for (uint32_t v = 0; v < k.nchunk; ++v) {
      const pr_view& pv = views[k.view0 + v];
      frame_matrix(pv.view, pv.proj, pv.w, pv.h, k.v[v].Pm);
      k.v[v].W = pv.w;
      k.v[v].H = pv.h;
    }
    HIP_TRY(ptr::launch_classify_views(k, o.counters ? 1 : 0, ctx->stream), "classify views");
  }

  ptr::RenderViewsArgs r;
  std::memset(&r, 0, sizeof r);
  r.low = static_cast<const uint32_t*>(cloud->bufs.low);
  r.med = static_cast<const uint32_t*>(cloud->bufs.med);
  r.high = static_cast<const uint32_t*>(cloud->bufs.high);
  r.sub = sub;
  r.runs = runs;
  r.hdr = hdr;
  r.stats = ctx->dev->stats;
  r.nviews = nviews;
  r.grid = shape_grid(ctx, tune, 1);
  r.cap = (uint32_t)(nb * nchunks);
  for (uint32_t v = 0; v < nviews; ++v) r.v[v] = {views[v].visbuf, views[v].w, views[v].h};
  HIP_TRY(timed_launch(ctx, [&] { return shape_of(tune).render_views(r, nb * nchunks, o.counters ? 1 : 0, ctx->stream); }),
          "render views");
  return PR_OK;
}

}  // namespace

pr_status pr_render_views(pr_ctx* ctx, const pr_cloud* cloud, const pr_view* views, uint32_t nviews,
                          const pr_render_opts* opts, void* work, uint64_t work_bytes) {
  if (!ctx || !cloud || !views || !work) return fail(PR_EINVAL, "pr_render_views: NULL argument");
  return render_views(ctx, cloud, views, nviews, opts, work, work_bytes);
}

pr_status pr_render_views_static(pr_ctx* ctx, const pr_cloud* cloud, const pr_view* views, uint32_t nviews,
                                 const pr_render_opts* opts) {
  if (!ctx || !cloud || !views) return fail(PR_EINVAL, "pr_render_views_static: NULL argument");
  if (!cloud->built) return fail(PR_ESTATE, "pr_render_views_static: cloud is not built (call pr_build_batches)");
  if (nviews < 1 || nviews > PR_MAX_VIEWS)
    return fail(PR_ERANGE, "pr_render_views_static: nviews %u not in 1..%d", nviews, PR_MAX_VIEWS);
  const uint64_t need = ptr::views_work_bytes(cloud->nb, nviews);
  if (need > (uint64_t)PR_STATIC_WORK_BYTES)
    return fail(PR_ERANGE,
                "pr_render_views_static: %llu batches x %u views need %llu bytes of work area; the library's "
                "static area holds %llu (use pr_render_views with a work buffer)",
                (unsigned long long)cloud->nb, nviews, (unsigned long long)need,
                (unsigned long long)PR_STATIC_WORK_BYTES);
  void* work = ptr::static_work_addr(ctx->device);
  if (!work) return fail(PR_ESTATE, "pr_render_views_static: no static work area on device %d", ctx->device);
  return render_views(ctx, cloud, views, nviews, opts, work, PR_STATIC_WORK_BYTES);
}

pr_status pr_clear(pr_ctx* ctx, uint64_t* visbuf, uint32_t w, uint32_t h) {
  if (!ctx || !visbuf) return fail(PR_EINVAL, "pr_clear: NULL argument");
  if (pr_status s = check_dims(w, h)) return s;
  if (reinterpret_cast<uintptr_t>(visbuf) & 15u) return fail(PR_EINVAL, "pr_clear: visbuf must be 16-byte aligned");
  if (pr_status s = set_device(ctx)) return s;
  HIP_TRY(ptr::launch_clear(visbuf, (uint64_t)w * h, ctx->dev, nullptr, 0, ctx->stream), "clear");
  return PR_OK;
}

pr_status pr_resolve(pr_ctx* ctx, const pr_cloud* cloud, const uint64_t* visbuf, uint32_t w, uint32_t h,
                     uint32_t clear_rgba, uint32_t* rgba_out) {
  if (!ctx || !cloud || !visbuf || !rgba_out) return fail(PR_EINVAL, "pr_resolve: NULL argument");
  if (cloud->ctx->device != ctx->device) return fail(PR_EINVAL, "pr_resolve: cloud lives on another device");
  if (!cloud->built) return fail(PR_ESTATE, "pr_resolve: cloud is not built");
  if (pr_status s = check_dims(w, h)) return s;
  if (pr_status s = set_device(ctx)) return s;
  if ((reinterpret_cast<uintptr_t>(visbuf) & 15u) || (reinterpret_cast<uintptr_t>(rgba_out) & 15u))
    return fail(PR_EINVAL, "pr_resolve: visbuf and rgba_out must be 16-byte aligned");
  HIP_TRY(ptr::launch_resolve(visbuf, (uint64_t)w * h, static_cast<const uint32_t*>(cloud->bufs.colors), cloud->n,
                              clear_rgba, rgba_out, ctx->stream),
          "resolve");
  return PR_OK;
}

pr_status pr_get_stats(pr_ctx* ctx, pr_stats* out) {
  if (!ctx || !out) return fail(PR_EINVAL, "pr_get_stats: NULL argument");
  if (pr_status s = set_device(ctx)) return s;
  uint64_t st[16];
  HIP_TRY(hipMemcpyAsync(st, ctx->dev->stats, sizeof st, hipMemcpyDeviceToHost, ctx->stream), "read counters");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "pr_get_stats");
  out->batches = st[ptr::ST_BATCHES];
  out->culled = st[ptr::ST_CULLED];
  out->points = st[ptr::ST_POINTS];
  for (int i = 0; i < 3; ++i) {
    out->level_batches[i] = st[ptr::ST_LB0 + i];
    out->level_points[i] = st[ptr::ST_LP0 + i];
  }
  out->atomics = st[ptr::ST_ATOMICS];
  out->words_bytes = st[ptr::ST_WORDS];
  return PR_OK;
}

pr_status pr_sync(pr_ctx* ctx) {
  if (!ctx) return fail(PR_EINVAL, "pr_sync: NULL context");
  if (pr_status s = set_device(ctx)) return s;
  HIP_TRY(hipStreamSynchronize(ctx->stream), "pr_sync");
  HIP_TRY(hipGetLastError(), "pr_sync");
  return PR_OK;
}

pr_status pr_time_kernels(pr_ctx* ctx, uint32_t n) {
  if (!ctx) return fail(PR_EINVAL, "pr_time_kernels: NULL context");
  if (n > PR_MAX_TIMED_LAUNCHES)
    return fail(PR_EINVAL, "pr_time_kernels: %u launches above the maximum of %u", n, PR_MAX_TIMED_LAUNCHES);
  if (pr_status s = set_device(ctx)) return s;
  // events still pending on the stream are not destroyed under it
  HIP_TRY(hipStreamSynchronize(ctx->stream), "pr_time_kernels");
  for (hipEvent_t e : ctx->tev) (void)hipEventDestroy(e);
  ctx->tev.clear();
  ctx->t_used = 0;
  for (uint32_t i = 0; i < 2 * n; ++i) {
    hipEvent_t e;
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      for (hipEvent_t d : ctx->tev) (void)hipEventDestroy(d);
      ctx->tev.clear();
      return hip_fail(r, "pr_time_kernels: hipEventCreate");
    }
    ctx->tev.push_back(e);
  }
  return PR_OK;
}

pr_status pr_kernel_times(pr_ctx* ctx, float* ms_out, uint32_t capacity, uint32_t* count) {
  if (!ctx || !count || (capacity && !ms_out)) return fail(PR_EINVAL, "pr_kernel_times: NULL argument");
  if (pr_status s = set_device(ctx)) return s;
  const uint32_t m = ctx->t_used < capacity ? ctx->t_used : capacity;
  if (m) HIP_TRY(hipEventSynchronize(ctx->tev[2 * (m - 1) + 1]), "pr_kernel_times: hipEventSynchronize");
  for (uint32_t i = 0; i < m; ++i)
    HIP_TRY(hipEventElapsedTime(&ms_out[i], ctx->tev[2 * i], ctx->tev[2 * i + 1]), "pr_kernel_times: hipEventElapsedTime");
  *count = m;
  return PR_OK;
}

pr_status pr_cloud_info(const pr_cloud* cloud, uint64_t* n, uint64_t* nbatches, uint32_t* batch_size) {
  if (!cloud) return fail(PR_EINVAL, "pr_cloud_info: NULL cloud");
  if (n) *n = cloud->n;
  if (nbatches) *nbatches = cloud->built ? cloud->nb : 0;
  if (batch_size) *batch_size = cloud->built ? cloud->batch_size : 0;
  return PR_OK;
}

void pr_cloud_free(pr_cloud* cloud) { delete cloud; }

pr_status pr_stream_probe(pr_ctx* ctx, const void* src, void* dst, uint64_t bytes) {
  if (!ctx || !src) return fail(PR_EINVAL, "pr_stream_probe: NULL argument");
  if ((bytes & 15u) || (reinterpret_cast<uintptr_t>(src) & 15u) || (reinterpret_cast<uintptr_t>(dst) & 15u))
    return fail(PR_EINVAL, "pr_stream_probe: size and pointers must be multiples of 16");
  if (pr_status s = set_device(ctx)) return s;
  HIP_TRY(ptr::launch_stream(src, dst, bytes, &ctx->dev->sink, 256u * ctx->cus, ctx->stream), "stream probe");
  return PR_OK;
}

pr_status pr_raster_shapes(const pr_ctx* ctx, pr_raster_shape* out, uint32_t cap, uint32_t* count) {
  if (!ctx || !count || (cap && !out)) return fail(PR_EINVAL, "pr_raster_shapes: NULL argument");
  for (uint32_t i = 0; i < kNumShapes && i < cap; ++i)
    out[i] = {shape_at(i).waves, shape_at(i).depth, shape_at(i).tile, ctx->per_cu[i][0]};
  *count = kNumShapes;
  return PR_OK;
}

pr_status pr_set_tuning(pr_ctx* ctx, const pr_tuning* tuning) {
  if (!ctx) return fail(PR_EINVAL, "pr_set_tuning: NULL context");
  const pr_tuning t = tuning ? *tuning : pr_tuning{0, 0, 0, 0};
  if (t.shape >= kNumShapes) return fail(PR_EINVAL, "pr_set_tuning: shape %u not in 0..%u", t.shape, kNumShapes - 1);
  if (t.tile_px > shape_at(t.shape).tile)
    return fail(PR_EINVAL, "pr_set_tuning: tile_px %u above the shape's tile of %u", t.tile_px, shape_at(t.shape).tile);
  const uint32_t fit = ctx->per_cu[t.shape][0] > ctx->per_cu[t.shape][1] ? ctx->per_cu[t.shape][0]
                                                                          : ctx->per_cu[t.shape][1];
  if (t.wg_per_cu > fit) return fail(PR_EINVAL, "pr_set_tuning: wg_per_cu %u above the %u that fit", t.wg_per_cu, fit);
  if (t.max_bands > ptr::MAX_BANDS)
    return fail(PR_EINVAL, "pr_set_tuning: max_bands %u above %u", t.max_bands, ptr::MAX_BANDS);
  ctx->tuning = t;
  return PR_OK;
}

pr_status pr_get_tuning(const pr_ctx* ctx, pr_tuning* out) {
  if (!ctx || !out) return fail(PR_EINVAL, "pr_get_tuning: NULL argument");
  *out = ctx->tuning;
  return PR_OK;
}

pr_status pr_autotune(pr_ctx* ctx, const pr_cloud* cloud, const pr_view* views, uint32_t nviews,
                      const pr_render_opts* opts, void* work, uint64_t work_bytes, uint32_t reps,
                      pr_tune_trial* trials, uint32_t cap, uint32_t* ntrials, pr_tuning* best) {
  if (!ctx || !ntrials || (cap && !trials)) return fail(PR_EINVAL, "pr_autotune: NULL argument");
  if (opts && (opts->accumulate || opts->counters))
    return fail(PR_EINVAL, "pr_autotune: accumulate and counters must be 0");
  if (pr_status s = set_device(ctx)) return s;
  if (reps == 0) reps = 3;
  const pr_tuning saved = ctx->tuning;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  pr_status st = PR_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = fail(PR_EDEVICE, "pr_autotune: events");
  uint32_t n = 0;
  float best_ms = 0.0f;
  pr_tuning win = saved;
  // one candidate: an untimed frame (caches, clocks), then reps timed frames
  auto trial = [&](const pr_tuning& t) {
    if (st != PR_OK) return;
    ctx->tuning = t;
    st = pr_render_views(ctx, cloud, views, nviews, opts, work, work_bytes);
    hipError_t e = hipSuccess;
    if (st == PR_OK) e = hipEventRecord(e0, ctx->stream);
    for (uint32_t r = 0; r < reps && st == PR_OK && e == hipSuccess; ++r)
      st = pr_render_views(ctx, cloud, views, nviews, opts, work, work_bytes);
    if (st != PR_OK) return;
    if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      st = hip_fail(e, "pr_autotune: timing");
      return;
    }
    ms /= (float)reps;
    if (n < cap) trials[n] = {t, ms, 0};
    if (n == 0 || ms < best_ms) {
      best_ms = ms;
      win = t;
    }
    ++n;
  };
  // stage 1: every shape with its full and half tile bound, all and half the workgroups that fit
  for (uint32_t i = 0; i < kNumShapes; ++i) {
    const uint32_t fit = ctx->per_cu[i][1];
    for (uint32_t tile : {0u, shape_at(i).tile / 2})
      for (uint32_t wg : {0u, fit / 2})
        if (wg == 0 || wg < fit) trial({i, tile, wg, 0});
  }
  // stage 2: the band limit for the winner of stage 1
  const pr_tuning w1 = win;
  for (uint32_t bands : {1u, 2u, 8u, 16u}) trial({w1.shape, w1.tile_px, w1.wg_per_cu, bands});
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != PR_OK) {
    ctx->tuning = saved;
    return st;
  }
  ctx->tuning = win;
  *ntrials = n;
  if (best) *best = win;
  return PR_OK;
}

}  // extern "C"

/* CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded reference for what the GPU rasterizer of
 * Schuetz, Kerbl & Wimmer, "Software Rasterization of 2 Billion Points in
 * Real Time" (HPG 2022) computes.  Only the test suite, the smoke check and
 * the bench's CPU-baseline leg may load this library.  It shares no source,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * What is computed (the reading of the paper is spelled out per function):
 *   O1 validate          -- every coordinate finite, n < 2^32.
 *   O2 Morton order      -- Sec. 3.1 (group consecutive points, optionally
 *                           sorted by Morton code / z-order); optionally each
 *                           batch in a spread order (this build's own option).
 *   O3 batches           -- Sec. 3.1 and Fig. "batches memory": fixed-size
 *                           runs of consecutive points plus their bounding box.
 *   O4 quantise + split  -- Sec. 3.3, Eq. 1 and the 10-bit packing listing.
 *   O5 frame matrix      -- Sec. 3.2 point projection (toPixelID undefined in
 *                           the paper: viewport folded into the matrix).
 *   O6 per-batch prologue-- Sec. 3.2 (workgroup-wise frustum culling) and
 *                           Sec. 3.3 (500-pixel precision rule).
 *   O7 per-point raster  -- Sec. 3.2 point rasterization listing: project,
 *                           64-bit key (depth bits << 32 | index), atomicMin.
 *   O8 resolve           -- Sec. 3.3 visibility buffer: index -> colour.
 *   O10 shading          -- Sec. 3.6 high-quality shading: colour sums and
 *                           counts within a depth window, then the average.
 *
 * Arithmetic rules (both sides follow the same written definition):
 *   - binary64 steps use plain + - * / with no fused multiply-add
 *     (compiled with -ffp-contract=off), evaluated left to right;
 *   - per-point projection is binary32 with explicit fmaf in a fixed order;
 *   - the pixel is the exact floor of the real quotient hx/hw (computed as
 *     floor of the binary64 quotient, which is exact: see or_render).
 *
 * Parity pins: tests/test_oracle_*.py (hand-placed example, exact-rational
 * brute force, closed forms and invariants).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint32_t first, count;
  float min[3], max[3];
} or_batch; /* 32 bytes */

typedef struct {
  int precision; /* 0 adaptive, 10/20/30 forced */
  int cull;      /* 1 = batch frustum culling */
  float t10, t20;
  float lod_px; /* > 0: LOD culling of nodes below this projected size (Sec. 3.5) */
} or_opts;

typedef struct {
  int culled;
  int level; /* 10, 20 or 30 */
  float P[3][3];
  float t[3];
} or_decision;

typedef struct {
  uint64_t batches, culled, points;
  uint64_t level_batches[3], level_points[3];
} or_stats;

#define OR_EMPTY 0xFFFFFFFFFFFFFFFFull

static inline uint32_t f32_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}
static inline float f32_from_bits(uint32_t u) {
  float f;
  memcpy(&f, &u, 4);
  return f;
}

/* Order used for bounding boxes: IEEE 754 totalOrder restricted to finite
 * values, i.e. the usual order with -0 below +0.  (The paper does not say
 * which zero a box takes when both occur; a fixed total order makes the box
 * independent of the order in which points are visited.) */
static inline int f32_less(float a, float b) {
  return a < b || (a == b && signbit(a) && !signbit(b));
}

/* ---------------------------------------------------------------- O1 */
/* Returns -1 if every coordinate is finite, else the index of the first
 * point with a non-finite coordinate. */
int64_t or_validate(const float* xyz, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a)
      if (!isfinite(xyz[3 * i + a])) return (int64_t)i;
  return -1;
}

/* ---------------------------------------------------------------- O2 */
/* Cloud bounding box (exact fp32 min / max in the order of f32_less). */
void or_cloud_aabb(const float* xyz, uint64_t n, float mn[3], float mx[3]) {
  for (int a = 0; a < 3; ++a) {
    mn[a] = INFINITY;
    mx[a] = -INFINITY;
  }
  for (uint64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      float v = xyz[3 * i + a];
      if (f32_less(v, mn[a])) mn[a] = v;
      if (f32_less(mx[a], v)) mx[a] = v;
    }
}

/* Morton code (Sec. 3.1 names z-order without defining it; reading):
 * per axis q = min(floor(2^21 (x - cmin) / (cmax - cmin)), 2^21 - 1) in
 * binary64 (q = 0 when the extent is 0); bit b of x, y, z goes to code bit
 * 3b, 3b+1, 3b+2. */
void or_morton_codes(const float* xyz, uint64_t n, const float mn[3], const float mx[3],
                     uint64_t* codes) {
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
      double d = (double)xyz[3 * i + a] - (double)mn[a];
      double s = (double)mx[a] - (double)mn[a];
      if (s == 0.0) {
        q[a] = 0;
      } else {
        double f = floor((d * 2097152.0) / s);
        q[a] = f > 2097151.0 ? 2097151u : (uint32_t)f;
      }
    }
    uint64_t c = 0;
    for (int b = 0; b < 21; ++b)
      for (int a = 0; a < 3; ++a) c |= (uint64_t)((q[a] >> b) & 1u) << (3 * b + a);
    codes[i] = c;
  }
}

typedef struct {
  uint64_t code;
  uint64_t idx;
} or_pair;
static int cmp_pair(const void* a, const void* b) {
  const or_pair* x = (const or_pair*)a;
  const or_pair* y = (const or_pair*)b;
  if (x->code != y->code) return x->code < y->code ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}
/* Stable order by code: perm[sorted position] = original index.  Sorting the
 * pairs (code, index) lexicographically is the same as a stable sort. */
int or_morton_order(const uint64_t* codes, uint64_t n, uint32_t* perm) {
  or_pair* p = (or_pair*)malloc(sizeof(or_pair) * (n ? n : 1));
  if (!p) return -2;
  for (uint64_t i = 0; i < n; ++i) {
    p[i].code = codes[i];
    p[i].idx = i;
  }
  qsort(p, n, sizeof(or_pair), cmp_pair);
  for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)p[i].idx;
  free(p);
  return 0;
}

/* ---------------------------------------------------------------- O3 */
/* Batch b holds points [b S, min((b+1) S, n)) and their fp32 bounding box
 * (Sec. 3.1: first index, count, bounding box per batch), min and max in the
 * order of f32_less. */
uint64_t or_batch_count(uint64_t n, uint32_t S) { return (n + S - 1) / S; }

/* The record of the batch of points [lo, hi): first, count and the fp32
 * bounding box (totalOrder min/max). */
static void or_batch_of(const float* xyz, uint64_t lo, uint64_t hi, or_batch* B) {
  B->first = (uint32_t)lo;
  B->count = (uint32_t)(hi - lo);
  for (int a = 0; a < 3; ++a) {
    B->min[a] = INFINITY;
    B->max[a] = -INFINITY;
  }
  for (uint64_t i = lo; i < hi; ++i)
    for (int a = 0; a < 3; ++a) {
      float v = xyz[3 * i + a];
      if (f32_less(v, B->min[a])) B->min[a] = v;
      if (f32_less(B->max[a], v)) B->max[a] = v;
    }
}

void or_make_batches(const float* xyz, uint64_t n, uint32_t S, or_batch* out) {
  uint64_t nb = or_batch_count(n, S);
  for (uint64_t b = 0; b < nb; ++b) {
    uint64_t lo = b * S, hi = lo + S < n ? lo + S : n;
    or_batch_of(xyz, lo, hi, &out[b]);
  }
}

/* Variable-size batches (Sec. 3.5: each batch stores its first point and its
 * number of points): spans[2b] = first, spans[2b + 1] = count. */
void or_make_batches_spans(const float* xyz, const uint32_t* spans, uint64_t nb, or_batch* out) {
  for (uint64_t b = 0; b < nb; ++b)
    or_batch_of(xyz, spans[2 * b], (uint64_t)spans[2 * b] + spans[2 * b + 1], &out[b]);
}

/* ---------------------------------------------------------------- O4 */
/* Eq. 1: X30 = min(floor(2^30 (x - boxMin) / boxSize), 2^30 - 1), per axis,
 * relative to the point's batch box, in binary64 with one correctly rounded
 * division; 0 when boxSize is 0.  Split (Sec. 3.3): low = bits 29..20,
 * medium = bits 19..10, high = bits 9..0, each packed x | y << 10 | z << 20
 * as in the packing listing, bits 30-31 zero. */
uint32_t or_eq1(float x, float bmin, float bmax) {
  double d = (double)x - (double)bmin;
  double s = (double)bmax - (double)bmin;
  if (s == 0.0) return 0;
  double f = floor((d * 1073741824.0) / s);
  return f > 1073741823.0 ? 1073741823u : (uint32_t)f;
}

void or_quantize(const float* xyz, const or_batch* batches, uint64_t nb, uint32_t* low,
                 uint32_t* med, uint32_t* high) {
  for (uint64_t b = 0; b < nb; ++b) {
    const or_batch* B = &batches[b];
    for (uint64_t i = B->first; i < (uint64_t)B->first + B->count; ++i) {
      uint32_t lw = 0, mw = 0, hw = 0;
      for (int a = 0; a < 3; ++a) {
        uint32_t X30 = or_eq1(xyz[3 * i + a], B->min[a], B->max[a]);
        lw |= ((X30 >> 20) & 1023u) << (10 * a);
        mw |= ((X30 >> 10) & 1023u) << (10 * a);
        hw |= (X30 & 1023u) << (10 * a);
      }
      low[i] = lw;
      med[i] = mw;
      high[i] = hw;
    }
  }
}

/* Spread order inside a batch (this build's own option, not the paper's):
 * the batch's c points, in Morton order, are stored so that position r
 * holds Morton rank (r * m) mod c, m the first integer >= floor(c / 4) + 1
 * with gcd(m, c) = 1.  Position 4q + j then holds rank 4q + j m (mod c):
 * the j-th points of consecutive quadruples are Morton neighbours in the
 * j-th quarter of the batch, and the four points of one quadruple lie in
 * four different quarters.  The batch keeps its points. */
static uint64_t gcd_u64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}
uint64_t or_spread_multiplier(uint64_t c) {
  uint64_t m = c / 4 + 1;
  while (gcd_u64(m, c) != 1) ++m;
  return m;
}

/* Whole load-time build: optional Morton order (morton = 1; 2: Morton order
 * with every batch in the spread order above), batches, Eq. 1 split.
 * Outputs are in render order; perm[render index] = input index. */
int or_build(const float* xyz, const uint32_t* rgba, uint64_t n, uint32_t S, int morton,
             float* xyz_out, uint32_t* colors, uint32_t* perm, or_batch* batches, uint32_t* low,
             uint32_t* med, uint32_t* high) {
  if (n >= 0xFFFFFFFFull || S == 0 || morton < 0 || morton > 2) return -1;
  if (or_validate(xyz, n) >= 0) return -5;
  if (morton) {
    float mn[3], mx[3];
    or_cloud_aabb(xyz, n, mn, mx);
    uint64_t* codes = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    if (!codes) return -2;
    or_morton_codes(xyz, n, mn, mx, codes);
    int rc = or_morton_order(codes, n, perm);
    free(codes);
    if (rc) return rc;
    if (morton == 2) {
      uint32_t* sorted = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
      if (!sorted) return -2;
      memcpy(sorted, perm, sizeof(uint32_t) * n);
      for (uint64_t b0 = 0; b0 < n; b0 += S) {
        const uint64_t c = (n - b0 < S) ? n - b0 : S;
        const uint64_t m = or_spread_multiplier(c);
        for (uint64_t r = 0; r < c; ++r) perm[b0 + r] = sorted[b0 + (r * m) % c];
      }
      free(sorted);
    }
  } else {
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
  }
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t s = perm[i];
    xyz_out[3 * i] = xyz[3 * s];
    xyz_out[3 * i + 1] = xyz[3 * s + 1];
    xyz_out[3 * i + 2] = xyz[3 * s + 2];
    colors[i] = rgba[s];
  }
  uint64_t nb = or_batch_count(n, S);
  or_make_batches(xyz_out, n, S, batches);
  or_quantize(xyz_out, batches, nb, low, med, high);
  return 0;
}

/* ---------------------------------------------------------------- O5 */
/* Pixel-space matrix.  view and proj: row-major storage, column vectors
 * (clip = proj * view * [x y z 1]^T), OpenGL clip space.  Window x =
 * (x_clip / w_clip + 1) W / 2, so hx = (W/2)(row0 + row3) . p, hy likewise
 * with H, and hw = row3 . p; rows of Pm: 0 -> hx, 1 -> hy, 2 -> hw.
 * binary64, no FMA, sums left to right. */
void or_frame_matrix(const float view[16], const float proj[16], uint32_t w, uint32_t h,
                     double Pm[3][4]) {
  double C[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      C[i][j] = (((double)proj[4 * i + 0] * (double)view[0 + j] +
                  (double)proj[4 * i + 1] * (double)view[4 + j]) +
                 (double)proj[4 * i + 2] * (double)view[8 + j]) +
                (double)proj[4 * i + 3] * (double)view[12 + j];
  for (int j = 0; j < 4; ++j) {
    Pm[0][j] = (0.5 * (double)w) * (C[0][j] + C[3][j]);
    Pm[1][j] = (0.5 * (double)h) * (C[1][j] + C[3][j]);
    Pm[2][j] = C[3][j];
  }
}

/* ---------------------------------------------------------------- O6 */
/* Per-batch prologue (Sec. 3.2 culling, Sec. 3.3 precision choice).
 *  corners: the 8 corners of [min, max]; per corner and row r:
 *      h_r = ((Pm[r][0] cx + Pm[r][1] cy) + Pm[r][2] cz) + Pm[r][3]
 *      a_r = ((|Pm[r][0] cx| + |Pm[r][1] cy|) + |Pm[r][2] cz|) + |Pm[r][3]|
 *  margin M_r = 2^-16 max over corners of a_r (covers every rounding of the
 *      fp32 per-point evaluation, which is below 2^-20 a_r);
 *  cull (conservative) iff for one plane all 8 corners are outside by the
 *      margin: hw < -Mw; hx < -Mx; hx - W hw > Mx + W Mw; hy < -My;
 *      hy - H hw > My + H Mw.  Near/far planes are not tested.
 *  level: E = +inf if any corner has hw <= 0, else the larger side of the
 *      screen-space box of the projected corners (correctly rounded binary64
 *      divisions); k = 10 if E < t10 (500 px), 20 if E < t20, else 30.
 *  fold (lower-corner decode: unknown low bits are zero, so a point decodes
 *      to min + F size 2^-k):  P[r][j] = fp32(Pm[r][j] (size_j 2^-k)),
 *      t[r] = fp32(((Pm[r][0] min_x + Pm[r][1] min_y) + Pm[r][2] min_z) + Pm[r][3]). */
/* Projected extent of the box [lo, hi] (8 corners, binary64, left-to-right
 * sums): +inf if a corner has hw <= 0, else the larger side of the screen
 * box of the projected corners. */
static double proj_extent(const double Pm[3][4], const double lo[3], const double hi[3]) {
  double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
  for (int c = 0; c < 8; ++c) {
    double cx = (c & 1) ? hi[0] : lo[0], cy = (c & 2) ? hi[1] : lo[1], cz = (c & 4) ? hi[2] : lo[2];
    double hx = ((Pm[0][0] * cx + Pm[0][1] * cy) + Pm[0][2] * cz) + Pm[0][3];
    double hy = ((Pm[1][0] * cx + Pm[1][1] * cy) + Pm[1][2] * cz) + Pm[1][3];
    double hw = ((Pm[2][0] * cx + Pm[2][1] * cy) + Pm[2][2] * cz) + Pm[2][3];
    if (!(hw > 0.0)) return INFINITY;
    double u = hx / hw, v = hy / hw;
    if (u < umin) umin = u;
    if (u > umax) umax = u;
    if (v < vmin) vmin = v;
    if (v > vmax) vmax = v;
  }
  double ex = umax - umin, ey = vmax - vmin;
  return ex > ey ? ex : ey;
}

/* node: NULL, or the batch's octree node (cube origin x, y, z, edge, level).
 * LOD (Sec. 3.5): with o->lod_px > 0, a batch of a node below the root
 * (level >= 1) is culled iff the projected extent of the node's cube is
 * below lod_px; the root is never culled this way. */
void or_decide(const double Pm[3][4], const or_batch* B, const double* node, uint32_t w, uint32_t h,
               const or_opts* o, or_decision* d) {
  double s[3];
  for (int a = 0; a < 3; ++a) s[a] = (double)B->max[a] - (double)B->min[a];
  double H[3][8], M[3];
  for (int r = 0; r < 3; ++r) {
    double amax = 0.0;
    for (int c = 0; c < 8; ++c) {
      double cx = (double)((c & 1) ? B->max[0] : B->min[0]);
      double cy = (double)((c & 2) ? B->max[1] : B->min[1]);
      double cz = (double)((c & 4) ? B->max[2] : B->min[2]);
      H[r][c] = ((Pm[r][0] * cx + Pm[r][1] * cy) + Pm[r][2] * cz) + Pm[r][3];
      double a = ((fabs(Pm[r][0] * cx) + fabs(Pm[r][1] * cy)) + fabs(Pm[r][2] * cz)) + fabs(Pm[r][3]);
      if (a > amax) amax = a;
    }
    M[r] = 0x1p-16 * amax;
  }
  double Wd = (double)w, Hd = (double)h;
  int behind = 1, left = 1, right = 1, bottom = 1, top = 1;
  for (int c = 0; c < 8; ++c) {
    if (!(H[2][c] < -M[2])) behind = 0;
    if (!(H[0][c] < -M[0])) left = 0;
    if (!(H[0][c] - Wd * H[2][c] > M[0] + Wd * M[2])) right = 0;
    if (!(H[1][c] < -M[1])) bottom = 0;
    if (!(H[1][c] - Hd * H[2][c] > M[1] + Hd * M[2])) top = 0;
  }
  d->culled = o->cull ? (behind | left | right | bottom | top) : 0;
  if (!d->culled && o->lod_px > 0.0f && node && node[4] >= 1.0) {
    double lo[3] = {node[0], node[1], node[2]};
    double hi[3] = {node[0] + node[3], node[1] + node[3], node[2] + node[3]};
    if (proj_extent(Pm, lo, hi) < (double)o->lod_px) d->culled = 1;
  }

  int k;
  if (o->precision == 10 || o->precision == 20 || o->precision == 30) {
    k = o->precision;
  } else {
    int front = 1;
    for (int c = 0; c < 8; ++c)
      if (!(H[2][c] > 0.0)) front = 0;
    double E = INFINITY;
    if (front) {
      double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
      for (int c = 0; c < 8; ++c) {
        double u = H[0][c] / H[2][c], v = H[1][c] / H[2][c];
        if (u < umin) umin = u;
        if (u > umax) umax = u;
        if (v < vmin) vmin = v;
        if (v > vmax) vmax = v;
      }
      double ex = umax - umin, ey = vmax - vmin;
      E = ex > ey ? ex : ey;
    }
    k = E < (double)o->t10 ? 10 : (E < (double)o->t20 ? 20 : 30);
  }
  d->level = k;
  double scale = k == 10 ? 0x1p-10 : (k == 20 ? 0x1p-20 : 0x1p-30);
  for (int r = 0; r < 3; ++r) {
    for (int j = 0; j < 3; ++j) d->P[r][j] = (float)(Pm[r][j] * (s[j] * scale));
    d->t[r] = (float)(((Pm[r][0] * (double)B->min[0] + Pm[r][1] * (double)B->min[1]) +
                       Pm[r][2] * (double)B->min[2]) +
                      Pm[r][3]);
  }
}

/* ---------------------------------------------------------------- O7 */
/* Render every non-culled batch into vb (w*h entries, row 0 = bottom).
 * vb must be filled with OR_EMPTY by the caller (or hold a previous partial
 * result: the operation is a running minimum).
 *  decode: F = low field (k=10); (low << 10) | med (k=20);
 *          (low << 20) | (med << 10) | high (k=30); X = (float)F (RNE).
 *  project: hx = fmaf(P02, Z, fmaf(P01, Y, fmaf(P00, X, t0))), same for hy, hw.
 *  keep iff hw > 0 and 0 <= hx < W hw and 0 <= hy < H hw (exact in binary64:
 *      W hw has at most 37 significant bits).
 *  pixel: px = floor(hx / hw) exactly.  floor of the binary64 quotient is
 *      exact here: for binary32 hx, hw with 0 <= q = hx/hw < 2^13, a
 *      non-integer q is at least 2^-25 away from every integer while the
 *      binary64 quotient is within 2^-40 of q, and an integer q is exact.
 *  key: (float bits of hw) << 32 | point index (Sec. 3.2 listing; hw > 0,
 *      so the bits order like the values); vb[p] = min(vb[p], key).
 * If batch_ids is non-NULL only those batches are rendered (any order). */
/* O7 steps 1-4 for point i of a batch with decision d: decode at the batch's
 * level, project with the three fmaf chains, reject unless hw > 0 and the
 * point is inside the image; the pixel is the exact floor of hx/hw, hy/hw
 * (floor of the binary64 quotient of two binary32 values, which is exact for
 * quotients below 2^26).  Returns 1 and (hw, pixel index) for a drawn point. */
static int or_point(const or_decision* d, const uint32_t* low, const uint32_t* med, const uint32_t* high,
                    uint64_t i, uint32_t w, uint32_t h, float* hw_out, uint64_t* p_out) {
  float XYZ[3];
  for (int a = 0; a < 3; ++a) {
    uint32_t lo = (low[i] >> (10 * a)) & 1023u;
    uint32_t F;
    if (d->level == 10) {
      F = lo;
    } else if (d->level == 20) {
      F = (lo << 10) | ((med[i] >> (10 * a)) & 1023u);
    } else {
      F = (lo << 20) | (((med[i] >> (10 * a)) & 1023u) << 10) | ((high[i] >> (10 * a)) & 1023u);
    }
    XYZ[a] = (float)F;
  }
  float hx = fmaf(d->P[0][2], XYZ[2], fmaf(d->P[0][1], XYZ[1], fmaf(d->P[0][0], XYZ[0], d->t[0])));
  float hy = fmaf(d->P[1][2], XYZ[2], fmaf(d->P[1][1], XYZ[1], fmaf(d->P[1][0], XYZ[0], d->t[1])));
  float hw = fmaf(d->P[2][2], XYZ[2], fmaf(d->P[2][1], XYZ[1], fmaf(d->P[2][0], XYZ[0], d->t[2])));
  if (!(hw > 0.0f)) return 0;
  double dx = (double)hx, dy = (double)hy, dw = (double)hw;
  if (!(dx >= 0.0 && dx < (double)w * dw && dy >= 0.0 && dy < (double)h * dw)) return 0;
  uint64_t px = (uint64_t)floor(dx / dw), py = (uint64_t)floor(dy / dw);
  *hw_out = hw;
  *p_out = py * w + px;
  return 1;
}

void or_render(const or_batch* batches, const double* nodes, uint64_t nb, const uint64_t* batch_ids, uint64_t nids,
               const uint32_t* low, const uint32_t* med, const uint32_t* high, const float view[16],
               const float proj[16], uint32_t w, uint32_t h, const or_opts* o, uint64_t* vb,
               or_stats* st) {
  double Pm[3][4];
  or_frame_matrix(view, proj, w, h, Pm);
  uint64_t n_iter = batch_ids ? nids : nb;
  if (st) memset(st, 0, sizeof *st);
  for (uint64_t it = 0; it < n_iter; ++it) {
    uint64_t b = batch_ids ? batch_ids[it] : it;
    const or_batch* B = &batches[b];
    or_decision d;
    or_decide(Pm, B, nodes ? nodes + 5 * b : NULL, w, h, o, &d);
    if (st) st->batches++;
    if (d.culled) {
      if (st) st->culled++;
      continue;
    }
    int li = d.level / 10 - 1;
    if (st) {
      st->points += B->count;
      st->level_batches[li]++;
      st->level_points[li] += B->count;
    }
    for (uint64_t i = B->first; i < (uint64_t)B->first + B->count; ++i) {
      float hw;
      uint64_t p;
      if (!or_point(&d, low, med, high, i, w, h, &hw, &p)) continue;
      uint64_t key = ((uint64_t)f32_bits(hw) << 32) | (uint64_t)i;
      if (key < vb[p]) vb[p] = key;
    }
  }
}

/* Per-batch decisions only (for counters and sampled checks). */
void or_decide_all(const or_batch* batches, const double* nodes, uint64_t nb, const float view[16],
                   const float proj[16], uint32_t w, uint32_t h, const or_opts* o, or_decision* out) {
  double Pm[3][4];
  or_frame_matrix(view, proj, w, h, Pm);
  for (uint64_t b = 0; b < nb; ++b) or_decide(Pm, &batches[b], nodes ? nodes + 5 * b : NULL, w, h, o, &out[b]);
}

/* ---------------------------------------------------------------- O8 */
/* Visibility-buffer resolve (Sec. 3.3): the colour of the winning point, or
 * the clear colour where no point landed.  An index that is not a point of
 * this cloud (a buffer rendered from another cloud) also gives the clear
 * colour; a buffer rendered from this cloud never holds one. */
void or_resolve(const uint64_t* vb, uint64_t npix, const uint32_t* colors, uint64_t ncolors,
                uint32_t clear_rgba, uint32_t* fb) {
  for (uint64_t p = 0; p < npix; ++p) {
    uint32_t idx = (uint32_t)(vb[p] & 0xFFFFFFFFull);
    fb[p] = (vb[p] == OR_EMPTY || idx >= ncolors) ? clear_rgba : colors[idx];
  }
}

/* ------------------------------------------------------- high-quality shading */
/* Sec. 3.6: the colours of the points within a depth range behind each
 * pixel's closest point are summed with a counter, and a final pass divides.
 * Reading taken here:
 *   - the closest depth of pixel p is the depth of its visibility-buffer key,
 *     hw_min = bits (vb[p] >> 32) as binary32 (vb from or_render, same opts);
 *   - point i (drawn by O7 at pixel p) joins iff hw_i <= fl32(hw_min * window),
 *     one binary32 multiplication (window >= 1; 1.01 admits points up to one percent
 *     farther than the closest one);
 *   - the sums are the paper's two 64-bit words per pixel holding four 32-bit
 *     fields: acc[2p] += R + G * 2^32, acc[2p + 1] += B + 2^32 (count), with
 *     R, G, B the low three bytes of the point's colour; additions wrap
 *     modulo 2^64 (exact while a pixel's sums stay below 2^32). */
void or_accumulate(const or_batch* batches, const double* nodes, uint64_t nb, const uint64_t* batch_ids, uint64_t nids,
                   const uint32_t* low, const uint32_t* med, const uint32_t* high, const uint32_t* colors,
                   const float view[16], const float proj[16], uint32_t w, uint32_t h, const or_opts* o,
                   float window, const uint64_t* vb, uint64_t* acc) {
  double Pm[3][4];
  or_frame_matrix(view, proj, w, h, Pm);
  uint64_t n_iter = batch_ids ? nids : nb;
  for (uint64_t it = 0; it < n_iter; ++it) {
    uint64_t b = batch_ids ? batch_ids[it] : it;
    const or_batch* B = &batches[b];
    or_decision d;
    or_decide(Pm, B, nodes ? nodes + 5 * b : NULL, w, h, o, &d);
    if (d.culled) continue;
    for (uint64_t i = B->first; i < (uint64_t)B->first + B->count; ++i) {
      float hw;
      uint64_t p;
      if (!or_point(&d, low, med, high, i, w, h, &hw, &p)) continue;
      float hw_min = f32_from_bits((uint32_t)(vb[p] >> 32));
      float thr = hw_min * window;
      if (!(hw <= thr)) continue;
      uint32_t c = colors[i];
      acc[2 * p] += (uint64_t)(c & 255u) + ((uint64_t)((c >> 8) & 255u) << 32);
      acc[2 * p + 1] += (uint64_t)((c >> 16) & 255u) + (1ull << 32);
    }
  }
}

/* The average: each channel (sum + count / 2) / count (rounded to nearest,
 * halves up), alpha 255; pixels with no point get the clear colour. */
void or_resolve_hqs(const uint64_t* acc, uint64_t npix, uint32_t clear_rgba, uint32_t* fb) {
  for (uint64_t p = 0; p < npix; ++p) {
    uint64_t n = acc[2 * p + 1] >> 32;
    if (n == 0) {
      fb[p] = clear_rgba;
      continue;
    }
    uint64_t r = ((acc[2 * p] & 0xFFFFFFFFull) + n / 2) / n;
    uint64_t g = ((acc[2 * p] >> 32) + n / 2) / n;
    uint64_t b = ((acc[2 * p + 1] & 0xFFFFFFFFull) + n / 2) / n;
    fb[p] = (uint32_t)r | ((uint32_t)g << 8) | ((uint32_t)b << 16) | (255u << 24);
  }
}

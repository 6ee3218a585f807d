/* Seeded synthetic point clouds: the stand-ins for the paper's scanned data
 * sets (Eclepens, Morro Bay, Banyunibo, Niederweiden are not available).
 *
 * This file generates positions and colours only.  It holds none of the
 * rasterizer's arithmetic (no quantisation, no projection, no ordering by
 * Morton code); both the CPU oracle and the GPU path consume its output.
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014).  The c-th output of a generator seeded
 * with s is mix(s + (c + 1) * 0x9E3779B97F4A7C15), so every (seed, counter)
 * pair can be evaluated on its own: point i of a cloud is a pure function of
 * (seed, i), and clouds can be produced by any number of threads in any
 * chunking with identical bytes.
 *
 * Build: gcc -O2 -fPIC -shared -pthread -ffp-contract=off (see build.py).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------ RNG */
static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static inline uint64_t sm_at(uint64_t seed, uint64_t ctr) {
  return sm_mix(seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull);
}
/* uniform in [0, 1) with 53 random bits */
static inline double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
/* uniform in (0, 1] (safe for log) */
static inline double u01_open0(uint64_t r) { return 1.0 - u01(r); }

/* One standard normal deviate pair by the Box-Muller transform. */
static inline void box_muller(uint64_t r1, uint64_t r2, double* a, double* b) {
  const double TWO_PI = 6.283185307179586476925286766559;
  double rad = sqrt(-2.0 * log(u01_open0(r1)));
  double th = TWO_PI * u01(r2);
  *a = rad * cos(th);
  *b = rad * sin(th);
}

/* Counters consumed per point (both generators). */
#define CTR_PER_POINT 24u

/* -------------------------------------------------------- thread helper */
typedef void (*range_fn)(void* arg, uint64_t lo, uint64_t hi);
typedef struct { range_fn fn; void* arg; uint64_t lo, hi; } range_job;
static void* range_thread(void* p) {
  range_job* j = (range_job*)p;
  j->fn(j->arg, j->lo, j->hi);
  return NULL;
}
static int pick_threads(int req) {
  if (req > 0) return req > 256 ? 256 : req;
  long c = sysconf(_SC_NPROCESSORS_ONLN);
  if (c < 1) c = 1;
  if (c > 16) c = 16;
  return (int)c;
}
static void parallel_for(uint64_t n, int nthreads, range_fn fn, void* arg) {
  int t = pick_threads(nthreads);
  if ((uint64_t)t > n) t = n ? (int)n : 1;
  pthread_t th[256];
  range_job jobs[256];
  for (int k = 0; k < t; ++k) {
    jobs[k].fn = fn;
    jobs[k].arg = arg;
    jobs[k].lo = n * (uint64_t)k / (uint64_t)t;
    jobs[k].hi = n * (uint64_t)(k + 1) / (uint64_t)t;
  }
  for (int k = 1; k < t; ++k) pthread_create(&th[k], NULL, range_thread, &jobs[k]);
  range_thread(&jobs[0]);
  for (int k = 1; k < t; ++k) pthread_join(th[k], NULL);
}

/* ============================================================ config 1
 * 8 primitives in the cube [0,100]^3 m.  Each is a plane patch or a sphere
 * (probability 1/2 each, from the seed).  Plane: centre U[20,80]^3, normal
 * uniform on the unit sphere, square patch of side U(20,80) m; samples that
 * leave the cube are redrawn (up to 8 times, then clamped).  Sphere: centre
 * U[20,80]^3, radius U(5,20) m, uniform on the surface.  Points are
 * primitive-major (point i belongs to primitive floor(8 i / n)).  Each axis
 * gets N(0, sigma) noise; colours are uniform 32-bit words.            */
typedef struct {
  int type; /* 0 plane, 1 sphere */
  double c[3], n[3], t1[3], t2[3], side, radius;
} prim_t;

static void make_prims(uint64_t seed, prim_t* P) {
  uint64_t ps = sm_mix(seed ^ 0xC1C1C1C1C1C1C1C1ull);
  for (int p = 0; p < 8; ++p) {
    uint64_t b = (uint64_t)p * 32u;
    prim_t* q = &P[p];
    q->type = (int)(sm_at(ps, b) & 1u);
    for (int a = 0; a < 3; ++a) q->c[a] = 20.0 + 60.0 * u01(sm_at(ps, b + 1 + a));
    if (q->type == 0) {
      double z = 2.0 * u01(sm_at(ps, b + 4)) - 1.0;
      double ph = 6.283185307179586 * u01(sm_at(ps, b + 5));
      double r = sqrt(1.0 - z * z);
      q->n[0] = r * cos(ph); q->n[1] = r * sin(ph); q->n[2] = z;
      double ax[3] = {0, 0, 1};
      if (fabs(z) > 0.9) { ax[0] = 1; ax[2] = 0; }
      /* t1 = normalize(n x ax), t2 = n x t1 */
      double t1[3] = {q->n[1] * ax[2] - q->n[2] * ax[1], q->n[2] * ax[0] - q->n[0] * ax[2],
                      q->n[0] * ax[1] - q->n[1] * ax[0]};
      double l = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
      for (int a = 0; a < 3; ++a) q->t1[a] = t1[a] / l;
      q->t2[0] = q->n[1] * q->t1[2] - q->n[2] * q->t1[1];
      q->t2[1] = q->n[2] * q->t1[0] - q->n[0] * q->t1[2];
      q->t2[2] = q->n[0] * q->t1[1] - q->n[1] * q->t1[0];
      q->side = 20.0 + 60.0 * u01(sm_at(ps, b + 6));
    } else {
      q->radius = 5.0 + 15.0 * u01(sm_at(ps, b + 6));
    }
  }
}

typedef struct {
  uint64_t seed, n;
  double sigma;
  prim_t P[8];
  float* xyz;
  uint32_t* rgba;
} prim_job;

static void prim_range(void* arg, uint64_t lo, uint64_t hi) {
  prim_job* J = (prim_job*)arg;
  for (uint64_t i = lo; i < hi; ++i) {
    uint64_t base = i * CTR_PER_POINT;
    const prim_t* q = &J->P[(i * 8u) / J->n];
    double pos[3];
    if (q->type == 0) {
      int ok = 0;
      for (int at = 0; at < 8 && !ok; ++at) {
        double u = u01(sm_at(J->seed, base + 2 * at)) - 0.5;
        double v = u01(sm_at(J->seed, base + 2 * at + 1)) - 0.5;
        ok = 1;
        for (int a = 0; a < 3; ++a) {
          pos[a] = q->c[a] + u * q->side * q->t1[a] + v * q->side * q->t2[a];
          if (pos[a] < 0.0 || pos[a] > 100.0) ok = 0;
        }
      }
      for (int a = 0; a < 3; ++a) pos[a] = pos[a] < 0.0 ? 0.0 : (pos[a] > 100.0 ? 100.0 : pos[a]);
    } else {
      double z = 2.0 * u01(sm_at(J->seed, base)) - 1.0;
      double ph = 6.283185307179586 * u01(sm_at(J->seed, base + 1));
      double r = sqrt(1.0 - z * z);
      pos[0] = q->c[0] + q->radius * r * cos(ph);
      pos[1] = q->c[1] + q->radius * r * sin(ph);
      pos[2] = q->c[2] + q->radius * z;
    }
    double g[4];
    box_muller(sm_at(J->seed, base + 16), sm_at(J->seed, base + 17), &g[0], &g[1]);
    box_muller(sm_at(J->seed, base + 18), sm_at(J->seed, base + 19), &g[2], &g[3]);
    for (int a = 0; a < 3; ++a) J->xyz[3 * i + a] = (float)(pos[a] + J->sigma * g[a]);
    J->rgba[i] = (uint32_t)(sm_at(J->seed, base + 20) >> 32);
  }
}

int synth_primitives(uint64_t seed, uint64_t n, double sigma, float* xyz, uint32_t* rgba,
                     int nthreads) {
  if (!xyz || !rgba) return -1;
  prim_job J;
  J.seed = seed; J.n = n; J.sigma = sigma; J.xyz = xyz; J.rgba = rgba;
  make_prims(seed, J.P);
  parallel_for(n, nthreads, prim_range, &J);
  return 0;
}

/* ============================================================ terrain
 * A 1 km x 1 km aerial-scan-like scene on [0,1000]^2 m:
 *   80 % ground: (x,y) uniform, z = fBm(x,y): 5 octaves of 2D gradient noise,
 *        base wavelength 250 m, lacunarity 2, gain 1/2, amplitude 60 m;
 *   16 % on 300 axis-aligned box "buildings" (footprint U(8,40) m per side,
 *        height U(5,60) m, standing on the terrain at their centre); a
 *        building is picked uniformly, then roof or one of the 4 walls with
 *        probability proportional to its area;
 *    4 % on 5000 vertical "poles" (height U(6,12) m, radius 0.1 m).
 * Every axis gets N(0, sigma) noise; colours are uniform 32-bit words.
 * Optional generation order: a stable bucket sort by 10 m tiles visited in
 * serpentine (boustrophedon) order, like aerial strips.                  */
#define N_BUILDINGS 300
#define N_POLES 5000

/* 8 unit gradient directions at multiples of 45 degrees */
static const double GRAD8[8][2] = {
    {1.0, 0.0}, {0.70710678118654752, 0.70710678118654752}, {0.0, 1.0},
    {-0.70710678118654752, 0.70710678118654752}, {-1.0, 0.0},
    {-0.70710678118654752, -0.70710678118654752}, {0.0, -1.0},
    {0.70710678118654752, -0.70710678118654752}};

static inline double fade(double t) { return t * t * t * (t * (t * 6.0 - 15.0) + 10.0); }

static inline double grad_dot(uint64_t oseed, int64_t ix, int64_t iy, double dx, double dy) {
  uint64_t h = sm_mix(oseed ^ sm_mix((uint64_t)ix * 0x632BE59BD9B4E019ull + (uint64_t)iy));
  const double* g = GRAD8[h & 7u];
  return g[0] * dx + g[1] * dy;
}

static double gradient_noise(uint64_t oseed, double x, double y) {
  double fx = floor(x), fy = floor(y);
  int64_t ix = (int64_t)fx, iy = (int64_t)fy;
  double dx = x - fx, dy = y - fy;
  double n00 = grad_dot(oseed, ix, iy, dx, dy);
  double n10 = grad_dot(oseed, ix + 1, iy, dx - 1.0, dy);
  double n01 = grad_dot(oseed, ix, iy + 1, dx, dy - 1.0);
  double n11 = grad_dot(oseed, ix + 1, iy + 1, dx - 1.0, dy - 1.0);
  double u = fade(dx), v = fade(dy);
  double a = n00 + u * (n10 - n00);
  double b = n01 + u * (n11 - n01);
  return a + v * (b - a);
}

double synth_terrain_height(uint64_t seed, double x, double y) {
  uint64_t ts = sm_mix(seed ^ 0x7E77A1A7E77A1A7Eull);
  double sum = 0.0, amp = 1.0, freq = 1.0 / 250.0;
  for (int o = 0; o < 5; ++o) {
    sum += amp * gradient_noise(sm_at(ts, (uint64_t)o), x * freq, y * freq);
    amp *= 0.5;
    freq *= 2.0;
  }
  return 60.0 * sum;
}

typedef struct { double cx, cy, wx, wy, h, z0; double a_roof, a_wx, a_wy, a_tot; } building_t;
typedef struct { double x, y, h, z0; } pole_t;

typedef struct {
  uint64_t seed, n, n_ground, n_build;
  double sigma;
  building_t* B;
  pole_t* Q;
  float* xyz;
  uint32_t* rgba;
  uint16_t* tile; /* optional: serpentine tile id per point */
  const uint32_t* idx; /* gather: point indices, output slot j holds point idx[j] */
} terrain_job;

static void make_scene(uint64_t seed, building_t* B, pole_t* Q) {
  uint64_t ps = sm_mix(seed ^ 0xB0B0B0B0B0B0B0B0ull);
  for (int b = 0; b < N_BUILDINGS; ++b) {
    uint64_t c = (uint64_t)b * 8u;
    building_t* q = &B[b];
    q->cx = 50.0 + 900.0 * u01(sm_at(ps, c));
    q->cy = 50.0 + 900.0 * u01(sm_at(ps, c + 1));
    q->wx = 8.0 + 32.0 * u01(sm_at(ps, c + 2));
    q->wy = 8.0 + 32.0 * u01(sm_at(ps, c + 3));
    q->h = 5.0 + 55.0 * u01(sm_at(ps, c + 4));
    q->z0 = synth_terrain_height(seed, q->cx, q->cy);
    q->a_roof = q->wx * q->wy;
    q->a_wx = q->wx * q->h; /* each of the two walls facing +-y */
    q->a_wy = q->wy * q->h; /* each of the two walls facing +-x */
    q->a_tot = q->a_roof + 2.0 * q->a_wx + 2.0 * q->a_wy;
  }
  uint64_t qs = sm_mix(seed ^ 0x9019019019019019ull);
  for (int p = 0; p < N_POLES; ++p) {
    uint64_t c = (uint64_t)p * 4u;
    Q[p].x = 10.0 + 980.0 * u01(sm_at(qs, c));
    Q[p].y = 10.0 + 980.0 * u01(sm_at(qs, c + 1));
    Q[p].h = 6.0 + 6.0 * u01(sm_at(qs, c + 2));
    Q[p].z0 = synth_terrain_height(seed, Q[p].x, Q[p].y);
  }
}

static inline uint16_t serpentine_tile(double x, double y) {
  int tx = (int)floor(x / 10.0), ty = (int)floor(y / 10.0);
  tx = tx < 0 ? 0 : (tx > 99 ? 99 : tx);
  ty = ty < 0 ? 0 : (ty > 99 ? 99 : ty);
  return (uint16_t)(ty * 100 + ((ty & 1) ? 99 - tx : tx));
}

/* Point i of the index-order terrain cloud: position f[3] and colour c; the
 * serpentine tile is written to J->tile[i] when requested. */
static void terrain_point(const terrain_job* J, uint64_t i, float f[3], uint32_t* c) {
  {
    uint64_t base = i * CTR_PER_POINT;
    double pos[3];
    if (i < J->n_ground) {
      pos[0] = 1000.0 * u01(sm_at(J->seed, base));
      pos[1] = 1000.0 * u01(sm_at(J->seed, base + 1));
      pos[2] = synth_terrain_height(J->seed, pos[0], pos[1]);
    } else if (i < J->n_build) {
      const building_t* q = &J->B[sm_at(J->seed, base) % N_BUILDINGS];
      double pick = q->a_tot * u01(sm_at(J->seed, base + 1));
      double u = u01(sm_at(J->seed, base + 2)), v = u01(sm_at(J->seed, base + 3));
      double x0 = q->cx - 0.5 * q->wx, y0 = q->cy - 0.5 * q->wy;
      if (pick < q->a_roof) {
        pos[0] = x0 + u * q->wx; pos[1] = y0 + v * q->wy; pos[2] = q->z0 + q->h;
      } else if (pick < q->a_roof + 2.0 * q->a_wx) {
        pos[0] = x0 + u * q->wx; pos[1] = (pick < q->a_roof + q->a_wx) ? y0 : y0 + q->wy;
        pos[2] = q->z0 + v * q->h;
      } else {
        pos[0] = (pick < q->a_roof + 2.0 * q->a_wx + q->a_wy) ? x0 : x0 + q->wx;
        pos[1] = y0 + u * q->wy; pos[2] = q->z0 + v * q->h;
      }
    } else {
      const pole_t* q = &J->Q[sm_at(J->seed, base) % N_POLES];
      double ph = 6.283185307179586 * u01(sm_at(J->seed, base + 1));
      pos[0] = q->x + 0.1 * cos(ph);
      pos[1] = q->y + 0.1 * sin(ph);
      pos[2] = q->z0 + q->h * u01(sm_at(J->seed, base + 2));
    }
    double g[4];
    box_muller(sm_at(J->seed, base + 16), sm_at(J->seed, base + 17), &g[0], &g[1]);
    box_muller(sm_at(J->seed, base + 18), sm_at(J->seed, base + 19), &g[2], &g[3]);
    for (int a = 0; a < 3; ++a) f[a] = (float)(pos[a] + J->sigma * g[a]);
    *c = (uint32_t)(sm_at(J->seed, base + 20) >> 32);
  }
}

static void terrain_range(void* arg, uint64_t lo, uint64_t hi) {
  terrain_job* J = (terrain_job*)arg;
  for (uint64_t i = lo; i < hi; ++i) {
    float f[3];
    uint32_t c;
    terrain_point(J, i, f, &c);
    J->xyz[3 * i] = f[0]; J->xyz[3 * i + 1] = f[1]; J->xyz[3 * i + 2] = f[2];
    J->rgba[i] = c;
    if (J->tile) J->tile[i] = serpentine_tile(f[0], f[1]);
  }
}

/* ---- stable bucket sort by serpentine tile (10000 buckets), threaded ---- */
#define N_TILES 10000
typedef struct {
  uint64_t n; int nchunks;
  const uint16_t* tile;
  uint64_t* hist; /* [chunk][N_TILES] counts, then start offsets */
  const float* sx; const uint32_t* sc;
  float* dx; uint32_t* dc;
} bucket_job;
typedef struct { bucket_job* J; int chunk; } bucket_arg;

static void bucket_hist(void* arg, uint64_t lo, uint64_t hi) {
  bucket_job* J = (bucket_job*)arg;
  for (uint64_t c = lo; c < hi; ++c) {
    uint64_t* h = J->hist + c * N_TILES;
    memset(h, 0, sizeof(uint64_t) * N_TILES);
    uint64_t a = J->n * c / (uint64_t)J->nchunks, b = J->n * (c + 1) / (uint64_t)J->nchunks;
    for (uint64_t i = a; i < b; ++i) h[J->tile[i]]++;
  }
}
static void bucket_scatter(void* arg, uint64_t lo, uint64_t hi) {
  bucket_job* J = (bucket_job*)arg;
  for (uint64_t c = lo; c < hi; ++c) {
    uint64_t* h = J->hist + c * N_TILES;
    uint64_t a = J->n * c / (uint64_t)J->nchunks, b = J->n * (c + 1) / (uint64_t)J->nchunks;
    for (uint64_t i = a; i < b; ++i) {
      uint64_t d = h[J->tile[i]]++;
      J->dx[3 * d] = J->sx[3 * i]; J->dx[3 * d + 1] = J->sx[3 * i + 1];
      J->dx[3 * d + 2] = J->sx[3 * i + 2];
      J->dc[d] = J->sc[i];
    }
  }
}

/* Points [lo, hi) of the index-order terrain cloud of n points, written to
 * xyz[0 .. 3(hi-lo)) and rgba[0 .. hi-lo): lets a very large cloud be produced
 * in chunks (identical bytes to synth_terrain(order = 0)). */
int synth_terrain_range(uint64_t seed, uint64_t n, uint64_t lo, uint64_t hi, double sigma, float* xyz,
                        uint32_t* rgba, int nthreads) {
  if (!xyz || !rgba || lo > hi || hi > n) return -1;
  terrain_job J;
  memset(&J, 0, sizeof J);
  J.seed = seed; J.n = n; J.sigma = sigma;
  J.n_ground = (uint64_t)((double)n * 0.80);
  J.n_build = (uint64_t)((double)n * 0.96);
  J.B = (building_t*)malloc(sizeof(building_t) * N_BUILDINGS);
  J.Q = (pole_t*)malloc(sizeof(pole_t) * N_POLES);
  if (!J.B || !J.Q) { free(J.B); free(J.Q); return -2; }
  make_scene(seed, J.B, J.Q);
  /* shift the output pointers so that point i lands at index i - lo */
  J.xyz = xyz - 3 * lo;
  J.rgba = rgba - lo;
  range_job jobs[256];
  pthread_t th[256];
  int t = pick_threads(nthreads);
  uint64_t cnt = hi - lo;
  if ((uint64_t)t > cnt) t = cnt ? (int)cnt : 1;
  for (int k = 0; k < t; ++k) {
    jobs[k].fn = terrain_range; jobs[k].arg = &J;
    jobs[k].lo = lo + cnt * (uint64_t)k / (uint64_t)t;
    jobs[k].hi = lo + cnt * (uint64_t)(k + 1) / (uint64_t)t;
  }
  for (int k = 1; k < t; ++k) pthread_create(&th[k], NULL, range_thread, &jobs[k]);
  range_thread(&jobs[0]);
  for (int k = 1; k < t; ++k) pthread_join(th[k], NULL);
  free(J.B); free(J.Q);
  return 0;
}

static void terrain_gather(void* arg, uint64_t lo, uint64_t hi) {
  terrain_job* J = (terrain_job*)arg;
  for (uint64_t j = lo; j < hi; ++j) {
    float f[3];
    uint32_t c;
    terrain_point(J, J->idx[j], f, &c);
    J->xyz[3 * j] = f[0]; J->xyz[3 * j + 1] = f[1]; J->xyz[3 * j + 2] = f[2];
    J->rgba[j] = c;
  }
}

/* Points idx[0 .. count) of the index-order terrain cloud of n points (each
 * index < n), written to xyz[3j ..] and rgba[j]: the same bytes as those
 * points of synth_terrain(order = 0).  Returns 0, -1 on bad arguments, -2 if
 * temporary memory is unavailable. */
int synth_terrain_gather(uint64_t seed, uint64_t n, const uint32_t* idx, uint64_t count, double sigma,
                         float* xyz, uint32_t* rgba, int nthreads) {
  if ((count && (!idx || !xyz || !rgba))) return -1;
  for (uint64_t j = 0; j < count; ++j)
    if ((uint64_t)idx[j] >= n) return -1;
  terrain_job J;
  memset(&J, 0, sizeof J);
  J.seed = seed; J.n = n; J.sigma = sigma;
  J.n_ground = (uint64_t)((double)n * 0.80);
  J.n_build = (uint64_t)((double)n * 0.96);
  J.B = (building_t*)malloc(sizeof(building_t) * N_BUILDINGS);
  J.Q = (pole_t*)malloc(sizeof(pole_t) * N_POLES);
  if (!J.B || !J.Q) { free(J.B); free(J.Q); return -2; }
  make_scene(seed, J.B, J.Q);
  J.xyz = xyz; J.rgba = rgba; J.idx = idx;
  range_job jobs[256];
  pthread_t th[256];
  int t = pick_threads(nthreads);
  if ((uint64_t)t > count) t = count ? (int)count : 1;
  for (int k = 0; k < t; ++k) {
    jobs[k].fn = terrain_gather; jobs[k].arg = &J;
    jobs[k].lo = count * (uint64_t)k / (uint64_t)t;
    jobs[k].hi = count * (uint64_t)(k + 1) / (uint64_t)t;
  }
  for (int k = 1; k < t; ++k) pthread_create(&th[k], NULL, range_thread, &jobs[k]);
  range_thread(&jobs[0]);
  for (int k = 1; k < t; ++k) pthread_join(th[k], NULL);
  free(J.B); free(J.Q);
  return 0;
}

/* order: 0 = index order (ground, then buildings, then poles);
 *        1 = stable serpentine 10 m tile order.
 * Returns 0, or -1 on bad arguments, -2 if temporary memory is unavailable. */
int synth_terrain(uint64_t seed, uint64_t n, double sigma, int order, float* xyz, uint32_t* rgba,
                  int nthreads) {
  if (!xyz || !rgba) return -1;
  terrain_job J;
  memset(&J, 0, sizeof J);
  J.seed = seed; J.n = n; J.sigma = sigma;
  J.n_ground = (uint64_t)((double)n * 0.80);
  J.n_build = (uint64_t)((double)n * 0.96);
  J.B = (building_t*)malloc(sizeof(building_t) * N_BUILDINGS);
  J.Q = (pole_t*)malloc(sizeof(pole_t) * N_POLES);
  if (!J.B || !J.Q) { free(J.B); free(J.Q); return -2; }
  make_scene(seed, J.B, J.Q);
  int rc = 0;
  if (order == 0) {
    J.xyz = xyz; J.rgba = rgba;
    parallel_for(n, nthreads, terrain_range, &J);
  } else {
    float* tx = (float*)malloc(sizeof(float) * 3 * (n ? n : 1));
    uint32_t* tc = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint16_t* tt = (uint16_t*)malloc(sizeof(uint16_t) * (n ? n : 1));
    int nch = pick_threads(nthreads) * 4;
    uint64_t* hist = (uint64_t*)malloc(sizeof(uint64_t) * N_TILES * (size_t)nch);
    if (!tx || !tc || !tt || !hist) {
      rc = -2;
    } else {
      J.xyz = tx; J.rgba = tc; J.tile = tt;
      parallel_for(n, nthreads, terrain_range, &J);
      bucket_job K;
      K.n = n; K.nchunks = nch; K.tile = tt; K.hist = hist;
      K.sx = tx; K.sc = tc; K.dx = xyz; K.dc = rgba;
      parallel_for((uint64_t)nch, nthreads, bucket_hist, &K);
      /* exclusive prefix in (tile, chunk) order: stable across chunks */
      uint64_t run = 0;
      for (int t = 0; t < N_TILES; ++t)
        for (int c = 0; c < nch; ++c) {
          uint64_t v = hist[(size_t)c * N_TILES + t];
          hist[(size_t)c * N_TILES + t] = run;
          run += v;
        }
      parallel_for((uint64_t)nch, nthreads, bucket_scatter, &K);
    }
    free(tx); free(tc); free(tt); free(hist);
  }
  free(J.B); free(J.Q);
  return rc;
}

/* ------------------------------------------------- layered point cloud */
/* Layered-point-cloud (LPC) layout: the Potree-style input of the LOD
 * renderer, produced here the way a converter would produce it (the paper
 * loads such files; the converter is not part of its method).
 *
 *   cube:    the cloud's box min corner and its largest extent (binary64);
 *   level:   L in 0..depth per point, drawn from SplitMix64(seed, i) with
 *            P(L) proportional to 4^L (each level roughly quadruples the
 *            points, like octree levels of a surface);
 *   node:    (L, octree cell of depth L), the cell from 20-bit-per-axis grid
 *            coordinates q = min(floor(2^20 (x - min) / size), 2^20 - 1);
 *   order:   by (L, Morton code of q), stable;
 *   batches: each node's points in chunks of at most cap, every chunk
 *            starting at a multiple of 4 (the slots in between are padding,
 *            zero, in no batch).
 * Outputs: xyz_out / rgba_out (npad points), spans[2b] = first,
 * spans[2b + 1] = count, nodes[5b ..] = cube origin x, y, z, edge, level.
 * Returns 0; -1 bad arguments; -2 no memory; -3 output capacity too small
 * (*npad_out, *nb_out then hold what is needed). */
static inline uint64_t spread3_20(uint64_t v) { /* bit b -> bit 3b, 20 bits */
  v &= 0xFFFFFull;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
static inline uint64_t compact3_20(uint64_t c) {
  uint64_t r = 0;
  for (int b = 0; b < 20; ++b) r |= ((c >> (3 * b)) & 1ull) << b;
  return r;
}

typedef struct {
  const float* xyz;
  uint64_t seed;
  int depth;
  double cdf[16], mn[3], size;
  uint64_t* key;
  uint32_t* idx;
} lpc_keys_job;

static void lpc_keys(void* arg, uint64_t lo, uint64_t hi) {
  lpc_keys_job* J = (lpc_keys_job*)arg;
  for (uint64_t i = lo; i < hi; ++i) {
    double u = u01(sm_at(J->seed ^ 0x4C50434C50434C50ull, i));
    int L = 0;
    while (L < J->depth && u >= J->cdf[L]) ++L;
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
      double f = floor((((double)J->xyz[3 * i + a] - J->mn[a]) * 1048576.0) / J->size);
      q[a] = f >= 1048575.0 ? 1048575u : (f <= 0.0 ? 0u : (uint64_t)f);
    }
    J->key[i] = ((uint64_t)L << 60) | spread3_20(q[0]) | (spread3_20(q[1]) << 1) | (spread3_20(q[2]) << 2);
    J->idx[i] = (uint32_t)i;
  }
}

/* Stable LSD radix sort of (key, idx) pairs, 8-bit digits, chunk-parallel:
 * per-chunk digit counts, offsets in (digit, chunk) order, scatter in chunk
 * order (each chunk keeps its input order). */
typedef struct {
  uint64_t *kin, *kout;
  uint32_t *iin, *iout;
  uint64_t n;
  int sh, nt;
  uint64_t* off; /* nt x 256 */
} radix_job;

static void radix_count(void* arg, uint64_t c0, uint64_t c1) {
  radix_job* R = (radix_job*)arg;
  for (uint64_t c = c0; c < c1; ++c) {
    uint64_t* h = R->off + 256 * c;
    memset(h, 0, 256 * sizeof(uint64_t));
    uint64_t lo = R->n * c / (uint64_t)R->nt, hi = R->n * (c + 1) / (uint64_t)R->nt;
    for (uint64_t i = lo; i < hi; ++i) h[(R->kin[i] >> R->sh) & 255u]++;
  }
}
static void radix_scatter(void* arg, uint64_t c0, uint64_t c1) {
  radix_job* R = (radix_job*)arg;
  for (uint64_t c = c0; c < c1; ++c) {
    uint64_t* h = R->off + 256 * c;
    uint64_t lo = R->n * c / (uint64_t)R->nt, hi = R->n * (c + 1) / (uint64_t)R->nt;
    for (uint64_t i = lo; i < hi; ++i) {
      uint64_t d = h[(R->kin[i] >> R->sh) & 255u]++;
      R->kout[d] = R->kin[i];
      R->iout[d] = R->iin[i];
    }
  }
}

typedef struct {
  const float* xyz;
  const uint32_t* rgba;
  const uint32_t* idx;     /* sorted order */
  const uint64_t* src;     /* per batch: first sorted position */
  const uint32_t* spans;
  float* xyz_out;
  uint32_t* rgba_out;
  int spread;
} lpc_gather_job;

/* Spread order of a batch of c points: slot t holds the batch's point of
 * sorted rank (t * m) mod c, m the first integer >= floor(c / 4) + 1 that is
 * coprime with c (a bijection of 0..c-1). */
static uint64_t lpc_spread_step(uint64_t c) {
  for (uint64_t m = c / 4 + 1;; ++m) {
    uint64_t a = m, b = c;
    while (b) {
      uint64_t r = a % b;
      a = b;
      b = r;
    }
    if (a == 1) return m;
  }
}

static void lpc_gather(void* arg, uint64_t b0, uint64_t b1) {
  lpc_gather_job* G = (lpc_gather_job*)arg;
  for (uint64_t b = b0; b < b1; ++b) {
    uint64_t pos = G->spans[2 * b], cnt = G->spans[2 * b + 1];
    const uint64_t m = G->spread ? lpc_spread_step(cnt) : 1;
    for (uint64_t t = 0; t < cnt; ++t) {
      uint64_t s = G->idx[G->src[b] + (t * m) % cnt], d = pos + t;
      G->xyz_out[3 * d] = G->xyz[3 * s];
      G->xyz_out[3 * d + 1] = G->xyz[3 * s + 1];
      G->xyz_out[3 * d + 2] = G->xyz[3 * s + 2];
      G->rgba_out[d] = G->rgba[s];
    }
  }
}

int synth_lpc_layout(uint64_t seed, const float* xyz, const uint32_t* rgba, uint64_t n, int depth, uint32_t cap,
                     int spread, float* xyz_out, uint32_t* rgba_out, uint64_t cap_points, uint32_t* spans,
                     double* nodes, uint64_t cap_batches, uint64_t* npad_out, uint64_t* nb_out) {
  if (!xyz || !rgba || !npad_out || !nb_out || depth < 0 || depth > 15 || cap < 4 || n >= (1ull << 32)) return -1;
  lpc_keys_job J;
  memset(&J, 0, sizeof J);
  J.xyz = xyz;
  J.seed = seed;
  J.depth = depth;
  double mx[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) {
    J.mn[a] = n ? (double)xyz[a] : 0.0;
    mx[a] = J.mn[a];
  }
  for (uint64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      double v = (double)xyz[3 * i + a];
      if (v < J.mn[a]) J.mn[a] = v;
      if (v > mx[a]) mx[a] = v;
    }
  J.size = 0.0;
  for (int a = 0; a < 3; ++a)
    if (mx[a] - J.mn[a] > J.size) J.size = mx[a] - J.mn[a];
  if (J.size == 0.0) J.size = 1.0;
  /* level CDF: P(L <= l) = (4^(l+1) - 1) / (4^(depth+1) - 1) */
  double tot = 0.0, acc = 0.0;
  for (int l = 0; l <= depth; ++l) tot += ldexp(1.0, 2 * l);
  for (int l = 0; l <= depth; ++l) {
    acc += ldexp(1.0, 2 * l);
    J.cdf[l] = acc / tot;
  }
  int nt = pick_threads(0);
  uint64_t m = n ? n : 1;
  uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * m);
  uint64_t* key2 = (uint64_t*)malloc(sizeof(uint64_t) * m);
  uint32_t* idx = (uint32_t*)malloc(sizeof(uint32_t) * m);
  uint32_t* idx2 = (uint32_t*)malloc(sizeof(uint32_t) * m);
  uint64_t* off = (uint64_t*)malloc(sizeof(uint64_t) * 256 * (uint64_t)nt);
  if (!key || !key2 || !idx || !idx2 || !off) {
    free(key); free(key2); free(idx); free(idx2); free(off);
    return -2;
  }
  J.key = key;
  J.idx = idx;
  parallel_for(n, nt, lpc_keys, &J);
  radix_job R;
  R.n = n;
  R.nt = nt;
  R.off = off;
  for (int pass = 0; pass < 8; ++pass) {
    R.kin = key; R.iin = idx; R.kout = key2; R.iout = idx2; R.sh = 8 * pass;
    parallel_for((uint64_t)nt, nt, radix_count, &R);
    uint64_t s = 0;
    for (int d = 0; d < 256; ++d)
      for (int c = 0; c < nt; ++c) {
        uint64_t v = off[256 * c + d];
        off[256 * c + d] = s;
        s += v;
      }
    parallel_for((uint64_t)nt, nt, radix_scatter, &R);
    uint64_t* tk = key; key = key2; key2 = tk;
    uint32_t* ti = idx; idx = idx2; idx2 = ti;
  }
  free(off);
  free(key2);
  free(idx2);
  /* nodes and batches (a serial walk over the sorted keys) */
  uint64_t* src = (uint64_t*)malloc(sizeof(uint64_t) * (cap_batches ? cap_batches : 1));
  if (!src) {
    free(key); free(idx);
    return -2;
  }
  uint64_t pos = 0, nb = 0;
  int fits = 1;
  uint64_t i = 0;
  while (i < n) {
    int L = (int)(key[i] >> 60);
    uint64_t cell = (key[i] & ((1ull << 60) - 1)) >> (3 * (20 - L));
    uint64_t j = i;
    while (j < n && (int)(key[j] >> 60) == L && ((key[j] & ((1ull << 60) - 1)) >> (3 * (20 - L))) == cell) ++j;
    double edge = ldexp(J.size, -L);
    for (uint64_t c0 = i; c0 < j; c0 += cap) {
      uint64_t c1 = c0 + cap < j ? c0 + cap : j;
      pos = (pos + 3) & ~3ull;
      if (nb < cap_batches && pos + (c1 - c0) <= cap_points && xyz_out && rgba_out && spans && nodes) {
        spans[2 * nb] = (uint32_t)pos;
        spans[2 * nb + 1] = (uint32_t)(c1 - c0);
        src[nb] = c0;
        for (int a = 0; a < 3; ++a) {
          uint64_t k = compact3_20(cell << (3 * (20 - L)) >> a) >> (20 - L);
          nodes[5 * nb + a] = J.mn[a] + (double)k * edge;
        }
        nodes[5 * nb + 3] = edge;
        nodes[5 * nb + 4] = (double)L;
      } else {
        fits = 0;
      }
      pos += c1 - c0;
      ++nb;
    }
    i = j;
  }
  if (fits) {
    lpc_gather_job G = {xyz, rgba, idx, src, spans, xyz_out, rgba_out, spread};
    parallel_for(nb, nt, lpc_gather, &G);
  }
  free(src);
  free(key);
  free(idx);
  *npad_out = pos;
  *nb_out = nb;
  return fits ? 0 : -3;
}

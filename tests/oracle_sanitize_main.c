/* Drives every entry point of the CPU oracle on small random inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure; the oracle's source is compiled into this program).  Exits
 * 0 when every call returned; the sanitizers abort on the first error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/ptoracle.c"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void) { /* SplitMix64 */
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double uniform(double a, double b) { return a + (b - a) * (double)(next_u64() >> 11) * 0x1p-53; }

/* Row-major look-at view and OpenGL perspective projection. */
static void camera(const double eye[3], const double at[3], double fovy_deg, uint32_t w, uint32_t h, float view[16],
                   float proj[16]) {
  double f[3] = {at[0] - eye[0], at[1] - eye[1], at[2] - eye[2]};
  double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (int i = 0; i < 3; ++i) f[i] /= fl;
  const double up[3] = {0.0, 0.0, 1.0};
  double s[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
  double sl = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  if (sl < 1e-9) {
    s[0] = 1.0;
    s[1] = s[2] = 0.0;
    sl = 1.0;
  }
  for (int i = 0; i < 3; ++i) s[i] /= sl;
  const double u[3] = {s[1] * f[2] - s[2] * f[1], s[2] * f[0] - s[0] * f[2], s[0] * f[1] - s[1] * f[0]};
  const double m[16] = {s[0], s[1], s[2], -(s[0] * eye[0] + s[1] * eye[1] + s[2] * eye[2]),
                        u[0], u[1], u[2], -(u[0] * eye[0] + u[1] * eye[1] + u[2] * eye[2]),
                        -f[0], -f[1], -f[2], f[0] * eye[0] + f[1] * eye[1] + f[2] * eye[2],
                        0.0, 0.0, 0.0, 1.0};
  const double t = 1.0 / tan(fovy_deg * 0.5 * 3.14159265358979323846 / 180.0), a = (double)w / (double)h;
  const double n = 0.05, fr = 1000.0;
  const double p[16] = {t / a, 0, 0, 0, 0, t, 0, 0, 0, 0, (fr + n) / (n - fr), 2 * fr * n / (n - fr), 0, 0, -1, 0};
  for (int i = 0; i < 16; ++i) {
    view[i] = (float)m[i];
    proj[i] = (float)p[i];
  }
}

int main(void) {
  const uint64_t n = 3000;
  const uint32_t S = 64, w = 37, h = 29;
  float* xyz = malloc(sizeof(float) * 3 * n);
  uint32_t* rgba = malloc(sizeof(uint32_t) * n);
  for (uint64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) xyz[3 * i + a] = (float)uniform(0.0, 10.0);
    rgba[i] = (uint32_t)next_u64();
  }
  xyz[0] = xyz[1] = xyz[2] = 0.0f; /* duplicates and box corners */
  memcpy(xyz + 3, xyz, 3 * sizeof(float));
  const uint64_t nb = or_batch_count(n, S);
  float* xo = malloc(sizeof(float) * 3 * n);
  uint32_t *col = malloc(4 * n), *perm = malloc(4 * n), *low = malloc(4 * n), *med = malloc(4 * n),
           *high = malloc(4 * n);
  or_batch* bat = malloc(sizeof(or_batch) * nb);
  uint64_t* vb = malloc(8ull * w * h);
  uint64_t* acc = malloc(16ull * w * h);
  uint32_t* fb = malloc(4ull * w * h);
  or_decision* dec = malloc(sizeof(or_decision) * nb);
  const double eyes[4][3] = {{5, -20, 15}, {5, 5, 5}, {30, 30, 2}, {5, 5, 40}};
  for (int morton = 0; morton < 3; ++morton) {  // input order, Morton order, Morton + spread order
    if (or_build(xyz, rgba, n, S, morton, xo, col, perm, bat, low, med, high) != 0) return 2;
    for (int c = 0; c < 4; ++c) {
      float view[16], proj[16];
      const double at[3] = {5, 5, 5.5};
      camera(eyes[c], at, 60.0 + 20.0 * c, w, h, view, proj);
      const or_opts modes[4] = {{0, 1, 500.0f, 512000.0f, 0.0f}, {30, 0, 500.0f, 512000.0f, 0.0f},
                                {10, 1, 500.0f, 512000.0f, 0.0f}, {0, 1, 1.0f, 2.0f, 0.0f}};
      for (int m = 0; m < 4; ++m) {
        or_stats st;
        for (uint64_t p = 0; p < (uint64_t)w * h; ++p) vb[p] = OR_EMPTY;
        or_render(bat, NULL, nb, NULL, 0, low, med, high, view, proj, w, h, &modes[m], vb, &st);
        or_decide_all(bat, NULL, nb, view, proj, w, h, &modes[m], dec);
        or_resolve(vb, (uint64_t)w * h, col, n, 0xFF000000u, fb);
        memset(acc, 0, 16ull * w * h);
        or_accumulate(bat, NULL, nb, NULL, 0, low, med, high, col, view, proj, w, h, &modes[m], 1.01f, vb, acc);
        or_resolve_hqs(acc, (uint64_t)w * h, 0xFF000000u, fb);
      }
    }
  }
  /* variable-size batches with padding and LOD nodes */
  const uint64_t nbs = n / 64;
  uint32_t* spans = malloc(8 * nbs);
  double* nodes = malloc(sizeof(double) * 5 * nbs);
  for (uint64_t b = 0; b < nbs; ++b) {
    spans[2 * b] = (uint32_t)(64 * b);
    spans[2 * b + 1] = (uint32_t)(1 + next_u64() % 60);
    nodes[5 * b + 0] = nodes[5 * b + 1] = nodes[5 * b + 2] = 0.0;
    nodes[5 * b + 3] = 10.0 / (double)(1u << (b % 4));
    nodes[5 * b + 4] = (double)(b % 4);
  }
  or_batch* sb = malloc(sizeof(or_batch) * nbs);
  or_make_batches_spans(xyz, spans, nbs, sb);
  memset(low, 0, 4 * n);
  memset(med, 0, 4 * n);
  memset(high, 0, 4 * n);
  or_quantize(xyz, sb, nbs, low, med, high);
  for (int c = 0; c < 4; ++c) {
    float view[16], proj[16];
    const double at[3] = {5, 5, 5};
    camera(eyes[c], at, 70.0, w, h, view, proj);
    const or_opts o = {0, 1, 500.0f, 512000.0f, 8.0f};
    or_stats st;
    for (uint64_t p = 0; p < (uint64_t)w * h; ++p) vb[p] = OR_EMPTY;
    or_render(sb, nodes, nbs, NULL, 0, low, med, high, view, proj, w, h, &o, vb, &st);
    or_decide_all(sb, nodes, nbs, view, proj, w, h, &o, dec);
  }
  uint64_t* codes = malloc(8 * n);
  float mn[3], mx[3];
  or_cloud_aabb(xyz, n, mn, mx);
  or_morton_codes(xyz, n, mn, mx, codes);
  if (or_morton_order(codes, n, perm) != 0) return 3;
  xyz[7] = NAN;
  if (or_validate(xyz, n) != 2) return 4; /* the first non-finite point */
  free(codes); free(sb); free(nodes); free(spans); free(dec); free(fb); free(acc); free(vb); free(bat);
  free(high); free(med); free(low); free(perm); free(col); free(xo); free(rgba); free(xyz);
  printf("oracle sanitizer run ok\n");
  return 0;
}

// Load-time build kernels for gfx950 (Sec. 3.1 data structure, Sec. 3.3 Eq. 1).
//
//  finite check (with the Morton order: on the cloud box's loads) -> [cloud
//  box -> 63-bit Morton codes -> stable LSD radix sort
//  (8 passes of 8 bits) -> gather] -> per-batch boxes -> Eq. 1 quantise and
//  split into low / med / high words.
//
// Boxes order binary32 values by IEEE totalOrder (-0 below +0) through the
// monotone integer map okey(), so a box depends only on the point set, not on
// the order of a parallel reduction.
#include "internal.h"

namespace ptr {
namespace {

__device__ __forceinline__ uint32_t okey(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float okey_inv(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// ---------------------------------------------------------- finite check
__global__ void __launch_bounds__(256) k_finite(const uint32_t* __restrict__ w, uint64_t nwords,
                                                uint32_t* __restrict__ flag) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride)
    bad |= (w[i] & 0x7F800000u) == 0x7F800000u;
  if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

__global__ void __launch_bounds__(256) k_iota(uint32_t* __restrict__ p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = (uint32_t)i;
}

// ------------------------------------------------------------- cloud box
__global__ void k_aabb_init(uint32_t* aabb) {
  if (threadIdx.x < 6) aabb[threadIdx.x] = threadIdx.x < 3 ? 0xFFFFFFFFu : 0u;
}

// The cloud box, and the finite check on the same loads (flag: set if a
// coordinate is NaN or Inf).
__global__ void __launch_bounds__(256) k_aabb(const float* __restrict__ xyz, uint64_t n, uint32_t* __restrict__ aabb,
                                              uint32_t* __restrict__ flag) {
  uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0, 0, 0};
  bool bad = false;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float f = xyz[3 * i + a];
      bad |= (__float_as_uint(f) & 0x7F800000u) == 0x7F800000u;
      const uint32_t k = okey(f);
      mn[a] = min(mn[a], k);
      mx[a] = max(mx[a], k);
    }
  }
  if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    for (int o = 32; o > 0; o >>= 1) {
      mn[a] = min(mn[a], (uint32_t)__shfl_xor((int)mn[a], o));
      mx[a] = max(mx[a], (uint32_t)__shfl_xor((int)mx[a], o));
    }
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      atomicMin(&aabb[a], mn[a]);
      atomicMax(&aabb[3 + a], mx[a]);
    }
  }
}

// ---------------------------------------------------------- Morton codes
__device__ __forceinline__ uint64_t spread3(uint64_t x) {  // bit b -> bit 3b (21 bits)
  x &= 0x1FFFFFull;
  x = (x | (x << 32)) & 0x1F00000000FFFFull;
  x = (x | (x << 16)) & 0x1F0000FF0000FFull;
  x = (x | (x << 8)) & 0x100F00F00F00F00Full;
  x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// q = min(floor(2^21 (x - cmin) / (cmax - cmin)), 2^21 - 1) in binary64; 0 for an empty extent.
__device__ __forceinline__ uint32_t morton_q(float x, float cmin, float cmax) {
  const double d = (double)x - (double)cmin;
  const double s = (double)cmax - (double)cmin;
  if (s == 0.0) return 0u;
  const double f = floor((d * 2097152.0) / s);
  return f > 2097151.0 ? 2097151u : (uint32_t)f;
}

__global__ void __launch_bounds__(256) k_morton(const float* __restrict__ xyz, uint64_t n,
                                                const uint32_t* __restrict__ aabb, uint64_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals) {
  const float cmin[3] = {okey_inv(aabb[0]), okey_inv(aabb[1]), okey_inv(aabb[2])};
  const float cmax[3] = {okey_inv(aabb[3]), okey_inv(aabb[4]), okey_inv(aabb[5])};
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t qx = morton_q(xyz[3 * i], cmin[0], cmax[0]);
    const uint64_t qy = morton_q(xyz[3 * i + 1], cmin[1], cmax[1]);
    const uint64_t qz = morton_q(xyz[3 * i + 2], cmin[2], cmax[2]);
    keys[i] = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
    vals[i] = (uint32_t)i;
  }
}

// ------------------------------------------------------------ radix sort
// Stable LSD radix sort of (u64 key, u32 value) pairs, 8 bits per pass.
// Each block owns a tile of RS_TILE consecutive elements.  count: per-block
// digit histogram, stored digit-major (hist[d * nblk + blk]); an exclusive
// scan of that array gives every (digit, block) its output offset; scatter:
// the tile is ranked chunk by chunk in input order (wave ballots give the
// rank among equal digits inside a wave, LDS counters carry it across waves
// and chunks), which keeps equal keys in input order.
constexpr int RS_THREADS = 256;
constexpr int RS_CHUNKS = 16;
constexpr uint64_t RS_TILE = (uint64_t)RS_THREADS * RS_CHUNKS;
constexpr uint64_t SCAN_CHUNK = 4096;

__global__ void __launch_bounds__(256) k_radix_count(const uint64_t* __restrict__ keys, uint64_t n, int shift,
                                                     uint32_t* __restrict__ hist, uint64_t nblk) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
  for (int it = 0; it < RS_CHUNKS; ++it) {
    const uint64_t i = base + (uint64_t)it * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of m u32 values: partial sums, top-level scan, apply
__global__ void __launch_bounds__(256) k_scan_partials(const uint32_t* __restrict__ x, uint64_t m,
                                                       uint32_t* __restrict__ part) {
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_CHUNK;
  uint32_t s = 0;
  for (uint64_t i = base + threadIdx.x; i < base + SCAN_CHUNK && i < m; i += 256) s += x[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  __shared__ uint32_t ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Block-wide exclusive scan of one value per thread (256 threads); returns the
// exclusive prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t ws[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) ws[wave] = inc;
  __syncthreads();
  uint32_t wbase = 0;
  for (int w = 0; w < wave; ++w) wbase += ws[w];
  const uint32_t tot = ws[0] + ws[1] + ws[2] + ws[3];
  __syncthreads();
  *total = tot;
  return wbase + inc - v;
}

__global__ void __launch_bounds__(256) k_scan_top(uint32_t* __restrict__ part, uint64_t np) {
  uint32_t carry = 0;
  for (uint64_t base = 0; base < np; base += 256) {
    const uint64_t i = base + threadIdx.x;
    const uint32_t v = i < np ? part[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, &tot);
    if (i < np) part[i] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(256) k_scan_apply(uint32_t* __restrict__ x, uint64_t m,
                                                    const uint32_t* __restrict__ part) {
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_CHUNK;
  uint32_t carry = part[blockIdx.x];
  for (uint64_t off = 0; off < SCAN_CHUNK; off += 256) {
    const uint64_t i = base + off + threadIdx.x;
    const uint32_t v = i < m ? x[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, &tot);
    if (i < m) x[i] = carry + ex;
    carry += tot;
  }
}

// Scatter of one pass: the tile is first ranked stably into LDS, ordered by
// digit (equal digits in input order: wave ballots give the rank inside a
// wave, LDS counters carry it across waves and chunks), then written out from
// LDS so that consecutive threads write consecutive slots of one digit's
// range: the tile's elements of a digit (about RS_TILE / 256) leave as one run
// instead of one scattered 8-byte store each.
__global__ void __launch_bounds__(256) k_radix_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                       uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                       uint64_t n, int shift, const uint32_t* __restrict__ offs,
                                                       uint64_t nblk) {
  __shared__ uint64_t skey[RS_TILE];
  __shared__ uint32_t sval[RS_TILE];
  __shared__ uint32_t goff[256];    // first output slot of this tile's digit d
  __shared__ uint32_t tstart[256];  // first LDS slot of digit d in the tile
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[4][256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint64_t m = 256 * nblk;
  const uint64_t at = (uint64_t)tid * nblk + blockIdx.x;  // (digit tid, this block) in the digit-major scan
  const uint32_t g0 = offs[at];
  const uint32_t g1 = at + 1 < m ? offs[at + 1] : (uint32_t)n;  // next (digit, block) starts where this ends
  goff[tid] = g0;
  uint32_t total;
  tstart[tid] = block_exclusive_scan(g1 - g0, &total);
  run[tid] = 0;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
  // the whole tile's loads are issued before the ranking starts, so that the
  // chunks' barriers do not each wait for a memory round trip
  uint64_t keys[RS_CHUNKS];
  uint32_t vals[RS_CHUNKS];
#pragma unroll
  for (int it = 0; it < RS_CHUNKS; ++it) {
    const uint64_t i = base + (uint64_t)it * RS_THREADS + tid;
    keys[it] = i < n ? kin[i] : 0ull;
    vals[it] = i < n ? vin[i] : 0u;
  }
#pragma unroll
  for (int it = 0; it < RS_CHUNKS; ++it) {
    wcnt[0][tid] = 0;
    wcnt[1][tid] = 0;
    wcnt[2][tid] = 0;
    wcnt[3][tid] = 0;
    __syncthreads();
    const uint64_t i = base + (uint64_t)it * RS_THREADS + tid;
    const bool valid = i < n;
    const uint64_t key = keys[it];
    const uint32_t val = vals[it];
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool set = (d >> bit) & 1u;
      const uint64_t mk = __ballot(set);
      peers &= set ? mk : ~mk;
    }
    const uint32_t rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = tstart[d] + run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      if (pos < RS_TILE) {  // always true for a consistent histogram; never write outside
        skey[pos] = key;
        sval[pos] = val;
      }
    }
    __syncthreads();
    run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
  }
  __syncthreads();
  const uint32_t nt = total < (uint32_t)RS_TILE ? total : (uint32_t)RS_TILE;
  for (uint32_t p = tid; p < nt; p += RS_THREADS) {
    const uint64_t key = skey[p];
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    const uint64_t pos = (uint64_t)goff[d] + (p - tstart[d]);
    if (pos < n) {  // always true for a consistent histogram; never write outside
      kout[pos] = key;
      vout[pos] = sval[p];
    }
  }
}

// ----------------------------------------------------------------- gather
// Positions and colours of the input as one 16-byte record per point, in
// input order: the gather then reads one record (one cache line) per output
// instead of a position and a colour from two arrays.
__global__ void __launch_bounds__(256) k_interleave(const float* __restrict__ xyz, const uint32_t* __restrict__ rgba,
                                                    uint64_t n, uint4* __restrict__ rec) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    rec[i] = make_uint4(__float_as_uint(xyz[3 * i]), __float_as_uint(xyz[3 * i + 1]), __float_as_uint(xyz[3 * i + 2]),
                        rgba[i]);
}

// The batches of a spread build: each batch of c points is stored in the
// order position r <- Morton rank (r * m) mod c (m: step for a full batch,
// m_last for the last batch when it is shorter).
struct Spread {
  uint64_t S, m, c_last, m_last;
};
__device__ __forceinline__ uint64_t spread_source(uint64_t i, const Spread& sp, uint64_t n) {
  const uint64_t b0 = i - i % sp.S;
  const bool full = b0 + sp.S <= n;
  const uint64_t c = full ? sp.S : sp.c_last, m = full ? sp.m : sp.m_last;
  return b0 + ((i - b0) * m) % c;
}

// Four consecutive outputs per thread: one 16-byte load of their sources, the
// four record reads in flight together, 48 + 16 contiguous bytes written.
// The outputs past the last multiple of four go one per thread.  SPREAD: the
// sources come from the Morton positions of the spread order (perm_in), and
// perm_out receives them.
template <bool SPREAD>
__global__ void __launch_bounds__(256) k_gather(const uint4* __restrict__ rec, const uint32_t* __restrict__ perm,
                                                uint32_t* __restrict__ perm_out, Spread sp, uint64_t n,
                                                float* __restrict__ xyz_out, uint32_t* __restrict__ colors) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t n4 = n / 4;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n4; g += stride) {
    uint64_t s[4];
    if constexpr (SPREAD) {
      uint32_t q[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint64_t src = spread_source(4 * g + j, sp, n);
        q[j] = perm[src < n ? src : 4 * g + j];
        s[j] = q[j];
      }
      reinterpret_cast<uint4*>(perm_out)[g] = make_uint4(q[0], q[1], q[2], q[3]);
    } else {
      const uint4 p = reinterpret_cast<const uint4*>(perm)[g];
      s[0] = p.x;
      s[1] = p.y;
      s[2] = p.z;
      s[3] = p.w;
    }
    uint4 r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (s[j] >= n) s[j] = 4 * g + j;  // a permutation never triggers this; it keeps reads in bounds
      r[j] = rec[s[j]];
    }
    float4* const xo = reinterpret_cast<float4*>(xyz_out + 12 * g);
    xo[0] = make_float4(__uint_as_float(r[0].x), __uint_as_float(r[0].y), __uint_as_float(r[0].z), __uint_as_float(r[1].x));
    xo[1] = make_float4(__uint_as_float(r[1].y), __uint_as_float(r[1].z), __uint_as_float(r[2].x), __uint_as_float(r[2].y));
    xo[2] = make_float4(__uint_as_float(r[2].z), __uint_as_float(r[3].x), __uint_as_float(r[3].y), __uint_as_float(r[3].z));
    reinterpret_cast<uint4*>(colors)[g] = make_uint4(r[0].w, r[1].w, r[2].w, r[3].w);
  }
  for (uint64_t i = 4 * n4 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t s;
    if constexpr (SPREAD) {
      const uint64_t src = spread_source(i, sp, n);
      s = perm[src < n ? src : i];
      perm_out[i] = (uint32_t)s;
    } else {
      s = perm[i];
    }
    if (s >= n) s = i;
    const uint4 r = rec[s];
    xyz_out[3 * i] = __uint_as_float(r.x);
    xyz_out[3 * i + 1] = __uint_as_float(r.y);
    xyz_out[3 * i + 2] = __uint_as_float(r.z);
    colors[i] = r.w;
  }
}

// ------------------------------------------------------------ batch boxes
// One block per batch: batch b is [b S, min((b + 1) S, n)), or, with spans,
// [out[b].first, out[b].first + out[b].count) as set by the host.
__global__ void __launch_bounds__(256) k_batch_bbox(const float* __restrict__ xyz, uint64_t n, uint32_t S,
                                                    BatchRec* __restrict__ out, int spans) {
  const uint64_t first = spans ? out[blockIdx.x].first : (uint64_t)blockIdx.x * S;
  const uint64_t end = spans ? first + out[blockIdx.x].count : (first + S < n ? first + S : n);
  uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0, 0, 0};
  for (uint64_t i = first + threadIdx.x; i < end; i += 256) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const uint32_t k = okey(xyz[3 * i + a]);
      mn[a] = min(mn[a], k);
      mx[a] = max(mx[a], k);
    }
  }
  __shared__ uint32_t red[4][6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    for (int o = 32; o > 0; o >>= 1) {
      mn[a] = min(mn[a], (uint32_t)__shfl_xor((int)mn[a], o));
      mx[a] = max(mx[a], (uint32_t)__shfl_xor((int)mx[a], o));
    }
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    for (int a = 0; a < 3; ++a) {
      red[wave][a] = mn[a];
      red[wave][3 + a] = mx[a];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    BatchRec r;
    r.first = (uint32_t)first;
    r.count = (uint32_t)(end - first);
    for (int a = 0; a < 3; ++a) {
      uint32_t lo = red[0][a], hi = red[0][3 + a];
      for (int w = 1; w < 4; ++w) {
        lo = min(lo, red[w][a]);
        hi = max(hi, red[w][3 + a]);
      }
      r.mn[a] = okey_inv(lo);
      r.mx[a] = okey_inv(hi);
    }
    out[blockIdx.x] = r;
  }
}

// --------------------------------------------------------------- quantise
// Eq. 1: X30 = min(floor(2^30 (x - min) / size), 2^30 - 1) in binary64 with
// one correctly rounded division (0 for size 0); low = bits 29..20, med =
// bits 19..10, high = bits 9..0, each packed x | y << 10 | z << 20.
__device__ __forceinline__ uint32_t eq1(float x, float bmin, float bmax) {
  const double d = (double)x - (double)bmin;
  const double s = (double)bmax - (double)bmin;
  if (s == 0.0) return 0u;
  const double f = floor((d * 1073741824.0) / s);
  return f > 1073741823.0 ? 1073741823u : (uint32_t)f;
}

__global__ void __launch_bounds__(256) k_quantize(const float* __restrict__ xyz, uint64_t n, uint32_t S,
                                                  const BatchRec* __restrict__ batches, uint32_t* __restrict__ low,
                                                  uint32_t* __restrict__ med, uint32_t* __restrict__ high) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const BatchRec& B = batches[(uint32_t)i / S];  // i < 2^32
    uint32_t lw = 0, mw = 0, hw = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const uint32_t X30 = eq1(xyz[3 * i + a], B.mn[a], B.mx[a]);
      lw |= ((X30 >> 20) & 1023u) << (10 * a);
      mw |= ((X30 >> 10) & 1023u) << (10 * a);
      hw |= (X30 & 1023u) << (10 * a);
    }
    low[i] = lw;
    med[i] = mw;
    high[i] = hw;
  }
}

// Variable-size batches: one block per batch, Eq. 1 relative to its box.
__global__ void __launch_bounds__(256) k_quantize_spans(const float* __restrict__ xyz,
                                                        const BatchRec* __restrict__ batches,
                                                        uint32_t* __restrict__ low, uint32_t* __restrict__ med,
                                                        uint32_t* __restrict__ high) {
  const BatchRec B = batches[blockIdx.x];
  for (uint64_t i = (uint64_t)B.first + threadIdx.x; i < (uint64_t)B.first + B.count; i += 256) {
    uint32_t lw = 0, mw = 0, hw = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const uint32_t X30 = eq1(xyz[3 * i + a], B.mn[a], B.mx[a]);
      lw |= ((X30 >> 20) & 1023u) << (10 * a);
      mw |= ((X30 >> 10) & 1023u) << (10 * a);
      hw |= (X30 & 1023u) << (10 * a);
    }
    low[i] = lw;
    med[i] = mw;
    high[i] = hw;
  }
}

inline uint32_t grid_for(uint64_t work, uint32_t per_block = 256, uint32_t cap = 65536) {
  uint64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (uint32_t)b;
}

inline uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

}  // namespace

uint64_t small_scratch_bytes() { return 4096; }

uint64_t sort_scratch_layout(uint64_t n, uint8_t* base, SortScratch* out) {
  SortScratch s{};
  s.nblk = (n + RS_TILE - 1) / RS_TILE;
  if (s.nblk == 0) s.nblk = 1;
  const uint64_t m = 256 * s.nblk;
  s.npart = (m + SCAN_CHUNK - 1) / SCAN_CHUNK;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = align256(off + bytes);
    return base ? base + o : nullptr;
  };
  s.aabb = reinterpret_cast<uint32_t*>(take(64));
  s.keys0 = reinterpret_cast<uint64_t*>(take(8 * n));
  s.keys1 = reinterpret_cast<uint64_t*>(take(8 * n));
  s.vals1 = reinterpret_cast<uint32_t*>(take(4 * n));
  s.hist = reinterpret_cast<uint32_t*>(take(4 * m));
  s.part = reinterpret_cast<uint32_t*>(take(4 * s.npart));
  if (out) *out = s;
  return off;
}

hipError_t launch_finite_check(const float* xyz, uint64_t n, uint32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_finite, dim3(grid_for(3 * n, 256 * 8)), dim3(256), 0, s,
                     reinterpret_cast<const uint32_t*>(xyz), 3 * n, flag);
  return hipGetLastError();
}

hipError_t launch_iota(uint32_t* p, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256 * 4)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_morton_codes(const float* xyz, uint64_t n, uint32_t* aabb, uint64_t* keys, uint32_t* vals,
                               uint32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_aabb_init, dim3(1), dim3(64), 0, s, aabb);
  hipLaunchKernelGGL(k_aabb, dim3(grid_for(n, 256 * 8, 4096)), dim3(256), 0, s, xyz, n, aabb, flag);
  hipLaunchKernelGGL(k_morton, dim3(grid_for(n, 256 * 4)), dim3(256), 0, s, xyz, n, aabb, keys, vals);
  return hipGetLastError();
}

hipError_t radix_sort_pairs(const SortScratch& sc, uint32_t* vals0, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t* kin = sc.keys0;
  uint64_t* kout = sc.keys1;
  uint32_t* vin = vals0;
  uint32_t* vout = sc.vals1;
  const uint64_t m = 256 * sc.nblk;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_radix_count, dim3((uint32_t)sc.nblk), dim3(256), 0, s, kin, n, shift, sc.hist, sc.nblk);
    hipLaunchKernelGGL(k_scan_partials, dim3((uint32_t)sc.npart), dim3(256), 0, s, sc.hist, m, sc.part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, sc.part, sc.npart);
    hipLaunchKernelGGL(k_scan_apply, dim3((uint32_t)sc.npart), dim3(256), 0, s, sc.hist, m, sc.part);
    hipLaunchKernelGGL(k_radix_scatter, dim3((uint32_t)sc.nblk), dim3(256), 0, s, kin, vin, kout, vout, n, shift,
                       sc.hist, sc.nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t* tk = kin;
    kin = kout;
    kout = tk;
    uint32_t* tv = vin;
    vin = vout;
    vout = tv;
  }
  // 8 passes: the sorted pairs are back in keys0 / vals0
  return hipSuccess;
}

uint64_t spread_step(uint64_t c) {
  uint64_t m = c / 4 + 1;
  for (;;) {
    uint64_t a = m, b = c;
    while (b) {
      const uint64_t t = a % b;
      a = b;
      b = t;
    }
    if (a == 1) return m;
    ++m;
  }
}

hipError_t launch_gather(const SortScratch& sc, const float* xyz, const uint32_t* rgba, uint32_t* perm,
                         uint64_t n, uint32_t batch_size, bool spread, float* xyz_out, uint32_t* colors,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  // the records take the two key buffers, free once the sort is done (keys0 then keys1: 16 n bytes)
  uint4* const rec = reinterpret_cast<uint4*>(sc.keys0);
  if (reinterpret_cast<uint8_t*>(sc.keys1) + 8 * n < reinterpret_cast<uint8_t*>(rec) + 16 * n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_interleave, dim3(grid_for(n, 256 * 4)), dim3(256), 0, s, xyz, rgba, n, rec);
  const dim3 grid(grid_for(n, 256 * 4));
  if (!spread) {
    hipLaunchKernelGGL(k_gather<false>, grid, dim3(256), 0, s, rec, perm, perm, Spread{}, n, xyz_out, colors);
    return hipGetLastError();
  }
  // the sorted order moves to the free value buffer; the spread order is written to perm
  hipError_t e = hipMemcpyAsync(sc.vals1, perm, 4 * n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  Spread sp;
  sp.S = batch_size;
  sp.m = spread_step(batch_size);
  sp.c_last = n % batch_size ? n % batch_size : batch_size;
  sp.m_last = spread_step(sp.c_last);
  hipLaunchKernelGGL(k_gather<true>, grid, dim3(256), 0, s, rec, sc.vals1, perm, sp, n, xyz_out, colors);
  return hipGetLastError();
}

hipError_t launch_batch_bbox(const float* xyz, uint64_t n, uint32_t S, uint64_t nb, BatchRec* out, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_bbox, dim3((uint32_t)nb), dim3(256), 0, s, xyz, n, S, out, 0);
  return hipGetLastError();
}

hipError_t launch_quantize(const float* xyz, uint64_t n, uint32_t S, const BatchRec* batches, uint32_t* low,
                           uint32_t* med, uint32_t* high, hipStream_t s) {
  hipLaunchKernelGGL(k_quantize, dim3(grid_for(n, 256 * 4)), dim3(256), 0, s, xyz, n, S, batches, low, med, high);
  return hipGetLastError();
}

hipError_t launch_batch_bbox_spans(const float* xyz, uint64_t nb, BatchRec* recs, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_bbox, dim3((uint32_t)nb), dim3(256), 0, s, xyz, (uint64_t)0, 0u, recs, 1);
  return hipGetLastError();
}

hipError_t launch_quantize_spans(const float* xyz, uint64_t nb, const BatchRec* recs, uint32_t* low, uint32_t* med,
                                 uint32_t* high, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_quantize_spans, dim3((uint32_t)nb), dim3(256), 0, s, xyz, recs, low, med, high);
  return hipGetLastError();
}

}  // namespace ptr

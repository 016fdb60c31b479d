// Secondary rays through the face soup: a bounding-volume hierarchy over the
// faces and two ray queries, transmittance (product of 1 - alpha over every
// hit in the ray's interval; order-free) and closest hit (smallest t with
// alpha >= alpha_min, ties to the smaller face id). This is the ray-traced use
// of the converted soup that the paper's abstract and introduction name
// (shadow and secondary rays); the hit test is Moller-Trumbore with closed
// triangles and an open interval, alpha the renderer's interpolation.
//
// Build (one pass per scene, all on the GPU):
//   1. scene box of the face centroids (per-block partial min/max, then one block)
//   2. 30-bit Morton code of each centroid in that box, value = face id
//   3. stable LSD radix sort, 8-bit digits, four passes (ranks inside a tile
//      from wavefront ballots, tile offsets from a digit-major scan)
//   4. leaf records in sorted order: v0, e1 = v1 - v0, e2 = v2 - v0, the
//      three opacities and the face id (64 bytes)
//   5. hierarchy of Karras (2012): internal node i of the N - 1 finds its
//      range and split from the longest common prefixes of neighbouring
//      codes (equal codes are told apart by their index)
//   6. boxes bottom-up, one launch per depth from the deepest: each node
//      unites its children's boxes and writes the result into its parent
//      (no atomics: the launch boundaries order the levels)
// Internal node record (64 bytes): both children's boxes side by side and the
// two child references (>= 0 internal node, < 0 leaf ~index), so one node
// visit is four 16-byte loads. The common prefix of a child's range is longer
// than its parent's and is at most 64 bits (32 code bits + 32 index bits),
// so a root-to-leaf path has at most 64 internal nodes and the traversal
// stack (one pending sibling per level) never holds more than 64 entries.

#include "common.h"

namespace {

constexpr int kRsThreads = 256;
constexpr int kRsRounds = 8;
constexpr int kRsTile = kRsThreads * kRsRounds;
constexpr int kTraceThreads = 128;
constexpr int kStack = 64;

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > 65535 * 16) g = 65535 * 16;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---- 1. scene box of the centroids ----
__device__ __forceinline__ void centroid(const float* __restrict__ pos, const int32_t* __restrict__ idx, int64_t V,
                                         int64_t F, int64_t f, float c[3]) {
  const int32_t i0 = idx[f], i1 = idx[F + f], i2 = idx[2 * F + f];
  const bool ok = i0 >= 0 && i0 < V && i1 >= 0 && i1 < V && i2 >= 0 && i2 < V;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    c[d] = ok ? (pos[d * V + i0] + pos[d * V + i1] + pos[d * V + i2]) * (1.f / 3.f) : __int_as_float(0x7fc00000);
}

__device__ __forceinline__ float wave_min(float x) {
  for (int d = 32; d >= 1; d >>= 1) x = fminf(x, __shfl_xor(x, d));
  return x;
}
__device__ __forceinline__ float wave_max(float x) {
  for (int d = 32; d >= 1; d >>= 1) x = fmaxf(x, __shfl_xor(x, d));
  return x;
}

// the points a hierarchy or an order is built over: face centroids, or Gaussian means
struct FaceCentroids {
  const float* pos;
  const int32_t* idx;
  int64_t V, F;
  __device__ __forceinline__ void get(int64_t f, float c[3]) const { centroid(pos, idx, V, F, f, c); }
};

struct Points {
  const float* p;  // [3][n]
  int64_t n;
  __device__ __forceinline__ void get(int64_t i, float c[3]) const {
    c[0] = p[i];
    c[1] = p[n + i];
    c[2] = p[2 * n + i];
  }
};

// per block: min and max of the points (NaN points are ignored by fminf / fmaxf)
template <class Src>
__global__ __launch_bounds__(256) void k_box_partial(Src src, int64_t F, float* __restrict__ part) {
  __shared__ float red[4][6];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t f = blockIdx.x * 256ll + threadIdx.x; f < F; f += (int64_t)gridDim.x * 256) {
    float c[3];
    src.get(f, c);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fminf(lo[d], c[d]);
      hi[d] = fmaxf(hi[d], c[d]);
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = wave_min(lo[d]);
    hi[d] = wave_max(hi[d]);
  }
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red[w][d] = lo[d];
      red[w][3 + d] = hi[d];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int d = threadIdx.x;
    float v = red[0][d];
    for (int k = 1; k < 4; ++k) v = d < 3 ? fminf(v, red[k][d]) : fmaxf(v, red[k][d]);
    part[blockIdx.x * 6ll + d] = v;
  }
}

__global__ __launch_bounds__(256) void k_box_final(const float* __restrict__ part, int nparts, float* __restrict__ box) {
  __shared__ float red[4][6];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int p = threadIdx.x; p < nparts; p += 256) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fminf(lo[d], part[p * 6ll + d]);
      hi[d] = fmaxf(hi[d], part[p * 6ll + 3 + d]);
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = wave_min(lo[d]);
    hi[d] = wave_max(hi[d]);
  }
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red[w][d] = lo[d];
      red[w][3 + d] = hi[d];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int d = threadIdx.x;
    float v = red[0][d];
    for (int k = 1; k < 4; ++k) v = d < 3 ? fminf(v, red[k][d]) : fmaxf(v, red[k][d]);
    box[d] = v;
  }
}

// ---- 2. Morton codes ----
__device__ __forceinline__ uint32_t spread10(uint32_t x) {
  // bit k of x moves to bit 3k
  x &= 1023u;
  x = (x | (x << 16)) & 0x030000FFu;
  x = (x | (x << 8)) & 0x0300F00Fu;
  x = (x | (x << 4)) & 0x030C30C3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

__device__ __forceinline__ uint32_t quant10(float c, float lo, float hi) {
  const float ext = hi - lo;
  float x = ext > 0.f ? (c - lo) / ext : 0.f;
  x = x >= 0.f ? x : 0.f;  // also NaN -> 0
  x = x <= 1.f ? x : 1.f;
  return (uint32_t)fminf(x * 1024.f, 1023.f);
}

template <class Src>
__global__ __launch_bounds__(256) void k_morton(Src src, int64_t F, const float* __restrict__ box,
                                                uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const float lo0 = box[0], lo1 = box[1], lo2 = box[2], hi0 = box[3], hi1 = box[4], hi2 = box[5];
  for (int64_t f = blockIdx.x * 256ll + threadIdx.x; f < F; f += (int64_t)gridDim.x * 256) {
    float c[3];
    src.get(f, c);
    keys[f] = (spread10(quant10(c[0], lo0, hi0)) << 2) | (spread10(quant10(c[1], lo1, hi1)) << 1) |
              spread10(quant10(c[2], lo2, hi2));
    vals[f] = (uint32_t)f;
  }
}

// ---- 3. stable LSD radix sort (8-bit digit per pass) ----
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                        uint32_t* __restrict__ counts, int64_t nblk) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsRounds; ++r) {
    const int64_t i = b0 + r * kRsThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Each round places 256 consecutive keys: the rank of a key among the keys of
// its wavefront with the same digit comes from eight ballots, the keys of
// earlier wavefronts with that digit from per-wave counts in LDS, and the
// keys of earlier rounds and tiles from the running digit base.
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                           int64_t n, int shift, const int64_t* __restrict__ offs,
                                                           int64_t nblk) {
  __shared__ int64_t base[256];
  __shared__ uint32_t wcnt[kRsThreads / 64][256];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  base[t] = offs[(int64_t)t * nblk + blockIdx.x];
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t b0 = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsRounds; ++r) {
#pragma unroll
    for (int w = 0; w < kRsThreads / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const int64_t i = b0 + r * kRsThreads + t;
    const bool ok = i < n;
    uint32_t k = 0, v = 0, d = 0;
    if (ok) {
      k = kin[i];
      v = vin[i];
      d = (k >> shift) & 255u;
    }
    uint64_t m = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(ok && bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(m & below);
    if (ok && rank == 0) wcnt[wid][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (ok) {
      int64_t pos = base[d] + rank;
      for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
      if (pos >= 0 && pos < n) {
        kout[pos] = k;
        vout[pos] = v;
      }
    }
    __syncthreads();
    int64_t add = 0;
#pragma unroll
    for (int w = 0; w < kRsThreads / 64; ++w) add += wcnt[w][t];
    base[t] += add;
    __syncthreads();
  }
}

// ---- 4. leaf records ----
__global__ __launch_bounds__(256) void k_leaves(const float* __restrict__ pos, const float* __restrict__ op,
                                                const int32_t* __restrict__ idx, int64_t V, int64_t F,
                                                const uint32_t* __restrict__ order, float4* __restrict__ leaves) {
  for (int64_t j = blockIdx.x * 256ll + threadIdx.x; j < F; j += (int64_t)gridDim.x * 256) {
    const int64_t f = order[j];
    const int32_t i0 = idx[f], i1 = idx[F + f], i2 = idx[2 * F + f];
    const bool ok = i0 >= 0 && i0 < V && i1 >= 0 && i1 < V && i2 >= 0 && i2 < V;
    const float nan = __int_as_float(0x7fc00000);
    float p[3][3], o[3];
    const int32_t ii[3] = {i0, i1, i2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int d = 0; d < 3; ++d) p[c][d] = ok ? pos[d * V + ii[c]] : nan;
      o[c] = ok ? op[ii[c]] : 0.f;
    }
    leaves[4 * j + 0] = make_float4(p[0][0], p[0][1], p[0][2], o[0]);
    leaves[4 * j + 1] = make_float4(p[1][0] - p[0][0], p[1][1] - p[0][1], p[1][2] - p[0][2], o[1]);
    leaves[4 * j + 2] = make_float4(p[2][0] - p[0][0], p[2][1] - p[0][1], p[2][2] - p[0][2], o[2]);
    leaves[4 * j + 3] = make_float4(__int_as_float((int32_t)f), 0.f, 0.f, 0.f);
  }
}

// ---- 5. hierarchy ----
// longest common prefix of sorted codes i and j, with the index breaking ties; -1 outside [0, n)
__device__ __forceinline__ int lcp(const uint32_t* __restrict__ k, int64_t n, int64_t i, int64_t j) {
  if (j < 0 || j >= n) return -1;
  const uint32_t a = k[i], b = k[j];
  if (a != b) return __clz(a ^ b);
  return 32 + __clz((uint32_t)i ^ (uint32_t)j);
}

__global__ __launch_bounds__(256) void k_hierarchy(const uint32_t* __restrict__ k, int64_t n,
                                                   float4* __restrict__ nodes, int32_t* __restrict__ parent,
                                                   int32_t* __restrict__ lparent) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n - 1; i += (int64_t)gridDim.x * 256) {
    const int d = lcp(k, n, i, i + 1) - lcp(k, n, i, i - 1) >= 0 ? 1 : -1;
    const int dmin = lcp(k, n, i, i - d);
    int64_t lmax = 2;
    while (lcp(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
      if (lcp(k, n, i, i + (l + t) * d) > dmin) l += t;
    const int64_t j = i + l * d;
    const int dnode = lcp(k, n, i, j);
    int64_t s = 0;
    for (int64_t div = 2;; div <<= 1) {
      const int64_t t = (l + div - 1) / div;
      if (lcp(k, n, i, i + (s + t) * d) > dnode) s += t;
      if (t <= 1) break;
    }
    const int64_t g = i + s * d + (d < 0 ? -1 : 0);
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    const int32_t c0 = lo == g ? ~(int32_t)g : (int32_t)g;
    const int32_t c1 = hi == g + 1 ? ~(int32_t)(g + 1) : (int32_t)(g + 1);
    nodes[4 * i + 3] = make_float4(__int_as_float(c0), __int_as_float(c1), 0.f, 0.f);
    if (c0 < 0) lparent[g] = (int32_t)i; else parent[g] = (int32_t)i;
    if (c1 < 0) lparent[g + 1] = (int32_t)i; else parent[g + 1] = (int32_t)i;
  }
}

// ---- 6. boxes, bottom-up ----
__device__ __forceinline__ void put_box(float* nd, int slot, const float (&lo)[3], const float (&hi)[3]) {
  // slot 0: floats 0..5 = lo0, hi0; slot 1: floats 6..11 = lo1, hi1
  float* b = nd + 6 * slot;
  b[0] = lo[0];
  b[1] = lo[1];
  b[2] = lo[2];
  b[3] = hi[0];
  b[4] = hi[1];
  b[5] = hi[2];
}

__device__ __forceinline__ void leaf_bounds(const float4* __restrict__ leaves, int64_t j, float (&lo)[3],
                                            float (&hi)[3]) {
  const float4 a = leaves[4 * j], e1 = leaves[4 * j + 1], e2 = leaves[4 * j + 2];
  const float p[3][3] = {{a.x, a.y, a.z}, {a.x + e1.x, a.y + e1.y, a.z + e1.z}, {a.x + e2.x, a.y + e2.y, a.z + e2.z}};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = fminf(p[0][d], fminf(p[1][d], p[2][d]));
    hi[d] = fmaxf(p[0][d], fmaxf(p[1][d], p[2][d]));
  }
}

// depth of every internal node: parent steps to the root (at most 64, see the header;
// the bound only guards the walk)
__global__ __launch_bounds__(256) void k_depth(const int32_t* __restrict__ parent, int64_t n_int,
                                               uint32_t* __restrict__ depth) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n_int; i += (int64_t)gridDim.x * 256) {
    int32_t j = (int32_t)i;
    uint32_t d = 0;
    while (j != 0 && d < 4 * kStack) {
      j = parent[j];
      ++d;
    }
    depth[i] = d;
  }
}

// Boxes level by level, deepest first (one launch per depth; the launch boundary
// orders the levels): a node of this depth writes its leaf children's boxes into
// its own slots, reads the slots its internal children filled one launch
// earlier, and writes their union into its slot of its parent. Every slot has
// one writer.
__global__ __launch_bounds__(256) void k_level_boxes(const float4* __restrict__ leaves, int64_t n_int, float* nodes,
                                                     const int32_t* __restrict__ parent,
                                                     const uint32_t* __restrict__ depth, uint32_t level,
                                                     float* __restrict__ root_box) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n_int; i += (int64_t)gridDim.x * 256) {
    if (depth[i] != level) continue;
    float* nd = nodes + 16 * i;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int slot = 0; slot < 2; ++slot) {
      const int32_t c = __float_as_int(nd[12 + slot]);
      float blo[3], bhi[3];
      if (c < 0) {
        leaf_bounds(leaves, ~(int64_t)c, blo, bhi);
        put_box(nd, slot, blo, bhi);
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          blo[d] = nd[6 * slot + d];
          bhi[d] = nd[6 * slot + 3 + d];
        }
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = fminf(lo[d], blo[d]);
        hi[d] = fmaxf(hi[d], bhi[d]);
      }
    }
    if (i == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        root_box[d] = lo[d];
        root_box[3 + d] = hi[d];
      }
    } else {
      float* pd = nodes + 16ll * parent[i];
      put_box(pd, __float_as_int(pd[12]) == (int32_t)i ? 0 : 1, lo, hi);
    }
  }
}

// a hierarchy of one face: its box is the root box
__global__ void k_single_leaf_box(const float4* __restrict__ leaves, float* __restrict__ root_box) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float lo[3], hi[3];
  leaf_bounds(leaves, 0, lo, hi);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    root_box[d] = lo[d];
    root_box[3 + d] = hi[d];
  }
}

// ---- queries ----
struct RayIn {
  const float* o;
  const float* d;
  const float* t0;
  const float* t1;
  const int32_t* order;
  int64_t n;
};

// the ray a thread traces: order[j] when an order is given (-1 outside [0, n))
__device__ __forceinline__ int64_t ray_of(const RayIn& r, int64_t j) {
  if (!r.order) return j;
  const int32_t i = r.order[j];
  return (i >= 0 && (int64_t)i < r.n) ? (int64_t)i : -1;
}

struct Ray {
  float o[3], d[3], id[3], t0, t1;
};

__device__ __forceinline__ Ray load_ray(const RayIn& r, int64_t i) {
  Ray y;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    y.o[c] = r.o[c * r.n + i];
    y.d[c] = r.d[c * r.n + i];
    const float dc = y.d[c];
    y.id[c] = 1.f / (fabsf(dc) > 1e-30f ? dc : copysignf(1e-30f, dc));
  }
  y.t0 = r.t0[i];
  y.t1 = r.t1[i];
  return y;
}

// slab test against [t0, tmax]; the far distance is widened by 1 + 2 gamma_3 so
// that rounding never drops a box a hit lies on
__device__ __forceinline__ bool box_hit(const Ray& y, float lx, float ly, float lz, float hx, float hy, float hz,
                                        float tmax) {
  const float ax = (lx - y.o[0]) * y.id[0], bx = (hx - y.o[0]) * y.id[0];
  const float ay = (ly - y.o[1]) * y.id[1], by = (hy - y.o[1]) * y.id[1];
  const float az = (lz - y.o[2]) * y.id[2], bz = (hz - y.o[2]) * y.id[2];
  const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), y.t0));
  const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), tmax)) * 1.0000004f;
  return tn <= tf;
}

struct Hit {
  float t, u, v, alpha;
  int32_t face;
  bool hit;
};

__device__ __forceinline__ Hit leaf_hit(const Ray& y, const float4* __restrict__ leaves, int32_t j) {
  const float4 a = leaves[4ll * j], e1 = leaves[4ll * j + 1], e2 = leaves[4ll * j + 2], w = leaves[4ll * j + 3];
  Hit h;
  h.hit = false;
  h.face = __float_as_int(w.x);
  const float pv0 = y.d[1] * e2.z - y.d[2] * e2.y;
  const float pv1 = y.d[2] * e2.x - y.d[0] * e2.z;
  const float pv2 = y.d[0] * e2.y - y.d[1] * e2.x;
  const float det = e1.x * pv0 + e1.y * pv1 + e1.z * pv2;
  if (!(det != 0.f)) return h;
  const float inv = 1.f / det;
  const float tv0 = y.o[0] - a.x, tv1 = y.o[1] - a.y, tv2 = y.o[2] - a.z;
  h.u = (tv0 * pv0 + tv1 * pv1 + tv2 * pv2) * inv;
  const float qv0 = tv1 * e1.z - tv2 * e1.y;
  const float qv1 = tv2 * e1.x - tv0 * e1.z;
  const float qv2 = tv0 * e1.y - tv1 * e1.x;
  h.v = (y.d[0] * qv0 + y.d[1] * qv1 + y.d[2] * qv2) * inv;
  h.t = (e2.x * qv0 + e2.y * qv1 + e2.z * qv2) * inv;
  h.hit = h.u >= 0.f && h.v >= 0.f && h.u + h.v <= 1.f && h.t > y.t0 && h.t < y.t1;
  const float al = (1.f - h.u - h.v) * a.w + h.u * e1.w + h.v * e2.w;
  h.alpha = fminf(fmaxf(al, 0.f), 1.f);
  return h;
}

// work counters of a query: err[2..3] node visits, err[4..5] leaf tests (uint64, one atomic per wave)
__device__ __forceinline__ void count_visits(uint64_t nn, uint64_t nl, uint32_t* err) {
  for (int d = 32; d >= 1; d >>= 1) {
    nn += __shfl_xor(nn, d);
    nl += __shfl_xor(nl, d);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd((unsigned long long*)(err + 2), (unsigned long long)nn);
    atomicAdd((unsigned long long*)(err + 4), (unsigned long long)nl);
  }
}

__global__ __launch_bounds__(kTraceThreads) void k_trace_transmittance(const float4* __restrict__ nodes,
                                                                       const float4* __restrict__ leaves, int64_t n_leaves,
                                                                       const float* __restrict__ root_box, RayIn rin,
                                                                       float t_eps, float* __restrict__ T_out,
                                                                       uint32_t* __restrict__ err) {
  __shared__ int32_t stk[kStack][kTraceThreads];
  const int tid = threadIdx.x;
  uint64_t n_nodes = 0, n_leaf = 0;
  for (int64_t r = blockIdx.x * (int64_t)kTraceThreads + tid; r < rin.n; r += (int64_t)gridDim.x * kTraceThreads) {
    const int64_t ri = ray_of(rin, r);
    if (ri < 0) continue;
    const Ray y = load_ray(rin, ri);
    float T = 1.f;
    bool overflow = false;
    if (n_leaves > 0 && box_hit(y, root_box[0], root_box[1], root_box[2], root_box[3], root_box[4], root_box[5], y.t1)) {
      int sp = 0;
      int32_t cur = n_leaves == 1 ? ~0 : 0;
      for (;;) {
        if (cur >= 0) {
          ++n_nodes;
          const float4 q0 = nodes[4ll * cur], q1 = nodes[4ll * cur + 1], q2 = nodes[4ll * cur + 2],
                       q3 = nodes[4ll * cur + 3];
          const bool h0 = box_hit(y, q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, y.t1);
          const bool h1 = box_hit(y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w, y.t1);
          const int32_t c0 = __float_as_int(q3.x), c1 = __float_as_int(q3.y);
          if (h0 && h1) {
            if (sp == kStack) {
              overflow = true;
              break;
            }
            stk[sp++][tid] = c1;
            cur = c0;
            continue;
          }
          if (h0 || h1) {
            cur = h0 ? c0 : c1;
            continue;
          }
        } else {
          ++n_leaf;
          const Hit h = leaf_hit(y, leaves, ~cur);
          if (h.hit) {
            T *= 1.f - h.alpha;
            if (T < t_eps) break;
          }
        }
        if (sp == 0) break;
        cur = stk[--sp][tid];
      }
    }
    if (overflow) {
      T = __int_as_float(0x7fc00000);
      atomicOr(err, 1u);
    }
    T_out[ri] = T;
  }
  count_visits(n_nodes, n_leaf, err);
}

__global__ __launch_bounds__(kTraceThreads) void k_trace_closest(const float4* __restrict__ nodes,
                                                                 const float4* __restrict__ leaves, int64_t n_leaves,
                                                                 const float* __restrict__ root_box, RayIn rin,
                                                                 float alpha_min, float* __restrict__ t_out,
                                                                 int32_t* __restrict__ f_out, float* __restrict__ u_out,
                                                                 float* __restrict__ v_out, uint32_t* __restrict__ err) {
  __shared__ int32_t stk[kStack][kTraceThreads];
  const int tid = threadIdx.x;
  uint64_t n_nodes = 0, n_leaf = 0;
  for (int64_t r = blockIdx.x * (int64_t)kTraceThreads + tid; r < rin.n; r += (int64_t)gridDim.x * kTraceThreads) {
    const int64_t ri = ray_of(rin, r);
    if (ri < 0) continue;
    const Ray y = load_ray(rin, ri);
    float bt = INFINITY, bu = 0.f, bv = 0.f;
    int32_t bf = -1;
    bool overflow = false;
    if (n_leaves > 0 && box_hit(y, root_box[0], root_box[1], root_box[2], root_box[3], root_box[4], root_box[5], y.t1)) {
      int sp = 0;
      int32_t cur = n_leaves == 1 ? ~0 : 0;
      for (;;) {
        const float tmax = fminf(bt, y.t1);
        if (cur >= 0) {
          ++n_nodes;
          const float4 q0 = nodes[4ll * cur], q1 = nodes[4ll * cur + 1], q2 = nodes[4ll * cur + 2],
                       q3 = nodes[4ll * cur + 3];
          const bool h0 = box_hit(y, q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, tmax);
          const bool h1 = box_hit(y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w, tmax);
          int32_t c0 = __float_as_int(q3.x), c1 = __float_as_int(q3.y);
          if (h0 && h1) {
            // nearer box first: compare the entry distances along the ray
            const float e0 = fmaxf(fmaxf(fminf((q0.x - y.o[0]) * y.id[0], (q0.w - y.o[0]) * y.id[0]),
                                         fminf((q0.y - y.o[1]) * y.id[1], (q1.x - y.o[1]) * y.id[1])),
                                   fminf((q0.z - y.o[2]) * y.id[2], (q1.y - y.o[2]) * y.id[2]));
            const float e1 = fmaxf(fmaxf(fminf((q1.z - y.o[0]) * y.id[0], (q2.y - y.o[0]) * y.id[0]),
                                         fminf((q1.w - y.o[1]) * y.id[1], (q2.z - y.o[1]) * y.id[1])),
                                   fminf((q2.x - y.o[2]) * y.id[2], (q2.w - y.o[2]) * y.id[2]));
            if (e1 < e0) {
              const int32_t tmp = c0;
              c0 = c1;
              c1 = tmp;
            }
            if (sp == kStack) {
              overflow = true;
              break;
            }
            stk[sp++][tid] = c1;
            cur = c0;
            continue;
          }
          if (h0 || h1) {
            cur = h0 ? c0 : c1;
            continue;
          }
        } else {
          ++n_leaf;
          const Hit h = leaf_hit(y, leaves, ~cur);
          if (h.hit && h.alpha >= alpha_min && (h.t < bt || (h.t == bt && h.face < bf))) {
            bt = h.t;
            bu = h.u;
            bv = h.v;
            bf = h.face;
          }
        }
        if (sp == 0) break;
        cur = stk[--sp][tid];
      }
    }
    if (overflow) {
      bt = __int_as_float(0x7fc00000);
      bf = -1;
      atomicOr(err, 1u);
    }
    t_out[ri] = bt;
    f_out[ri] = bf;
    if (u_out) u_out[ri] = bu;
    if (v_out) v_out[ri] = bv;
  }
  count_visits(n_nodes, n_leaf, err);
}


// Morton codes of the points in their own box, then the stable radix sort:
// codes and point indices sorted in keys[0] / vals[0] (four passes)
template <class Src>
hipError_t morton_sort(hipStream_t s, Src src, int64_t F, const BvhBufs& b, uint32_t* vals0) {
  const unsigned gb = grid_for(F, 256) > 1024 ? 1024 : grid_for(F, 256);
  hipLaunchKernelGGL(k_box_partial<Src>, dim3(gb), dim3(256), 0, s, src, F, b.part);
  hipLaunchKernelGGL(k_box_final, dim3(1), dim3(256), 0, s, b.part, (int)gb, b.scene_box);
  hipLaunchKernelGGL(k_morton<Src>, dim3(grid_for(F, 256)), dim3(256), 0, s, src, F, b.scene_box, b.keys[0], vals0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nblk = (F + kRsTile - 1) / kRsTile;
  uint32_t* vals[2] = {vals0, b.vals[1]};
  int cur = 0;
  for (int shift = 0; shift < 32; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblk), dim3(kRsThreads), 0, s, b.keys[cur], F, shift, b.counts, nblk);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_scan_u32(s, b.counts, b.offs, 256 * nblk, b.scan);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nblk), dim3(kRsThreads), 0, s, b.keys[cur], vals[cur],
                       b.keys[cur ^ 1], vals[cur ^ 1], F, shift, b.offs, nblk);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur ^= 1;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_spatial_order(hipStream_t s, const float* mean, int64_t n, const BvhBufs& b, int32_t* order) {
  if (n == 0) return hipSuccess;
  return morton_sort(s, Points{mean, n}, n, b, reinterpret_cast<uint32_t*>(order));
}

hipError_t launch_bvh_build(hipStream_t s, const msp_faces* f, const BvhBufs& b) {
  const int64_t F = f->n_faces, V = f->n_verts;
  if (F == 0) return hipSuccess;
  hipError_t e = morton_sort(s, FaceCentroids{f->pos, f->idx, V, F}, F, b, b.vals[0]);
  if (e != hipSuccess) return e;
  const int cur = 0;
  // four passes: the sorted codes and face ids are back in buffer 0
  hipLaunchKernelGGL(k_leaves, dim3(grid_for(F, 256)), dim3(256), 0, s, f->pos, f->opacity, f->idx, V, F,
                     b.vals[cur], (float4*)b.leaves);
  if (F > 1)
    hipLaunchKernelGGL(k_hierarchy, dim3(grid_for(F - 1, 256)), dim3(256), 0, s, b.keys[cur], F, (float4*)b.nodes,
                       b.parent, b.lparent);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (F == 1) {
    hipLaunchKernelGGL(k_single_leaf_box, dim3(1), dim3(64), 0, s, (const float4*)b.leaves, b.root_box);
    return hipGetLastError();
  }
  // b.flags holds the depths
  hipLaunchKernelGGL(k_depth, dim3(grid_for(F - 1, 256)), dim3(256), 0, s, b.parent, F - 1, b.flags);
  for (int level = kStack; level >= 0; --level)
    hipLaunchKernelGGL(k_level_boxes, dim3(grid_for(F - 1, 256)), dim3(256), 0, s, (const float4*)b.leaves, F - 1,
                       b.nodes, b.parent, b.flags, (uint32_t)level, b.root_box);
  return hipGetLastError();
}

hipError_t launch_trace_transmittance(hipStream_t s, const BvhBufs& b, int64_t n_leaves, const msp_rays* r,
                                      float t_eps, float* T, uint32_t* err) {
  if (r->n == 0) return hipSuccess;
  RayIn rin{r->origin, r->dir, r->tmin, r->tmax, r->order, r->n};
  hipLaunchKernelGGL(k_trace_transmittance, dim3(grid_for(r->n, kTraceThreads)), dim3(kTraceThreads), 0, s,
                     (const float4*)b.nodes, (const float4*)b.leaves, n_leaves, b.root_box, rin, t_eps, T, err);
  return hipGetLastError();
}

hipError_t launch_trace_closest(hipStream_t s, const BvhBufs& b, int64_t n_leaves, const msp_rays* r, float alpha_min,
                                float* t, int32_t* face, float* u, float* v, uint32_t* err) {
  if (r->n == 0) return hipSuccess;
  RayIn rin{r->origin, r->dir, r->tmin, r->tmax, r->order, r->n};
  hipLaunchKernelGGL(k_trace_closest, dim3(grid_for(r->n, kTraceThreads)), dim3(kTraceThreads), 0, s,
                     (const float4*)b.nodes, (const float4*)b.leaves, n_leaves, b.root_box, rin, alpha_min, t, face, u,
                     v, err);
  return hipGetLastError();
}

// Tile-binned, exactly depth-ordered rendering of a triangle soup, forward and
// adjoint (rendering section of the paper: MVP transform, layers peeled in
// depth order, interpolated vertex attributes, front-to-back blending through
// alpha; the adjoint feeds the fine-tuning section's optimiser).
//
// Pipeline per render (all views in one launch per stage):
//   setup      per (view, face): fixed-order float32 projection, near cull,
//              pixel footprint with a 2^-8 px margin, nearest depth; writes a
//              48-byte geometry record; per-tile counts gathered in a
//              per-workgroup LDS tile table, then one global atomic per
//              (workgroup, tile).
//   attr       per face: corner opacities, colours and vertex ids packed in a
//              64-byte record (view independent).
//   scan       tile counts -> tile-list offsets (scan.hip).
//   emit       per face: its key (bits(zmin) << 32 | face id) into every
//              tile it touches; each workgroup reserves one range per tile
//              and hands out its slots from LDS.
//   tile_sort  each tile list sorted ascending: per-thread register sorts
//              merged in LDS by merge path; lists longer than one chunk are
//              chunk-sorted, then merged pairwise through global memory.
//   composite  persistent: each wavefront pulls (view, 8x8 pixel block) work
//              items; the block's tile list is staged 64 entries at a time in
//              a per-wave LDS slab (ballot-compacted to the faces whose
//              footprint meets the block; the next chunk's records are
//              fetched while the current one is processed) and streamed in
//              nearest-depth order. Each lane keeps a register buffer of up
//              to KB fragments sorted by (depth, face id); a fragment is
//              composited once the next entry's nearest depth exceeds its
//              depth, because no later face can then come in front of it. If
//              the buffer overflows, the largest keys are dropped and
//              remembered, everything smaller is still composited in exact
//              order, and the lane re-scans the list for the keys after the
//              last one it composited: exact (depth, face id) order at any
//              depth complexity.
//   backward   pass 1 recomputes each pixel's ordered list with the same code
//              into a per-block [k][64] slab (face id, transmittance);
//              pass 2 walks it back to front with S_i = a_i c_i +
//              (1 - a_i) S_{i+1} and P_i = (1 - a_i) P_{i+1} (no division by
//              1 - a), takes d position through the ray/triangle Jacobian,
//              and sums per-face gradients in a per-wave LDS hash table; a
//              flush combines the vertices neighbouring lanes share and adds
//              each face's and vertex's sums to global memory once.
#include "common.h"

namespace {

constexpr float kMargin = 0.00390625f;  // 2^-8 pixel
constexpr int kRec = 28;                // floats per staged face record
constexpr int kWavesPerWG = 4;
constexpr int kHashSlots = 128;         // per-wave gradient table (8 blocks of 16 slots)
constexpr int kHashBits = 7;            // log2(kHashSlots)
constexpr int kHashFill = 64;           // flushed once it holds more faces than this (free slots stay likely)
static_assert(kHashSlots == 2 * MSP_WAVE, "a flush takes two slots per lane");
static_assert((1 << kHashBits) == kHashSlots, "slot bits");
constexpr uint32_t kEmpty = 0xffffffffu;

enum : int { DONE = 0, ACTIVE = 1, RESTART = 2 };

struct Proj {
  float xc, yc, zc, u, v;
};

// Camera coordinates and pixel coordinates, one IEEE float32 operation at a
// time in a fixed order (no contraction), so binning is reproducible bit for bit.
__device__ __forceinline__ Proj project(const msp_camera& c, float x, float y, float z) {
#pragma clang fp contract(off)
  Proj p;
  const float* W = c.world_to_cam;
  p.xc = ((W[0] * x + W[1] * y) + W[2] * z) + W[3];
  p.yc = ((W[4] * x + W[5] * y) + W[6] * z) + W[7];
  p.zc = ((W[8] * x + W[9] * y) + W[10] * z) + W[11];
  p.u = c.fx * (p.xc / p.zc) + c.cx;
  p.v = c.fy * (p.yc / p.zc) + c.cy;
  return p;
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (MSP_WAVE - 1); }

// Per-workgroup table of the tiles its faces touch (open addressing in LDS).
// Binning through it turns one global atomic per (face, tile) into one per
// (workgroup, tile): the 256 faces of a workgroup are 16 fans whose tiles repeat.
constexpr int kTableSlots = 1024;

__device__ __forceinline__ uint32_t table_hash(int32_t t) { return ((uint32_t)t * 2654435761u) >> 22; }

// slot of tile t, inserting it if absent; -1 if the table is full
__device__ __forceinline__ int table_insert(int32_t* key, int32_t t) {
  const uint32_t h = table_hash(t);
  for (int i = 0; i < kTableSlots; ++i) {
    const int sl = (int)((h + i) & (kTableSlots - 1));
    int32_t k = __atomic_load_n(&key[sl], __ATOMIC_RELAXED);
    if (k == -1) k = atomicCAS(&key[sl], -1, t);
    if (k == -1 || k == t) return sl;
  }
  return -1;
}

// slot of tile t after all insertions, -1 if it was not inserted
__device__ __forceinline__ int table_find(const int32_t* key, int32_t t) {
  const uint32_t h = table_hash(t);
  for (int i = 0; i < kTableSlots; ++i) {
    const int sl = (int)((h + i) & (kTableSlots - 1));
    const int32_t k = key[sl];
    if (k == t) return sl;
    if (k == -1) return -1;
  }
  return -1;
}

// tile rectangle of a footprint record (xr, yr packed pixel bounds); empty if culled
struct TileRect {
  int tx0, tx1, ty0, ty1;
};

__device__ __forceinline__ TileRect tile_rect(const RasterArgs& a, const float4& g2) {
  const uint32_t xr = __float_as_uint(g2.y), yr = __float_as_uint(g2.z);
  const int px0 = xr & 0xffff, px1 = xr >> 16, py0 = yr & 0xffff, py1 = yr >> 16;
  TileRect r;
  if (px0 > px1 || py0 > py1) {
    r.tx0 = r.ty0 = 0;
    r.tx1 = r.ty1 = -1;
  } else {
    r.tx0 = px0 / a.tile_w;
    r.tx1 = px1 / a.tile_w;
    r.ty0 = py0 / a.tile_h;
    r.ty1 = py1 / a.tile_h;
  }
  return r;
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
// geometry record (3 float4): (u0, v0, u1, v1) (u2, v2, 1/z0, 1/z1) (1/z2, xr, yr, zbits)
// with xr = px0 | px1 << 16, yr = py0 | py1 << 16; a culled face has px0 > px1.
// Projection, cull and footprint of face f in one view; writes its geometry
// record and returns its tile rectangle (empty when culled) and footprint pixels.
__device__ __forceinline__ void setup_face(const RasterArgs& a, const msp_camera& c, int view, int64_t f, TileRect& tr,
                                           unsigned long long& area) {
  const int64_t F = a.n_faces, V = a.n_verts;
  float4 g0 = make_float4(0, 0, 0, 0), g1 = g0;
  float4 g2 = make_float4(0.f, __uint_as_float(1u), __uint_as_float(0u), 0.f);
  const int32_t i0 = a.idx[f], i1 = a.idx[F + f], i2 = a.idx[2 * F + f];
  if ((uint64_t)i0 < (uint64_t)V && (uint64_t)i1 < (uint64_t)V && (uint64_t)i2 < (uint64_t)V) {
    const Proj p0 = project(c, a.pos[i0], a.pos[V + i0], a.pos[2 * V + i0]);
    const Proj p1 = project(c, a.pos[i1], a.pos[V + i1], a.pos[2 * V + i1]);
    const Proj p2 = project(c, a.pos[i2], a.pos[V + i2], a.pos[2 * V + i2]);
    const bool vis = p0.zc > c.znear && p1.zc > c.znear && p2.zc > c.znear;
    const bool fin = isfinite(p0.u) && isfinite(p1.u) && isfinite(p2.u) && isfinite(p0.v) &&
                     isfinite(p1.v) && isfinite(p2.v);
    if (vis && fin) {
#pragma clang fp contract(off)
      const float umin = fminf(fminf(p0.u, p1.u), p2.u), umax = fmaxf(fmaxf(p0.u, p1.u), p2.u);
      const float vmin = fminf(fminf(p0.v, p1.v), p2.v), vmax = fmaxf(fmaxf(p0.v, p1.v), p2.v);
      float fx0 = ceilf((umin - 0.5f) - kMargin), fx1 = floorf((umax - 0.5f) + kMargin);
      float fy0 = ceilf((vmin - 0.5f) - kMargin), fy1 = floorf((vmax - 0.5f) + kMargin);
      fx0 = fmaxf(fx0, 0.f);
      fy0 = fmaxf(fy0, 0.f);
      fx1 = fminf(fx1, (float)(a.W - 1));
      fy1 = fminf(fy1, (float)(a.H - 1));
      if (fx0 <= fx1 && fy0 <= fy1) {
        const int px0 = (int)fx0, px1 = (int)fx1, py0 = (int)fy0, py1 = (int)fy1;
        area = (unsigned long long)(px1 - px0 + 1) * (unsigned long long)(py1 - py0 + 1);
        const float zmin = fminf(fminf(p0.zc, p1.zc), p2.zc);
        tr = TileRect{px0 / a.tile_w, px1 / a.tile_w, py0 / a.tile_h, py1 / a.tile_h};
        g0 = make_float4(p0.u, p0.v, p1.u, p1.v);
        // reciprocal depths (the perspective weights of the barycentrics), divided
        // once per (view, face) here instead of in every block that stages the face
        g1 = make_float4(p2.u, p2.v, 1.f / p0.zc, 1.f / p1.zc);
        g2 = make_float4(1.f / p2.zc, __uint_as_float((uint32_t)px0 | ((uint32_t)px1 << 16)),
                         __uint_as_float((uint32_t)py0 | ((uint32_t)py1 << 16)), __uint_as_float(__float_as_uint(zmin)));
      }
    }
  }
  float4* geo = a.geo + ((int64_t)view * F + f) * 3;
  geo[0] = g0;
  geo[1] = g1;
  geo[2] = g2;
}

// Each thread takes kSetupFaces faces (a workgroup that many groups of 256
// consecutive ones), so that their loads overlap and the workgroup's table
// and barriers serve more faces (per 8-view 1080p step of 8M faces: 2.04 ms at
// one face per thread, 1.79 at two, 1.67 at four, 2.08 at eight).
constexpr int kSetupFaces = 4;

__global__ __launch_bounds__(256) void k_setup(RasterArgs a) {
  const int view = blockIdx.y;
  const int64_t F = a.n_faces;
  const msp_camera c = a.cams[view];
  TileRect tr[kSetupFaces];
  unsigned long long area[kSetupFaces];
#pragma unroll
  for (int k = 0; k < kSetupFaces; ++k) {
    const int64_t f = ((int64_t)blockIdx.x * kSetupFaces + k) * blockDim.x + threadIdx.x;
    tr[k] = TileRect{0, -1, 0, -1};
    area[k] = 0;
    if (f < F) setup_face(a, c, view, f, tr[k], area[k]);
  }
  // footprint pixels of the drawn faces per group of 256 faces (statistics: the
  // coverage tests the pixels ask for); summed on the host when statistics are read
  __shared__ unsigned long long fsum[kSetupFaces][256 / MSP_WAVE];
#pragma unroll
  for (int k = 0; k < kSetupFaces; ++k) {
    unsigned long long s = area[k];
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if (lane_id() == 0) fsum[k][threadIdx.x / MSP_WAVE] = s;
  }
  // per-tile counts through the workgroup's tile table
  __shared__ int32_t tkey[kTableSlots];
  __shared__ uint32_t tcnt[kTableSlots];
  for (int i = threadIdx.x; i < kTableSlots; i += blockDim.x) {
    tkey[i] = -1;
    tcnt[i] = 0;
  }
  __syncthreads();
  if (threadIdx.x < kSetupFaces) {
    const int64_t groups = (F + 255) / 256;
    const int64_t g = (int64_t)blockIdx.x * kSetupFaces + threadIdx.x;
    unsigned long long t = 0;
    for (int w = 0; w < (int)(blockDim.x / MSP_WAVE); ++w) t += fsum[threadIdx.x][w];
    if (g < groups) a.fp_part[(int64_t)view * groups + g] = t;
  }
  uint32_t* cnt = a.tile_cnt + (int64_t)view * a.n_tiles;
#pragma unroll
  for (int k = 0; k < kSetupFaces; ++k)
    for (int ty = tr[k].ty0; ty <= tr[k].ty1; ++ty)
      for (int tx = tr[k].tx0; tx <= tr[k].tx1; ++tx) {
        const int32_t t = ty * a.ntx + tx;
        const int sl = table_insert(tkey, t);
        if (sl >= 0) atomicAdd(&tcnt[sl], 1u);
        else atomicAdd(&cnt[t], 1u);
      }
  __syncthreads();
  for (int i = threadIdx.x; i < kTableSlots; i += blockDim.x)
    if (tkey[i] >= 0) atomicAdd(&cnt[tkey[i]], tcnt[i]);
}

// attribute record (4 float4, view independent): (o0, o1, o2, id0) (p0, id1) (p1, id2) (p2, 0),
// the corner opacities, world positions and vertex ids; in RGB mode also the
// corner colours (3 float4): (r0, g0, b0, r1) (g1, b1, r2, g2) (b2, 0, 0, 0)
__global__ __launch_bounds__(256) void k_face_attr(RasterArgs a) {
  const int64_t F = a.n_faces, V = a.n_verts;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  int32_t id[3] = {a.idx[f], a.idx[F + f], a.idx[2 * F + f]};
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if ((uint64_t)id[k] >= (uint64_t)V) id[k] = 0;  // such faces are culled in setup and never drawn
  float4* r = a.attr + f * 4;
  r[0] = make_float4(a.opacity[id[0]], a.opacity[id[1]], a.opacity[id[2]], __int_as_float(id[0]));
  r[1] = make_float4(a.pos[id[0]], a.pos[V + id[0]], a.pos[2 * V + id[0]], __int_as_float(id[1]));
  r[2] = make_float4(a.pos[id[1]], a.pos[V + id[1]], a.pos[2 * V + id[1]], __int_as_float(id[2]));
  r[3] = make_float4(a.pos[id[2]], a.pos[V + id[2]], a.pos[2 * V + id[2]], 0.f);
  if (a.rgb && a.crec) {
    float4* c = a.crec + f * 3;
    c[0] = make_float4(a.rgb[id[0]], a.rgb[V + id[0]], a.rgb[2 * V + id[0]], a.rgb[id[1]]);
    c[1] = make_float4(a.rgb[V + id[1]], a.rgb[2 * V + id[1]], a.rgb[id[2]], a.rgb[V + id[2]]);
    c[2] = make_float4(a.rgb[2 * V + id[2]], 0.f, 0.f, 0.f);
  }
}

// ---------------------------------------------------------------------------
// emit: scatter keys into the tile segments
// ---------------------------------------------------------------------------
// Each thread takes kEmitFaces faces (a workgroup 2048 consecutive ones): the
// kernel is bound by the latency chain of a workgroup (footprint loads, table,
// barrier, reservation atomics, barrier, offsets, stores), so fewer, fuller
// workgroups finish it sooner (per 8-view 1080p step of 8M faces: 2.3 ms at
// one face per thread, 1.86 at two, 1.53 at four, 1.38 at eight, 1.95 at 16).
constexpr int kEmitFaces = 8;

__global__ __launch_bounds__(256) void k_emit(RasterArgs a) {
  if (*a.ovf & 3u) return;  // uniform: set before this launch
  const int view = blockIdx.y;
  const int64_t F = a.n_faces;
  TileRect r[kEmitFaces];
  uint64_t key[kEmitFaces];
#pragma unroll
  for (int k = 0; k < kEmitFaces; ++k) {
    const int64_t f = ((int64_t)blockIdx.x * kEmitFaces + k) * blockDim.x + threadIdx.x;
    r[k] = TileRect{0, -1, 0, -1};
    key[k] = 0;
    if (f < F) {
      const float4 g2 = a.geo[((int64_t)view * F + f) * 3 + 2];
      r[k] = tile_rect(a, g2);
      key[k] = ((uint64_t)__float_as_uint(g2.w) << 32) | (uint32_t)f;
    }
  }
  __shared__ int32_t tkey[kTableSlots];
  __shared__ uint32_t tcnt[kTableSlots];
  __shared__ uint32_t tbase[kTableSlots];
  for (int i = threadIdx.x; i < kTableSlots; i += blockDim.x) {
    tkey[i] = -1;
    tcnt[i] = 0;
  }
  __syncthreads();
  // 1: this workgroup's count per tile
#pragma unroll
  for (int k = 0; k < kEmitFaces; ++k)
    for (int ty = r[k].ty0; ty <= r[k].ty1; ++ty)
      for (int tx = r[k].tx0; tx <= r[k].tx1; ++tx) {
        const int sl = table_insert(tkey, ty * a.ntx + tx);
        if (sl >= 0) atomicAdd(&tcnt[sl], 1u);
      }
  __syncthreads();
  // 2: one reservation per tile in the tile's segment
  const int64_t tb = (int64_t)view * a.n_tiles;
  for (int i = threadIdx.x; i < kTableSlots; i += blockDim.x) {
    if (tkey[i] >= 0) tbase[i] = atomicAdd(&a.cursor[tb + tkey[i]], tcnt[i]);
    tcnt[i] = 0;
  }
  __syncthreads();
  // 3: every (face, tile) takes a slot of its workgroup's range (faces whose tile
  // did not fit the table reserve their slot on their own)
#pragma unroll
  for (int k = 0; k < kEmitFaces; ++k)
    for (int ty = r[k].ty0; ty <= r[k].ty1; ++ty)
      for (int tx = r[k].tx0; tx <= r[k].tx1; ++tx) {
        const int32_t t = ty * a.ntx + tx;
        const int sl = table_find(tkey, t);
        const uint32_t slot = sl >= 0 ? tbase[sl] + atomicAdd(&tcnt[sl], 1u) : atomicAdd(&a.cursor[tb + t], 1u);
        const int64_t p = a.tile_off[tb + t] + slot;
        if (p < a.tile_off[tb + t + 1] && p < a.key_cap) a.keys[p] = key[k];
      }
}

// ---------------------------------------------------------------------------
// tile_sort: per-tile ascending sort of 64-bit keys
// ---------------------------------------------------------------------------
// A chunk of up to kSortChunk keys is sorted by one workgroup: each thread
// sorts kSortItems keys in registers (bitonic network, no barriers), then runs
// of kSortItems, 2 kSortItems, ... are merged in LDS, every thread producing
// kSortItems outputs of its merge from a merge-path split. Lists longer than a
// chunk are chunk-sorted, then merged pairwise through global memory, one
// chunk of output at a time (split found by a cooperative search, both input
// ranges staged in LDS).
constexpr int kSortThreads = 512;
constexpr int kSortItems = 16;
constexpr int kSortChunk = kSortThreads * kSortItems;  // 8192 keys, 64 KiB (+ padding) of LDS
constexpr uint64_t kSentinel = ~0ull;                 // above every key (float bits of a finite z)

__device__ __forceinline__ int spad(int j) { return j + (j >> 5); }  // one pad word per 32 keys: no bank conflicts

__device__ __forceinline__ void sort_regs(uint64_t (&x)[kSortItems]) {
#pragma unroll
  for (int k = 2; k <= kSortItems; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < kSortItems; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const uint64_t u = x[i], v = x[l];
          const bool sw = ((i & k) == 0) ? (u > v) : (u < v);
          x[i] = sw ? v : u;
          x[l] = sw ? u : v;
        }
      }
}

// kSortItems outputs starting at merge-path diagonal `diag` of runs
// A = s[spad(oa + i)], i < na and B = s[spad(ob + j)], j < nb (A first on ties).
__device__ __forceinline__ void merge_lds(const uint64_t* s, int oa, int na, int ob, int nb, int diag,
                                          uint64_t (&x)[kSortItems]) {
  int lo = diag > nb ? diag - nb : 0, hi = diag < na ? diag : na;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (s[spad(oa + mid)] <= s[spad(ob + diag - 1 - mid)]) lo = mid + 1;
    else hi = mid;
  }
  int i = lo, j = diag - lo;
  uint64_t av = i < na ? s[spad(oa + i)] : kSentinel;
  uint64_t bv = j < nb ? s[spad(ob + j)] : kSentinel;
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const bool ta = av <= bv;
    x[k] = ta ? av : bv;
    if (ta) {
      ++i;
      av = i < na ? s[spad(oa + i)] : kSentinel;
    } else {
      ++j;
      bv = j < nb ? s[spad(ob + j)] : kSentinel;
    }
  }
}

// out[0, m) = in[0, m) sorted, m <= kSortChunk; in and out may be the same (all
// threads of the workgroup call it)
__device__ void sort_chunk(const uint64_t* in, uint64_t* out, int m, uint64_t* s) {
  const int t = threadIdx.x;
  int P = 1;  // threads in use: a power of two with P * kSortItems >= m
  while (P * kSortItems < m) P <<= 1;
  const int n = P * kSortItems;
  for (int j = t; j < n; j += kSortThreads) s[spad(j)] = j < m ? in[j] : kSentinel;
  __syncthreads();
  uint64_t x[kSortItems];
  if (t < P) {
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) x[i] = s[spad(t * kSortItems + i)];
    sort_regs(x);
  }
  for (int L = kSortItems; L < n; L <<= 1) {
    __syncthreads();
    if (t < P) {
#pragma unroll
      for (int i = 0; i < kSortItems; ++i) s[spad(t * kSortItems + i)] = x[i];
    }
    __syncthreads();
    if (t < P) {
      const int g = 2 * L / kSortItems;  // threads per merge
      const int base = (t / g) * 2 * L;
      merge_lds(s, base, L, base + L, L, (t % g) * kSortItems, x);
    }
  }
  __syncthreads();
  if (t < P) {
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) s[spad(t * kSortItems + i)] = x[i];
  }
  __syncthreads();
  for (int j = t; j < m; j += kSortThreads) out[j] = s[spad(j)];
  __syncthreads();
}

// merge-path split of diagonal d over global runs A (na) and B (nb): the number
// of A elements among the first d outputs. Cooperative: each round tests
// kSortThreads candidates, so two rounds cover 65536 positions.
__device__ int coop_split(const uint64_t* A, int64_t na, const uint64_t* B, int64_t nb, int64_t d, int64_t* sh) {
  const int t = threadIdx.x;
  int64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  while (hi > lo) {  // uniform
    const int64_t span = hi - lo;
    const int64_t m = lo + (span * t) / kSortThreads;  // candidates in [lo, hi)
    const bool below = A[m] <= B[d - 1 - m];             // true: the split is above m
    __syncthreads();
    if (t == 0) {
      sh[0] = lo;
      sh[1] = hi;
    }
    __syncthreads();
    if (below) atomicMax((unsigned long long*)&sh[0], (unsigned long long)(m + 1));
    else atomicMin((unsigned long long*)&sh[1], (unsigned long long)m);
    __syncthreads();
    lo = sh[0];
    hi = sh[1];
  }
  return (int)lo;
}

// out[0, cnt) = outputs [o0, o0 + cnt) of merging global runs A and B
__device__ void merge_chunk(const uint64_t* A, int64_t na, const uint64_t* B, int64_t nb, int64_t o0, int cnt,
                            uint64_t* out, uint64_t* s, int64_t* sh) {
  const int t = threadIdx.x;
  const int64_t a0 = coop_split(A, na, B, nb, o0, sh);
  const int64_t a1 = coop_split(A, na, B, nb, o0 + cnt, sh);
  const int la = (int)(a1 - a0), lb = cnt - la;
  const int64_t b0 = o0 - a0;
  for (int j = t; j < la; j += kSortThreads) s[spad(j)] = A[a0 + j];
  for (int j = t; j < lb; j += kSortThreads) s[spad(la + j)] = B[b0 + j];
  __syncthreads();
  uint64_t x[kSortItems];
  const bool busy = t * kSortItems < cnt;
  if (busy) merge_lds(s, 0, la, la, lb, t * kSortItems, x);
  __syncthreads();
  if (busy) {
#pragma unroll
    for (int i = 0; i < kSortItems; ++i)
      if (t * kSortItems + i < cnt) s[spad(t * kSortItems + i)] = x[i];
  }
  __syncthreads();
  for (int j = t; j < cnt; j += kSortThreads) out[j] = s[spad(j)];
  __syncthreads();
}

__global__ __launch_bounds__(kSortThreads) void k_tile_sort(RasterArgs a, int64_t n_seg) {
  __shared__ uint64_t s[kSortChunk + kSortChunk / 32];
  __shared__ int64_t sh[2];
  const int64_t seg = blockIdx.x;
  if (seg >= n_seg || (*a.ovf & 3u)) return;  // uniform
  const int64_t beg = a.tile_off[seg];
  const int64_t n = a.tile_off[seg + 1] - beg;
  if (n <= 1) return;
  // the merge passes alternate between the keys and tmp; with an odd number of
  // them the sorted chunks go to tmp, so that the last pass writes the keys
  int passes = 0;
  for (int64_t w = kSortChunk; w < n; w <<= 1) ++passes;
  uint64_t* const keys = a.keys + beg;
  uint64_t* src = (passes & 1) ? a.tmp + beg : keys;
  for (int64_t c0 = 0; c0 < n; c0 += kSortChunk)
    sort_chunk(keys + c0, src + c0, (int)(n - c0 < kSortChunk ? n - c0 : kSortChunk), s);
  if (n <= kSortChunk) return;
  uint64_t* dst = src == keys ? a.tmp + beg : keys;
  for (int64_t w = kSortChunk; w < n; w <<= 1) {
    for (int64_t s0 = 0; s0 < n; s0 += 2 * w) {
      const int64_t na = n - s0 < w ? n - s0 : w;
      const int64_t rest = n - s0 - na;
      const int64_t nb = rest < w ? rest : w;
      for (int64_t o0 = 0; o0 < na + nb; o0 += kSortChunk) {
        const int cnt = (int)(na + nb - o0 < kSortChunk ? na + nb - o0 : kSortChunk);
        if (nb == 0) {
          for (int j = threadIdx.x; j < cnt; j += kSortThreads) dst[s0 + o0 + j] = src[s0 + o0 + j];
        } else {
          merge_chunk(src + s0, na, src + s0 + na, nb, o0, cnt, dst + s0 + o0, s, sh);
        }
      }
    }
    __syncthreads();
    uint64_t* tswap = src;
    src = dst;
    dst = tswap;
  }
}

// ---------------------------------------------------------------------------
// composite forward / backward
// ---------------------------------------------------------------------------

// Staged face record (floats): 0 zmin | 1..3 edge 0 (e0, ex, ey) | 4..6 edge 1 |
// 7..9 edge 2 | 10..12 1/z of the corners | 13..15 corner opacities | 16 face id bits |
// 17..25 corner colours (r,g,b per corner) or the face colour in 17..19 | 26, 27 pad.
// Edge k is the one opposite corner k, oriented so that inside is >= 0 and
// evaluated relative to the centre of the block's first pixel.
struct Fetched {
  float4 g0, g1, g2;  // geometry record of the view
  float4 a0;          // corner opacities (and vertex id 0)
  float4 c0, c1, c2;  // colours: the corners' (RGB mode) or the face's for the view in c0 (SH mode)
};

__device__ __forceinline__ bool build_record(const Fetched& q, uint32_t f, float rx, float ry, float* R) {
#pragma clang fp contract(off)
  const float u[3] = {q.g0.x, q.g0.z, q.g1.x};
  const float v[3] = {q.g0.y, q.g0.w, q.g1.y};
  const float iz[3] = {q.g1.z, q.g1.w, q.g2.x};  // 1 / z of the corners
  const float area2 = (u[1] - u[0]) * (v[2] - v[0]) - (v[1] - v[0]) * (u[2] - u[0]);
  if (!(area2 != 0.f) || !isfinite(area2)) return false;
  const float sg = area2 > 0.f ? 1.f : -1.f;
  R[0] = q.g2.w;  // nearest depth (same bits as the sort key)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int ia = (k + 1) % 3, ib = (k + 2) % 3;
    const float du = u[ib] - u[ia], dv = v[ib] - v[ia];
    R[1 + 3 * k] = sg * (du * (ry - v[ia]) - dv * (rx - u[ia]));
    R[2 + 3 * k] = -sg * dv;
    R[3 + 3 * k] = sg * du;
    R[10 + k] = iz[k];
  }
  R[13] = q.a0.x;
  R[14] = q.a0.y;
  R[15] = q.a0.z;
  R[16] = __uint_as_float(f);
  R[17] = q.c0.x; R[18] = q.c0.y; R[19] = q.c0.z;
  R[20] = q.c0.w; R[21] = q.c1.x; R[22] = q.c1.y;
  R[23] = q.c1.z; R[24] = q.c1.w; R[25] = q.c2.x;
  R[26] = 0.f;
  R[27] = 0.f;
  return true;
}

// False when one edge function is negative at every pixel centre of the 8x8
// block (the face covers none of them). The largest value of a linear function
// over the block is at a corner; the test allows a relative 2^-20 of the
// terms' magnitudes for the rounding of the per-pixel evaluation, so it never
// drops a face that covers a pixel.
__device__ __forceinline__ bool meets_block(const float* R) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float e0 = R[1 + 3 * k], ex = R[2 + 3 * k], ey = R[3 + 3 * k];
    const float mx = e0 + fmaxf(ex, 0.f) * 7.f + fmaxf(ey, 0.f) * 7.f;
    const float tol = (fabsf(e0) + 7.f * fabsf(ex) + 7.f * fabsf(ey)) * 0x1p-20f;
    if (mx < -tol) return false;
  }
  return true;
}

// Edge functions of the pixel at block offset (dx, dy).
__device__ __forceinline__ void edges(const float* R, float dx, float dy, float& E0, float& E1, float& E2) {
  E0 = fmaf(R[3], dy, fmaf(R[2], dx, R[1]));
  E1 = fmaf(R[6], dy, fmaf(R[5], dx, R[4]));
  E2 = fmaf(R[9], dy, fmaf(R[8], dx, R[7]));
}

// Closed-edge coverage test (the first test pixel_eval makes).
__device__ __forceinline__ bool covers(const float* R, float dx, float dy) {
  float E0, E1, E2;
  edges(R, dx, dy, E0, E1, E2);
  return E0 >= 0.f && E1 >= 0.f && E2 >= 0.f;
}

// Coverage and perspective-correct barycentrics of the pixel at block offset (dx, dy).
__device__ __forceinline__ bool pixel_eval(const float* R, float dx, float dy, float& z, float& b0, float& b1,
                                           float& b2) {
#pragma clang fp contract(off)
  float E0, E1, E2;
  edges(R, dx, dy, E0, E1, E2);
  if (E0 < 0.f || E1 < 0.f || E2 < 0.f) return false;
  const float w0 = E0 * R[10], w1 = E1 * R[11], w2 = E2 * R[12];
  const float s = (w0 + w1) + w2;
  if (!(s > 0.f)) return false;
  const float inv = 1.f / s;
  b0 = w0 * inv;
  b1 = w1 * inv;
  b2 = w2 * inv;
  z = fmaxf(((E0 + E1) + E2) * inv, R[0]);
  return true;
}

__device__ __forceinline__ void frag_attr(const float* R, bool sh, float b0, float b1, float b2, float& raw,
                                          float& al, float& cr, float& cg, float& cb) {
#pragma clang fp contract(off)
  raw = (b0 * R[13] + b1 * R[14]) + b2 * R[15];
  al = fminf(fmaxf(raw, 0.f), 1.f);
  if (sh) {
    cr = R[17];
    cg = R[18];
    cb = R[19];
  } else {
    cr = (b0 * R[17] + b1 * R[20]) + b2 * R[23];
    cg = (b0 * R[18] + b1 * R[21]) + b2 * R[24];
    cb = (b0 * R[19] + b1 * R[22]) + b2 * R[25];
  }
}

__device__ __forceinline__ uint64_t mkkey(float z, uint32_t f) {
  return ((uint64_t)__float_as_uint(z) << 32) | f;
}

struct Item {
  int view, bx0, by0;
  int64_t seg;  // tile segment index
  int64_t blk;  // global 8x8 block index
};

__device__ __forceinline__ bool decode_item(const RasterArgs& a, uint32_t item, Item& it) {
  const int bpx = a.tile_w / 8, bpy = a.tile_h / 8;
  const int64_t per_view = a.n_tiles * bpx * bpy;
  it.view = (int)(item / per_view);
  const int64_t r = item - (int64_t)it.view * per_view;
  const int64_t tile = r / (bpx * bpy);
  const int sb = (int)(r - tile * (bpx * bpy));
  const int tx = (int)(tile % a.ntx), ty = (int)(tile / a.ntx);
  it.bx0 = tx * a.tile_w + (sb % bpx) * 8;
  it.by0 = ty * a.tile_h + (sb / bpx) * 8;
  it.seg = (int64_t)it.view * a.n_tiles + tile;
  const int nbx = (a.W + 7) / 8, nby = (a.H + 7) / 8;
  it.blk = ((int64_t)it.view * nby + it.by0 / 8) * nbx + it.bx0 / 8;
  return it.bx0 < a.W && it.by0 < a.H;
}


// XCD-aware work queues. The chip runs workgroups on eight XCDs, each with its
// own L2, and hands consecutive workgroups to the XCDs in turn. Work is split
// into eight queues by a spatial group g (queue g mod 8); a workgroup starts
// at queue blockIdx.x mod 8, so the items of one group (the blocks of one
// tile, which read the same tile list and face records) run on one XCD and
// share its L2. A workgroup whose queue is empty moves on to the next one, so
// the load stays balanced; placement affects speed only, never results.
// q8: eight counters; per_group items per group, n_groups groups; returns the
// item index group * per_group + k (k < per_group) or false when all are done.
__device__ __forceinline__ bool take_item(unsigned long long* q8, int64_t n_groups, uint32_t per_group, uint32_t home,
                                          uint32_t& qi, int lane, uint32_t& item) {
  while (qi < 8) {
    const uint32_t q = (home + qi) & 7u;
    const int64_t nq = (int64_t)q < n_groups ? ((n_groups - q + 7) / 8) * per_group : 0;
    uint32_t k = 0;
    if (lane == 0) k = (uint32_t)atomicAdd(&q8[q], 1ull);
    k = __shfl(k, 0);
    if ((int64_t)k < nq) {
      item = (uint32_t)(((int64_t)q + 8 * (int64_t)(k / per_group)) * per_group + k % per_group);
      return true;
    }
    ++qi;
  }
  return false;
}

// Per-lane ordering buffer in registers: up to KB fragments sorted by key
// (depth bits, face id), with alpha and (COL) the interpolated colour.
// Insertion is a compare-select network, popping a shift.
template <int KB, bool COL>
struct RegBuf {
  float z[KB];
  uint32_t f[KB];
  float al[KB], cr[KB], cg[KB], cb[KB];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      z[i] = __uint_as_float(0x7f800000u);
      f[i] = kEmpty;
    }
  }
  __device__ __forceinline__ void init() {
    clear();
#pragma unroll
    for (int i = 0; i < KB; ++i) al[i] = cr[i] = cg[i] = cb[i] = 0.f;
  }
  __device__ __forceinline__ bool empty() const { return f[0] == kEmpty; }
  __device__ __forceinline__ float front_z() const { return z[0]; }
  __device__ __forceinline__ uint32_t front_f() const { return f[0]; }
  __device__ __forceinline__ float front_al() const { return al[0]; }
  __device__ __forceinline__ uint64_t front_key() const { return mkkey(z[0], f[0]); }
  __device__ __forceinline__ void front_col(float& r, float& g, float& b) const {
    r = cr[0];
    g = cg[0];
    b = cb[0];
  }
  __device__ __forceinline__ void pop() {
#pragma unroll
    for (int i = 0; i < KB - 1; ++i) {
      z[i] = z[i + 1];
      f[i] = f[i + 1];
      al[i] = al[i + 1];
      if (COL) {
        cr[i] = cr[i + 1];
        cg[i] = cg[i + 1];
        cb[i] = cb[i + 1];
      }
    }
    z[KB - 1] = __uint_as_float(0x7f800000u);
    f[KB - 1] = kEmpty;
  }
  // inserts (nk, ...) in order; when full, the largest of buffer + new is
  // dropped and `drop` lowered to it
  __device__ __forceinline__ void insert(uint64_t nk, float zz, uint32_t fid, float a_, float r, float g, float b,
                                         uint64_t& drop) {
    const bool full = f[KB - 1] != kEmpty;
    const uint64_t lastk = mkkey(z[KB - 1], f[KB - 1]);
    if (full) drop = nk < lastk ? lastk : nk;
    if (full && nk > lastk) return;
    bool cpos[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) cpos[i] = nk < mkkey(z[i], f[i]);
#pragma unroll
    for (int i = KB - 1; i >= 1; --i) {
      const bool up = cpos[i - 1];
      const bool put = !up && cpos[i];
      z[i] = up ? z[i - 1] : (put ? zz : z[i]);
      f[i] = up ? f[i - 1] : (put ? fid : f[i]);
      al[i] = up ? al[i - 1] : (put ? a_ : al[i]);
      if (COL) {
        cr[i] = up ? cr[i - 1] : (put ? r : cr[i]);
        cg[i] = up ? cg[i - 1] : (put ? g : cg[i]);
        cb[i] = up ? cb[i - 1] : (put ? b : cb[i]);
      }
    }
    if (cpos[0]) {
      z[0] = zz;
      f[0] = fid;
      al[0] = a_;
      if (COL) {
        cr[0] = r;
        cg[0] = g;
        cb[0] = b;
      }
    }
  }
};

// Ordered traversal of one 8x8 block. MODE 0 composites into C/T; MODE 1
// records each composited fragment (face id, transmittance before it) into the
// block's list slab. Buf is the ordering buffer.
template <int KB, int MODE, bool SHP, class Buf>
__device__ void trace_block(const RasterArgs& a, const Item& it, float* slab, Buf& kb, int lane, float& T,
                            float& Cr, float& Cg, float& Cb, int& nf, uint32_t& restarts, uint2* list,
                            int64_t list_rows) {
  const int px = it.bx0 + (lane & 7), py = it.by0 + (lane >> 3);
  const bool valid = px < a.W && py < a.H;
  const int64_t beg = a.tile_off[it.seg];
  const int64_t n = a.tile_off[it.seg + 1] - beg;
  const float rx = (float)it.bx0 + 0.5f, ry = (float)it.by0 + 0.5f;
  const float dx = (float)(lane & 7), dy = (float)(lane >> 3);
  const bool sh = a.col4 != nullptr;
  const float eps = a.t_eps;

  kb.init();
  T = 1.f;
  Cr = Cg = Cb = 0.f;
  nf = 0;
  // SH colours are fetched when a fragment is composited and added one pop later,
  // so the load overlaps the work up to the next pop instead of stalling this one
  float pw = 0.f;
  float4 pc = make_float4(0.f, 0.f, 0.f, 0.f);
  uint64_t lo = 0, drop = ~0ull, last = 0;
  int state = valid ? ACTIVE : DONE;

  auto pop_front = [&]() {
    const uint32_t f0 = kb.front_f();
    const float al0 = kb.front_al();
    if (list != nullptr) {
      if (nf < list_rows) list[(int64_t)nf * MSP_WAVE + lane] = make_uint2(f0, __float_as_uint(T));
    }
    if (MODE == 0) {
      const float w = T * al0;
      if (SHP) {
        Cr = fmaf(pw, pc.x, Cr);
        Cg = fmaf(pw, pc.y, Cg);
        Cb = fmaf(pw, pc.z, Cb);
        pw = w;
        pc = a.col4[(int64_t)it.view * a.n_faces + f0];
      } else {
        float r, g, b;
        kb.front_col(r, g, b);
        Cr = fmaf(w, r, Cr);
        Cg = fmaf(w, g, Cg);
        Cb = fmaf(w, b, Cb);
      }
    }
    T = T * (1.f - al0);
    last = kb.front_key();
    ++nf;
    kb.pop();
  };
  // composite every buffered fragment (all keys below the drop threshold are final)
  auto flush_all = [&]() {
    while (!kb.empty() && T >= eps) pop_front();
    kb.clear();
  };

  while (__any(state != DONE)) {
    if (state == RESTART) {
      state = ACTIVE;
      lo = last;
      drop = ~0ull;
      ++restarts;
    }
    // keys run two chunks ahead and footprints one chunk ahead of the staging, so
    // the dependent loads overlap the processing of the current chunk
    const float4* geo_v = a.geo + (int64_t)it.view * a.n_faces * 3;
    uint64_t key_cur = lane < n ? a.keys[beg + lane] : ~0ull;
    uint64_t key_nxt = MSP_WAVE + lane < n ? a.keys[beg + MSP_WAVE + lane] : ~0ull;
    float4 fp_cur = geo_v[(int64_t)((uint64_t)(uint32_t)key_cur < (uint64_t)a.n_faces ? (uint32_t)key_cur : 0) * 3 + 2];
    for (int64_t base = 0; base < n; base += MSP_WAVE) {
      if (!__any(state == ACTIVE)) break;
      // ---- stage this chunk (ballot-compacted to faces meeting the block) ----
      const uint64_t key = key_cur;
      const float4 g2 = fp_cur;
      const uint32_t fk = (uint32_t)key;
      const bool ok = base + lane < n && (uint64_t)fk < (uint64_t)a.n_faces;
      // prefetch: footprints of the next chunk, keys of the one after
      const uint32_t fn = (uint32_t)key_nxt;
      fp_cur = geo_v[(int64_t)((uint64_t)fn < (uint64_t)a.n_faces ? fn : 0) * 3 + 2];
      key_cur = key_nxt;
      key_nxt = base + 2 * MSP_WAVE + lane < n ? a.keys[beg + base + 2 * MSP_WAVE + lane] : ~0ull;
      bool keep = false;
      float R[kRec];
      if (ok) {
        const uint32_t xr = __float_as_uint(g2.y), yr = __float_as_uint(g2.z);
        const int px0 = xr & 0xffff, px1 = xr >> 16, py0 = yr & 0xffff, py1 = yr >> 16;
        keep = px0 <= px1 && px0 <= it.bx0 + 7 && px1 >= it.bx0 && py0 <= it.by0 + 7 && py1 >= it.by0;
      }
      if (keep) {
        // full records only for the faces that meet this block
        Fetched q;
        const float4* gp = geo_v + (int64_t)fk * 3;
        q.g0 = gp[0];
        q.g1 = gp[1];
        q.g2 = g2;
        q.a0 = a.attr[(int64_t)fk * 4];
        if (a.col4) {
          q.c0 = a.col4[(int64_t)it.view * a.n_faces + fk];
          q.c1 = q.c2 = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
          const float4* cp = a.crec + (int64_t)fk * 3;
          q.c0 = cp[0];
          q.c1 = cp[1];
          q.c2 = cp[2];
        }
        keep = build_record(q, fk, rx, ry, R) && meets_block(R);
      }
      const uint64_t m = __ballot(keep);
      const int cnt = __popcll(m);
      if (keep) {
        float4* dst = reinterpret_cast<float4*>(slab + __popcll(m & lanemask_lt(lane)) * kRec);
#pragma unroll
        for (int q = 0; q < kRec / 4; ++q) dst[q] = make_float4(R[4 * q], R[4 * q + 1], R[4 * q + 2], R[4 * q + 3]);
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      // ---- coverage of this lane's pixel by every staged face (the edge tests
      // pixel_eval repeats, bit for bit), so that each lane walks only the
      // faces that cover it: a sliver face meets a handful of the 64 pixels ----
      uint64_t cov = 0;
      if (state == ACTIVE) {
        for (int j = 0; j < cnt; ++j)
          if (covers(slab + j * kRec, dx, dy)) cov |= 1ull << j;
      }
      // ---- each lane streams its covering faces in nearest-depth order; pops
      // owed to the faces it skips happen at its next covering face (whose
      // nearest depth is no smaller), which composites the same fragments ----
      while (cov) {
        const int j = __builtin_ctzll(cov);
        cov &= cov - 1;
        const float* S = slab + j * kRec;
        const float W = S[0];
        if (W > __uint_as_float((uint32_t)(drop >> 32))) {
          // everything below the drop threshold has been seen: finish it, then re-scan
          flush_all();
          state = RESTART;
          cov = 0;
          continue;
        }
        while (kb.front_z() < W && T >= eps) pop_front();
        if (T < eps) {
          state = DONE;
          cov = 0;
          continue;
        }
        float z, b0, b1, b2;
        if (!pixel_eval(S, dx, dy, z, b0, b1, b2)) continue;
        const uint32_t fid = __float_as_uint(S[16]);
        const uint64_t nk = mkkey(z, fid);
        if (!(nk > lo && nk < drop)) continue;
        float raw, al, cr, cg, cb;
        frag_attr(S, sh, b0, b1, b2, raw, al, cr, cg, cb);
        kb.insert(nk, z, fid, al, cr, cg, cb, drop);
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (state == ACTIVE) {
      flush_all();
      state = (T < eps || drop == ~0ull) ? DONE : RESTART;
    } else if (state == RESTART && T < eps) {
      state = DONE;
    }
  }
  if (MODE == 0 && SHP) {
    Cr = fmaf(pw, pc.x, Cr);
    Cg = fmaf(pw, pc.y, Cg);
    Cb = fmaf(pw, pc.z, Cb);
  }
}

template <int KB, bool SHP>
__device__ __forceinline__ void composite_items(const RasterArgs& a, uint32_t n_items, float* slab) {
  const int lane = lane_id();
  RegBuf<KB, !SHP> kb;  // with SH the colour comes from the face when a fragment is composited
  uint64_t frags = 0;
  uint32_t restarts = 0;
  if (*a.ovf & 3u) return;
  const uint32_t bpt = (uint32_t)((a.tile_w / 8) * (a.tile_h / 8));
  uint32_t qi = 0;
  for (;;) {
    uint32_t item = 0;
    if (!take_item(a.counters + 8, a.n_tiles * a.n_views, bpt, blockIdx.x & 7u, qi, lane, item)) break;
    if (item >= n_items) break;
    Item it;
    if (!decode_item(a, item, it)) continue;
    float T, Cr, Cg, Cb;
    int nf;
    uint2* list = a.store_rows ? a.frag_list + it.blk * a.store_rows * MSP_WAVE : nullptr;
    trace_block<KB, 0, SHP>(a, it, slab, kb, lane, T, Cr, Cg, Cb, nf, restarts, list, a.store_rows);
    if (a.store_rows) {
      // a block whose longest list does not fit is recomputed by the backward pass
      int mx = nf;
      for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d));
      if (lane == 0 && mx > a.store_rows) atomicOr(a.ovf, 4u);
    }
    const int px = it.bx0 + (lane & 7), py = it.by0 + (lane >> 3);
    if (px < a.W && py < a.H) {
      const int64_t plane = (int64_t)a.H * a.W;
      const int64_t o = (int64_t)it.view * 4 * plane + (int64_t)py * a.W + px;
      a.img[o] = Cr + T * a.bg0;
      a.img[o + plane] = Cg + T * a.bg1;
      a.img[o + 2 * plane] = Cb + T * a.bg2;
      a.img[o + 3 * plane] = 1.f - T;
      a.nfrag[(int64_t)it.view * plane + (int64_t)py * a.W + px] = nf;
      frags += (uint64_t)nf;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) frags += __shfl_xor(frags, d);
  if (lane == 0) {
    atomicAdd(&a.counters[0], (unsigned long long)frags);
    if (restarts) atomicAdd(&a.counters[1], (unsigned long long)restarts);
  }
}

// The SH kernel keeps only depth, id and alpha per buffer slot (the colour is
// fetched when a fragment is composited), which at a budget of 168 registers
// runs three waves per SIMD with a few spills: faster than two without. The
// RGB kernel keeps the interpolated colour per slot as well.
template <int KB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_composite_sh(RasterArgs a,
                                                                                            uint32_t n_items) {
  __shared__ float slabs[kWavesPerWG][MSP_WAVE * kRec];
  composite_items<KB, true>(a, n_items, slabs[threadIdx.x / MSP_WAVE]);
}

template <int KB>
__global__ __launch_bounds__(256) void k_composite_rgb(RasterArgs a, uint32_t n_items) {
  __shared__ float slabs[kWavesPerWG][MSP_WAVE * kRec];
  composite_items<KB, false>(a, n_items, slabs[threadIdx.x / MSP_WAVE]);
}

// per 8x8 block: the longest fragment list of its pixels (rows of the backward slab)
__global__ void k_block_max(RasterArgs a, int64_t n_blocks) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_blocks) return;
  const int nbx = (a.W + 7) / 8, nby = (a.H + 7) / 8;
  const int64_t view = b / ((int64_t)nbx * nby);
  const int64_t r = b - view * nbx * nby;
  const int by0 = (int)(r / nbx) * 8, bx0 = (int)(r % nbx) * 8;
  int mx = 0;
  const int64_t plane = (int64_t)a.H * a.W;
  for (int y = by0; y < by0 + 8 && y < a.H; ++y)
    for (int x = bx0; x < bx0 + 8 && x < a.W; ++x) {
      const int v = a.nfrag[view * plane + (int64_t)y * a.W + x];
      mx = v > mx ? v : mx;
    }
  a.blk_cap[b] = (uint32_t)mx;
}

// backward pass 1: recompute the ordered fragment lists. Like the SH composite
// it keeps depth, id and alpha per buffer slot, and at three waves per SIMD
// (a 168-register budget) it runs faster than at the two its 185 registers
// would give (9.7 against 12.7 ms per 8-view 1080p step of 343M fragments).
template <int KB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_bwd_lists(RasterArgs a,
                                                                                         uint32_t n_items) {
  __shared__ float slabs[kWavesPerWG][MSP_WAVE * kRec];
  const int lane = lane_id();
  float* slab = slabs[threadIdx.x / MSP_WAVE];
  RegBuf<KB, false> kb;  // lists record face ids and transmittance only
  uint32_t restarts = 0;
  if (*a.ovf & 3u) return;
  const uint32_t bpt = (uint32_t)((a.tile_w / 8) * (a.tile_h / 8));
  uint32_t qi = 0;
  for (;;) {
    uint32_t item = 0;
    if (!take_item(a.counters + 16, a.n_tiles * a.n_views, bpt, blockIdx.x & 7u, qi, lane, item)) break;
    if (item >= n_items) break;
    Item it;
    if (!decode_item(a, item, it)) continue;
    const int64_t row0 = a.blk_off[it.blk];
    const int64_t rows = a.blk_off[it.blk + 1] - row0;
    float T, Cr, Cg, Cb;
    int nf;
    trace_block<KB, 1, false>(a, it, slab, kb, lane, T, Cr, Cg, Cb, nf, restarts, a.frag_list + row0 * MSP_WAVE,
                              rows);
  }
}

// backward pass 2: back-to-front walk with per-wave LDS reduction of the face gradients.
// Table values per face: RGB mode: dop[3] | drgb[3 corners][3] | dpos[3 corners][3]
//                        SH mode:  dop[3] | dcol[3]            | dpos[3 corners][3]
// (positions in world space).
template <bool SH>
struct GradLayout {
  static constexpr int NV = SH ? 15 : 21;
  static constexpr int NS = SH ? 16 : 24;  // floats per face slot (whole float4s)
  static constexpr int COL = 3;
  static constexpr int POS = SH ? 6 : 12;
  // per-vertex entry: dop | (RGB: drgb[3]) | dpos world[3]
  static constexpr int VW = SH ? 4 : 7;
  static constexpr int VS = SH ? 4 : 8;   // floats per vertex slot (whole float4s)
  // vertex table slots (a wave's two tables fit three workgroups per CU in SH
  // mode, two in RGB mode), flushed above three quarters full
  static constexpr int VSLOTS = SH ? 224 : 160;
  static constexpr int VFILL = VSLOTS * 3 / 4;
};
constexpr int kVertBits = 8;  // slot bits of a vertex table index (VSLOTS <= 256)

// How a wave's sums reach global memory. ACC_F32: float atomics (the order of
// additions from different waves varies between runs). Deterministic mode runs
// the kernel twice: ACC_MAX finds, per value class, the largest magnitude any
// wave adds and how many values it adds; ACC_FIX then adds every value as a
// 64-bit fixed-point integer with a per-class scale 2^s chosen so that no sum
// can leave the integer range. Integer addition is associative, so the sums do
// not depend on the order of the atomics, and the per-wave sums that feed them
// are themselves computed in a fixed order (tables private to one wave).
enum : int { ACC_F32 = 0, ACC_MAX = 1, ACC_FIX = 2 };

struct DetTrack {
  float mx[DT_N];
  uint32_t n[DT_N];
  bool bad;
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int c = 0; c < DT_N; ++c) {
      mx[c] = 0.f;
      n[c] = 0u;
    }
    bad = false;
  }
};

// adds x to element kf of the float sums fp (ACC_F32; skipped when the caller
// asked for no such output) or to element ki of the fixed-point sums ip (ACC_FIX)
template <int ACC>
__device__ __forceinline__ void gadd(float* fp, int64_t kf, unsigned long long* ip, int64_t ki, int cls, float x,
                                     const RasterArgs& a, DetTrack& d) {
  if constexpr (ACC == ACC_F32) {
    if (fp) atomicAdd(fp + kf, x);
  } else if constexpr (ACC == ACC_MAX) {
    if (!isfinite(x)) d.bad = true;
    else d.mx[cls] = fmaxf(d.mx[cls], fabsf(x));
    d.n[cls] += 1u;
  } else {
    atomicAdd(ip + ki, (unsigned long long)__double2ll_rn((double)x * a.det_scale[cls]));
  }
}

// wave-wide maxima and counts of ACC_MAX, one atomic per wave and class
__device__ __forceinline__ void det_publish(const RasterArgs& a, DetTrack& d, int lane) {
#pragma unroll
  for (int c = 0; c < DT_N; ++c) {
    float m = d.mx[c];
    uint32_t n = d.n[c];
    for (int o = 32; o >= 1; o >>= 1) {
      m = fmaxf(m, __shfl_xor(m, o));
      n += __shfl_xor(n, o);
    }
    if (lane == 0 && n) {
      atomicMax(&a.det_max[c], __float_as_uint(m));
      atomicAdd(&a.det_cnt[c], (unsigned long long)n);
    }
  }
  if (__any(d.bad) && lane == 0) atomicOr(&a.det_max[DT_N], 1u);
}

// one vertex's values c[VW] into the global sums. Each value class is a plane of
// its own (dpos x, y, z, dop, drgb r, g, b), so the atomics of one flush go to
// separate cache lines instead of queueing on one line (putting a vertex's
// values side by side was measured slower).
template <bool SH, int ACC>
__device__ __forceinline__ void vert_global(const RasterArgs& a, int32_t v, const float* c, DetTrack& d) {
  using L = GradLayout<SH>;
  const int64_t V = a.n_verts;
  gadd<ACC>(a.dpos, v, a.acc64, v, DT_POS, c[L::VW - 3], a, d);
  gadd<ACC>(a.dpos, V + v, a.acc64, V + v, DT_POS, c[L::VW - 2], a, d);
  gadd<ACC>(a.dpos, 2 * V + v, a.acc64, 2 * V + v, DT_POS, c[L::VW - 1], a, d);
  gadd<ACC>(a.dop, v, a.acc64, 3 * V + v, DT_OP, c[0], a, d);
  if (!SH) {
    gadd<ACC>(a.drgb, v, a.acc64, 4 * V + v, DT_RGB, c[1], a, d);
    gadd<ACC>(a.drgb, V + v, a.acc64, 5 * V + v, DT_RGB, c[2], a, d);
    gadd<ACC>(a.drgb, 2 * V + v, a.acc64, 6 * V + v, DT_RGB, c[3], a, d);
  }
}

// A wave's face table has kHashSlots slots in blocks of 16; face f may sit only
// at offset f & 15 of a block (the first free one of its eight blocks, starting
// at a hash of f >> 4). The faces of a fan have consecutive ids, so those of one
// fan usually share a block and sit at neighbouring offsets: at a flush their
// shared vertices are then held by neighbouring lanes.
constexpr int kSlotBlocks = kHashSlots / 16;

// slot of face f in the wave's table (inserted if absent; the fill count grows), -1 if none
__device__ __forceinline__ int face_slot(uint32_t* keys, uint32_t* fill, uint32_t f) {
  const uint32_t b0 = ((f >> 4) * 0x9E3779B1u) >> (32 - 3);  // 3 bits: kSlotBlocks = 8
  static_assert(kSlotBlocks == 8, "block hash bits");
  for (int p = 0; p < kSlotBlocks; ++p) {
    const uint32_t s = (((b0 + p) & (kSlotBlocks - 1)) << 4) | (f & 15u);
    const uint32_t k = keys[s];
    if (k == f) return (int)s;
    if (k == kEmpty) {
      const uint32_t prev = atomicCAS(&keys[s], kEmpty, f);
      if (prev == kEmpty) atomicAdd(fill, 1u);
      if (prev == kEmpty || prev == f) return (int)s;
    }
  }
  return -1;
}

// Per-wave vertex table: a flush of the face table pours its faces' vertex
// entries in here, so a vertex that faces flushed at different times share
// (the centre of a fan above all) costs one set of global atomics per table
// lifetime instead of one per face.
template <bool SH>
struct VertTable {
  uint32_t* keys;
  float* vals;
  uint32_t* fill;
};

// slot of vertex v (inserted if absent; the fill count grows), -1 if none within the probe limit
template <bool SH>
__device__ __forceinline__ int vert_slot(const VertTable<SH>& t, uint32_t v) {
  using L = GradLayout<SH>;
  uint32_t s = (uint32_t)(((uint64_t)(v * 0x9E3779B1u) * (uint32_t)L::VSLOTS) >> 32);
  for (int p = 0; p < 16; ++p) {
    const uint32_t k = t.keys[s];
    if (k == v) return (int)s;
    if (k == kEmpty) {
      const uint32_t prev = atomicCAS(&t.keys[s], kEmpty, v);
      if (prev == kEmpty) atomicAdd(t.fill, 1u);
      if (prev == kEmpty || prev == v) return (int)s;
    }
    s = s + 1 == (uint32_t)L::VSLOTS ? 0u : s + 1;
  }
  return -1;
}

// rank of this lane among the lanes of the wave that hold the same slot (got),
// lower lanes first; -1 without a slot. Whole wave.
template <int BITS>
__device__ __forceinline__ int slot_rank(bool got, int slot, int lane) {
  uint64_t same = __ballot(got);
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const bool bit = got && ((slot >> b) & 1);
    const uint64_t bbm = __ballot(bit);
    same &= bit ? bbm : ~bbm;
  }
  return got ? (int)__popcll(same & lanemask_lt(lane)) : -1;
}

// adds the vertex entries c of the lanes with `want` set to vertex v in the
// wave's vertex table: lanes that share a slot update it in turn, by rank (plain
// reads and writes, no LDS float atomics); a lane that finds no slot adds its
// entry to global memory. Whole wave.
template <bool SH, int ACC>
__device__ __forceinline__ void vert_put(const RasterArgs& a, const VertTable<SH>& t, bool want, int32_t v,
                                         const float* c, int lane, DetTrack& d) {
  using L = GradLayout<SH>;
  const int slot = want ? vert_slot(t, (uint32_t)v) : -1;
  const bool got = slot >= 0;
  if (want && !got) vert_global<SH, ACC>(a, v, c, d);
  const int rank = slot_rank<kVertBits>(got, slot, lane);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  for (int r = 0; __any(rank >= r); ++r) {
    if (rank == r) {
      float4* p4 = reinterpret_cast<float4*>(t.vals + slot * L::VS);
#pragma unroll
      for (int q = 0; q < L::VS / 4; ++q) {
        float4 x = p4[q];
        if (4 * q < L::VW) x.x += c[4 * q];
        if (4 * q + 1 < L::VW) x.y += c[4 * q + 1];
        if (4 * q + 2 < L::VW) x.z += c[4 * q + 2];
        if (4 * q + 3 < L::VW) x.w += c[4 * q + 3];
        p4[q] = x;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  }
}

// empties the wave's vertex table into the global sums
template <bool SH, int ACC>
__device__ __forceinline__ void flush_verts(const RasterArgs& a, const VertTable<SH>& t, int lane, DetTrack& d) {
  using L = GradLayout<SH>;
  for (int sl = lane; sl < L::VSLOTS; sl += MSP_WAVE) {
    const uint32_t v = t.keys[sl];
    if (v == kEmpty) continue;
    float c[L::VS];
    float4* p4 = reinterpret_cast<float4*>(t.vals + sl * L::VS);
#pragma unroll
    for (int q = 0; q < L::VS / 4; ++q) {
      const float4 x = p4[q];
      c[4 * q] = x.x;
      c[4 * q + 1] = x.y;
      c[4 * q + 2] = x.z;
      c[4 * q + 3] = x.w;
      p4[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    t.keys[sl] = kEmpty;
    vert_global<SH, ACC>(a, (int32_t)v, c, d);
  }
  if (lane == 0) *t.fill = 0;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
}

// lane i receives lane i - d's value (lanes below d: their own)
__device__ __forceinline__ float lane_up(float x, int d) { return __shfl_up(x, d); }
__device__ __forceinline__ int lane_up(int x, int d) { return __shfl_up(x, d); }
__device__ __forceinline__ int lane_down(int x, int d) { return __shfl_down(x, d); }

// Empties the wave's face table: per face its view's colour gradient (SH) to
// global memory and three vertex entries to the vertex table. Lane l takes slots
// l and l + 64.
// Vertex entries of neighbouring lanes that name the same vertex are combined
// first: the second corner of lane l - 1 into the first corner of lane l (the
// boundary vertex two neighbouring fan faces share), and the centres by a
// segmented scan over runs of equal centre ids; each run adds its centre once.
// The combination order is fixed, so the sums are the same on every run.
template <bool SH, int ACC>
__device__ __forceinline__ void flush_table(const RasterArgs& a, int view, uint32_t* keys, float* vals,
                                            uint32_t* fill, const VertTable<SH>& vt, int lane, DetTrack& d) {
  using L = GradLayout<SH>;
  for (int it = 0; it < kHashSlots / MSP_WAVE; ++it) {
    const int s = it * MSP_WAVE + lane;
    const uint32_t f = keys[s];
    float v[L::NS];
    float4* v4 = reinterpret_cast<float4*>(vals + s * L::NS);
#pragma unroll
    for (int q = 0; q < L::NS / 4; ++q) {
      const float4 x = v4[q];
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
      v4[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    keys[s] = kEmpty;
    int id[3] = {-1, -1, -1};
    if (f != kEmpty) {
      const float4* r = a.attr + (int64_t)f * 4;
      id[0] = __float_as_int(r[0].w);
      id[1] = __float_as_int(r[1].w);
      id[2] = __float_as_int(r[2].w);
      if (SH) {
        // the view's colour gradient of the face, planes [view][channel][F]
        const int64_t o = (int64_t)view * 3 * a.n_faces + f;
        gadd<ACC>(a.dcol, o, a.dcol64, o, DT_COL, v[3], a, d);
        gadd<ACC>(a.dcol, o + a.n_faces, a.dcol64, o + a.n_faces, DT_COL, v[4], a, d);
        gadd<ACC>(a.dcol, o + 2 * a.n_faces, a.dcol64, o + 2 * a.n_faces, DT_COL, v[5], a, d);
      }
    }
    // corner entries: dop | (RGB: drgb[3]) | dpos[3]; an empty slot holds zeros
    float c[3][L::VW];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      c[k][0] = v[k];
      if (!SH) {
        c[k][1] = v[L::COL + 3 * k];
        c[k][2] = v[L::COL + 3 * k + 1];
        c[k][3] = v[L::COL + 3 * k + 2];
      }
      c[k][L::VW - 3] = v[L::POS + 3 * k];
      c[k][L::VW - 2] = v[L::POS + 3 * k + 1];
      c[k][L::VW - 1] = v[L::POS + 3 * k + 2];
    }
    // Every lane exchange runs with all lanes active: a shuffle inside a
    // short-circuited condition would execute under a partial exec mask, and
    // reads from inactive lanes return 0.
    const int id2p = lane_up(id[2], 1);
    const int id1n = lane_down(id[1], 1);
    const int id0p = lane_up(id[0], 1);
    const int id0n = lane_down(id[0], 1);
    // boundary: the previous lane's second corner joins this lane's first corner
    const bool take = lane > 0 && id[1] >= 0 && id2p == id[1];
    const bool gave = lane < MSP_WAVE - 1 && id[2] >= 0 && id1n == id[2];
#pragma unroll
    for (int q = 0; q < L::VW; ++q) {
      const float x = lane_up(c[2][q], 1);
      if (take) c[1][q] += x;
    }
    // centres: inclusive scan within runs of equal centre ids (head = first lane of a run)
    int head = (lane == 0 || id0p != id[0]) ? 1 : 0;
    const bool tail = lane == MSP_WAVE - 1 || id0n != id[0];
#pragma unroll
    for (int dd = 1; dd < MSP_WAVE; dd <<= 1) {
      const int hp = lane_up(head, dd);
      float xp[L::VW];
#pragma unroll
      for (int q = 0; q < L::VW; ++q) xp[q] = lane_up(c[0][q], dd);
      if (lane >= dd) {
        if (!head) {
#pragma unroll
          for (int q = 0; q < L::VW; ++q) c[0][q] = xp[q] + c[0][q];
        }
        head |= hp;
      }
    }
    vert_put<SH, ACC>(a, vt, id[0] >= 0 && tail, id[0], c[0], lane, d);
    vert_put<SH, ACC>(a, vt, id[1] >= 0, id[1], c[1], lane, d);
    vert_put<SH, ACC>(a, vt, id[2] >= 0 && !gave, id[2], c[2], lane, d);
    if (*vt.fill > (uint32_t)L::VFILL) flush_verts<SH, ACC>(a, vt, lane, d);
  }
  if (lane == 0) *fill = 0;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
}

// One step of a segmented merge across lanes: lane l and its DPP partner
// (l ^ D for the given control) that both still hold values of the same face
// combine them in the lane with bit D clear; the other lane drops out. Must be
// executed by the whole wave (DPP reads the partner's registers); the values
// move only if some pair matches.
template <int CTRL, int D, int NV>
__device__ __forceinline__ void merge_step(uint32_t f, bool& alive, float (&val)[NV], int lane) {
  const uint32_t fp = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, CTRL, 0xf, 0xf, false);
  const int ap = __builtin_amdgcn_mov_dpp(alive ? 1 : 0, CTRL, 0xf, 0xf, false);
  const bool same = alive && ap != 0 && fp == f;
  if (!__any(same)) return;
  const bool take = same && (lane & D) == 0;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const float vp = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(val[q]), CTRL, 0xf, 0xf, false));
    val[q] = take ? val[q] + vp : val[q];
  }
  if (same && (lane & D) != 0) alive = false;
}

// The adjoint's geometry is computed in float64 from the faces' float32 world
// corners: the pixel ray (camera centre o, direction D = R^-1 d_cam, both from
// the host in double) is intersected with the face plane by Moller-Trumbore,
// giving the barycentrics b = (1 - u - v, u, v) and the Jacobian of (u, v)
// with respect to the corners. A face seen nearly edge-on makes both
// ill-conditioned (the determinant is proportional to the cosine between the
// face normal and the ray); the float32 rounding of its corners' projections
// would then be amplified by 1 / |cos|, double precision keeps it below 1e-12.
template <bool SH, int ACC>
__global__ __launch_bounds__(256) void k_bwd_grads(RasterArgs a, uint32_t n_items) {
  using L = GradLayout<SH>;
  // [slot][value]: one face's values side by side, NS floats apart (16-byte aligned slots)
  __shared__ __align__(16) float hvals[kWavesPerWG][L::NS * kHashSlots];
  __shared__ __align__(16) float vvals[kWavesPerWG][L::VS * L::VSLOTS];
  __shared__ uint32_t hkeys[kWavesPerWG][kHashSlots];
  __shared__ uint32_t vkeys[kWavesPerWG][L::VSLOTS];
  __shared__ uint32_t hfill[kWavesPerWG];
  __shared__ uint32_t vfill[kWavesPerWG];
  const int lane = lane_id();
  const int wid = threadIdx.x / MSP_WAVE;
  uint32_t* keys = hkeys[wid];
  float* vals = hvals[wid];
  uint32_t* fill = &hfill[wid];
  const VertTable<SH> vt{vkeys[wid], vvals[wid], &vfill[wid]};
  DetTrack dt;
  dt.init();
  for (int s = lane; s < kHashSlots; s += MSP_WAVE) keys[s] = kEmpty;
  for (int s = lane; s < L::NS * kHashSlots; s += MSP_WAVE) vals[s] = 0.f;
  for (int s = lane; s < L::VSLOTS; s += MSP_WAVE) vt.keys[s] = kEmpty;
  for (int s = lane; s < L::VS * L::VSLOTS; s += MSP_WAVE) vt.vals[s] = 0.f;
  if (lane == 0) {
    *fill = 0;
    *vt.fill = 0;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  if (*a.ovf & (a.store_rows ? 7u : 3u)) return;
  const int nbx = (a.W + 7) / 8, nby = (a.H + 7) / 8;
  const int nrx = (nbx + 1) / 2, nry = (nby + 1) / 2;
  // queue groups: 4x4 regions (64x64 pixels) of one view, whose regions share face records
  const int nsx = (nrx + 3) / 4, nsy = (nry + 3) / 4;
  const int64_t n_groups = (int64_t)nsx * nsy * a.n_views;
  const int64_t F = a.n_faces;
  uint32_t qi = 0;
  for (;;) {
    // work item: a 2x2 group of 8x8 blocks of one view; the tables persist over the group
    uint32_t item = 0;
    if (!take_item(a.counters + 24, n_groups, 16u, blockIdx.x & 7u, qi, lane, item)) break;
    const uint32_t grp = item / 16u, sub16 = item % 16u;
    const int view = (int)(grp / ((uint32_t)nsx * nsy));
    const int gr = (int)(grp - (uint32_t)view * nsx * nsy);
    const int rx = (gr % nsx) * 4 + (int)(sub16 & 3u), ry = (gr / nsx) * 4 + (int)(sub16 >> 2);
    if (view >= a.n_views || rx >= nrx || ry >= nry) continue;
    const msp_camera c = a.cams[view];
    const double* cd = a.camd + (int64_t)view * 12;  // camera centre (3), R^-1 row-major (9)
    const double Ox = cd[0], Oy = cd[1], Oz = cd[2];
    for (int sub = 0; sub < 4; ++sub) {
    const int bx = 2 * rx + (sub & 1), by = 2 * ry + (sub >> 1);
    if (bx >= nbx || by >= nby) continue;
    const int64_t blk = ((int64_t)view * nby + by) * nbx + bx;
    int64_t row0, rows;
    if (a.store_rows) {
      row0 = blk * a.store_rows;
      rows = a.store_rows;
    } else {
      row0 = a.blk_off[blk];
      rows = a.blk_off[blk + 1] - row0;
    }
    const uint2* list = a.frag_list + row0 * MSP_WAVE;
    const int px = bx * 8 + (lane & 7), py = by * 8 + (lane >> 3);
    const bool valid = px < a.W && py < a.H;
    const int64_t plane = (int64_t)a.H * a.W;
    int nf = 0;
    float gr_ = 0.f, gg = 0.f, gb = 0.f, gA = 0.f;
    if (valid) {
      nf = a.nfrag[(int64_t)view * plane + (int64_t)py * a.W + px];
      if (nf > rows) nf = (int)rows;
      const int64_t o = (int64_t)view * 4 * plane + (int64_t)py * a.W + px;
      gr_ = a.dimg[o];
      gg = a.dimg[o + plane];
      gb = a.dimg[o + 2 * plane];
      gA = a.dimg[o + 3 * plane];
    }
    // this pixel's ray in world space: D = R^-1 ((px + 1/2 - cx) / fx, (py + 1/2 - cy) / fy, 1)
    const double dcx = ((double)px + 0.5 - (double)c.cx) / (double)c.fx;
    const double dcy = ((double)py + 0.5 - (double)c.cy) / (double)c.fy;
    const double Dx = cd[3] * dcx + cd[4] * dcy + cd[5];
    const double Dy = cd[6] * dcx + cd[7] * dcy + cd[8];
    const double Dz = cd[9] * dcx + cd[10] * dcy + cd[11];
    float Sr = a.bg0, Sg = a.bg1, Sb = a.bg2, P = 1.f;
    int maxn = nf;
    for (int d = 32; d >= 1; d >>= 1) maxn = max(maxn, __shfl_xor(maxn, d));
    // Each lane walks its own list back to front from its own last fragment, so
    // the pixels a large face covers reach it at different steps (their list
    // lengths differ) instead of all at once: fewer same-address LDS atomics.
    // the list entry of the next step is loaded one step ahead, so that its latency
    // overlaps the current step's record loads instead of adding to them
    uint2 e_next = nf > 0 ? list[(int64_t)(nf - 1) * MSP_WAVE + lane] : make_uint2(kEmpty, 0u);
    for (int t = 0; t < maxn; ++t) {
      bool act = t < nf;
      float val[L::NV];
      uint32_t f = kEmpty;
      const uint2 e = e_next;
      if (t + 1 < nf) e_next = list[(int64_t)(nf - 2 - t) * MSP_WAVE + lane];
      if (act) {
        f = e.x;
        const float Ti = __uint_as_float(e.y);
        act = (uint64_t)f < (uint64_t)F;
        const float4* r = a.attr + (int64_t)(act ? f : 0u) * 4;
        const float4 A0 = r[0], P0 = r[1], P1 = r[2], P2 = r[3];
        float4 C0, C1 = make_float4(0.f, 0.f, 0.f, 0.f), C2 = C1;
        if (SH) {
          C0 = a.col4[(int64_t)view * F + (act ? f : 0u)];
        } else {
          const float4* cp = a.crec + (int64_t)(act ? f : 0u) * 3;
          C0 = cp[0];
          C1 = cp[1];
          C2 = cp[2];
        }
        // Moller-Trumbore in double: e1 = p1 - p0, e2 = p2 - p0, s = o - p0,
        // pv = D x e2, det = e1 . pv, u = s . pv / det, v = D . (s x e1) / det
        const double e1x = (double)P1.x - P0.x, e1y = (double)P1.y - P0.y, e1z = (double)P1.z - P0.z;
        const double e2x = (double)P2.x - P0.x, e2y = (double)P2.y - P0.y, e2z = (double)P2.z - P0.z;
        const double sx = Ox - P0.x, sy = Oy - P0.y, sz = Oz - P0.z;
        const double pvx = Dy * e2z - Dz * e2y, pvy = Dz * e2x - Dx * e2z, pvz = Dx * e2y - Dy * e2x;
        const double det = e1x * pvx + e1y * pvy + e1z * pvz;
        // a zero determinant (the ray in the face's plane) cannot come from a drawn
        // fragment of a non-degenerate face; such a fragment is left out
        if (act) act = det != 0.0 && isfinite(det);
        if (act) {
          // 1 / det: the hardware reciprocal refined by two Newton steps (relative error near 2^-52)
          double inv = __builtin_amdgcn_rcp(det);
          inv = fma(inv, fma(-det, inv, 1.0), inv);
          inv = fma(inv, fma(-det, inv, 1.0), inv);
          const double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
          const double uu = (sx * pvx + sy * pvy + sz * pvz) * inv;
          const double vv = (Dx * qx + Dy * qy + Dz * qz) * inv;
          const float b0 = (float)(1.0 - uu - vv), b1 = (float)uu, b2 = (float)vv;
          float raw, al, cr, cg, cb;
          {
#pragma clang fp contract(off)
            raw = (b0 * A0.x + b1 * A0.y) + b2 * A0.z;
            al = fminf(fmaxf(raw, 0.f), 1.f);
            if (SH) {
              cr = C0.x;
              cg = C0.y;
              cb = C0.z;
            } else {
              cr = (b0 * C0.x + b1 * C0.w) + b2 * C1.z;
              cg = (b0 * C0.y + b1 * C1.x) + b2 * C1.w;
              cb = (b0 * C0.z + b1 * C1.y) + b2 * C2.x;
            }
          }
          const float wgt = Ti * al;
          const float dcr = gr_ * wgt, dcg = gg * wgt, dcb = gb * wgt;
          const float dal = Ti * (gr_ * (cr - Sr) + gg * (cg - Sg) + gb * (cb - Sb)) + gA * Ti * P;
          Sr = al * cr + (1.f - al) * Sr;
          Sg = al * cg + (1.f - al) * Sg;
          Sb = al * cb + (1.f - al) * Sb;
          P = (1.f - al) * P;
          const float dalr = (raw > 0.f && raw < 1.f) ? dal : 0.f;
          const float bb[3] = {b0, b1, b2};
          float dLdb[3];
          dLdb[0] = A0.x * dalr;
          dLdb[1] = A0.y * dalr;
          dLdb[2] = A0.z * dalr;
          if (!SH) {
            dLdb[0] += C0.x * dcr + C0.y * dcg + C0.z * dcb;
            dLdb[1] += C0.w * dcr + C1.x * dcg + C1.y * dcb;
            dLdb[2] += C1.z * dcr + C1.w * dcg + C2.x * dcb;
          }
#pragma unroll
          for (int qq = 0; qq < 3; ++qq) val[qq] = bb[qq] * dalr;
          if (SH) {
            val[3] = dcr;
            val[4] = dcg;
            val[5] = dcb;
          } else {
#pragma unroll
            for (int qq = 0; qq < 3; ++qq) {
              val[L::COL + 3 * qq] = bb[qq] * dcr;
              val[L::COL + 3 * qq + 1] = bb[qq] * dcg;
              val[L::COL + 3 * qq + 2] = bb[qq] * dcb;
            }
          }
          // dL/dp_k = -b_k y with y = (g_u (D x e2) + g_v (e1 x D)) / det, the
          // solution of [-D, e1, e2]^T y = (0, g_u, g_v)
          const double gu = (double)dLdb[1] - dLdb[0], gv = (double)dLdb[2] - dLdb[0];
          const double cxx = e1y * Dz - e1z * Dy, cxy = e1z * Dx - e1x * Dz, cxz = e1x * Dy - e1y * Dx;
          const float w0 = (float)((gu * pvx + gv * cxx) * inv);
          const float w1 = (float)((gu * pvy + gv * cxy) * inv);
          const float w2 = (float)((gu * pvz + gv * cxz) * inv);
#pragma unroll
          for (int qq = 0; qq < 3; ++qq) {
            val[L::POS + 3 * qq] = -bb[qq] * w0;
            val[L::POS + 3 * qq + 1] = -bb[qq] * w1;
            val[L::POS + 3 * qq + 2] = -bb[qq] * w2;
          }
        }
      }
      // Accumulate into the wave's table. LDS float atomics run one lane at a
      // time, so lanes of neighbouring pixels that hold the same face first merge
      // their values through DPP moves (x neighbours, then x+2, then y neighbours).
      if (*fill > (uint32_t)kHashFill) flush_table<SH, ACC>(a, view, keys, vals, fill, vt, lane, dt);
      if (!act) {
#pragma unroll
        for (int qq = 0; qq < L::NV; ++qq) val[qq] = 0.f;
      }
      merge_step<0xB1, 1, L::NV>(f, act, val, lane);   // quad_perm [1,0,3,2]: lane ^ 1
      merge_step<0x4E, 2, L::NV>(f, act, val, lane);   // quad_perm [2,3,0,1]: lane ^ 2
      merge_step<0x128, 8, L::NV>(f, act, val, lane);  // row_ror:8: lane ^ 8 within 16 lanes
      // Slots for the remaining lanes, then plain read-add-write instead of LDS
      // float atomics: the lanes that share a slot are ranked once (one ballot
      // per slot bit; lower lanes first) and update it in rounds, rank r in
      // round r. Lanes that found no slot retry after a flush, which empties the
      // table so that every face finds a slot.
      bool pend = act;
      for (;;) {
        const int slot = pend ? face_slot(keys, fill, f) : -1;
        const bool got = pend && slot >= 0;
        const int rank = slot_rank<kHashBits>(got, slot, lane);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        for (int r = 0; __any(rank >= r); ++r) {
          if (rank == r) {
            float4* p4 = reinterpret_cast<float4*>(vals + slot * L::NS);
#pragma unroll
            for (int q = 0; q < L::NS / 4; ++q) {
              float4 x = p4[q];
              if (4 * q < L::NV) x.x += val[4 * q];
              if (4 * q + 1 < L::NV) x.y += val[4 * q + 1];
              if (4 * q + 2 < L::NV) x.z += val[4 * q + 2];
              if (4 * q + 3 < L::NV) x.w += val[4 * q + 3];
              p4[q] = x;
            }
          }
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        }
        pend = pend && !got;
        if (!__any(pend)) break;
        flush_table<SH, ACC>(a, view, keys, vals, fill, vt, lane, dt);
      }
    }
    }  // sub-block
    flush_table<SH, ACC>(a, view, keys, vals, fill, vt, lane, dt);
    flush_verts<SH, ACC>(a, vt, lane, dt);
  }
  if constexpr (ACC == ACC_MAX) det_publish(a, dt, lane);
}

// Deterministic mode: per class c the scale 2^s with max |value| <= 2^e_M and
// count <= 2^e_N, s = 62 - e_M - e_N, so every partial sum stays below 2^62 in
// magnitude. Classes with a non-finite value get scale 0 (their outputs become NaN).
__global__ void k_det_scales(const uint32_t* det_max, const unsigned long long* det_cnt, double* scale, int c0, int c1) {
  const int c = c0 + (int)threadIdx.x;
  if (c >= c1) return;
  if (det_max[DT_N] & 1u) {
    scale[c] = 0.0;
    scale[DT_N + c] = __longlong_as_double(0x7ff8000000000000ll);
    return;
  }
  const float M = __uint_as_float(det_max[c]);
  const unsigned long long N = det_cnt[c];
  if (!(M > 0.f) || N == 0) {
    scale[c] = 1.0;
    scale[DT_N + c] = 1.0;
    return;
  }
  int eM = 0;
  (void)frexpf(M, &eM);  // M < 2^eM
  int eN = 0;
  while (eN < 63 && (1ull << eN) < N) ++eN;  // N <= 2^eN
  const int s = 62 - eM - eN;
  scale[c] = ldexp(1.0, s);
  scale[DT_N + c] = ldexp(1.0, -s);
}

__device__ __forceinline__ float det_value(unsigned long long x, double inv) {
  return (float)((double)(long long)x * inv);
}

// SH mode: the fixed-point colour gradients -> float [views][3][F] for the SH adjoint
__global__ __launch_bounds__(256) void k_dcol_finalize(const unsigned long long* __restrict__ dcol64, int64_t n,
                                                       const double* __restrict__ scale, float* dcol) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dcol[i] = det_value(dcol64[i], scale[DT_N + DT_COL]);
}

// Deterministic mode: fixed-point vertex sums (planes dpos x, y, z, dop, drgb r, g, b)
// -> the caller's gradients; the SH adjoint's position terms (their own class and
// planes) are added last.
__global__ __launch_bounds__(256) void k_det_finalize(const unsigned long long* __restrict__ acc64,
                                                      const unsigned long long* __restrict__ accsh64,
                                                      const double* __restrict__ scale, int64_t V, float* dpos,
                                                      float* dop, float* drgb) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const double ip = scale[DT_N + DT_POS], io = scale[DT_N + DT_OP], ir = scale[DT_N + DT_RGB];
  if (dpos) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float x = det_value(acc64[c * V + v], ip);
      if (accsh64) x += det_value(accsh64[c * V + v], scale[DT_N + DT_SHPOS]);
      dpos[c * V + v] = x;
    }
  }
  if (dop) dop[v] = det_value(acc64[3 * V + v], io);
  if (drgb) {
#pragma unroll
    for (int c = 0; c < 3; ++c) drgb[c * V + v] = det_value(acc64[(4 + c) * V + v], ir);
  }
}

__global__ void k_cap_guard(const int64_t* total, int64_t cap, uint32_t* flag, uint32_t bit) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && *total > cap) atomicOr(flag, bit);
}

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

template <class K>
int persistent_grid(K kernel, int n_cu, uint32_t n_items) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  int64_t g = (int64_t)n_cu * per_cu;
  const int64_t need = ((int64_t)n_items + kWavesPerWG - 1) / kWavesPerWG;
  if (g > need) g = need;
  return (int)(g < 1 ? 1 : g);
}

uint32_t n_items_of(const RasterArgs& a) {
  return (uint32_t)(a.n_tiles * (a.tile_w / 8) * (a.tile_h / 8) * a.n_views);
}

}  // namespace

hipError_t launch_cap_guard(hipStream_t s, const int64_t* total, int64_t cap, uint32_t* flag, uint32_t bit) {
  hipLaunchKernelGGL(k_cap_guard, dim3(1), dim3(64), 0, s, total, cap, flag, bit);
  return hipGetLastError();
}

hipError_t launch_setup(hipStream_t s, const RasterArgs& a) {
  if (a.n_faces == 0) return hipSuccess;
  hipLaunchKernelGGL(k_setup, dim3(grid_for(a.n_faces, 256 * kSetupFaces), a.n_views), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_face_attr, dim3(grid_for(a.n_faces, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_emit(hipStream_t s, const RasterArgs& a) {
  if (a.n_faces == 0) return hipSuccess;
  hipLaunchKernelGGL(k_emit, dim3(grid_for(a.n_faces, 256 * kEmitFaces), a.n_views), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tile_sort(hipStream_t s, const RasterArgs& a) {
  const int64_t n_seg = a.n_tiles * a.n_views;
  if (n_seg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)n_seg), dim3(kSortThreads), 0, s, a, n_seg);
  return hipGetLastError();
}

template <int KB, bool SHP>
static void launch_comp(hipStream_t s, const RasterArgs& a, int n_cu, uint32_t n_items) {
  if (SHP) {
    const int g = persistent_grid(k_composite_sh<KB>, n_cu, n_items);
    hipLaunchKernelGGL((k_composite_sh<KB>), dim3(g), dim3(256), 0, s, a, n_items);
  } else {
    const int g = persistent_grid(k_composite_rgb<KB>, n_cu, n_items);
    hipLaunchKernelGGL((k_composite_rgb<KB>), dim3(g), dim3(256), 0, s, a, n_items);
  }
}

hipError_t launch_composite(hipStream_t s, const RasterArgs& a, int kbuf, int n_cu) {
  const uint32_t n_items = n_items_of(a);
  const bool sh = a.col4 != nullptr;
  if (kbuf == 8) {
    if (sh) launch_comp<8, true>(s, a, n_cu, n_items);
    else launch_comp<8, false>(s, a, n_cu, n_items);
  } else if (kbuf == 12) {
    if (sh) launch_comp<12, true>(s, a, n_cu, n_items);
    else launch_comp<12, false>(s, a, n_cu, n_items);
  } else {
    if (sh) launch_comp<16, true>(s, a, n_cu, n_items);
    else launch_comp<16, false>(s, a, n_cu, n_items);
  }
  return hipGetLastError();
}

hipError_t launch_block_max(hipStream_t s, const RasterArgs& a) {
  const int64_t nb = (int64_t)a.n_views * ((a.W + 7) / 8) * ((a.H + 7) / 8);
  hipLaunchKernelGGL(k_block_max, dim3(grid_for(nb, 256)), dim3(256), 0, s, a, nb);
  return hipGetLastError();
}

hipError_t launch_bwd_lists(hipStream_t s, const RasterArgs& a, int kbuf, int n_cu) {
  const uint32_t n_items = n_items_of(a);
  if (kbuf == 8) {
    const int g = persistent_grid(k_bwd_lists<8>, n_cu, n_items);
    hipLaunchKernelGGL(k_bwd_lists<8>, dim3(g), dim3(256), 0, s, a, n_items);
  } else if (kbuf == 12) {
    const int g = persistent_grid(k_bwd_lists<12>, n_cu, n_items);
    hipLaunchKernelGGL(k_bwd_lists<12>, dim3(g), dim3(256), 0, s, a, n_items);
  } else {
    const int g = persistent_grid(k_bwd_lists<16>, n_cu, n_items);
    hipLaunchKernelGGL(k_bwd_lists<16>, dim3(g), dim3(256), 0, s, a, n_items);
  }
  return hipGetLastError();
}

template <int ACC>
static void launch_grads_mode(hipStream_t s, const RasterArgs& a, int n_cu, uint32_t n_items) {
  if (a.col4) {
    const int g = persistent_grid(k_bwd_grads<true, ACC>, n_cu, n_items);
    hipLaunchKernelGGL((k_bwd_grads<true, ACC>), dim3(g), dim3(256), 0, s, a, n_items);
  } else {
    const int g = persistent_grid(k_bwd_grads<false, ACC>, n_cu, n_items);
    hipLaunchKernelGGL((k_bwd_grads<false, ACC>), dim3(g), dim3(256), 0, s, a, n_items);
  }
}

hipError_t launch_bwd_grads(hipStream_t s, const RasterArgs& a, int n_cu, int mode) {
  const uint32_t nbx = (uint32_t)((a.W + 7) / 8), nby = (uint32_t)((a.H + 7) / 8);
  const uint32_t n_items = ((nbx + 1) / 2) * ((nby + 1) / 2) * (uint32_t)a.n_views;
  if (mode == 0) launch_grads_mode<ACC_F32>(s, a, n_cu, n_items);
  else if (mode == 1) launch_grads_mode<ACC_MAX>(s, a, n_cu, n_items);
  else launch_grads_mode<ACC_FIX>(s, a, n_cu, n_items);
  return hipGetLastError();
}

hipError_t launch_det_scales(hipStream_t s, const uint32_t* det_max, const unsigned long long* det_cnt, double* scale,
                             int c0, int c1) {
  hipLaunchKernelGGL(k_det_scales, dim3(1), dim3(64), 0, s, det_max, det_cnt, scale, c0, c1);
  return hipGetLastError();
}

hipError_t launch_dcol_finalize(hipStream_t s, const unsigned long long* dcol64, int64_t n, const double* scale,
                                float* dcol) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dcol_finalize, dim3(grid_for(n, 256)), dim3(256), 0, s, dcol64, n, scale, dcol);
  return hipGetLastError();
}

hipError_t launch_det_finalize(hipStream_t s, const unsigned long long* acc64, const unsigned long long* accsh64,
                               const double* scale, int64_t V, float* dpos, float* dop, float* drgb) {
  if (V == 0) return hipSuccess;
  hipLaunchKernelGGL(k_det_finalize, dim3(grid_for(V, 256)), dim3(256), 0, s, acc64, accsh64, scale, V, dpos, dop,
                     drgb);
  return hipGetLastError();
}

// Gaussian -> triangle-fan conversion (flat-Gaussian transformation section of
// the paper: Eq. 2d_scaledrot for the two scaled axes, the vertex equation for
// the boundary points, the fan construction, and the opacity paragraph for the
// centre/boundary opacities; the 3D-Gaussian section for the three-fan
// variant: Eq. 3d_scaledrot and one fan on each plane of two scaled axes).
// Streaming and HBM-bound: one thread per output vertex and one per output
// face, structure-of-arrays writes, coalesced.
#include "common.h"

namespace {

constexpr int kMaxK = 64;

struct CosSin {
  float c[kMaxK];
  float s[kMaxK];
};

// Columns of the rotation of a (w, x, y, z) quaternion, normalised in float32.
__device__ inline void rot_column(float w, float x, float y, float z, int col, float& r0, float& r1,
                                  float& r2) {
  const float n = sqrtf(w * w + x * x + y * y + z * z);
  w /= n; x /= n; y /= n; z /= n;
  if (col == 0) {
    r0 = 1.f - 2.f * (y * y + z * z); r1 = 2.f * (x * y + w * z); r2 = 2.f * (x * z - w * y);
  } else if (col == 1) {
    r0 = 2.f * (x * y - w * z); r1 = 1.f - 2.f * (x * x + z * z); r2 = 2.f * (y * z + w * x);
  } else {
    r0 = 2.f * (x * z + w * y); r1 = 2.f * (y * z - w * x); r2 = 1.f - 2.f * (x * x + y * y);
  }
}

// Gaussian behind output block g: order[g] when an order is given (an index
// outside [0, n) gives -1: NaN positions, zero opacity and colour, gid -1).
__device__ __forceinline__ int64_t source_of(const int32_t* __restrict__ order, int64_t g, int64_t n) {
  if (!order) return g;
  const int32_t o = order[g];
  return (o >= 0 && (int64_t)o < n) ? (int64_t)o : -1;
}

// The fan spans the two largest scales (ties to the lower index), in index order.
__device__ inline void pick_axes(float s0, float s1, float s2, int& a, int& b) {
  int drop;
  if (s2 <= s0 && s2 <= s1) drop = 2;
  else if (s1 <= s0) drop = 1;
  else drop = 0;
  a = drop == 0 ? 1 : 0;
  b = drop == 2 ? 1 : 2;
}

__device__ __forceinline__ void invalid_vertex(float* pos, float* vop, float* vrgb, int64_t V, int64_t v) {
  const float nan = __int_as_float(0x7fc00000);
  pos[v] = pos[V + v] = pos[2 * V + v] = nan;
  vop[v] = 0.f;
  vrgb[v] = vrgb[V + v] = vrgb[2 * V + v] = 0.f;
}

__global__ void k_convert_vertices(const float* __restrict__ mean, const float* __restrict__ scale,
                                   const float* __restrict__ quat, const float* __restrict__ opacity,
                                   const float* __restrict__ rgb, int64_t n, int K, float sigma,
                                   float opac_mul, CosSin cs, const int32_t* __restrict__ order,
                                   float* __restrict__ pos, float* __restrict__ vop, float* __restrict__ vrgb) {
  const int64_t V = n * (K + 1);
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int64_t blk = v / (K + 1);
  const int j = (int)(v - blk * (K + 1));
  const int64_t g = source_of(order, blk, n);
  if (g < 0) {
    invalid_vertex(pos, vop, vrgb, V, v);
    return;
  }
  const float mx = mean[g], my = mean[n + g], mz = mean[2 * n + g];
  float px = mx, py = my, pz = mz;
  const float o = opacity[g];
  if (j > 0) {
    const float s[3] = {scale[g], scale[n + g], scale[2 * n + g]};
    int a, b;
    pick_axes(s[0], s[1], s[2], a, b);
    const float qw = quat[g], qx = quat[n + g], qy = quat[2 * n + g], qz = quat[3 * n + g];
    float ra0, ra1, ra2, rb0, rb1, rb2;
    rot_column(qw, qx, qy, qz, a, ra0, ra1, ra2);
    rot_column(qw, qx, qy, qz, b, rb0, rb1, rb2);
    const float la = sigma * s[a], lb = sigma * s[b];
    const float c = cs.c[j - 1], sn = cs.s[j - 1];
    px = mx + c * (la * ra0) + sn * (lb * rb0);
    py = my + c * (la * ra1) + sn * (lb * rb1);
    pz = mz + c * (la * ra2) + sn * (lb * rb2);
  }
  pos[v] = px;
  pos[V + v] = py;
  pos[2 * V + v] = pz;
  vop[v] = j == 0 ? o : opac_mul * o;
  vrgb[v] = rgb[g];
  vrgb[V + v] = rgb[n + g];
  vrgb[2 * V + v] = rgb[2 * n + g];
}

__global__ void k_convert_faces(int64_t n, int K, const float* __restrict__ sh, const int32_t* __restrict__ order,
                                int32_t* __restrict__ idx, int32_t* __restrict__ gid, float* __restrict__ fsh) {
  const int64_t F = n * K;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const int64_t blk = f / K;
  const int k = (int)(f - blk * K);
  const int32_t c = (int32_t)(blk * (K + 1));
  idx[f] = c;
  idx[F + f] = c + 1 + k;
  idx[2 * F + f] = c + 1 + (k + 1) % K;
  const int64_t g = source_of(order, blk, n);
  if (gid) gid[f] = (int32_t)g;
  if (sh && fsh) {
#pragma unroll 4
    for (int r = 0; r < 48; ++r) fsh[r * F + f] = g >= 0 ? sh[r * n + g] : 0.f;
  }
}

// Three-fan conversion of 3D Gaussians. Per Gaussian, P = 7 + 3 (K - 4)
// vertices: the centre; the six axis points m + A_i, m - A_i (i = 0, 1, 2,
// A_i = sigma s_i r_i), which the three planes share at their quarter turns;
// then per plane p = (0,1), (0,2), (1,2) its K - 4 other boundary points
// m + cos(t_k) A_i + sin(t_k) A_j in angle order. Face g 3K + p K + k is
// (centre, ring_p(k), ring_p((k+1) mod K)). K is a multiple of 4.
__device__ __forceinline__ void plane_axes(int p, int& i, int& j) {
  i = p == 2 ? 1 : 0;
  j = p == 0 ? 1 : 2;
}

__global__ void k_convert3_vertices(const float* __restrict__ mean, const float* __restrict__ scale,
                                    const float* __restrict__ quat, const float* __restrict__ opacity,
                                    const float* __restrict__ rgb, int64_t n, int K, float sigma,
                                    float opac_mul, CosSin cs, const int32_t* __restrict__ order,
                                    float* __restrict__ pos, float* __restrict__ vop, float* __restrict__ vrgb) {
  const int per = 7 + 3 * (K - 4);
  const int64_t V = n * per;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int64_t blk = v / per;
  const int j = (int)(v - blk * per);
  const int64_t g = source_of(order, blk, n);
  if (g < 0) {
    invalid_vertex(pos, vop, vrgb, V, v);
    return;
  }
  const float mx = mean[g], my = mean[n + g], mz = mean[2 * n + g];
  float px = mx, py = my, pz = mz;
  const float o = opacity[g];
  if (j > 0) {
    const float qw = quat[g], qx = quat[n + g], qy = quat[2 * n + g], qz = quat[3 * n + g];
    int ia, ib;
    float ca, cb;  // coefficients of A_ia and A_ib
    if (j <= 6) {
      ia = (j - 1) / 2;
      ib = ia;
      ca = ((j - 1) & 1) ? -1.f : 1.f;
      cb = 0.f;
    } else {
      const int q4 = K / 4;
      const int p = (j - 7) / (K - 4), r = (j - 7) - p * (K - 4);
      const int k = (r / (q4 - 1)) * q4 + 1 + r % (q4 - 1);  // the r-th angle off the quarter turns
      plane_axes(p, ia, ib);
      ca = cs.c[k];
      cb = cs.s[k];
    }
    float a0, a1, a2, b0, b1, b2;
    rot_column(qw, qx, qy, qz, ia, a0, a1, a2);
    rot_column(qw, qx, qy, qz, ib, b0, b1, b2);
    const float la = sigma * scale[ia * n + g], lb = sigma * scale[ib * n + g];
    px = mx + ca * (la * a0) + cb * (lb * b0);
    py = my + ca * (la * a1) + cb * (lb * b1);
    pz = mz + ca * (la * a2) + cb * (lb * b2);
  }
  pos[v] = px;
  pos[V + v] = py;
  pos[2 * V + v] = pz;
  vop[v] = j == 0 ? o : opac_mul * o;
  vrgb[v] = rgb[g];
  vrgb[V + v] = rgb[n + g];
  vrgb[2 * V + v] = rgb[2 * n + g];
}

__device__ __forceinline__ int32_t ring3(int32_t base, int p, int k, int K) {
  const int q4 = K / 4;
  int i, j;
  plane_axes(p, i, j);
  if (k % q4 == 0) {
    switch (k / q4) {  // t_k = -pi, -pi/2, 0, pi/2
      case 0: return base + 2 + 2 * i;
      case 1: return base + 2 + 2 * j;
      case 2: return base + 1 + 2 * i;
      default: return base + 1 + 2 * j;
    }
  }
  return base + 7 + p * (K - 4) + (k - k / q4 - 1);
}

__global__ void k_convert3_faces(int64_t n, int K, const float* __restrict__ sh, const int32_t* __restrict__ order,
                                 int32_t* __restrict__ idx, int32_t* __restrict__ gid, float* __restrict__ fsh) {
  const int64_t F = n * 3 * K;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const int64_t blk = f / (3 * K);
  const int rem = (int)(f - blk * 3 * K);
  const int p = rem / K, k = rem - p * K;
  const int32_t base = (int32_t)(blk * (7 + 3 * (K - 4)));
  idx[f] = base;
  idx[F + f] = ring3(base, p, k, K);
  idx[2 * F + f] = ring3(base, p, (k + 1) % K, K);
  const int64_t g = source_of(order, blk, n);
  if (gid) gid[f] = (int32_t)g;
  if (sh && fsh) {
#pragma unroll 4
    for (int r = 0; r < 48; ++r) fsh[r * F + f] = g >= 0 ? sh[r * n + g] : 0.f;
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_f32(float* p, float v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_fill_u32(hipStream_t s, uint32_t* p, uint32_t v, int64_t n) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(hipStream_t s, float* p, float v, int64_t n) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_convert_three(hipStream_t s, const msp_gaussians* g, int K, float sigma, float opac_mul,
                                const float* cos_sin, const int32_t* order, msp_faces* out) {
  if (g->n == 0) return hipSuccess;
  CosSin cs;
  for (int k = 0; k < kMaxK; ++k) {
    cs.c[k] = k < K ? cos_sin[k] : 0.f;
    cs.s[k] = k < K ? cos_sin[K + k] : 0.f;
  }
  const int64_t V = g->n * (7 + 3 * (K - 4)), F = g->n * 3 * K;
  hipLaunchKernelGGL(k_convert3_vertices, dim3(grid_for(V, 256)), dim3(256), 0, s, g->mean, g->scale, g->quat,
                     g->opacity, g->rgb, g->n, K, sigma, opac_mul, cs, order, out->pos, out->opacity, out->rgb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_convert3_faces, dim3(grid_for(F, 256)), dim3(256), 0, s, g->n, K, g->sh, order, out->idx,
                     out->gid, out->sh);
  return hipGetLastError();
}

hipError_t launch_convert_flat(hipStream_t s, const msp_gaussians* g, int K, float sigma, float opac_mul,
                               const float* cos_sin, const int32_t* order, msp_faces* out) {
  if (g->n == 0) return hipSuccess;
  CosSin cs;
  for (int k = 0; k < kMaxK; ++k) {
    cs.c[k] = k < K ? cos_sin[k] : 0.f;
    cs.s[k] = k < K ? cos_sin[K + k] : 0.f;
  }
  const int64_t V = g->n * (K + 1), F = g->n * K;
  hipLaunchKernelGGL(k_convert_vertices, dim3(grid_for(V, 256)), dim3(256), 0, s, g->mean, g->scale, g->quat,
                     g->opacity, g->rgb, g->n, K, sigma, opac_mul, cs, order, out->pos, out->opacity, out->rgb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_convert_faces, dim3(grid_for(F, 256)), dim3(256), 0, s, g->n, K, g->sh, order, out->idx,
                     out->gid, out->sh);
  return hipGetLastError();
}

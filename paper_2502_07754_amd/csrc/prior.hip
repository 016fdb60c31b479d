// Mesh-prior mode (section "MeshSplats with Mesh Prior"): secondary triangles
// living on the faces of a fixed geometry mesh. Each secondary vertex is a
// convex combination of its mesh face's three corners with weights
// a = softmax(theta) (three logits per vertex, so the weights stay on the
// simplex); training moves the logits, colours and opacities.
//
// Layout: the mesh face mf carries T = n^2 secondary faces f = mf T + t, and
// face f owns vertices 3f, 3f + 1, 3f + 2 in corner order. Logits are [3][V]
// (row j: weight of mesh corner j). Sub-triangle t of the regular n-segment
// subdivision: row a = 0..n-1 holds 2(n - a) - 1 triangles, alternating the
// upward ((a,b), (a+1,b), (a,b+1)) and downward ((a+1,b), (a+1,b+1), (a,b+1))
// ones for b = 0, 1, ..., where grid point (a, b) weighs the corners
// ((n - a - b)/n, a/n, b/n).
//
// All three kernels are elementwise and HBM-bound: one thread per secondary
// vertex (or face), reading its logits as coalesced rows and its mesh face's
// corners through L2 (the 3T vertices of a mesh face are adjacent lanes).
// Mesh indices outside [0, n_verts) produce NaN positions and zero logit
// gradients for that face's vertices instead of an out-of-bounds read.

#include "common.h"

namespace {

inline unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65535 * 16) g = 65535 * 16;
  return (unsigned)(g < 1 ? 1 : g);
}

struct Corners {
  float m[3][3];  // [corner][xyz]
  bool ok;
};

__device__ __forceinline__ Corners load_corners(const float* __restrict__ mpos, const int32_t* __restrict__ midx,
                                                int64_t Vm, int64_t Fm, int64_t mf) {
  Corners c;
  c.ok = true;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int32_t i = midx[j * Fm + mf];
    const bool in = i >= 0 && (int64_t)i < Vm;
    c.ok = c.ok && in;
#pragma unroll
    for (int d = 0; d < 3; ++d) c.m[j][d] = in ? mpos[d * Vm + i] : 0.f;
  }
  return c;
}

__device__ __forceinline__ void weights(float t0, float t1, float t2, float a[3]) {
  const float mx = fmaxf(t0, fmaxf(t1, t2));
  const float e0 = expf(t0 - mx), e1 = expf(t1 - mx), e2 = expf(t2 - mx);
  const float inv = 1.f / (e0 + e1 + e2);
  a[0] = e0 * inv;
  a[1] = e1 * inv;
  a[2] = e2 * inv;
}

// grid point (a, b) of the n-segment subdivision as weights on the three corners
__device__ __forceinline__ void grid_weights(int a, int b, int n, float w[3]) {
  const float inv = 1.f / (float)n;
  w[0] = (float)(n - a - b) * inv;
  w[1] = (float)a * inv;
  w[2] = (float)b * inv;
}

__global__ void k_prior_init(int64_t Fm, int n, float shrink, float op0, float r0, float g0, float b0,
                             const int32_t* __restrict__ midx, const float* __restrict__ mrgb, int64_t Vm,
                             float* __restrict__ logits, int32_t* __restrict__ idx, int32_t* __restrict__ gid,
                             float* __restrict__ vop, float* __restrict__ vrgb) {
  const int T = n * n;
  const int64_t F = Fm * T, V = 3 * F;
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t mf = f / T;
    int r = (int)(f - mf * T), a = 0;
    while (r >= 2 * (n - a) - 1) {
      r -= 2 * (n - a) - 1;
      ++a;
    }
    const int b = r >> 1;
    float w[3][3];
    if ((r & 1) == 0) {
      grid_weights(a, b, n, w[0]);
      grid_weights(a + 1, b, n, w[1]);
      grid_weights(a, b + 1, n, w[2]);
    } else {
      grid_weights(a + 1, b, n, w[0]);
      grid_weights(a + 1, b + 1, n, w[1]);
      grid_weights(a, b + 1, n, w[2]);
    }
    float cen[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) cen[j] = (w[0][j] + w[1][j] + w[2][j]) * (1.f / 3.f);
    float crgb[3][3];
    bool have_rgb = false;
    if (mrgb) {
      have_rgb = true;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int32_t i = midx[j * Fm + mf];
        const bool in = i >= 0 && (int64_t)i < Vm;
        have_rgb = have_rgb && in;
#pragma unroll
        for (int d = 0; d < 3; ++d) crgb[j][d] = in ? mrgb[d * Vm + i] : 0.f;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t v = 3 * f + c;
      float al[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        al[j] = (1.f - shrink) * w[c][j] + shrink * cen[j];
        logits[j * V + v] = logf(al[j]);
      }
      idx[c * F + f] = (int32_t)v;
      vop[v] = op0;
      float rgb[3] = {r0, g0, b0};
      if (mrgb) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
          rgb[d] = have_rgb ? al[0] * crgb[0][d] + al[1] * crgb[1][d] + al[2] * crgb[2][d] : __int_as_float(0x7fc00000);
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) vrgb[d * V + v] = rgb[d];
    }
    if (gid) gid[f] = (int32_t)mf;
  }
}

__global__ void k_prior_vertices(const float* __restrict__ mpos, const int32_t* __restrict__ midx, int64_t Vm,
                                 int64_t Fm, int T3, const float* __restrict__ logits, float* __restrict__ pos) {
  const int64_t V = Fm * T3;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < V; v += (int64_t)gridDim.x * blockDim.x) {
    const Corners c = load_corners(mpos, midx, Vm, Fm, v / T3);
    float a[3];
    weights(logits[v], logits[V + v], logits[2 * V + v], a);
#pragma unroll
    for (int d = 0; d < 3; ++d)
      pos[d * V + v] = c.ok ? a[0] * c.m[0][d] + a[1] * c.m[1][d] + a[2] * c.m[2][d] : __int_as_float(0x7fc00000);
  }
}

__global__ void k_prior_backward(const float* __restrict__ mpos, const int32_t* __restrict__ midx, int64_t Vm,
                                 int64_t Fm, int T3, const float* __restrict__ logits, const float* __restrict__ dpos,
                                 float* __restrict__ dlogits) {
  const int64_t V = Fm * T3;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < V; v += (int64_t)gridDim.x * blockDim.x) {
    const Corners c = load_corners(mpos, midx, Vm, Fm, v / T3);
    float a[3];
    weights(logits[v], logits[V + v], logits[2 * V + v], a);
    const float dx = dpos[v], dy = dpos[V + v], dz = dpos[2 * V + v];
    float g[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) g[j] = dx * c.m[j][0] + dy * c.m[j][1] + dz * c.m[j][2];
    const float mean = a[0] * g[0] + a[1] * g[1] + a[2] * g[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) dlogits[j * V + v] = c.ok ? a[j] * (g[j] - mean) : 0.f;
  }
}

}  // namespace

hipError_t launch_prior_init(hipStream_t s, const msp_mesh* m, int n, float shrink, float op0, const float rgb0[3],
                             float* logits, msp_faces* out) {
  const int64_t F = m->n_faces * (int64_t)n * n;
  if (F == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prior_init, dim3(grid_for(F)), dim3(256), 0, s, m->n_faces, n, shrink, op0, rgb0[0], rgb0[1],
                     rgb0[2], m->idx, m->rgb, m->n_verts, logits, out->idx, out->gid, out->opacity, out->rgb);
  return hipGetLastError();
}

hipError_t launch_prior_vertices(hipStream_t s, const msp_mesh* m, int n, const float* logits, float* pos) {
  const int T3 = 3 * n * n;
  const int64_t V = m->n_faces * T3;
  if (V == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prior_vertices, dim3(grid_for(V)), dim3(256), 0, s, m->pos, m->idx, m->n_verts, m->n_faces,
                     T3, logits, pos);
  return hipGetLastError();
}

hipError_t launch_prior_backward(hipStream_t s, const msp_mesh* m, int n, const float* logits, const float* dpos,
                                 float* dlogits) {
  const int T3 = 3 * n * n;
  const int64_t V = m->n_faces * T3;
  if (V == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prior_backward, dim3(grid_for(V)), dim3(256), 0, s, m->pos, m->idx, m->n_verts, m->n_faces,
                     T3, logits, dpos, dlogits);
  return hipGetLastError();
}

// View-dependent face colour from degree-3 real spherical harmonics, and its
// adjoint. The coefficients ([48][F], row 3 b + c) are read once for all views
// of a render (forward) and the coefficient gradient is written once after all
// views (backward): the SH read/write is the dominant HBM traffic of a
// many-view render, so it is never repeated per view.
//
// Basis (b = l^2 + l + m, l <= 3): Y = c_lm P_l^(m)(z) Q_m(x, y) with P_l^(m) the
// m-th derivative of the Legendre polynomial, Q_0 = 1, Q_m = Re (x + i y)^m for
// m > 0 and Im (x + i y)^|m| for m < 0, and c_lm = K_lm (m = 0) or
// sqrt(2) K_lm (-1)^m, K_lm = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!): the real,
// orthonormal SH with the Condon-Shortley phase. The host derives the
// polynomial coefficients from the Legendre recurrence and the factorials.
// colour_c = max(0, 1/2 + sum_b k[3b+c] Y_b(d)), d = normalize(centroid - eye).
#include <cmath>

#include "common.h"

namespace {

constexpr int kMaxViews = 64;

struct ShArgs {
  float poly[16][4];          // ascending powers of z
  int m[16];
  float eye[kMaxViews][3];    // camera centres (world)
};

// (x + i y)^|m| split into Re/Im for |m| = 0..3
__device__ __forceinline__ void wpow(float x, float y, float re[4], float im[4]) {
  re[0] = 1.f; im[0] = 0.f;
  re[1] = x; im[1] = y;
  re[2] = x * x - y * y; im[2] = 2.f * x * y;
  re[3] = re[2] * x - im[2] * y; im[3] = re[2] * y + im[2] * x;
}

__device__ __forceinline__ float polyval(const float* p, float z) { return ((p[3] * z + p[2]) * z + p[1]) * z + p[0]; }
__device__ __forceinline__ float polyder(const float* p, float z) { return (3.f * p[3] * z + 2.f * p[2]) * z + p[1]; }

// face centroid (read once per face for all views); false for a face with a
// vertex id out of range, which is never drawn and whose colour is not used
__device__ __forceinline__ bool face_centroid(const float* __restrict__ pos, int64_t V,
                                              const int32_t* __restrict__ idx, int64_t F, int64_t f, float& cx,
                                              float& cy, float& cz) {
  const int32_t i0 = idx[f], i1 = idx[F + f], i2 = idx[2 * F + f];
  if ((uint64_t)i0 >= (uint64_t)V || (uint64_t)i1 >= (uint64_t)V || (uint64_t)i2 >= (uint64_t)V) {
    cx = cy = cz = 0.f;
    return false;
  }
  cx = (pos[i0] + pos[i1] + pos[i2]) * (1.f / 3.f);
  cy = (pos[V + i0] + pos[V + i1] + pos[V + i2]) * (1.f / 3.f);
  cz = (pos[2 * V + i0] + pos[2 * V + i1] + pos[2 * V + i2]) * (1.f / 3.f);
  return true;
}

// unit direction from the eye to the centroid and the inverse distance
__device__ __forceinline__ void face_dir(float cx, float cy, float cz, const float* eye, float& dx, float& dy,
                                         float& dz, float& inv_len) {
  const float vx = cx - eye[0], vy = cy - eye[1], vz = cz - eye[2];
  inv_len = 1.f / sqrtf(vx * vx + vy * vy + vz * vz);
  dx = vx * inv_len;
  dy = vy * inv_len;
  dz = vz * inv_len;
}

__global__ __launch_bounds__(256) void k_sh_eval(const float* __restrict__ sh, const float* __restrict__ pos,
                                                 int64_t V, const int32_t* __restrict__ idx, int64_t F, int n_views,
                                                 ShArgs t, float4* __restrict__ col4) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  float k[48];
#pragma unroll
  for (int r = 0; r < 48; ++r) k[r] = sh[r * F + f];
  float ccx, ccy, ccz;
  if (!face_centroid(pos, V, idx, F, f, ccx, ccy, ccz)) {
    for (int v = 0; v < n_views; ++v) col4[(int64_t)v * F + f] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  for (int v = 0; v < n_views; ++v) {
    float x, y, z, il;
    face_dir(ccx, ccy, ccz, t.eye[v], x, y, z, il);
    float re[4], im[4];
    wpow(x, y, re, im);
    float cr = 0.5f, cg = 0.5f, cb = 0.5f;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      const int m = t.m[b];
      const float q = m == 0 ? 1.f : (m > 0 ? re[m] : im[-m]);
      const float Y = polyval(t.poly[b], z) * q;
      cr = fmaf(k[3 * b], Y, cr);
      cg = fmaf(k[3 * b + 1], Y, cg);
      cb = fmaf(k[3 * b + 2], Y, cb);
    }
    col4[(int64_t)v * F + f] = make_float4(fmaxf(cr, 0.f), fmaxf(cg, 0.f), fmaxf(cb, 0.f), 0.f);
  }
}

__global__ __launch_bounds__(256) void k_sh_bwd(const float* __restrict__ sh, const float* __restrict__ pos,
                                                int64_t V, const int32_t* __restrict__ idx, int64_t F, int n_views,
                                                ShArgs t, const float* __restrict__ dcol, float* __restrict__ dsh,
                                                float* dpos, float4* gvout, uint32_t* det_max,
                                                unsigned long long* det_cnt) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float gvx = 0.f, gvy = 0.f, gvz = 0.f;  // d L / d (centroid), summed over views
  if (f < F) {
    float k[48], dk[48];
#pragma unroll
    for (int r = 0; r < 48; ++r) {
      k[r] = sh[r * F + f];
      dk[r] = 0.f;
    }
    float ccx, ccy, ccz;
    const bool drawn = face_centroid(pos, V, idx, F, f, ccx, ccy, ccz);
    for (int v = 0; v < n_views && drawn; ++v) {
      const int64_t o = (int64_t)v * 3 * F + f;
      const float g0 = dcol[o], g1 = dcol[o + F], g2 = dcol[o + 2 * F];
      if (g0 == 0.f && g1 == 0.f && g2 == 0.f) continue;
      float x, y, z, il;
      face_dir(ccx, ccy, ccz, t.eye[v], x, y, z, il);
      float re[4], im[4];
      wpow(x, y, re, im);
      float Y[16], pre0 = 0.5f, pre1 = 0.5f, pre2 = 0.5f;
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const int m = t.m[b];
        const float q = m == 0 ? 1.f : (m > 0 ? re[m] : im[-m]);
        Y[b] = polyval(t.poly[b], z) * q;
        pre0 = fmaf(k[3 * b], Y[b], pre0);
        pre1 = fmaf(k[3 * b + 1], Y[b], pre1);
        pre2 = fmaf(k[3 * b + 2], Y[b], pre2);
      }
      const float h0 = pre0 > 0.f ? g0 : 0.f, h1 = pre1 > 0.f ? g1 : 0.f, h2 = pre2 > 0.f ? g2 : 0.f;
      float ddx = 0.f, ddy = 0.f, ddz = 0.f;
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        dk[3 * b] = fmaf(Y[b], h0, dk[3 * b]);
        dk[3 * b + 1] = fmaf(Y[b], h1, dk[3 * b + 1]);
        dk[3 * b + 2] = fmaf(Y[b], h2, dk[3 * b + 2]);
        const float s = k[3 * b] * h0 + k[3 * b + 1] * h1 + k[3 * b + 2] * h2;
        const int m = t.m[b];
        const int am = m < 0 ? -m : m;
        const float p = polyval(t.poly[b], z), dp = polyder(t.poly[b], z);
        float yx, yy, yz;
        if (m == 0) {
          yx = 0.f; yy = 0.f; yz = dp;
        } else if (m > 0) {
          yx = p * am * re[am - 1];
          yy = -p * am * im[am - 1];
          yz = dp * re[am];
        } else {
          yx = p * am * im[am - 1];
          yy = p * am * re[am - 1];
          yz = dp * im[am];
        }
        ddx = fmaf(s, yx, ddx);
        ddy = fmaf(s, yy, ddy);
        ddz = fmaf(s, yz, ddz);
      }
      // through d = v / |v|: (I - d d^T) dd / |v|
      const float dot = ddx * x + ddy * y + ddz * z;
      gvx += (ddx - dot * x) * il;
      gvy += (ddy - dot * y) * il;
      gvz += (ddz - dot * z) * il;
    }
    if (dsh) {
#pragma unroll
      for (int r = 0; r < 48; ++r) dsh[r * F + f] = dk[r];
    }
  }
  // each corner moves the centroid by a third of its own motion
  const float tx = gvx * (1.f / 3.f), ty = gvy * (1.f / 3.f), tz = gvz * (1.f / 3.f);
  if (gvout) {
    // deterministic mode: per-face terms, their largest magnitude and count (one atomic per wave)
    if (f < F) gvout[f] = make_float4(tx, ty, tz, 0.f);
    const bool fin = isfinite(tx) && isfinite(ty) && isfinite(tz);
    float m = (f < F && fin) ? fmaxf(fmaxf(fabsf(tx), fabsf(ty)), fabsf(tz)) : 0.f;
    uint32_t n = f < F ? 9u : 0u;
    for (int o = 32; o >= 1; o >>= 1) {
      m = fmaxf(m, __shfl_xor(m, o));
      n += __shfl_xor(n, o);
    }
    const bool bad = __any(f < F && !fin);
    if ((threadIdx.x & 63) == 0) {
      if (n) {
        atomicMax(&det_max[DT_SHPOS], __float_as_uint(m));
        atomicAdd(&det_cnt[DT_SHPOS], (unsigned long long)n);
      }
      if (bad) atomicOr(&det_max[DT_N], 1u);
    }
    return;
  }
  if (f < F && dpos && (gvx != 0.f || gvy != 0.f || gvz != 0.f)) {
    const int32_t id[3] = {idx[f], idx[F + f], idx[2 * F + f]};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if ((uint64_t)id[q] >= (uint64_t)V) continue;
      atomicAdd(&dpos[id[q]], tx);
      atomicAdd(&dpos[V + id[q]], ty);
      atomicAdd(&dpos[2 * V + id[q]], tz);
    }
  }
}

// deterministic mode: the per-face position terms as fixed-point sums per vertex
__global__ __launch_bounds__(256) void k_sh_fix(const int32_t* __restrict__ idx, int64_t F, int64_t V,
                                                const float4* __restrict__ gv, const double* __restrict__ scale,
                                                unsigned long long* accsh64) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const float4 g = gv[f];
  if (g.x == 0.f && g.y == 0.f && g.z == 0.f) return;
  const double sc = scale[DT_SHPOS];
  const long long x = __double2ll_rn((double)g.x * sc), y = __double2ll_rn((double)g.y * sc),
                  z = __double2ll_rn((double)g.z * sc);
  const int32_t id[3] = {idx[f], idx[F + f], idx[2 * F + f]};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if ((uint64_t)id[q] >= (uint64_t)V) continue;
    atomicAdd(&accsh64[id[q]], (unsigned long long)x);
    atomicAdd(&accsh64[V + id[q]], (unsigned long long)y);
    atomicAdd(&accsh64[2 * V + id[q]], (unsigned long long)z);
  }
}

bool make_table(const msp_camera* cams, int n_views, ShArgs& t) {
  if (n_views > kMaxViews) return false;
  double P[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  for (int n = 1; n < 3; ++n)  // (n+1) P_{n+1} = (2n+1) z P_n - n P_{n-1}
    for (int c = 0; c < 4; ++c)
      P[n + 1][c] = ((2.0 * n + 1.0) * (c > 0 ? P[n][c - 1] : 0.0) - n * P[n - 1][c]) / (n + 1.0);
  auto fact = [](int n) {
    double r = 1;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
  };
  const double pi = 3.14159265358979323846;
  for (int b = 0; b < 16; ++b) {
    int l = 0;
    while ((l + 1) * (l + 1) <= b) ++l;
    const int m = b - l * l - l, am = m < 0 ? -m : m;
    double D[4];
    for (int c = 0; c < 4; ++c) D[c] = P[l][c];
    for (int r = 0; r < am; ++r)
      for (int c = 0; c < 4; ++c) D[c] = c + 1 < 4 ? (c + 1) * D[c + 1] : 0.0;
    const double K = std::sqrt((2 * l + 1) / (4 * pi) * fact(l - am) / fact(l + am));
    const double cm = m == 0 ? K : std::sqrt(2.0) * K * ((am & 1) ? -1.0 : 1.0);
    for (int c = 0; c < 4; ++c) t.poly[b][c] = (float)(cm * D[c]);
    t.m[b] = m;
  }
  for (int v = 0; v < n_views; ++v) {
    // eye = -W^{-1} t for the 3x3 part W of world_to_cam, solved in double
    const float* w = cams[v].world_to_cam;
    const double a = w[0], b = w[1], c = w[2], d = w[4], e = w[5], f = w[6], g = w[8], h = w[9], i = w[10];
    const double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
    const double inv[9] = {(e * i - f * h) / det, (c * h - b * i) / det, (b * f - c * e) / det,
                           (f * g - d * i) / det, (a * i - c * g) / det, (c * d - a * f) / det,
                           (d * h - e * g) / det, (b * g - a * h) / det, (a * e - b * d) / det};
    const double tx = w[3], ty = w[7], tz = w[11];
    for (int r = 0; r < 3; ++r)
      t.eye[v][r] = (float)(-(inv[3 * r] * tx + inv[3 * r + 1] * ty + inv[3 * r + 2] * tz));
  }
  return true;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

}  // namespace

int sh_max_views() { return kMaxViews; }

hipError_t launch_sh_eval(hipStream_t s, const msp_faces* f, const msp_camera* h_cams, int n_views, float4* col4) {
  if (f->n_faces == 0) return hipSuccess;
  ShArgs t;
  if (!make_table(h_cams, n_views, t)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sh_eval, dim3(grid_for(f->n_faces)), dim3(256), 0, s, f->sh, f->pos, f->n_verts, f->idx,
                     f->n_faces, n_views, t, col4);
  return hipGetLastError();
}

hipError_t launch_sh_bwd(hipStream_t s, const msp_faces* f, const msp_camera* h_cams, int n_views, const float* dcol,
                         float* dsh, float* dpos, float4* gv, uint32_t* det_max, unsigned long long* det_cnt) {
  if (f->n_faces == 0) return hipSuccess;
  ShArgs t;
  if (!make_table(h_cams, n_views, t)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sh_bwd, dim3(grid_for(f->n_faces)), dim3(256), 0, s, f->sh, f->pos, f->n_verts, f->idx,
                     f->n_faces, n_views, t, dcol, dsh, dpos, gv, det_max, det_cnt);
  return hipGetLastError();
}

hipError_t launch_sh_fix(hipStream_t s, const msp_faces* f, const float4* gv, const double* scale,
                         unsigned long long* accsh64) {
  if (f->n_faces == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sh_fix, dim3(grid_for(f->n_faces)), dim3(256), 0, s, f->idx, f->n_faces, f->n_verts, gv, scale,
                     accsh64);
  return hipGetLastError();
}

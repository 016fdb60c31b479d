// Fine-tuning kernels (fine-tuning section of the paper): image losses and
// their gradients (MSE, L1, and L1 mixed with SSIM as in Eq. loss), the Adam
// update with per-group learning rates and opacity projection, face/vertex
// pruning with stable compaction, and the multi-ring conversion used to
// render fine-tuning targets. All streaming and HBM-bound.
#include <cmath>

#include "common.h"

namespace {

constexpr int kWin = 11;  // SSIM window (Gaussian, sigma 1.5)

struct Win {
  float g[kWin];
};

inline unsigned grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  if (g > 65535 * 16) g = 65535 * 16;
  return (unsigned)(g < 1 ? 1 : g);
}

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[256 / MSP_WAVE];
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  const int lane = threadIdx.x & (MSP_WAVE - 1), wid = threadIdx.x / MSP_WAVE;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x / MSP_WAVE); ++w) t += red[w];
  __syncthreads();
  return t;
}

// MSE / L1 over the three colour planes; partial sums per block (summed by k_sum_partials)
__global__ __launch_bounds__(256) void k_pointwise_loss(const float* __restrict__ img, const float* __restrict__ tgt,
                                                        int V, int H, int W, int kind, float gscale,
                                                        float* __restrict__ dimg, double* __restrict__ part) {
  const int64_t plane = (int64_t)H * W;
  const int64_t n = (int64_t)V * 3 * plane;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = i / (3 * plane), r = i - v * 3 * plane;  // r = c * plane + p
    const float x = img[v * 4 * plane + r], y = tgt[i];
    const float d = x - y;
    float g;
    if (kind == MSP_LOSS_MSE) {
      acc += (double)d * d;
      g = 2.f * d;
    } else {
      acc += fabs((double)d);
      g = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
    }
    if (dimg) dimg[v * 4 * plane + r] = g * gscale;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_sum_partials(const double* __restrict__ part, int n, double scale, double add, int accumulate,
                               double* __restrict__ acc, float* __restrict__ out) {
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) t += part[i];
  t = block_sum(t);
  if (threadIdx.x == 0) {
    const double v = t * scale + add + (accumulate ? *acc : 0.0);
    *acc = v;
    *out = (float)v;
  }
}

// SSIM pass 1: horizontal window sums of x, y, x^2, y^2, xy for every row and
// every valid column: h[k][v][c][row][x], x in [0, W-10).
__global__ __launch_bounds__(256) void k_ssim_h(const float* __restrict__ img, const float* __restrict__ tgt, int V,
                                                int H, int W, Win w, float* __restrict__ h) {
  const int Wv = W - (kWin - 1);
  const int64_t n = (int64_t)V * 3 * H * Wv;
  const int64_t plane = (int64_t)H * W;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % Wv);
    const int64_t rowid = i / Wv;  // (v*3 + c)*H + row
    const int row = (int)(rowid % H);
    const int64_t vc = rowid / H;
    const int64_t v = vc / 3, c = vc - v * 3;
    const float* X = img + v * 4 * plane + c * plane + (int64_t)row * W + x;
    const float* Y = tgt + vc * plane + (int64_t)row * W + x;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
    for (int u = 0; u < kWin; ++u) {
      const float a = X[u], b = Y[u], g = w.g[u];
      s0 = fmaf(g, a, s0);
      s1 = fmaf(g, b, s1);
      s2 = fmaf(g, a * a, s2);
      s3 = fmaf(g, b * b, s3);
      s4 = fmaf(g, a * b, s4);
    }
    h[i] = s0;
    h[n + i] = s1;
    h[2 * n + i] = s2;
    h[3 * n + i] = s3;
    h[4 * n + i] = s4;
  }
}

// SSIM pass 2: vertical window sums -> SSIM map and the per-window partials
// dS/dmu_x, dS/dE[x^2], dS/dE[xy] (written to q[3][...]); sum of S per block.
__global__ __launch_bounds__(256) void k_ssim_v(const float* __restrict__ h, int V, int H, int W, Win w,
                                                float* __restrict__ q, double* __restrict__ part) {
  const int Wv = W - (kWin - 1), Hv = H - (kWin - 1);
  const int64_t nh = (int64_t)V * 3 * H * Wv;
  const int64_t n = (int64_t)V * 3 * Hv * Wv;
  const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % Wv);
    const int64_t r = i / Wv;
    const int y = (int)(r % Hv);
    const int64_t vc = r / Hv;
    const int64_t base = (vc * H + y) * Wv + x;
    float m[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < kWin; ++u) {
      const float g = w.g[u];
#pragma unroll
      for (int k = 0; k < 5; ++k) m[k] = fmaf(g, h[k * nh + base + (int64_t)u * Wv], m[k]);
    }
    const float mx = m[0], my = m[1];
    const float A1 = 2.f * mx * my + C1, A2 = 2.f * (m[4] - mx * my) + C2;
    const float B1 = mx * mx + my * my + C1, B2 = (m[2] - mx * mx) + (m[3] - my * my) + C2;
    const float iB = 1.f / (B1 * B2);
    const float S = A1 * A2 * iB;
    acc += S;
    const float dA1 = A2 * iB, dA2 = A1 * iB, dB1 = -S / B1, dB2 = -S / B2;
    q[i] = dA1 * 2.f * my - dA2 * 2.f * my + dB1 * 2.f * mx - dB2 * 2.f * mx;  // d/d mu_x
    q[n + i] = dB2;                                                            // d/d E[x^2]
    q[2 * n + i] = 2.f * dA2;                                                  // d/d E[xy]
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// SSIM adjoint, vertical part: t[k][v][c][row][x] = sum over valid windows y of q[k](y, x) w(row - y)
__global__ __launch_bounds__(256) void k_ssim_adj_v(const float* __restrict__ q, int V, int H, int W, Win w,
                                                    float* __restrict__ t) {
  const int Wv = W - (kWin - 1), Hv = H - (kWin - 1);
  const int64_t nq = (int64_t)V * 3 * Hv * Wv;
  const int64_t n = (int64_t)V * 3 * H * Wv;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % Wv);
    const int64_t r = i / Wv;
    const int row = (int)(r % H);
    const int64_t vc = r / H;
    float s[3] = {0, 0, 0};
#pragma unroll
    for (int u = 0; u < kWin; ++u) {
      const int y = row - u;
      if (y < 0 || y >= Hv) continue;
      const int64_t o = (vc * Hv + y) * Wv + x;
#pragma unroll
      for (int k = 0; k < 3; ++k) s[k] = fmaf(w.g[u], q[k * nq + o], s[k]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k * n + i] = s[k];
  }
}

// SSIM adjoint, horizontal part and combination into dimg (added to what is there).
__global__ __launch_bounds__(256) void k_ssim_adj_h(const float* __restrict__ t, const float* __restrict__ img,
                                                    const float* __restrict__ tgt, int V, int H, int W, Win w,
                                                    float scale, float* __restrict__ dimg) {
  const int Wv = W - (kWin - 1);
  const int64_t nt = (int64_t)V * 3 * H * Wv;
  const int64_t plane = (int64_t)H * W;
  const int64_t n = (int64_t)V * 3 * plane;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % W);
    const int64_t r = i / W;  // (v*3 + c)*H + row
    float s[3] = {0, 0, 0};
#pragma unroll
    for (int u = 0; u < kWin; ++u) {
      const int xx = x - u;
      if (xx < 0 || xx >= Wv) continue;
      const int64_t o = r * Wv + xx;
#pragma unroll
      for (int k = 0; k < 3; ++k) s[k] = fmaf(w.g[u], t[k * nt + o], s[k]);
    }
    const int64_t vc = r / H, v = vc / 3, c = vc - v * 3, p = i - vc * plane;
    const float a = img[v * 4 * plane + c * plane + p], b = tgt[i];
    dimg[v * 4 * plane + c * plane + p] += scale * (s[0] + 2.f * a * s[1] + b * s[2]);
  }
}

__global__ void k_zero_alpha(float* dimg, int V, int64_t plane) {
  const int64_t n = (int64_t)V * plane;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = i / plane, p = i - v * plane;
    dimg[v * 4 * plane + 3 * plane + p] = 0.f;
  }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                                              float eps, float bc1, float bc2, float lo, float hi, int clamp) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float x = p[i] - lr * (mi * bc1) / (sqrtf(vi * bc2) + eps);
    if (clamp) x = fminf(fmaxf(x, lo), hi);
    p[i] = x;
  }
}

// ---- pruning ----
__global__ void k_face_keep(const int32_t* __restrict__ idx, const float* __restrict__ op, int64_t F, int64_t V,
                            float thresh, uint32_t* __restrict__ keep, uint32_t* __restrict__ used) {
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = idx[f], b = idx[F + f], c = idx[2 * F + f];
    // a face with an out-of-range vertex id is dropped
    const bool ok = (uint64_t)a < (uint64_t)V && (uint64_t)b < (uint64_t)V && (uint64_t)c < (uint64_t)V;
    const bool k = ok && (op[a] >= thresh || op[b] >= thresh || op[c] >= thresh);
    keep[f] = k ? 1u : 0u;
    if (k) {
      used[a] = 1u;
      used[b] = 1u;
      used[c] = 1u;
    }
  }
}

__global__ void k_compact_faces(const int32_t* __restrict__ idx, const int32_t* __restrict__ gid,
                                const float* __restrict__ sh, int64_t F, const uint32_t* __restrict__ keep,
                                const int64_t* __restrict__ foff, const int64_t* __restrict__ voff,
                                int32_t* __restrict__ idx2, int32_t* __restrict__ gid2, float* __restrict__ sh2) {
  const int64_t F2 = foff[F];
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x) {
    if (!keep[f]) continue;
    const int64_t o = foff[f];
    for (int k = 0; k < 3; ++k) idx2[k * F2 + o] = (int32_t)voff[idx[k * F + f]];
    if (gid) gid2[o] = gid[f];
    if (sh)
      for (int r = 0; r < 48; ++r) sh2[r * F2 + o] = sh[r * F + f];
  }
}

// copies rows x V vertex array into rows x V2 packed, keeping used vertices
__global__ void k_compact_rows(const float* __restrict__ src, int rows, int64_t V, const uint32_t* __restrict__ used,
                               const int64_t* __restrict__ voff, float* __restrict__ dst) {
  const int64_t V2 = voff[V];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)rows * V;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / V, v = i - r * V;
    if (used[v]) dst[r * V2 + voff[v]] = src[i];
  }
}

// ---- multi-ring conversion (fine-tuning targets) ----
struct RingArgs {
  float c[64], s[64];
  float radius[16], ofall[16];
};

__device__ inline void rot_col(float w, float x, float y, float z, int col, float& r0, float& r1, float& r2) {
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

__global__ void k_rings_vertices(const float* __restrict__ mean, const float* __restrict__ scale,
                                 const float* __restrict__ quat, const float* __restrict__ opacity,
                                 const float* __restrict__ rgb, int64_t n, int K, int rings, RingArgs ra,
                                 float* __restrict__ pos, float* __restrict__ vop, float* __restrict__ vrgb) {
  const int per = 1 + rings * K;
  const int64_t V = n * per;
  for (int64_t vid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; vid < V; vid += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = vid / per;
    const int j = (int)(vid - g * per);
    float px = mean[g], py = mean[n + g], pz = mean[2 * n + g];
    float o = opacity[g];
    if (j > 0) {
      const int ring = (j - 1) / K, k = (j - 1) % K;
      const float s0 = scale[g], s1 = scale[n + g], s2 = scale[2 * n + g];
      const int drop = (s2 <= s0 && s2 <= s1) ? 2 : (s1 <= s0 ? 1 : 0);
      const int a = drop == 0 ? 1 : 0, b = drop == 2 ? 1 : 2;
      const float sa = a == 0 ? s0 : s1, sb = b == 1 ? s1 : s2;
      const float qw = quat[g], qx = quat[n + g], qy = quat[2 * n + g], qz = quat[3 * n + g];
      float ra0, ra1, ra2, rb0, rb1, rb2;
      rot_col(qw, qx, qy, qz, a, ra0, ra1, ra2);
      rot_col(qw, qx, qy, qz, b, rb0, rb1, rb2);
      const float r = ra.radius[ring];
      const float ca = r * ra.c[k] * sa, cb = r * ra.s[k] * sb;
      px += ca * ra0 + cb * rb0;
      py += ca * ra1 + cb * rb1;
      pz += ca * ra2 + cb * rb2;
      o *= ra.ofall[ring];
    }
    pos[vid] = px;
    pos[V + vid] = py;
    pos[2 * V + vid] = pz;
    vop[vid] = o;
    vrgb[vid] = rgb[g];
    vrgb[V + vid] = rgb[n + g];
    vrgb[2 * V + vid] = rgb[2 * n + g];
  }
}

__global__ void k_rings_faces(int64_t n, int K, int rings, int32_t* __restrict__ idx, int32_t* __restrict__ gid) {
  const int per = 1 + rings * K;
  const int nf = K * (2 * rings - 1);
  const int64_t F = n * nf;
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = f / nf;
    const int l = (int)(f - g * nf);
    int a, b, c;
    if (l < K) {
      a = 0;
      b = 1 + l;
      c = 1 + (l + 1) % K;
    } else {
      const int q = l - K, j = q / (2 * K), r = q % (2 * K), k = r / 2;
      const int a0 = 1 + j * K + k, a1 = 1 + j * K + (k + 1) % K;
      const int b0 = 1 + (j + 1) * K + k, b1 = 1 + (j + 1) * K + (k + 1) % K;
      if ((r & 1) == 0) {
        a = a0; b = b0; c = b1;
      } else {
        a = a0; b = b1; c = a1;
      }
    }
    const int32_t base = (int32_t)(g * per);
    idx[f] = base + a;
    idx[F + f] = base + b;
    idx[2 * F + f] = base + c;
    if (gid) gid[f] = (int32_t)g;
  }
}

Win ssim_window() {
  Win w;
  double s = 0;
  double g[kWin];
  for (int u = 0; u < kWin; ++u) {
    const double x = u - (kWin - 1) / 2.0;
    g[u] = std::exp(-x * x / (2 * 1.5 * 1.5));
    s += g[u];
  }
  for (int u = 0; u < kWin; ++u) w.g[u] = (float)(g[u] / s);
  return w;
}

}  // namespace

size_t loss_scratch_bytes(int V, int H, int W, int kind) {
  size_t b = 8 * 4096 * 2;  // partial sums
  if (kind == MSP_LOSS_L1_DSSIM && W > kWin - 1 && H > kWin - 1)
    b += sizeof(float) * ((size_t)5 * V * 3 * H * (W - kWin + 1) + (size_t)3 * V * 3 * (H - kWin + 1) * (W - kWin + 1) +
                          (size_t)3 * V * 3 * H * (W - kWin + 1)) + 1024;
  return b;
}

hipError_t launch_loss(hipStream_t s, int kind, float lambda, const float* img, const float* tgt, int V, int H, int W,
                       float* loss_out, float* dimg, void* scratch) {
  const int64_t n = (int64_t)V * 3 * H * W;
  const unsigned G = grid_for(n) > 4096 ? 4096 : grid_for(n);
  double* part = (double*)scratch;
  double* acc = part + 4096;
  hipError_t e;
  const bool dssim = kind == MSP_LOSS_L1_DSSIM;
  const float wl1 = dssim ? lambda : 1.f;
  hipLaunchKernelGGL(k_pointwise_loss, dim3(G), dim3(256), 0, s, img, tgt, V, H, W,
                     kind == MSP_LOSS_MSE ? (int)MSP_LOSS_MSE : (int)MSP_LOSS_L1, wl1 / (float)n, dimg, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, (int)G, (double)wl1 / (double)n, 0.0, 0, acc,
                     loss_out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (dimg) {
    hipLaunchKernelGGL(k_zero_alpha, dim3(grid_for((int64_t)V * H * W)), dim3(256), 0, s, dimg, V, (int64_t)H * W);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (!dssim || H < kWin || W < kWin) return hipSuccess;
  const Win w = ssim_window();
  const int Wv = W - (kWin - 1), Hv = H - (kWin - 1);
  float* h = (float*)(acc + 16);
  const int64_t nh = (int64_t)V * 3 * H * Wv, nq = (int64_t)V * 3 * Hv * Wv;
  float* q = h + 5 * nh;
  float* t = q + 3 * nq;
  hipLaunchKernelGGL(k_ssim_h, dim3(grid_for(nh)), dim3(256), 0, s, img, tgt, V, H, W, w, h);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned Gq = grid_for(nq) > 4096 ? 4096 : grid_for(nq);
  hipLaunchKernelGGL(k_ssim_v, dim3(Gq), dim3(256), 0, s, h, V, H, W, w, q, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // loss += (1 - lambda) (1 - mean S) = (1 - lambda) - (1 - lambda)/nq * sum S
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, (int)Gq, -(double)(1.f - lambda) / (double)nq,
                     (double)(1.f - lambda), 1, acc, loss_out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (!dimg) return hipSuccess;
  hipLaunchKernelGGL(k_ssim_adj_v, dim3(grid_for(nh)), dim3(256), 0, s, q, V, H, W, w, t);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_ssim_adj_h, dim3(grid_for(n)), dim3(256), 0, s, t, img, tgt, V, H, W, w,
                     -(1.f - lambda) / (float)nq, dimg);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, const msp_adam_group& g, int step, float b1, float b2, float eps) {
  if (g.n <= 0) return hipSuccess;
  const double bc1 = 1.0 / (1.0 - std::pow((double)b1, step));
  const double bc2 = 1.0 / (1.0 - std::pow((double)b2, step));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(g.n)), dim3(256), 0, s, g.param, g.grad, g.m, g.v, g.n, g.lr, b1, b2, eps,
                     (float)bc1, (float)bc2, g.lo, g.hi, g.clamp);
  return hipGetLastError();
}

hipError_t launch_face_keep(hipStream_t s, const int32_t* idx, const float* op, int64_t F, int64_t V, float thresh,
                            uint32_t* keep, uint32_t* used) {
  if (F == 0) return hipSuccess;
  hipLaunchKernelGGL(k_face_keep, dim3(grid_for(F)), dim3(256), 0, s, idx, op, F, V, thresh, keep, used);
  return hipGetLastError();
}

hipError_t launch_compact_faces(hipStream_t s, const int32_t* idx, const int32_t* gid, const float* sh, int64_t F,
                                const uint32_t* keep, const int64_t* foff, const int64_t* voff, int32_t* idx2,
                                int32_t* gid2, float* sh2) {
  if (F == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact_faces, dim3(grid_for(F)), dim3(256), 0, s, idx, gid, sh, F, keep, foff, voff, idx2,
                     gid2, sh2);
  return hipGetLastError();
}

hipError_t launch_compact_rows(hipStream_t s, const float* src, int rows, int64_t V, const uint32_t* used,
                               const int64_t* voff, float* dst) {
  if (V == 0 || rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact_rows, dim3(grid_for((int64_t)rows * V)), dim3(256), 0, s, src, rows, V, used, voff,
                     dst);
  return hipGetLastError();
}

hipError_t launch_convert_rings(hipStream_t s, const msp_gaussians* g, int K, int rings, float sigma_max,
                                msp_faces* out) {
  if (g->n == 0) return hipSuccess;
  RingArgs ra;
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < 64; ++k) {
    const double th = -pi + 2.0 * pi * k / K;
    ra.c[k] = k < K ? (float)std::cos(th) : 0.f;
    ra.s[k] = k < K ? (float)std::sin(th) : 0.f;
  }
  for (int j = 0; j < 16; ++j) {
    const double r = sigma_max * (j + 1) / rings;
    ra.radius[j] = (float)r;
    ra.ofall[j] = (float)std::exp(-r * r / 2);
  }
  const int64_t V = g->n * (1 + rings * K), F = g->n * K * (2 * rings - 1);
  hipLaunchKernelGGL(k_rings_vertices, dim3(grid_for(V)), dim3(256), 0, s, g->mean, g->scale, g->quat, g->opacity,
                     g->rgb, g->n, K, rings, ra, out->pos, out->opacity, out->rgb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rings_faces, dim3(grid_for(F)), dim3(256), 0, s, g->n, K, rings, out->idx, out->gid);
  return hipGetLastError();
}

// Refiner MLP on the matrix cores: 15 -> 256 -> 256 -> (3K+4), ReLU, bfloat16
// operands with float32 accumulation (v_mfma_f32_16x16x32_bf16), the one dense
// contraction of the path. Not in the paper: it predicts corrections of each
// Gaussian's fan so fine-tuning starts nearer its optimum; a zero last layer
// reproduces the plain conversion.
//
// Inference (k_mlp_infer_lds) computes each layer transposed, so the hidden
// activations stay in registers, over weight copies whose k-blocks are stored
// in the matching slot order and held in LDS.
// Training (k_mlp_train) recomputes the forward one 32-sample group (two row
// tiles) per wavefront, the hidden activations going through a per-wave LDS
// tile (bfloat16) to turn the MFMA output layout into the next operand
// layout; its weights come from global memory (L2-resident, 155 KB in
// bfloat16) as 16-byte operand fragments, pre-packed as [out][in] rows (and
// transposed copies) so every fragment is contiguous, each applied to both
// row tiles. Then dH2 = (dY W3) * [h2>0] and dH1 = (dH2 W2) * [h1>0] (masks
// as register bits), bias gradients summed per wave in LDS, and bfloat16
// feature-major copies of x, h1, h2, dy, dh2, dh1 for the weight-gradient
// products dW = dH^T H, which k_wgrad_blocks computes per range of samples
// (each operand read once, partial products summed by k_wgrad_sum).
//
// MFMA 16x16x32 operand layout (lane l = 0..63, q = l / 16, r = l % 16):
//   A[i][k]: lane (i, q) holds k = 8q..8q+7;  B[k][j]: lane (j, q) holds k = 8q..8q+7;
//   D[i][j]: lane (j, q) holds i = 4q..4q+3.
#include <cmath>

#include "common.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int HID = 256;
constexpr int LDH = HID + 8;  // LDS row stride (bf16 elements) of a 16 x 256 tile
constexpr int WPB = 2;        // waves per block

// float -> bfloat16, round to nearest even (NaN stays a quiet NaN): one
// v_cvt_pk_bf16_f32 on gfx950.
__device__ __forceinline__ uint16_t bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ bf16x8 frag_from_u4(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ bf16x8 load_frag(const uint16_t* p) {  // 16-byte aligned
  return frag_from_u4(*reinterpret_cast<const u32x4*>(p));
}

__device__ __forceinline__ bf16x8 pack8(const float* v) {
  const bf16x8 b = {(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3],
                    (__bf16)v[4], (__bf16)v[5], (__bf16)v[6], (__bf16)v[7]};
  return b;
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Feature held by slot s = 8q + p of a 32-wide k-block in the transposed
// inference layout: slots 8q..8q+3 are features 4q..4q+3, slots 8q+4..8q+7
// are features 16+4q..16+4q+3.
__host__ __device__ constexpr int slot_feature(int s) {  // s = 8q + p within a 32-wide k-block
  return (s & 7) < 4 ? 4 * (s >> 3) + (s & 7) : 16 + 4 * (s >> 3) + (s & 7) - 4;
}

struct MlpArgs {
  const uint16_t* w1;   // [256][32]
  const uint16_t* w2;   // [256][256]
  const uint16_t* w3;   // [32][256]
  const uint16_t* w2t;  // [256][256]  w2t[i][o] = W2[o][i]
  const uint16_t* w3t;  // [256][32]   w3t[j][o] = W3[o][j]
  const uint16_t* w1t;  // [32][256]   w1t[k][i] = W1[i][k] (k < n_in, else 0)
  const float* b1;      // [256]
  const float* b2;      // [256]
  const float* b3;      // [32]
  int n_out;
};

struct TrainBufs {
  const float* dy;  // [N][n_out]
  uint16_t *xt, *h1t, *h2t, *dyt, *dh2t, *dh1t;  // feature-major, row length n_pad
  int64_t n_pad;
  float* bpart;            // [waves][2 HID + 32] per-wave bias-gradient sums (db1 | db2 | db3)
  float* dx;               // [N][16] input gradient (column 15 zero), or null
};

// Writes a D fragment (+bias, optional relu) of column block nb into an LDS tile as bf16.
__device__ __forceinline__ void store_tile(uint16_t* T, int nb, int lane, const float v[4]) {
  const int j = nb * 16 + (lane & 15), q = lane >> 4;
#pragma unroll
  for (int e = 0; e < 4; ++e) T[(4 * q + e) * LDH + j] = bf16_rne(v[e]);
}

__device__ __forceinline__ bf16x8 tile_frag(const uint16_t* T, int kb, int lane) {
  return load_frag(T + (lane & 15) * LDH + kb * 32 + 8 * (lane >> 4));
}

// feature-major bf16 store of a D fragment: dst[j][s0 + 4q + e]
__device__ __forceinline__ void store_t(uint16_t* dst, int64_t n_pad, int j, int64_t s, const float v[4]) {
  uint16_t* p = dst + (int64_t)j * n_pad + s;
  const uint32_t lo = (uint32_t)bf16_rne(v[0]) | ((uint32_t)bf16_rne(v[1]) << 16);
  const uint32_t hi = (uint32_t)bf16_rne(v[2]) | ((uint32_t)bf16_rne(v[3]) << 16);
  *reinterpret_cast<uint2*>(p) = make_uint2(lo, hi);
}

// sum of the 16 rows of a D fragment for column j (lanes sharing lane % 16)
__device__ __forceinline__ float col_sum(const float v[4]) {
  float s = (v[0] + v[1]) + (v[2] + v[3]);
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s;
}

// bit e set when v[e], rounded to bfloat16, is positive (sign clear, not zero)
__device__ __forceinline__ uint64_t positive_bits(const float v[4]) {
  uint64_t bits = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint16_t h = bf16_rne(v[e]);
    bits |= (uint64_t)((h & 0x7fffu) != 0 && !(h & 0x8000u)) << e;
  }
  return bits;
}

// One wavefront takes RT tiles of 16 samples at a time and applies every
// weight fragment it loads to all of them.
template <int RT>
__global__ __launch_bounds__(64 * WPB) void k_mlp_train(const float* __restrict__ x, int64_t N, MlpArgs m,
                                                        TrainBufs tb) {
  __shared__ uint16_t lds[WPB][RT][16 * LDH];
  __shared__ float dbl[WPB][2 * HID + 32];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int q = lane >> 4, r = lane & 15;
  // one LDS tile per wave and row tile: H1 (re-laid out as layer 2's
  // operand), then dH2 (as the operand of dH1); the ReLU masks stay in
  // registers, one bit per element this lane holds (block nb, row 4q + e ->
  // bit 4 nb + e)
  uint16_t* T[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) T[rt] = lds[wid][rt];
  // this wave's bias-gradient sums (db1, db2, db3), each address owned by one
  // lane; added to the global sums once, after the wave's last group
  float* dbw = dbl[wid];
  for (int i = lane; i < 2 * HID + 32; i += 64) dbw[i] = 0.f;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  const int64_t groups = (N + 16 * RT - 1) / (16 * RT);
  const int64_t g0 = (int64_t)blockIdx.x * WPB + wid;
  for (int64_t gi = g0; gi < groups; gi += (int64_t)gridDim.x * WPB) {
    const int64_t s0 = gi * 16 * RT;
    // ---- layer 1: A = x rows (16 features, padded to K = 32) ----
    bf16x8 ax[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int64_t srow = s0 + 16 * rt + r;  // the sample whose A row this lane carries
      float xv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) xv[e] = (q == 0 || q == 1) && srow < N ? x[srow * 16 + 8 * q + e] : 0.f;
      ax[rt] = pack8(xv);
      if (q < 2) {  // x^T for dW1 (features 0..15)
#pragma unroll
        for (int e = 0; e < 8; ++e) tb.xt[(int64_t)(8 * q + e) * tb.n_pad + srow] = bf16_rne(xv[e]);
      }
    }
    uint64_t m1[RT], m2[RT];  // [h1 > 0], [h2 > 0] as rounded to bfloat16
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) m1[rt] = m2[rt] = 0;
#pragma unroll 2
    for (int nb = 0; nb < 16; ++nb) {
      const bf16x8 w = load_frag(m.w1 + (nb * 16 + r) * 32 + 8 * q);
      const float b = m.b1[nb * 16 + r];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(ax[rt], w, acc);
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = fmaxf(acc[e] + b, 0.f);
        m1[rt] |= positive_bits(v) << (4 * nb);
        store_tile(T[rt], nb, lane, v);
        store_t(tb.h1t, tb.n_pad, nb * 16 + r, s0 + 16 * rt + 4 * q, v);
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    // ---- layer 2 ----
    bf16x8 a[RT][8];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) a[rt][kb] = tile_frag(T[rt], kb, lane);
    for (int nb = 0; nb < 16; ++nb) {
      f32x4 acc[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
      const uint16_t* wb = m.w2 + (nb * 16 + r) * HID + 8 * q;
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) {
        const bf16x8 w = load_frag(wb + kb * 32);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = mfma(a[rt][kb], w, acc[rt]);
      }
      const float b = m.b2[nb * 16 + r];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = fmaxf(acc[rt][e] + b, 0.f);
        m2[rt] |= positive_bits(v) << (4 * nb);
        store_t(tb.h2t, tb.n_pad, nb * 16 + r, s0 + 16 * rt + 4 * q, v);
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    // ---- backward: dY (K = 32, outputs padded) ----
    bf16x8 ady[RT];
    float s3[8];  // db3: sums over this group's samples (lanes sharing q)
#pragma unroll
    for (int e = 0; e < 8; ++e) s3[e] = 0.f;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int64_t srow = s0 + 16 * rt + r;
      float dv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int o = 8 * q + e;
        dv[e] = (o < m.n_out && srow < N) ? tb.dy[srow * m.n_out + o] : 0.f;
      }
      ady[rt] = pack8(dv);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        tb.dyt[(int64_t)(8 * q + e) * tb.n_pad + srow] = bf16_rne(dv[e]);
        s3[e] += dv[e];
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float s = s3[e];
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      s += __shfl_xor(s, 4);
      s += __shfl_xor(s, 8);
      if (r == 0) dbw[2 * HID + 8 * q + e] += s;
    }
    // dH2 = (dY W3) * [h2 > 0]
    for (int nb = 0; nb < 16; ++nb) {
      const bf16x8 w = load_frag(m.w3t + (nb * 16 + r) * 32 + 8 * q);
      const int j = nb * 16 + r;
      float sj = 0.f;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(ady[rt], w, acc);
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (m2[rt] >> (4 * nb + e)) & 1u ? acc[e] : 0.f;  // h2 > 0
        sj += col_sum(v);
        store_tile(T[rt], nb, lane, v);
        store_t(tb.dh2t, tb.n_pad, j, s0 + 16 * rt + 4 * q, v);
      }
      if (q == 0) dbw[HID + j] += sj;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    // dH1 = (dH2 W2) * [h1 > 0]
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) a[rt][kb] = tile_frag(T[rt], kb, lane);
    // the tiles are read before dH1 overwrites them (when dX is wanted)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    for (int nb = 0; nb < 16; ++nb) {
      f32x4 acc[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
      const uint16_t* wb = m.w2t + (nb * 16 + r) * HID + 8 * q;
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) {
        const bf16x8 w = load_frag(wb + kb * 32);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = mfma(a[rt][kb], w, acc[rt]);
      }
      const int j = nb * 16 + r;
      float sj = 0.f;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (m1[rt] >> (4 * nb + e)) & 1u ? acc[rt][e] : 0.f;  // h1 > 0
        sj += col_sum(v);
        store_t(tb.dh1t, tb.n_pad, j, s0 + 16 * rt + 4 * q, v);
        if (tb.dx) store_tile(T[rt], nb, lane, v);  // dH1 as the operand of dX
      }
      if (q == 0) dbw[j] += sj;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (tb.dx) {  // dX = dH1 W1 (input features 0..15; feature 15 has zero weights)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) a[rt][kb] = tile_frag(T[rt], kb, lane);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) acc = mfma(a[rt][kb], load_frag(m.w1t + r * HID + kb * 32 + 8 * q), acc);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t sample = s0 + 16 * rt + 4 * q + e;
          if (sample < N) tb.dx[sample * 16 + r] = acc[e];
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    }
  }
  // every wave writes its partial sums (zeros if it had no group); k_bias_sum adds
  // them in wave order, so the bias gradients are the same on every run
  float* bp = tb.bpart + ((int64_t)blockIdx.x * WPB + wid) * (2 * HID + 32);
  for (int i = lane; i < 2 * HID + 32; i += 64) bp[i] = dbw[i];
}

// bias gradients: the per-wave partial sums added in wave order
__global__ __launch_bounds__(256) void k_bias_sum(const float* __restrict__ bpart, int n_waves, int n_out,
                                                  float* __restrict__ db1, float* __restrict__ db2,
                                                  float* __restrict__ db3) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * HID + 32) return;
  float acc = 0.f;
  for (int w = 0; w < n_waves; ++w) acc += bpart[(int64_t)w * (2 * HID + 32) + i];
  if (i < HID) db1[i] = acc;
  else if (i < 2 * HID) db2[i - HID] = acc;
  else if (i - 2 * HID < n_out) db3[i - 2 * HID] = acc;
}

// Weight gradients C = A B^T, C[m][n] = sum_s A[m][s] B[n][s] over all samples
// (A, B bf16 feature-major rows of length n_pad), each operand read once:
// every block takes a contiguous range of samples and the whole M x NC
// product. Per 32 samples it stages both operands' columns in LDS (rows padded
// to 80 bytes, so the 16 lanes r of a fragment read hit distinct bank groups;
// the next step's columns are loaded while this step's products run), and
// each wavefront computes a (16 TM) x (16 TN) part of C from them. The block
// writes its partial product to part[block]; k_wgrad_sum adds the partials in
// block order (no atomics, the same result on every run).
template <int M, int NC>
struct WgradShape {
  // 64 x 64 per wavefront for the 256 x 256 product, 32 x 32 (eight waves)
  // when one side is 32 wide
  static constexpr int TM = (M < 64 || NC < 64) ? 2 : 4, TN = TM;
  static constexpr int WM = M / (16 * TM), WN = NC / (16 * TN), WAVES = WM * WN;
  static constexpr int ROWS = M + NC, LDR = 40;  // LDS row stride in bf16 elements (80 bytes)
  static constexpr int CHUNKS = ROWS * 4;        // 16-byte chunks of one 32-sample step
  static constexpr int PER = (CHUNKS + 64 * WAVES - 1) / (64 * WAVES);
};

template <int M, int NC>
__global__ __launch_bounds__((64 * WgradShape<M, NC>::WAVES)) void k_wgrad_blocks(const uint16_t* __restrict__ A,
                                                                              const uint16_t* __restrict__ B,
                                                                              int64_t n_pad, int64_t span,
                                                                              float* __restrict__ part) {
  using S = WgradShape<M, NC>;
  constexpr int NT = 64 * S::WAVES;
  __shared__ __attribute__((aligned(16))) uint16_t st[2][S::ROWS * S::LDR];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, q = lane >> 4, r = lane & 15;
  const int wm = wid / S::WN, wn = wid % S::WN;
  const int64_t k0 = (int64_t)blockIdx.x * span;
  const int64_t k1 = k0 + span < n_pad ? k0 + span : n_pad;
  u32x4 v[S::PER];
#pragma unroll
  for (int i = 0; i < S::PER; ++i) v[i] = u32x4{0u, 0u, 0u, 0u};
  // columns [k, k + 32) of both operands: chunk c is 16 bytes of row c / 4
#pragma unroll
  for (int i = 0; i < S::PER; ++i) {
    const int c = tid + i * NT;
    if (c < S::CHUNKS && k0 < k1) {
      const int row = c >> 2;
      const uint16_t* src = row < M ? A + (int64_t)row * n_pad : B + (int64_t)(row - M) * n_pad;
      v[i] = *reinterpret_cast<const u32x4*>(src + k0 + (c & 3) * 8);
    }
  }
#pragma unroll
  for (int i = 0; i < S::PER; ++i) {
    const int c = tid + i * NT;
    if (c < S::CHUNKS) *reinterpret_cast<u32x4*>(st[0] + (c >> 2) * S::LDR + (c & 3) * 8) = v[i];
  }
  __syncthreads();
  f32x4 acc[S::TM][S::TN];
#pragma unroll
  for (int tm = 0; tm < S::TM; ++tm)
#pragma unroll
    for (int tn = 0; tn < S::TN; ++tn) acc[tm][tn] = f32x4{0.f, 0.f, 0.f, 0.f};
  int buf = 0;
  for (int64_t k = k0; k < k1; k += 32) {
    const bool more = k + 32 < k1;
    if (more) {
#pragma unroll
      for (int i = 0; i < S::PER; ++i) {
        const int c = tid + i * NT;
        if (c < S::CHUNKS) {
          const int row = c >> 2;
          const uint16_t* src = row < M ? A + (int64_t)row * n_pad : B + (int64_t)(row - M) * n_pad;
          v[i] = *reinterpret_cast<const u32x4*>(src + k + 32 + (c & 3) * 8);
        }
      }
    }
    const uint16_t* sa = st[buf] + (wm * 16 * S::TM + r) * S::LDR + 8 * q;
    const uint16_t* sb = st[buf] + (M + wn * 16 * S::TN + r) * S::LDR + 8 * q;
    bf16x8 fa[S::TM], fb[S::TN];
#pragma unroll
    for (int tm = 0; tm < S::TM; ++tm) fa[tm] = load_frag(sa + tm * 16 * S::LDR);
#pragma unroll
    for (int tn = 0; tn < S::TN; ++tn) fb[tn] = load_frag(sb + tn * 16 * S::LDR);
#pragma unroll
    for (int tm = 0; tm < S::TM; ++tm)
#pragma unroll
      for (int tn = 0; tn < S::TN; ++tn) acc[tm][tn] = mfma(fa[tm], fb[tn], acc[tm][tn]);
    if (more) {
#pragma unroll
      for (int i = 0; i < S::PER; ++i) {
        const int c = tid + i * NT;
        if (c < S::CHUNKS) *reinterpret_cast<u32x4*>(st[buf ^ 1] + (c >> 2) * S::LDR + (c & 3) * 8) = v[i];
      }
    }
    __syncthreads();  // the other buffer is complete, this one free for the step after
    buf ^= 1;
  }
  float* pb = part + (int64_t)blockIdx.x * M * NC;
#pragma unroll
  for (int tm = 0; tm < S::TM; ++tm)
#pragma unroll
    for (int tn = 0; tn < S::TN; ++tn) {
      const int col = (wn * S::TN + tn) * 16 + r;
#pragma unroll
      for (int e = 0; e < 4; ++e) pb[((wm * S::TM + tm) * 16 + 4 * q + e) * NC + col] = acc[tm][tn][e];
    }
}

// C[i] = sum over blocks b of part[b][i]: a workgroup of 256 threads takes 64
// outputs; thread (o, g) sums the partials b = g, g + 4, ... of output o with
// eight loads in flight, and the four sums of an output are added in a fixed
// order (the same result on every run).
__global__ __launch_bounds__(256) void k_wgrad_sum(const float* __restrict__ part, int nb, int64_t len,
                                                   float* __restrict__ C) {
  __shared__ float red[4][64];
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + o;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (i < len) {
    int b = g;
    for (; b + 28 < nb; b += 32) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += part[(int64_t)(b + 4 * u) * len + i];
    }
    for (; b < nb; b += 4) acc[0] += part[(int64_t)b * len + i];
  }
  red[g][o] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (g == 0 && i < len) C[i] = (red[0][o] + red[1][o]) + (red[2][o] + red[3][o]);
}

// ---- packing: fp32 masters -> padded bf16 operands and transposed copies ----
__global__ void k_pack(const float* __restrict__ W1, const float* __restrict__ W2, const float* __restrict__ W3,
                       const float* __restrict__ b3, int n_in, int n_out, uint16_t* w1, uint16_t* w2, uint16_t* w3,
                       uint16_t* w2t, uint16_t* w3t, uint16_t* w2p, uint16_t* w3p, uint16_t* w1t, float* b3p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < HID * 32) {
    const int o = i / 32, k = i % 32;
    w1[i] = k < n_in ? bf16_rne(W1[o * n_in + k]) : 0;
    const int j = i / 32, oo = i % 32;  // w3t[j][o]
    w3t[i] = oo < n_out ? bf16_rne(W3[oo * HID + j]) : 0;
    const int o3 = i / HID, k3 = i % HID;  // w3[o][k]
    w3[i] = o3 < n_out ? bf16_rne(W3[o3 * HID + k3]) : 0;
    const int f3 = (k3 & ~31) + slot_feature(k3 & 31);  // w3p[o][slot]
    w3p[i] = o3 < n_out ? bf16_rne(W3[o3 * HID + f3]) : 0;
    const int k1 = i / HID, j1 = i % HID;  // w1t[k][i]
    w1t[i] = k1 < n_in ? bf16_rne(W1[j1 * n_in + k1]) : 0;
  }
  if (i < HID * HID) {
    w2[i] = bf16_rne(W2[i]);
    const int a = i / HID, b = i % HID;  // w2t[a][b] = W2[b][a]
    w2t[i] = bf16_rne(W2[b * HID + a]);
    w2p[i] = bf16_rne(W2[a * HID + (b & ~31) + slot_feature(b & 31)]);  // w2p[o][slot]
  }
  if (i < 32) b3p[i] = i < n_out ? b3[i] : 0.f;
}

__global__ void k_unpack_grads(const float* __restrict__ g1, const float* __restrict__ g3, int n_in, int n_out,
                               float* __restrict__ dW1, float* __restrict__ dW3) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < HID * n_in) dW1[i] = g1[(i / n_in) * 32 + i % n_in];
  if (i < n_out * HID) dW3[i] = g3[i];
}

// ---- features and application of the refiner outputs ----
__device__ inline void rcol(float w, float x, float y, float z, int col, float& r0, float& r1, float& r2) {
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

__global__ void k_features(const float* __restrict__ mean, const float* __restrict__ scale,
                           const float* __restrict__ quat, const float* __restrict__ opacity,
                           const float* __restrict__ rgb, int64_t n, int K, float* __restrict__ x) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float qw = quat[g], qx = quat[n + g], qy = quat[2 * n + g], qz = quat[3 * n + g];
  const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float sg = qw < 0.f ? -1.f : 1.f;
  float* o = x + g * 16;
  o[0] = mean[g];
  o[1] = mean[n + g];
  o[2] = mean[2 * n + g];
  o[3] = scale[g] / 0.1f;
  o[4] = scale[n + g] / 0.1f;
  o[5] = scale[2 * n + g] / 0.1f;
  o[6] = sg * qw / qn;
  o[7] = sg * qx / qn;
  o[8] = sg * qy / qn;
  o[9] = sg * qz / qn;
  o[10] = opacity[g];
  o[11] = rgb[g];
  o[12] = rgb[n + g];
  o[13] = rgb[2 * n + g];
  o[14] = (float)K / 16.f;
  o[15] = 0.f;
}

struct CS {
  float c[64], s[64];
};

__global__ void k_apply(const float* __restrict__ mean, const float* __restrict__ scale,
                        const float* __restrict__ quat, const float* __restrict__ opacity,
                        const float* __restrict__ rgb, int64_t n, int K, float sigma, float opac_mul, CS cs,
                        const float* __restrict__ y, int n_out, float* __restrict__ pos, float* __restrict__ vop,
                        float* __restrict__ vrgb) {
  const int64_t V = n * (K + 1);
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int64_t g = v / (K + 1);
  const int j = (int)(v - g * (K + 1));
  const float* yg = y + g * n_out;
  float px = mean[g], py = mean[n + g], pz = mean[2 * n + g];
  const float o = fminf(fmaxf(opacity[g] + yg[3 * K], 0.f), 1.f);
  if (j > 0) {
    const int k = j - 1;
    const float s0 = scale[g], s1 = scale[n + g], s2 = scale[2 * n + g];
    const int drop = (s2 <= s0 && s2 <= s1) ? 2 : (s1 <= s0 ? 1 : 0);
    const int ia = drop == 0 ? 1 : 0, ib = drop == 2 ? 1 : 2;
    const float sa = ia == 0 ? s0 : s1, sb = ib == 1 ? s1 : s2;
    const float qw = quat[g], qx = quat[n + g], qy = quat[2 * n + g], qz = quat[3 * n + g];
    float a0, a1, a2, b0, b1, b2;
    rcol(qw, qx, qy, qz, ia, a0, a1, a2);
    rcol(qw, qx, qy, qz, ib, b0, b1, b2);
    const float n0 = a1 * b2 - a2 * b1, n1 = a2 * b0 - a0 * b2, n2 = a0 * b1 - a1 * b0;
    const float la = sigma * sa, lb = sigma * sb, lc = sqrtf(la * lb);
    const float ca = cs.c[k] * la + yg[3 * k] * la;
    const float cb = cs.s[k] * lb + yg[3 * k + 1] * lb;
    const float cn = yg[3 * k + 2] * lc;
    px += ca * a0 + cb * b0 + cn * n0;
    py += ca * a1 + cb * b1 + cn * n1;
    pz += ca * a2 + cb * b2 + cn * n2;
  }
  pos[v] = px;
  pos[V + v] = py;
  pos[2 * V + v] = pz;
  vop[v] = j == 0 ? o : opac_mul * o;
  vrgb[v] = rgb[g] + yg[3 * K + 1];
  vrgb[V + v] = rgb[n + g] + yg[3 * K + 2];
  vrgb[2 * V + v] = rgb[2 * n + g] + yg[3 * K + 3];
}

// adjoint of k_apply: dL/dy from the gradients of the refined fan's vertices
__global__ void k_apply_backward(const float* __restrict__ scale, const float* __restrict__ quat,
                                 const float* __restrict__ opacity, int64_t n, int K, float sigma, float opac_mul,
                                 const float* __restrict__ y, int n_out, const float* __restrict__ dpos,
                                 const float* __restrict__ dop, const float* __restrict__ drgb,
                                 float* __restrict__ dy) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int64_t V = n * (K + 1);
  const float s0 = scale[g], s1 = scale[n + g], s2 = scale[2 * n + g];
  const int drop = (s2 <= s0 && s2 <= s1) ? 2 : (s1 <= s0 ? 1 : 0);
  const int ia = drop == 0 ? 1 : 0, ib = drop == 2 ? 1 : 2;
  const float sa = ia == 0 ? s0 : s1, sb = ib == 1 ? s1 : s2;
  const float qw = quat[g], qx = quat[n + g], qy = quat[2 * n + g], qz = quat[3 * n + g];
  float a0, a1, a2, b0, b1, b2;
  rcol(qw, qx, qy, qz, ia, a0, a1, a2);
  rcol(qw, qx, qy, qz, ib, b0, b1, b2);
  const float n0 = a1 * b2 - a2 * b1, n1 = a2 * b0 - a0 * b2, n2 = a0 * b1 - a1 * b0;
  const float la = sigma * sa, lb = sigma * sb, lc = sqrtf(la * lb);
  const float* yg = y + g * n_out;
  float* dg = dy + g * n_out;
  const int64_t v0 = g * (K + 1);
  for (int k = 0; k < K; ++k) {
    const int64_t v = v0 + 1 + k;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if (dpos) {
      gx = dpos[v];
      gy = dpos[V + v];
      gz = dpos[2 * V + v];
    }
    dg[3 * k] = la * (gx * a0 + gy * a1 + gz * a2);
    dg[3 * k + 1] = lb * (gx * b0 + gy * b1 + gz * b2);
    dg[3 * k + 2] = lc * (gx * n0 + gy * n1 + gz * n2);
  }
  const float u = opacity[g] + yg[3 * K];
  float go = 0.f;
  if (dop && u > 0.f && u < 1.f) {
    float sb_ = 0.f;
    for (int k = 1; k <= K; ++k) sb_ += dop[v0 + k];
    go = dop[v0] + opac_mul * sb_;
  }
  dg[3 * K] = go;
  float cr = 0.f, cg = 0.f, cb = 0.f;
  if (drgb) {
    for (int j = 0; j <= K; ++j) {
      cr += drgb[v0 + j];
      cg += drgb[V + v0 + j];
      cb += drgb[2 * V + v0 + j];
    }
  }
  dg[3 * K + 1] = cr;
  dg[3 * K + 2] = cg;
  dg[3 * K + 3] = cb;
}

// least-squares refiner targets from fine-tuned fans (same vertex layout as the plain fan)
__global__ void k_targets(const float* __restrict__ mean, const float* __restrict__ scale,
                          const float* __restrict__ quat, const float* __restrict__ opacity,
                          const float* __restrict__ rgb, int64_t n, int K, float sigma, float opac_mul, CS cs,
                          const float* __restrict__ tpos, const float* __restrict__ top,
                          const float* __restrict__ trgb, float* __restrict__ y) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int64_t V = n * (K + 1);
  const int n_out = 3 * K + 4;
  const float s0 = scale[g], s1 = scale[n + g], s2 = scale[2 * n + g];
  const int drop = (s2 <= s0 && s2 <= s1) ? 2 : (s1 <= s0 ? 1 : 0);
  const int ia = drop == 0 ? 1 : 0, ib = drop == 2 ? 1 : 2;
  const float sa = ia == 0 ? s0 : s1, sb = ib == 1 ? s1 : s2;
  const float qw = quat[g], qx = quat[n + g], qy = quat[2 * n + g], qz = quat[3 * n + g];
  float a0, a1, a2, b0, b1, b2;
  rcol(qw, qx, qy, qz, ia, a0, a1, a2);
  rcol(qw, qx, qy, qz, ib, b0, b1, b2);
  const float n0 = a1 * b2 - a2 * b1, n1 = a2 * b0 - a0 * b2, n2 = a0 * b1 - a1 * b0;
  const float la = sigma * sa, lb = sigma * sb, lc = sqrtf(la * lb);
  const float mx = mean[g], my = mean[n + g], mz = mean[2 * n + g];
  float* yg = y + g * n_out;
  for (int k = 0; k < K; ++k) {
    const int64_t v = g * (K + 1) + 1 + k;
    // plain boundary position
    const float px = mx + cs.c[k] * la * a0 + cs.s[k] * lb * b0;
    const float py = my + cs.c[k] * la * a1 + cs.s[k] * lb * b1;
    const float pz = mz + cs.c[k] * la * a2 + cs.s[k] * lb * b2;
    const float dx = tpos[v] - px, dy = tpos[V + v] - py, dz = tpos[2 * V + v] - pz;
    yg[3 * k] = (dx * a0 + dy * a1 + dz * a2) / fmaxf(la, 1e-12f);
    yg[3 * k + 1] = (dx * b0 + dy * b1 + dz * b2) / fmaxf(lb, 1e-12f);
    yg[3 * k + 2] = (dx * n0 + dy * n1 + dz * n2) / fmaxf(lc, 1e-12f);
  }
  const float o0 = opacity[g];
  float acc = top[g * (K + 1)] - o0;
  float cr = 0.f, cg = 0.f, cb = 0.f;
  for (int j = 0; j <= K; ++j) {
    const int64_t v = g * (K + 1) + j;
    if (j > 0) acc += opac_mul * (top[v] - opac_mul * o0);
    cr += trgb[v];
    cg += trgb[V + v];
    cb += trgb[2 * V + v];
  }
  yg[3 * K] = acc / (1.f + opac_mul * opac_mul * K);
  yg[3 * K + 1] = cr / (K + 1) - rgb[g];
  yg[3 * K + 2] = cg / (K + 1) - rgb[n + g];
  yg[3 * K + 3] = cb / (K + 1) - rgb[2 * n + g];
}

// per-output loss weights: boundary offsets by the squared world length of a
// unit of that local coordinate (a^2, b^2, a b) / ref^2, opacity and colour
// deltas by the fan's area over the area of the same K-gon of radius ref
__global__ void k_weights(const float* __restrict__ scale, int64_t n, int K, float sigma, float inv_ref2,
                          float* __restrict__ w) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const float s0 = scale[g], s1 = scale[n + g], s2 = scale[2 * n + g];
  const int drop = (s2 <= s0 && s2 <= s1) ? 2 : (s1 <= s0 ? 1 : 0);
  const float sa = drop == 0 ? s1 : s0, sb = drop == 2 ? s1 : s2;
  const float la = sigma * sa, lb = sigma * sb;
  const float wa = la * la * inv_ref2, wb = lb * lb * inv_ref2, wab = la * lb * inv_ref2;
  float* wg = w + g * (int64_t)(3 * K + 4);
  for (int k = 0; k < K; ++k) {
    wg[3 * k] = wa;
    wg[3 * k + 1] = wb;
    wg[3 * k + 2] = wab;
  }
  for (int q = 0; q < 4; ++q) wg[3 * K + q] = wab;
}

// (weighted) mean squared error over n values and its gradient; partial sums per block
__global__ __launch_bounds__(256) void k_vec_mse(const float* __restrict__ y, const float* __restrict__ t,
                                                 const float* __restrict__ w, int64_t n, float gscale,
                                                 float* __restrict__ dy, double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    const float wi = w ? w[i] : 1.f;
    acc += (double)wi * d * d;
    if (dy) dy[i] = 2.f * wi * d * gscale;
  }
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_vec_mse_sum(const double* __restrict__ part, int nb, double scale, float* __restrict__ out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += part[i];
    *out = (float)(s * scale);
  }
}

inline unsigned gfor(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b > 0 ? (n + b - 1) / b : 1); }

// Inference computes every layer transposed, D = W H^T (output features x
// samples): the D fragments of output blocks 2c and 2c + 1 then hold, in lane
// (sample r, q), features 32c + 4q + e and 32c + 16 + 4q + e (e = 0..3), which
// is the B-operand layout of the k-block c of the next layer once the slots
// 8q..8q+7 of that block are read as those eight features. The packed copies
// w2p and w3p store each row's k-blocks in that slot order, so the hidden
// activations stay in registers and each product is over the same
// 32 features as in the training forward (the same sums; only the order in
// which the matrix core adds the 32 products of a block may differ).

__device__ __forceinline__ f32x4 ld_f4(const float* p) { return *reinterpret_cast<const f32x4*>(p); }

__device__ __forceinline__ bf16x8 relu_pack(f32x4 a, f32x4 b) {
  float v[8];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[e] = fmaxf(a[e], 0.f);
    v[4 + e] = fmaxf(b[e], 0.f);
  }
  return pack8(v);
}

// relu, then bfloat16 pairs: elements 0..3 of an operand fragment
__device__ __forceinline__ uint2 relu_pack4(f32x4 a) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 lo = {(__bf16)fmaxf(a[0], 0.f), (__bf16)fmaxf(a[1], 0.f)};
  const bf16x2 hi = {(__bf16)fmaxf(a[2], 0.f), (__bf16)fmaxf(a[3], 0.f)};
  return make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
}

// W2 and W3 (slot-ordered copies) stay resident in LDS: one block per CU
// copies them once (rows padded to 528 bytes, so the 16 lanes r of a fragment
// read hit distinct bank groups), then each of its wavefronts runs through
// groups of RT row tiles (16 RT samples) on its own, applying every weight
// fragment it reads to all RT tiles; layer 3 is folded into layer 2 (each
// pair of layer-2 output blocks, once rectified and rounded, is one k-block
// of layer 3). Fragments come from LDS rather than L2, so no registers hold
// prefetched weights and a SIMD runs three wavefronts. The biases and the
// nonzero half of W1 (input features 0..15, 8 KB) sit in LDS too, so after
// the copy the only global traffic is the inputs and the outputs.
constexpr int kInferWaves = 12;  // wavefronts per block (three per SIMD)
constexpr int LDW = HID + 8;     // LDS row stride (bf16 elements) of the weight copies
constexpr int kInferRows = HID + 32;  // W2 rows, then W3 rows

template <int RT>
__global__ __launch_bounds__(64 * kInferWaves) __attribute__((amdgpu_waves_per_eu(kInferWaves / 4))) void k_mlp_infer_lds(
    const float* __restrict__ x, int64_t N, MlpArgs m, const uint16_t* __restrict__ w2p,
    const uint16_t* __restrict__ w3p, float* __restrict__ y) {
  __shared__ __attribute__((aligned(16))) uint16_t wl[kInferRows * LDW];
  __shared__ __attribute__((aligned(16))) float bl[2 * HID + 32];  // b1, b2, b3 (padded to 32)
  __shared__ __attribute__((aligned(16))) uint16_t w1l[HID * 16];   // W1 rows, input features 0..15
  for (int i = threadIdx.x; i < kInferRows * 32; i += blockDim.x) {
    const int row = i >> 5, ch = i & 31;  // 16-byte chunk ch of the row
    const uint16_t* src = row < HID ? w2p + row * HID + ch * 8 : w3p + (row - HID) * HID + ch * 8;
    *reinterpret_cast<u32x4*>(wl + row * LDW + ch * 8) = *reinterpret_cast<const u32x4*>(src);
  }
  for (int i = threadIdx.x; i < HID * 2; i += blockDim.x)  // two 16-byte chunks per row
    *reinterpret_cast<u32x4*>(w1l + i * 8) = *reinterpret_cast<const u32x4*>(m.w1 + (i >> 1) * 32 + (i & 1) * 8);
  for (int i = threadIdx.x; i < 2 * HID + 32; i += blockDim.x)
    bl[i] = i < HID ? m.b1[i] : i < 2 * HID ? m.b2[i - HID] : m.b3[i - 2 * HID];
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int q = lane >> 4, r = lane & 15;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  const int64_t groups = (N + 16 * RT - 1) / (16 * RT);
  const int64_t stride = (int64_t)gridDim.x * kInferWaves;
  const uint16_t* wr = wl + r * LDW + 8 * q;  // this lane's fragment base
  // a group's inputs in the B-operand layout (lane (sample r, q < 2) holds
  // features 8q..8q+7), loaded one group ahead: the loop's only other global
  // accesses are the output stores, issued after them
  int64_t gi = (int64_t)blockIdx.x * kInferWaves + wid;
  f32x4 xlo[RT], xhi[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t srow = gi * 16 * RT + 16 * rt + r;
    xlo[rt] = xhi[rt] = zero;
    if (gi < groups && q < 2 && srow < N) {
      xlo[rt] = ld_f4(x + srow * 16 + 8 * q);
      xhi[rt] = ld_f4(x + srow * 16 + 8 * q + 4);
    }
  }
  for (; gi < groups; gi += stride) {
    const int64_t s0 = gi * 16 * RT;
    // ---- layer 1: H1^T = relu(W1 X^T + b1), natural k order (x is the B operand) ----
    bf16x8 h1[RT][8];
    {
      bf16x8 xb[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const float xv[8] = {xlo[rt][0], xlo[rt][1], xlo[rt][2], xlo[rt][3],
                             xhi[rt][0], xhi[rt][1], xhi[rt][2], xhi[rt][3]};
        xb[rt] = pack8(xv);
      }
      const int64_t gn = gi + stride;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int64_t srow = gn * 16 * RT + 16 * rt + r;
        xlo[rt] = xhi[rt] = zero;
        if (gn < groups && q < 2 && srow < N) {
          xlo[rt] = ld_f4(x + srow * 16 + 8 * q);
          xhi[rt] = ld_f4(x + srow * 16 + 8 * q + 4);
        }
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        // lanes q >= 2 carry input slots 16..31, where x is zero: they read the
        // same weights as q - 2, and their products vanish
        const bf16x8 wa = load_frag(w1l + (32 * c + r) * 16 + 8 * (q & 1));
        const bf16x8 wb = load_frag(w1l + (32 * c + 16 + r) * 16 + 8 * (q & 1));
        const f32x4 ba = ld_f4(bl + 32 * c + 4 * q), bb = ld_f4(bl + 32 * c + 16 + 4 * q);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          h1[rt][c] = relu_pack(mfma(wa, xb[rt], zero) + ba, mfma(wb, xb[rt], zero) + bb);
        if (c % 4 == 3) __builtin_amdgcn_sched_barrier(0);  // bounds the loads hoisted ahead
      }
    }
    // ---- layers 2 and 3 ----
    f32x4 acc3[RT][2];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc3[rt][0] = acc3[rt][1] = zero;
#pragma unroll 1
    for (int c = 0; c < 8; ++c) {
      uint2 h2p[2][RT];  // rectified bf16 halves: features 32c + 4q + e, then 32c + 16 + 4q + e
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int nb = 2 * c + h;
        const f32x4 b = ld_f4(bl + HID + nb * 16 + 4 * q);
        f32x4 acc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = zero;
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
          const bf16x8 w = load_frag(wr + nb * 16 * LDW + kb * 32);
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) acc[rt] = mfma(w, h1[rt][kb], acc[rt]);
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) h2p[h][rt] = relu_pack4(acc[rt] + b);
      }
      const bf16x8 w3a = load_frag(wr + HID * LDW + c * 32);
      const bf16x8 w3b = load_frag(wr + (HID + 16) * LDW + c * 32);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const u32x4 u = {h2p[0][rt].x, h2p[0][rt].y, h2p[1][rt].x, h2p[1][rt].y};
        const bf16x8 h2 = frag_from_u4(u);
        acc3[rt][0] = mfma(w3a, h2, acc3[rt][0]);
        acc3[rt][1] = mfma(w3b, h2, acc3[rt][1]);
      }
    }
    // ---- output: lane (sample r, q) holds outputs 16 h + 4q + e ----
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const f32x4 b = ld_f4(bl + 2 * HID + 16 * h + 4 * q);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int64_t srow = s0 + 16 * rt + r;
        if (srow >= N) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = 16 * h + 4 * q + e;
          if (j < m.n_out) y[srow * m.n_out + j] = acc3[rt][h][e] + b[e];
        }
      }
    }
  }
}

}  // namespace

struct msp_refiner {
  int n_in = 15, n_out = 0;
  DevBuf w1, w2, w3, w2t, w3t, w2p, w3p, w1t, b1, b2, b3p, train, grads, part, wpart;
  int64_t train_pad = 0;
};

msp_refiner* refiner_new(int n_out) {
  msp_refiner* r = new msp_refiner();
  r->n_out = n_out;
  return r;
}

void refiner_delete(msp_refiner* r) { delete r; }
int refiner_n_out(const msp_refiner* r) { return r->n_out; }
double* refiner_part(msp_refiner* r) { return (double*)r->part.p; }

hipError_t launch_refiner_pack(hipStream_t s, msp_refiner* r, const float* W1, const float* b1, const float* W2,
                               const float* b2, const float* W3, const float* b3) {
  hipLaunchKernelGGL(k_pack, dim3(gfor(HID * HID)), dim3(256), 0, s, W1, W2, W3, b3, r->n_in, r->n_out,
                     (uint16_t*)r->w1.p, (uint16_t*)r->w2.p, (uint16_t*)r->w3.p, (uint16_t*)r->w2t.p,
                     (uint16_t*)r->w3t.p, (uint16_t*)r->w2p.p, (uint16_t*)r->w3p.p, (uint16_t*)r->w1t.p,
                     (float*)r->b3p.p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(r->b1.p, b1, 4 * HID, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(r->b2.p, b2, 4 * HID, hipMemcpyDeviceToDevice, s);
}

static MlpArgs margs(const msp_refiner* r) {
  MlpArgs m;
  m.w1 = (const uint16_t*)r->w1.p;
  m.w2 = (const uint16_t*)r->w2.p;
  m.w3 = (const uint16_t*)r->w3.p;
  m.w2t = (const uint16_t*)r->w2t.p;
  m.w3t = (const uint16_t*)r->w3t.p;
  m.w1t = (const uint16_t*)r->w1t.p;
  m.b1 = (const float*)r->b1.p;
  m.b2 = (const float*)r->b2.p;
  m.b3 = (const float*)r->b3p.p;
  m.n_out = r->n_out;
  return m;
}

constexpr int kInferRT = 2;  // row tiles per wavefront in inference

hipError_t launch_refiner_forward(hipStream_t s, const msp_refiner* r, const float* x, int64_t N, float* y, int n_cu) {
  if (N == 0) return hipSuccess;
  const int64_t groups = (N + 16 * kInferRT - 1) / (16 * kInferRT);
  int64_t g = (groups + kInferWaves - 1) / kInferWaves;
  g = g < 1 ? 1 : (g > n_cu ? n_cu : g);  // the LDS copy of the weights allows one block per CU
  hipLaunchKernelGGL(k_mlp_infer_lds<kInferRT>, dim3((unsigned)g), dim3(64 * kInferWaves), 0, s, x, N, margs(r),
                     (const uint16_t*)r->w2p.p, (const uint16_t*)r->w3p.p, y);
  return hipGetLastError();
}

// Row tiles of 16 samples per wavefront in the training kernel; the samples
// are padded to whole groups of 16 kTrainRT (a multiple of 32), so that the
// groups write every column of the training copies.
constexpr int kTrainRT = 2;
static_assert((16 * kTrainRT) % 32 == 0, "the weight-gradient kernels step through 32 samples");
static int64_t train_pad(int64_t N) { return (N + 16 * kTrainRT - 1) / (16 * kTrainRT) * (16 * kTrainRT); }

size_t refiner_train_bytes(int64_t N) {
  const int64_t np = train_pad(N);
  return (size_t)2 * np * (32 + 256 + 256 + 32 + 256 + 256) + 256;
}

hipError_t launch_refiner_backward(hipStream_t s, msp_refiner* r, const float* x, const float* dy, int64_t N,
                                   float* dW1, float* db1, float* dW2, float* db2, float* dW3, float* db3, float* dx,
                                   int n_cu) {
  const int64_t np = train_pad(N);
  uint16_t* base = (uint16_t*)r->train.p;
  TrainBufs tb;
  tb.dy = dy;
  tb.n_pad = np;
  tb.xt = base;
  tb.h1t = tb.xt + 32 * np;
  tb.h2t = tb.h1t + 256 * np;
  tb.dyt = tb.h2t + 256 * np;
  tb.dh2t = tb.dyt + 32 * np;
  tb.dh1t = tb.dh2t + 256 * np;
  tb.bpart = (float*)r->wpart.p;  // before the weight-gradient kernels reuse the buffer
  tb.dx = dx;
  hipError_t e;
  // k_mlp_train writes every column (its groups end at np, padded
  // samples as zeros or as the zero-input activations, whose gradients are
  // zero) of every row except the input feature rows 16..31 of xt, which must
  // read as zero
  if ((e = hipMemsetAsync(tb.xt + 16 * np, 0, 2 * 16 * np, s)) != hipSuccess) return e;
  if (N == 0) {  // no samples: zero bias gradients
    if ((e = hipMemsetAsync(db1, 0, 4 * HID, s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(db2, 0, 4 * HID, s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(db3, 0, 4 * r->n_out, s)) != hipSuccess) return e;
  }
  float* g1 = (float*)r->grads.p;  // [256][32]
  float* g3 = g1 + HID * 32;       // [32][256]
  if (N == 0) {  // no samples: zero weight gradients
    if ((e = hipMemsetAsync(g1, 0, 4 * (HID * 32 * 2), s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(dW2, 0, 4 * HID * HID, s)) != hipSuccess) return e;
  }
  if (N > 0) {
    // kTrainRT row tiles per wavefront: the groups end at np
    const int64_t groups = np / (16 * kTrainRT);
    int64_t gb = (groups + WPB - 1) / WPB;
    gb = gb > (int64_t)n_cu * 8 ? (int64_t)n_cu * 8 : gb;
    hipLaunchKernelGGL(k_mlp_train<kTrainRT>, dim3((unsigned)gb), dim3(64 * WPB), 0, s, x, N, margs(r), tb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_sum, dim3(gfor(2 * HID + 32)), dim3(256), 0, s, tb.bpart, (int)(gb * WPB), r->n_out,
                       db1, db2, db3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // dW3 = dY^T H2 : [32][256];  dW2 = dH2^T H1 : [256][256];  dW1 = dH1^T X : [256][32]
    // each over nbk sample ranges of `span` samples, then the partials summed
    int64_t nbk = np / 32 < n_cu ? np / 32 : n_cu;
    const int64_t span = (np / 32 + nbk - 1) / nbk * 32;
    nbk = (np + span - 1) / span;
    float* part = (float*)r->wpart.p;
    hipLaunchKernelGGL((k_wgrad_blocks<32, HID>), dim3((unsigned)nbk), dim3(64 * WgradShape<32, HID>::WAVES), 0, s,
                       tb.dyt, tb.h2t, np, span, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_sum, dim3(gfor(32 * HID, 64)), dim3(256), 0, s, part, (int)nbk, (int64_t)32 * HID, g3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_wgrad_blocks<HID, HID>), dim3((unsigned)nbk), dim3(64 * WgradShape<HID, HID>::WAVES), 0, s,
                       tb.dh2t, tb.h1t, np, span, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_sum, dim3(gfor(HID * HID, 64)), dim3(256), 0, s, part, (int)nbk, (int64_t)HID * HID, dW2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_wgrad_blocks<HID, 32>), dim3((unsigned)nbk), dim3(64 * WgradShape<HID, 32>::WAVES), 0, s,
                       tb.dh1t, tb.xt, np, span, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_sum, dim3(gfor(HID * 32, 64)), dim3(256), 0, s, part, (int)nbk, (int64_t)HID * 32, g1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_unpack_grads, dim3(gfor(HID * 32)), dim3(256), 0, s, g1, g3, r->n_in, r->n_out, dW1, dW3);
  return hipGetLastError();
}

hipError_t launch_refiner_features(hipStream_t s, const msp_gaussians* g, int K, float* x) {
  if (g->n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3(gfor(g->n)), dim3(256), 0, s, g->mean, g->scale, g->quat, g->opacity, g->rgb,
                     g->n, K, x);
  return hipGetLastError();
}

hipError_t launch_refiner_apply(hipStream_t s, const msp_gaussians* g, int K, float sigma, float opac_mul,
                                const float* y, int n_out, msp_faces* out) {
  if (g->n == 0) return hipSuccess;
  CS cs;
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < 64; ++k) {
    const double th = -pi + 2.0 * pi * k / K;
    cs.c[k] = k < K ? (float)std::cos(th) : 0.f;
    cs.s[k] = k < K ? (float)std::sin(th) : 0.f;
  }
  const int64_t V = g->n * (K + 1);
  hipLaunchKernelGGL(k_apply, dim3(gfor(V)), dim3(256), 0, s, g->mean, g->scale, g->quat, g->opacity, g->rgb, g->n, K,
                     sigma, opac_mul, cs, y, n_out, out->pos, out->opacity, out->rgb);
  return hipGetLastError();
}

hipError_t launch_refiner_targets(hipStream_t s, const msp_gaussians* g, int K, float sigma, float opac_mul,
                                  const msp_faces* tuned, float* y) {
  if (g->n == 0) return hipSuccess;
  CS cs;
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < 64; ++k) {
    cs.c[k] = k < K ? (float)std::cos(-pi + 2.0 * pi * k / K) : 0.f;
    cs.s[k] = k < K ? (float)std::sin(-pi + 2.0 * pi * k / K) : 0.f;
  }
  hipLaunchKernelGGL(k_targets, dim3(gfor(g->n)), dim3(256), 0, s, g->mean, g->scale, g->quat, g->opacity, g->rgb,
                     g->n, K, sigma, opac_mul, cs, tuned->pos, tuned->opacity, tuned->rgb, y);
  return hipGetLastError();
}

hipError_t launch_refiner_apply_backward(hipStream_t s, const msp_gaussians* g, int K, float sigma, float opac_mul,
                                         const float* y, const msp_face_grads* gr, float* dy) {
  if (g->n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply_backward, dim3(gfor(g->n)), dim3(256), 0, s, g->scale, g->quat, g->opacity, g->n, K,
                     sigma, opac_mul, y, 3 * K + 4, gr->dpos, gr->dopacity, gr->drgb, dy);
  return hipGetLastError();
}

hipError_t launch_refiner_weights(hipStream_t s, const msp_gaussians* g, int K, float sigma, float ref_len, float* w) {
  if (g->n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_weights, dim3(gfor(g->n)), dim3(256), 0, s, g->scale, g->n, K, sigma,
                     1.f / (ref_len * ref_len), w);
  return hipGetLastError();
}

hipError_t launch_vec_mse(hipStream_t s, const float* y, const float* t, const float* w, int64_t n, float* loss,
                          float* dy, double* part) {
  const unsigned nb = n > 0 ? (unsigned)std::min<int64_t>(1024, (n + 255) / 256) : 1;
  hipLaunchKernelGGL(k_vec_mse, dim3(nb), dim3(256), 0, s, y, t, w, n, 1.f / (float)(n > 0 ? n : 1), dy, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vec_mse_sum, dim3(1), dim3(64), 0, s, part, (int)nb, 1.0 / (double)(n > 0 ? n : 1), loss);
  return hipGetLastError();
}

int refiner_alloc(msp_ctx* ctx, msp_refiner* r) {
  int rc;
  if ((rc = msp_ensure(ctx, r->part, 8 * 1024)) || (rc = msp_ensure(ctx, r->w1, 2 * HID * 32)) || (rc = msp_ensure(ctx, r->w2, 2 * HID * HID)) ||
      (rc = msp_ensure(ctx, r->w3, 2 * 32 * HID)) || (rc = msp_ensure(ctx, r->w2t, 2 * HID * HID)) ||
      (rc = msp_ensure(ctx, r->w3t, 2 * HID * 32)) || (rc = msp_ensure(ctx, r->w2p, 2 * HID * HID)) ||
      (rc = msp_ensure(ctx, r->w3p, 2 * 32 * HID)) || (rc = msp_ensure(ctx, r->w1t, 2 * 32 * HID)) ||
      (rc = msp_ensure(ctx, r->b1, 4 * HID)) ||
      (rc = msp_ensure(ctx, r->b2, 4 * HID)) || (rc = msp_ensure(ctx, r->b3p, 4 * 32)) ||
      (rc = msp_ensure(ctx, r->grads, 4 * HID * 32 * 2)))
    return rc;
  return MSP_OK;
}

int refiner_train_alloc(msp_ctx* ctx, msp_refiner* r, int64_t N) {
  int rc;
  if ((rc = msp_ensure(ctx, r->train, refiner_train_bytes(N)))) return rc;
  // one partial weight gradient (up to 256 x 256) per block of the weight-gradient products
  return msp_ensure(ctx, r->wpart, (size_t)4 * ctx->n_cu * HID * HID);
}

void refiner_free_bufs(msp_refiner* r) {
  DevBuf* b[] = {&r->w1, &r->w2, &r->w3, &r->w2t, &r->w3t, &r->w2p, &r->w3p, &r->w1t, &r->b1, &r->b2, &r->b3p, &r->train, &r->grads, &r->part, &r->wpart};
  for (DevBuf* x : b)
    if (x->p) (void)hipFree(x->p);
}

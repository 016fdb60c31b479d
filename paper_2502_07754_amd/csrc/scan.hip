// Device-wide exclusive prefix sum (reduce -> scan of block sums -> apply),
// used to turn per-tile entry counts into tile-list offsets and per-block
// fragment capacities into list offsets. Each block owns a 2048-element tile;
// within a block, 64-wide wavefront inclusive scans (shuffle-up ladder)
// combine through LDS.
#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;

__device__ inline int64_t wave_incl_scan(int64_t x) {
  const int lane = threadIdx.x & (MSP_WAVE - 1);
#pragma unroll
  for (int d = 1; d < MSP_WAVE; d <<= 1) {
    const int64_t y = __shfl_up(x, d, MSP_WAVE);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread across the block; returns the block total in `total`.
__device__ inline int64_t block_excl_scan(int64_t x, int64_t& total) {
  __shared__ int64_t wsum[kThreads / MSP_WAVE];
  const int lane = threadIdx.x & (MSP_WAVE - 1);
  const int wid = threadIdx.x / MSP_WAVE;
  const int64_t inc = wave_incl_scan(x);
  if (lane == MSP_WAVE - 1) wsum[wid] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kThreads / MSP_WAVE; ++w) {
    if (w < wid) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  total = all;
  return before + inc - x;
}

template <class T>
__global__ void k_reduce(const T* __restrict__ in, int64_t n, int64_t* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i)
    if (base + i < n) s += (int64_t)in[base + i];
  int64_t total;
  block_excl_scan(s, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

template <class T>
__global__ void k_apply(const T* __restrict__ in, int64_t n, const int64_t* __restrict__ part_off,
                        int64_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  int64_t v[kItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    v[i] = (base + i < n) ? (int64_t)in[base + i] : 0;
    s += v[i];
  }
  int64_t total;
  int64_t run = block_excl_scan(s, total) + (part_off ? part_off[blockIdx.x] : 0);
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    out[n] = (part_off ? part_off[blockIdx.x] : 0) + total;
}

int64_t n_blocks(int64_t n) { return n <= 0 ? 1 : (n + kTile - 1) / kTile; }

template <class T>
hipError_t scan_rec(hipStream_t s, const T* in, int64_t* out, int64_t n, int64_t* scratch) {
  const int64_t nb = n_blocks(n);
  if (nb == 1) {
    hipLaunchKernelGGL(k_apply<T>, dim3(1), dim3(kThreads), 0, s, in, n, (const int64_t*)nullptr, out);
    return hipGetLastError();
  }
  int64_t* part = scratch;
  int64_t* part_off = scratch + nb;
  int64_t* rest = scratch + 2 * nb + 1;
  hipLaunchKernelGGL(k_reduce<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_rec<int64_t>(s, part, part_off, nb, rest);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_apply<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, (const int64_t*)part_off, out);
  return hipGetLastError();
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
  size_t words = 0;
  int64_t m = n;
  while (true) {
    const int64_t nb = n_blocks(m);
    if (nb == 1) break;
    words += 2 * nb + 1;
    m = nb;
  }
  return (words + 1) * sizeof(int64_t);
}

hipError_t launch_scan_u32(hipStream_t s, const uint32_t* in, int64_t* out, int64_t n, void* scratch) {
  return scan_rec<uint32_t>(s, in, out, n, (int64_t*)scratch);
}

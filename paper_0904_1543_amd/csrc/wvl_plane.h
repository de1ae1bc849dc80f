// Device helpers shared by the two in-plane kernels (vector and matrix-core).
#pragma once

#include "wvl_kernels.h"

namespace wvl {

constexpr int kXyThreads = 512;   // threads of an in-plane workgroup (8 waves)
constexpr int kXyWaves = kXyThreads / 64;
constexpr int kU = 4;             // outputs per work item of the vector engine
constexpr int kMaxItems = 8;      // vector-engine work items per thread and pass (m <= 128)

// Points of the plane owned by this thread: e = threadIdx.x + k * kXyThreads,
// with its LDS position y * pitch + x stepped incrementally.
struct PtIter {
  int e, x, y, dx, dy, m1;
  __device__ PtIter(int m1_) : m1(m1_) {
    e = threadIdx.x;
    x = threadIdx.x % m1_;
    y = threadIdx.x / m1_;
    dx = kXyThreads % m1_;
    dy = kXyThreads / m1_;
  }
  __device__ int pos(int pitch) const { return y * pitch + x; }
  __device__ void next() {
    e += kXyThreads;
    x += dx;
    y += dy;
    if (x >= m1) { x -= m1; ++y; }
  }
};

// Visit the points of the plane owned by this thread in batches of B: the
// B global loads of a batch (load(e)) are issued before any of them is used
// (use(e, pos, value)), so their latencies overlap instead of adding up.
template <int B, typename L, typename U>
__device__ __forceinline__ void plane_batched(int m1, int npl, int pitch, L&& load, U&& use) {
  PtIter q(m1);
  while (q.e < npl) {
    decltype(load(0)) v[B];
    int e[B], pos[B];
    #pragma unroll
    for (int k = 0; k < B; ++k) {
      e[k] = q.e;
      pos[k] = q.pos(pitch);
      if (q.e < npl) v[k] = load(q.e);
      q.next();
    }
    #pragma unroll
    for (int k = 0; k < B; ++k)
      if (e[k] < npl) use(e[k], pos[k], v[k]);
  }
}
constexpr int kPlaneBatch = 8;

__device__ __forceinline__ double xy_block_sum(double v) {
  __shared__ double red[kXyThreads / 64];
  #pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  #pragma unroll
  for (int w = 0; w < kXyThreads / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

}  // namespace wvl

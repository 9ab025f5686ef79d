// Workgroup and wavefront reductions in a fixed order (bitwise reproducible).
#pragma once

#include <hip/hip_runtime.h>

namespace ba {

// ---------------------------------------------------------------------------
// reduction helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the workgroup; result valid in every thread.  sh: >= blockDim/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  return s;
}

// Three sums over the workgroup in one exchange (fixed order); results
// valid in every thread.  sh: >= 3 * blockDim/64 doubles.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[3 * wid] = a;
    sh[3 * wid + 1] = b;
    sh[3 * wid + 2] = c;
  }
  __syncthreads();
  double x = 0.0, y = 0.0, z = 0.0;
  for (int i = 0; i < nw; ++i) {
    x += sh[3 * i];
    y += sh[3 * i + 1];
    z += sh[3 * i + 2];
  }
  a = x;
  b = y;
  c = z;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s = fmax(s, sh[i]);
  return s;
}

// Sum of arr[0..n) by one workgroup in a fixed order; valid in every thread.
__device__ __forceinline__ double block_sum_array(const double* __restrict__ arr, int n, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += arr[i];
  return block_sum(s, sh);
}

// The same for long arrays: four strided loads in flight per thread (four
// running sums, added in a fixed order at the end), then the workgroup tree.
__device__ __forceinline__ double block_sum_array4(const double* __restrict__ arr, int n, double* sh) {
  const int nt = blockDim.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * nt < n; i += 4 * nt) {
    const double a0 = arr[i], a1 = arr[i + nt], a2 = arr[i + 2 * nt], a3 = arr[i + 3 * nt];
    s0 += a0;
    s1 += a1;
    s2 += a2;
    s3 += a3;
  }
  for (; i < n; i += nt) s0 += arr[i];
  return block_sum((s0 + s1) + (s2 + s3), sh);
}

}  // namespace ba

// reduce.hpp -- deterministic wavefront / workgroup reductions in FP64.
#pragma once
#include <hip/hip_runtime.h>

namespace odp {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum in a fixed order (deterministic); every thread gets the total.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) t += sh[i];
  return t;
}

}  // namespace odp

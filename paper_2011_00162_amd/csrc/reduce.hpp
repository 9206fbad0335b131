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

// One frequency's terms of the frame constraint's residuals (penalty balancing):
// |Gamma^{n+1} - Gamma^n|^2 and |Gamma^{n+1}|^2 in FP32 (they only steer a factor-of-tau
// decision), added to FP64 sums one after the other (see elem_measures).
__device__ __forceinline__ void frame_terms(float2 g_old, float2 g_new, double& del, double& nrm) {
  const float dx = g_new.x - g_old.x, dy = g_new.y - g_old.y;
  del += (double)(dx * dx + dy * dy);
  nrm += (double)(g_new.x * g_new.x + g_new.y * g_new.y);
  asm volatile("" : "+v"(del), "+v"(nrm));
}

// A frame's statistics, summed over the workgroup in a fixed order: out[0..3] = (L1
// misfit, G_eps, |Gamma^{n+1} - Gamma^n|^2, |Gamma^{n+1}|^2); the last two are 0 unless
// FRES (the frame residuals are formed only where a penalty rule reads them).
template <int NT, bool FRES>
__device__ __forceinline__ void frame_stats(double* out, double mis, double gsum, double del, double nrm,
                                            double* sh) {
  mis = block_sum<NT>(mis, sh);
  gsum = block_sum<NT>(gsum, sh);
  if (FRES) {
    del = block_sum<NT>(del, sh);
    nrm = block_sum<NT>(nrm, sh);
  }
  if (threadIdx.x == 0) {
    out[0] = mis;
    out[1] = gsum;
    out[2] = FRES ? del : 0.0;
    out[3] = FRES ? nrm : 0.0;
  }
}

}  // namespace odp

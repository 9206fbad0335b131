// blind.hip -- probe steps of OD2BP (Algorithm 3 of the paper, Sec. 3.2).
//
//  w^{n+1}   = P_O( (1/D) sum_d (w_d^n + Delta_d^n) )                  (eq. blind_w, 1/D for D copies)
//  w_d^{n+1} = (eta sum_{j in d} conj(S_j u_d^n) o phi_j + mu (w^{n+1} - Delta_d^n))
//              / (eta sum_{j in d} |S_j u_d^n|^2 + mu)                 (eq. blind_W)
//  Delta_d^{n+1} = Delta_d^n + w_d^{n+1} - w^{n+1}                     (eq. admm_Delta)
// with phi_j = F^{-1}(Z_j - Gamma_j) from the frame sweep and P_O = F^{-1} M F the
// projection onto probes whose spectrum vanishes off the support mask M.
// The frame sums run in FP64 over each subdomain's frames in ascending order.
#include <hip/hip_runtime.h>

#include "fft_frame.hpp"
#include "odp_internal.hpp"

namespace odp {

template <int P, bool MASK>
__global__ __launch_bounds__(Frame<P>::T) void k_probe_mean(ProbeArgs a) {
  using F = Frame<P>;
  __shared__ float2 lds[MASK ? F::LDS : 1];
  const int t = threadIdx.x;
  const int col = F::a_col(t), r2 = F::a_r2(t);
  const double invD = 1.0 / (double)a.D;
  float2 v[16];
#pragma unroll
  for (int r1 = 0; r1 < 16; ++r1) {
    const int k = (F::N2 * r1 + r2) * P + col;
    double sx = 0.0, sy = 0.0;
    for (int d = 0; d < a.D; ++d) {
      const float2 ws = a.w_sub[(size_t)d * P * P + k], dl = a.delta[(size_t)d * P * P + k];
      sx += (double)ws.x + dl.x;
      sy += (double)ws.y + dl.y;
    }
    v[r1] = make_float2((float)(sx * invD), (float)(sy * invD));
  }
  if (MASK) {
    F::forward(v, lds, a.tw, t);
    const float s = 1.0f / (float)(P * P);   // both unitary factors
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      int kr, kc;
      F::freq(t, e, kr, kc);
      v[e] = c_scale(v[e], s * a.fmask[kr * P + kc]);
    }
    __syncthreads();
    F::inverse(v, lds, a.tw, t);
  }
#pragma unroll
  for (int r1 = 0; r1 < 16; ++r1) a.w[(F::N2 * r1 + r2) * P + col] = v[r1];
}

__global__ __launch_bounds__(256) void k_probe_copies(ProbeArgs a) {
  const int p = a.p, d = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= p * p) return;
  const int ky = k / p, kx = k % p;
  double nr = 0.0, ni = 0.0, den = 0.0;
  for (int q = a.sub_first[d]; q < a.sub_first[d + 1]; ++q) {
    const int j = a.order[q];
    const FrameDesc fd = a.frames[j];
    const float2 pu = a.u[fd.base + (int64_t)ky * fd.pitch + kx];
    const float2 ph = a.phi[(size_t)j * p * p + k];
    nr += (double)pu.x * ph.x + (double)pu.y * ph.y;   // conj(S_j u) o phi
    ni += (double)pu.x * ph.y - (double)pu.y * ph.x;
    den += (double)pu.x * pu.x + (double)pu.y * pu.y;
  }
  const size_t o = (size_t)d * p * p + k;
  const float2 w = a.w[k], dl = a.delta[o];
  const double q = a.eta * den + a.mu;
  const double wx = (a.eta * nr + a.mu * ((double)w.x - dl.x)) / q;
  const double wy = (a.eta * ni + a.mu * ((double)w.y - dl.y)) / q;
  a.w_sub[o] = make_float2((float)wx, (float)wy);
  a.delta[o] = make_float2((float)((double)dl.x + wx - w.x), (float)((double)dl.y + wy - w.y));
}

hipError_t launch_probe_update(const ProbeArgs& a, hipStream_t s) {
  const bool mask = a.fmask != nullptr;
#define ODP_MEAN(PP)                                                                             \
  if (a.p == PP) {                                                                               \
    if (mask) hipLaunchKernelGGL((k_probe_mean<PP, true>), dim3(1), dim3(Frame<PP>::T), 0, s, a);  \
    else hipLaunchKernelGGL((k_probe_mean<PP, false>), dim3(1), dim3(Frame<PP>::T), 0, s, a);      \
  }
  ODP_MEAN(32)
  ODP_MEAN(64)
  ODP_MEAN(128)
#undef ODP_MEAN
  hipLaunchKernelGGL(k_probe_copies, dim3((a.p * a.p + 255) / 256, a.D), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace odp

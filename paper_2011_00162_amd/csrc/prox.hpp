// prox.hpp -- the ST-AGM metric of eq. obj-1 and its closed-form proximal map (eq. Prox_sol).
#pragma once
#include <hip/hip_runtime.h>

namespace odp {

// Closed-form proximal map of the ST-AGM (eq. Prox_sol), with precomputed
// coefficients: thr = eps - (1-eps)/lam (truncated branch when |y| < thr*sqrt f),
// ctr = lam/(lam - (1-eps)/eps) (only used when thr > 0), ca = 1/(1+lam),
// cb = lam/(1+lam).  sign(0) = +1.
struct ProxC {
  float thr, ctr, ca, cb;
};

__host__ __device__ inline ProxC prox_coeffs(double eps, double lam) {
  const double kappa = (1.0 - eps) / eps;
  ProxC c;
  c.thr = (float)(eps - (1.0 - eps) / lam);
  c.ctr = lam > kappa ? (float)(lam / (lam - kappa)) : 0.0f;
  c.ca = (float)(1.0 / (1.0 + lam));
  c.cb = (float)(lam / (1.0 + lam));
  return c;
}

// Branch-free: selects only, so a wavefront never splits on the data.
__device__ __forceinline__ float2 prox_stagm(float2 y, float sf, const ProxC& c) {
  const float a2 = y.x * y.x + y.y * y.y;
  const bool nz = a2 > 0.0f;
  const float inv = nz ? __builtin_amdgcn_rsqf(a2) : 0.0f;   // 1/|y|, about 1 ulp
  const float ay = a2 * inv;                                  // |y| (0 for y = 0)
  const float rho = (ay < c.thr * sf) ? fmaxf(0.0f, ay * c.ctr) : fmaf(sf, c.ca, ay * c.cb);
  const float s = rho * inv;
  // y = 0: every phase is a minimiser; sign(0) = +1
  return nz ? make_float2(y.x * s, y.y * s) : make_float2(rho, 0.0f);
}

// One frame element's terms of the iteration's measures (Sec. 4): the misfit
// | |X| - sqrt(f) | and g_eps(X; f), from the FP32 spectrum X in FP32 (|X| by the
// hardware square root, about an ulp; g_eps is continuous where its branch switches, so
// a switch near the threshold moves nothing).  gcoef = (1 - eps) / (2 eps): the truncated
// branch is gcoef (eps f - |X|^2).  Branch-free; each term is added to the caller's FP64
// sums, one element after the other (an empty asm on the sums keeps the scheduler from
// interleaving the temporaries of many elements, which spilled).
__device__ __forceinline__ void elem_measures(float2 X, float sf, float eps, float gcoef, double& mis,
                                              double& gsum) {
  const float ax2 = fmaf(X.x, X.x, X.y * X.y);
  const float ax = __builtin_amdgcn_sqrtf(ax2);
  const float d = ax - sf;
  const float esf = eps * sf;
  const float gt = gcoef * fmaf(esf, sf, -ax2);
  const float gq = 0.5f * d * d;
  mis += (double)fabsf(d);
  gsum += (double)(ax < esf ? gt : gq);
  asm volatile("" : "+v"(mis), "+v"(gsum));
}

}  // namespace odp

// kernels.hip -- HIP kernels of the OD2P / OD2Pm / OD2BP hot path for gfx950.
//
// Frame kernels run one workgroup per scan frame (p*p/16 threads, 16 complex
// values per thread, frame transform through LDS, see fft_frame.hpp).  The pixel
// update and the illumination reciprocals are in pixel.hip.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "fft_frame.hpp"
#include "fft_mfma.hpp"
#include "odp_internal.hpp"
#include "prox.hpp"
#include "reduce.hpp"

namespace odp {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ void atomic_add_c(float2* p, float2 v) {
  unsafeAtomicAdd(&p->x, v.x);
  unsafeAtomicAdd(&p->y, v.y);
}

__device__ __forceinline__ int sweep_pos(int32_t chunk, int xcd_slice) {
  // XCD-aware slicing: workgroup b runs on XCD b % 8; each XCD takes a
  // contiguous slice of the subdomain-grouped frame order, so neighbouring
  // windows (which share image patches) share one L2.  The autotuner may pick
  // the plain order instead.
  const int b = blockIdx.x;
  return xcd_slice ? (b % NXCD) * chunk + b / NXCD : b;
}

// ---------------------------------------------------------------------------
// K1: frame sweep (Alg. 2 Steps 1-2 for the frames, the A_d* half of Step 3)
//   X = F(w o S_j u_d); y = Gamma + X; z = Prox(y); Gamma <- y - z;
//   psi_j = conj(w) o F^{-1}(z - Gamma)   (blind: F^{-1}(z - Gamma), the probe
//   and image steps each apply their own probe copy)
// Each frame's output goes to its own slot of psi, so no two workgroups write
// the same address; the pixel update pulls the covering frames in a fixed order.
// ---------------------------------------------------------------------------
// ST: 0 no statistics, 1 the iteration's measures, 2 also the frame residuals.
// MF: radix-16 stages on the matrix cores (FrameMF, split BF16), else Frame's FP32 stages.
// NT: streaming (non-temporal) accesses to the frame arrays (ld_s / st_s).
template <int P, bool MF, bool BLIND, int ST, bool NT>
__global__ __launch_bounds__(Frame<P>::T, MF && P == 64 && ST == 0 ? 4 : 1) void k_sweep(SweepArgs a, ProxC pc) {
  using F = Frame<P>;
  using M = FrameMF<P>;    // instantiated only when MF
  constexpr bool STATS = ST > 0;
  __shared__ __align__(16) float2 lds[F::LDS];
  __shared__ __align__(16) float2 twl[F::N2 * TWL];   // stage-B twiddles, read from LDS so that no
                                       // wait on them also waits on the prefetches
  __shared__ double red[F::T / 64];
  const int pos = sweep_pos(a.chunk, a.xcd_slice);
  if (pos >= a.J) return;  // uniform over the workgroup
  const int t = threadIdx.x;
  const FrameDesc fd = a.fpos[pos];
  if (a.stop && a.stop[fd.probe].stopped) return;   // its problem met its stopping rule
  const int j = fd.j;
  const size_t woff = (size_t)(a.w_per_sub ? fd.sub : fd.probe) * P * P;
  const float2* w = a.w + woff;
  const int col = F::a_col(t), r2 = F::a_r2(t);
  const float inv_p = 1.0f / (float)P;

  // the thread's 16 spatial positions (the inverse returns its values to the same ones)
  auto prow = [&](int e) { if constexpr (MF) return M::row(t, e); else return F::N2 * e + r2; };
  auto pcol = [&](int e) { if constexpr (MF) return M::col(t, e); else return col; };
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int row = prow(e), c = pcol(e);
    v[e] = c_mul(a.u[fd.base + (int64_t)row * fd.pitch + c], w[row * P + c]);
  }
  if constexpr (MF) {
    M::forward_a(v, lds, a.mft, t);
  } else {
    // the stage-B twiddles go to LDS after the gather's loads are issued, so waiting for
    // this copy overlaps their latency; visible after the first barrier of forward_bc
    if (t < F::N2 * 16) twl[(t >> 4) * TWL + (t & 15)] = a.tw[t];
    F::forward_a(v, lds, a.tw, t);
  }
  // The thread's amplitudes (and, for P <= 64, multipliers) are fetched now, while
  // stages B and C run: between stages A and C the thread holds no frame data in
  // registers.  At P = 128 (1024 threads, 128 VGPRs) only the amplitudes fit.
  constexpr int PRE = 1;
  const size_t fbase = (size_t)j * P * P;
  float2 gpre[16];
  float spre[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    int kr, kc;
    F::freq(t, e, kr, kc);
    if (PRE >= 1) spre[e] = ld_s<NT>(a.sqrt_f + fbase + kr * P + kc);
    if (PRE >= 2) gpre[e] = ld_s<NT>(a.gamma + fbase + kr * P + kc);
  }
  if constexpr (MF) M::forward_bc(v, lds, a.mft, t);
  else F::template forward_bc<TWL>(v, lds, twl, t);

  // all 16 multipliers are read before any is written back, so the loads are in
  // flight together (the stores could otherwise alias later loads for the compiler)
  if (PRE < 2) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      int kr, kc;
      F::freq(t, e, kr, kc);
      gpre[e] = ld_s<NT>(a.gamma + fbase + kr * P + kc);
    }
  }
  double mis = 0.0, gsum = 0.0, gdel = 0.0, gnrm = 0.0;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    int kr, kc;
    F::freq(t, e, kr, kc);
    const size_t idx = fbase + kr * P + kc;
    const float2 X = c_scale(v[e], inv_p);
    const float sf = PRE >= 1 ? spre[e] : ld_s<NT>(a.sqrt_f + idx);
    const float2 y = c_add(gpre[e], X);
    const float2 z = prox_stagm(y, sf, pc);
    const float2 g = c_sub(y, z);
    if (STATS) {
      elem_measures(X, sf, a.eps, a.gcoef, mis, gsum);
      if (ST > 1) frame_terms(gpre[e], g, gdel, gnrm);
    }
    gpre[e] = g;
    v[e] = c_scale(c_sub(z, g), inv_p);   // both 1/p factors of the unitary pair applied here
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    int kr, kc;
    F::freq(t, e, kr, kc);
    st_s<NT>(a.gamma + fbase + kr * P + kc, gpre[e]);
  }
  if (STATS) frame_stats<F::T, (ST > 1)>(a.part + NFS * (size_t)j, mis, gsum, gdel, gnrm, red);
  __syncthreads();  // stage-C reads of all threads done before inverse writes reuse LDS
  if constexpr (MF) M::inverse(v, lds, a.mft, t);
  else F::template inverse<TWL>(v, lds, twl, t);
  // the inverse returns each thread's 16 points to the positions it gathered; the 16
  // probe values are read before any output is written, so they are in flight together
  if (!BLIND) {
    const float2* wo = a.w_out + woff;
    float2 wk[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) wk[e] = wo[prow(e) * P + pcol(e)];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = c_mulc(v[e], wk[e]);
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) st_s<NT>(a.psi + fbase + prow(e) * P + pcol(e), v[e]);
}

// K1 at p = 128: the same step on the two-half transform (Half128: 512 threads,
// 77 KB of LDS, two frames per CU).  The prox of each half runs between that half's
// forward and inverse stages B and C.
// MF: stages A and B on the matrix cores (Half128MF, split BF16).
template <bool MF, bool BLIND, int ST, bool NT>
__global__ __launch_bounds__(Half128::T) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_sweep128(SweepArgs a, ProxC pc) {
  using F = Half128;
  using M = Half128MF;
  constexpr bool STATS = ST > 0;
  constexpr int P = 128;
  __shared__ __align__(16) float2 lds[F::LDS];
  __shared__ __align__(16) float2 twl[F::N2 * TWL];
  __shared__ double red[F::T / 64];
  const int pos = sweep_pos(a.chunk, a.xcd_slice);
  if (pos >= a.J) return;  // uniform over the workgroup
  const int t = threadIdx.x;
  const FrameDesc fd = a.fpos[pos];
  if (a.stop && a.stop[fd.probe].stopped) return;   // its problem met its stopping rule
  const int j = fd.j;
  const size_t woff = (size_t)(a.w_per_sub ? fd.sub : fd.probe) * P * P;
  const float2* w = a.w + woff;
  // per-frame scalar bases; the per-element offsets below are 32-bit (a window spans
  // at most 128 rows of its subdomain, a frame 128 x 128 values)
  const float2* ub = a.u + fd.base;
  const size_t fbase = (size_t)j * P * P;
  float2* gb = a.gamma + fbase;
  const float* sb = a.sqrt_f + fbase;
  float2* pb = a.psi + fbase;
  const int col = F::a_col(t);
  const float inv_p = 1.0f / (float)P;

  // gather and stage A one line at a time; the second line's gather runs in groups of
  // 8 rows, so the first line's transform and 16 products stay in registers without
  // spilling
  float2 v[32];
  if constexpr (MF) {
    // gather and stage A two line blocks at a time (8 slots), the next group's loads
    // after the current group's products
    const mf::Tab A = M::tab_a(a.mft, 0, t);
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
#pragma unroll
      for (int e = 8 * grp; e < 8 * grp + 8; ++e) {
        const int row = M::row(t, e), c = M::col(t, e);
        const uint32_t ob = 8u * (uint32_t)(row * fd.pitch + c);
        v[e] = c_mul(*reinterpret_cast<const float2*>(reinterpret_cast<const char*>(ub) + ob),
                     w[(uint32_t)(row * P + c)]);
      }
      M::stage_a_fwd(v, A, grp);
#pragma unroll
      for (int e = 8 * grp; e < 8 * grp + 8; ++e) pin(v[e]);
      asm volatile("" ::: "memory");
    }
  } else
#pragma unroll
  for (int l = 0; l < 2; ++l) {
#pragma unroll
    for (int r0 = 0; r0 < 16; r0 += 8) {
#pragma unroll
      for (int r1 = r0; r1 < r0 + 8; ++r1) {
        const int row = F::row_of(t, 16 * l + r1);
        const uint32_t ob = 8u * (uint32_t)(row * fd.pitch + col);
        v[16 * l + r1] = c_mul(*reinterpret_cast<const float2*>(reinterpret_cast<const char*>(ub) + ob),
                               w[(uint32_t)(row * P + col)]);
      }
      if (l == 1) asm volatile("" ::: "memory");   // keep the next group's loads after these
    }
    // stage-B twiddles to LDS after the first line's loads are issued (visible after
    // the barrier that follows half_fwd's stage-A writes)
    if (l == 0 && t < F::N2 * 16) twl[(t >> 4) * TWL + (t & 15)] = a.tw[t];
    F::stage_a_fwd_line(v, a.tw, t, l);
    // the line's 16 outputs are complete here: the compiler may not sink parts of the
    // butterfly past the first half (their intermediates would outnumber the outputs)
#pragma unroll
    for (int k = 0; k < 16; ++k) pin(v[16 * l + k]);
    asm volatile("" ::: "memory");   // the second line's loads start after this transform
  }

  double mis = 0.0, gsum = 0.0, gdel = 0.0, gnrm = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // no leading barriers: every LDS slot a thread writes first in a half transform is
    // one that only this thread touched last (Half128::own_pair, the stage-A slots)
    if constexpr (MF) M::template half_fwd<false>(v, lds, a.mft, t, h);
    else F::template half_fwd<TWL, false>(v, lds, twl, t, h);
    // the other half's 16 values wait in the LDS buffer, idle between the stage-C reads
    // and the inverse; the 32 registers they free let all 16 amplitude and multiplier
    // loads of this half be in flight at once
    auto slot = [&](int hh, int k) { return MF ? 4 * (k >> 1) + 2 * hh + (k & 1) : 16 * (k >> 3) + 8 * hh + (k & 7); };
    // the frequency offsets below are computed here from an opaque copy of the thread
    // index: hoisted to the start of the kernel they would stay live across the
    // transforms and spill
    int tq = t;
    asm volatile("" : "+v"(tq));
    // the other half goes into the 16 LDS values this thread has just read in the last
    // stage-C pass (no other thread reads them, so no barrier)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float2 x0 = v[slot(1 - h, 2 * k)], x1 = v[slot(1 - h, 2 * k + 1)];
      *reinterpret_cast<float4*>(lds + F::own_pair(tq, k)) = make_float4(x0.x, x0.y, x1.x, x1.y);
    }
    asm volatile("" ::: "memory");
    float2 gpre[16];
    float spre[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      int kr, kc;
      F::freq(tq, 16 * (k >> 3) + 8 * h + (k & 7), kr, kc);
      spre[k] = ld_s<NT>(sb + (uint32_t)(kr * P + kc));
      gpre[k] = ld_s<NT>(gb + (uint32_t)(kr * P + kc));
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int e = slot(h, k);
      const float2 X = c_scale(v[e], inv_p);
      const float sf = spre[k];
      const float2 y = c_add(gpre[k], X);
      const float2 z = prox_stagm(y, sf, pc);
      const float2 g = c_sub(y, z);
      if (STATS) {
        elem_measures(X, sf, a.eps, a.gcoef, mis, gsum);
        if (ST > 1) frame_terms(gpre[k], g, gdel, gnrm);
      }
      gpre[k] = g;
      v[e] = c_scale(c_sub(z, g), inv_p);   // both 1/p factors of the unitary pair applied here
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      int kr, kc;
      F::freq(tq, 16 * (k >> 3) + 8 * h + (k & 7), kr, kc);
      st_s<NT>(gb + (uint32_t)(kr * P + kc), gpre[k]);
    }
    asm volatile("" ::: "memory");
    // each thread reads back only what it wrote; half_inv's first LDS writes go to these
    // same slots, after these reads in the thread's own program order
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float4 x = *reinterpret_cast<const float4*>(lds + F::own_pair(tq, k));
      v[slot(1 - h, 2 * k)] = make_float2(x.x, x.y);
      v[slot(1 - h, 2 * k + 1)] = make_float2(x.z, x.w);
    }
    if constexpr (MF) M::template half_inv<false>(v, lds, a.mft, t, h);
    else F::template half_inv<TWL, false>(v, lds, twl, t, h);
  }
  if (STATS) frame_stats<F::T, (ST > 1)>(a.part + NFS * (size_t)j, mis, gsum, gdel, gnrm, red);
  // inverse stage A and the output one line at a time; the second line's probe loads
  // are issued before the first line's stores (see the prox above)
  const float2* wo = a.w_out + woff;
  if constexpr (MF) {
    // inverse stage A two line blocks at a time; each group's probe values are loaded
    // before its products, its outputs stored after
    const mf::Tab A = M::tab_a(a.mft, 1, t);
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
      asm volatile("" ::: "memory");
      float2 wk[8];
      if (!BLIND) {
#pragma unroll
        for (int i = 0; i < 8; ++i) wk[i] = wo[(uint32_t)(M::row(t, 8 * grp + i) * P + M::col(t, 8 * grp + i))];
      }
      M::stage_a_inv(v, A, grp);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = 8 * grp + i;
        const float2 x = BLIND ? v[e] : c_mulc(v[e], wk[i]);
        st_s<NT>(pb + (uint32_t)(M::row(t, e) * P + M::col(t, e)), x);
      }
    }
    return;
  }
  float2 wk[2][16];
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    asm volatile("" ::: "memory");
    F::stage_a_inv_line(v, a.tw, t, l);
    if (!BLIND) {
      if (l == 0) {
#pragma unroll
        for (int r1 = 0; r1 < 16; ++r1) wk[0][r1] = wo[(uint32_t)(F::row_of(t, r1) * P + col)];
      }
#pragma unroll
      for (int r1 = 0; r1 < 16; ++r1) v[16 * l + r1] = c_mulc(v[16 * l + r1], wk[l][r1]);
      if (l == 0) {
#pragma unroll
        for (int r1 = 0; r1 < 16; ++r1) wk[1][r1] = wo[(uint32_t)(F::row_of(t, 16 + r1) * P + col)];
      }
    }
#pragma unroll
    for (int r1 = 0; r1 < 16; ++r1) st_s<NT>(pb + (uint32_t)(F::row_of(t, 16 * l + r1) * P + col), v[16 * l + r1]);
  }
}

// the five statistics / blind variants of one sweep kernel
template <int P, bool MF, bool NT>
static hipError_t go_sweep(const SweepArgs& a, const ProxC& pc, dim3 grid, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  const bool bl = a.blind != 0;
  const int st = a.part == nullptr ? 0 : (a.frame_res && !bl ? 2 : 1);
#define ODP_SWEEP_GO(K, T) hipExtLaunchKernelGGL(K, grid, dim3(T), 0, s, ev0, ev1, 0, a, pc)
  if constexpr (P == 128) {
    constexpr int T = Half128::T;
    if (bl && st) ODP_SWEEP_GO((k_sweep128<MF, true, 1, NT>), T);
    else if (bl) ODP_SWEEP_GO((k_sweep128<MF, true, 0, NT>), T);
    else if (st == 2) ODP_SWEEP_GO((k_sweep128<MF, false, 2, NT>), T);
    else if (st) ODP_SWEEP_GO((k_sweep128<MF, false, 1, NT>), T);
    else ODP_SWEEP_GO((k_sweep128<MF, false, 0, NT>), T);
  } else {
    constexpr int T = Frame<P>::T;
    if (bl && st) ODP_SWEEP_GO((k_sweep<P, MF, true, 1, NT>), T);
    else if (bl) ODP_SWEEP_GO((k_sweep<P, MF, true, 0, NT>), T);
    else if (st == 2) ODP_SWEEP_GO((k_sweep<P, MF, false, 2, NT>), T);
    else if (st) ODP_SWEEP_GO((k_sweep<P, MF, false, 1, NT>), T);
    else ODP_SWEEP_GO((k_sweep<P, MF, false, 0, NT>), T);
  }
#undef ODP_SWEEP_GO
  return hipGetLastError();
}

hipError_t launch_sweep(int p, const SweepArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const ProxC pc = prox_coeffs(a.eps, a.eta);
  const dim3 grid(NXCD * a.chunk);
  const bool nt = a.stream != 0;
#define ODP_SWEEP(PP, MF) \
  return nt ? go_sweep<PP, MF, true>(a, pc, grid, s, ev0, ev1) : go_sweep<PP, MF, false>(a, pc, grid, s, ev0, ev1);
  if (a.mft) {   // radix-16 stages on the matrix cores (hybrid transform)
    if (p == 64) ODP_SWEEP(64, true)
    if (p == 128) ODP_SWEEP(128, true)
    return hipErrorInvalidValue;
  }
  if (p == 32) ODP_SWEEP(32, false)
  if (p == 64) ODP_SWEEP(64, false)
  if (p == 128) ODP_SWEEP(128, false)
#undef ODP_SWEEP
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Operators A and A* on the whole image (Sec. 2)
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(Frame<P>::T) void k_forward(const float2* __restrict__ u, int W,
                                                         const float2* __restrict__ w,
                                                         const float2* __restrict__ tw,
                                                         const int32_t* __restrict__ off,
                                                         float2* __restrict__ out) {
  using F = Frame<P>;
  __shared__ __align__(16) float2 lds[F::LDS];
  const int j = blockIdx.x, t = threadIdx.x;
  const int col = F::a_col(t), r2 = F::a_r2(t);
  const int64_t base = (int64_t)off[2 * j] * W + off[2 * j + 1];
  float2 v[16];
#pragma unroll
  for (int r1 = 0; r1 < 16; ++r1) {
    const int row = F::N2 * r1 + r2;
    v[r1] = c_mul(u[base + (int64_t)row * W + col], w[row * P + col]);
  }
  F::forward(v, lds, tw, t);
  const float inv_p = 1.0f / (float)P;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    int kr, kc;
    F::freq(t, e, kr, kc);
    out[(size_t)j * P * P + kr * P + kc] = c_scale(v[e], inv_p);
  }
}

template <int P>
__global__ __launch_bounds__(Frame<P>::T) void k_adjoint(const float2* __restrict__ frames,
                                                         const float2* __restrict__ w,
                                                         const float2* __restrict__ tw,
                                                         const int32_t* __restrict__ off,
                                                         float2* __restrict__ u, int W) {
  using F = Frame<P>;
  __shared__ __align__(16) float2 lds[F::LDS];
  const int j = blockIdx.x, t = threadIdx.x;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    int kr, kc;
    F::freq(t, e, kr, kc);
    v[e] = frames[(size_t)j * P * P + kr * P + kc];
  }
  F::inverse(v, lds, tw, t);
  const int col = F::a_col(t), r2 = F::a_r2(t);
  const int64_t base = (int64_t)off[2 * j] * W + off[2 * j + 1];
  const float inv_p = 1.0f / (float)P;
#pragma unroll
  for (int r1 = 0; r1 < 16; ++r1) {
    const int row = F::N2 * r1 + r2;
    atomic_add_c(&u[base + (int64_t)row * W + col], c_mulc(c_scale(v[r1], inv_p), w[row * P + col]));
  }
}

hipError_t launch_forward(int p, const float2* u, int H, int W, const float2* w, const float2* tw,
                          const int32_t* offsets, int J, float2* out, hipStream_t s) {
  (void)H;
  if (p == 32) hipLaunchKernelGGL(k_forward<32>, dim3(J), dim3(Frame<32>::T), 0, s, u, W, w, tw, offsets, out);
  else if (p == 64) hipLaunchKernelGGL(k_forward<64>, dim3(J), dim3(Frame<64>::T), 0, s, u, W, w, tw, offsets, out);
  else if (p == 128) hipLaunchKernelGGL(k_forward<128>, dim3(J), dim3(Frame<128>::T), 0, s, u, W, w, tw, offsets, out);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_adjoint(int p, const float2* frames, const float2* w, const float2* tw,
                          const int32_t* offsets, int J, float2* u_out, int H, int W, hipStream_t s) {
  hipError_t e = launch_fill(u_out, (int64_t)H * W, make_float2(0.f, 0.f), s);
  if (e != hipSuccess) return e;
  if (p == 32) hipLaunchKernelGGL(k_adjoint<32>, dim3(J), dim3(Frame<32>::T), 0, s, frames, w, tw, offsets, u_out, W);
  else if (p == 64) hipLaunchKernelGGL(k_adjoint<64>, dim3(J), dim3(Frame<64>::T), 0, s, frames, w, tw, offsets, u_out, W);
  else if (p == 128) hipLaunchKernelGGL(k_adjoint<128>, dim3(J), dim3(Frame<128>::T), 0, s, frames, w, tw, offsets, u_out, W);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// elementwise prox, fills, copies
// ---------------------------------------------------------------------------
__global__ void k_prox(const float2* __restrict__ y, const float* __restrict__ sf, int64_t n, ProxC pc,
                       float2* z) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = prox_stagm(y[i], sf[i], pc);
}

hipError_t launch_prox(const float2* y, const float* sf, int64_t n, float eps, float lam, float2* z,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_prox, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, y, sf, n,
                     prox_coeffs(eps, lam), z);
  return hipGetLastError();
}

__global__ void k_fill(float2* p, int64_t n, float2 v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill(float2* p, int64_t n, float2 value, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

__global__ void k_copy(float2* d, const float2* src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = src[i];
}

hipError_t launch_copy(float2* dst, const float2* src, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// bind-time reductions: max of den (FP64) and sum of sqrt f (FP64), fixed order
// ---------------------------------------------------------------------------
constexpr int RED_BLOCKS = 1024;

__global__ __launch_bounds__(256) void k_sum_max_part(const double* x, int64_t n, const float* y, int64_t ny,
                                                      double* part) {
  __shared__ double sh[4];
  double mx = 0.0, sm = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * 256) mx = fmax(mx, x[i]);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ny; i += (int64_t)RED_BLOCKS * 256) sm += (double)y[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  sm = block_sum<256>(sm, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = mx;
    part[2 * blockIdx.x + 1] = sm;
  }
}

__global__ __launch_bounds__(256) void k_sum_max_final(const double* part, double* out) {
  __shared__ double sh[4];
  double mx = 0.0, sm = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += 256) {
    mx = fmax(mx, part[2 * i]);
    sm += part[2 * i + 1];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  sm = block_sum<256>(sm, sh);
  if (threadIdx.x == 0) {
    out[0] = mx;
    out[1] = sm;
  }
}

hipError_t launch_sum_max(const double* x, int64_t n, const float* y, int64_t ny, double* out, hipStream_t s) {
  // out[0] = max x, out[1] = sum y; out[2 .. 2 + 2*RED_BLOCKS) is scratch
  hipLaunchKernelGGL(k_sum_max_part, dim3(RED_BLOCKS), dim3(256), 0, s, x, n, y, ny, out + 2);
  hipLaunchKernelGGL(k_sum_max_final, dim3(1), dim3(256), 0, s, out + 2, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-iteration statistics: RF, RE, G_eps (Sec. 4, eq. STAGM), fixed order
// ---------------------------------------------------------------------------
// blocks [0, D): the NPS pixel statistics of subdomain b into scratch[NPS b ...];
// block D: the frames' (L1 misfit, G_eps) into scratch[NPS D], scratch[NPS D + 1]
__global__ __launch_bounds__(256) void k_stats_reduce(const double* frame_part, int J, const double* tile_part,
                                                      const int32_t* re_list, const int32_t* re_first, int D,
                                                      double* scratch) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  double v[NPS] = {};
  if (b < D) {
    for (int k = re_first[b] + threadIdx.x; k < re_first[b + 1]; k += 256) {
      const int e = re_list[k];
#pragma unroll
      for (int q = 0; q < NPS; ++q) v[q] += tile_part[NPS * (size_t)e + q];
    }
  } else {
    for (int k = threadIdx.x; k < J; k += 256)
#pragma unroll
      for (int q = 0; q < NFS; ++q) v[q] += frame_part[NFS * (size_t)k + q];
  }
  const int nq = b < D ? NPS : NFS;
  for (int q = 0; q < nq; ++q) {
    const double t = block_sum<256>(v[q], sh);
    if (threadIdx.x == 0) scratch[NPS * (size_t)b + q] = t;
  }
}

__global__ void k_stats_final(const double* scratch, int D, const double* sum_sf, double* out3) {
  if (threadIdx.x != 0) return;
  double re = 0.0;
  for (int d = 0; d < D; ++d) {
    const double num = scratch[NPS * d], den = scratch[NPS * d + 1];
    const double v = den > 0.0 ? sqrt(num / den) : 0.0;
    re = fmax(re, v);
  }
  out3[0] = scratch[NPS * D] / sum_sf[0];
  out3[1] = re;
  out3[2] = scratch[NPS * D + 1];
}

hipError_t launch_stats(const double* frame_part, int J, const double* tile_part, const int32_t* re_list,
                        const int32_t* re_first, int D, const double* sum_sf, double* out3, double* scratch,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_stats_reduce, dim3(D + 1), dim3(256), 0, s, frame_part, J, tile_part, re_list, re_first,
                     D, scratch);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, s, scratch, D, sum_sf, out3);
  return hipGetLastError();
}

// per problem (one thread each): its subdomains' sums in ascending order, then its frames'
// residual sums in ascending frame order
__global__ void k_residual_sums(const double* scratch, const double* frame_part, const int32_t* prob, int n,
                                double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int J0 = prob[4 * i], Jp = prob[4 * i + 1], D0 = prob[4 * i + 2], Dp = prob[4 * i + 3];
  double v[NRES] = {};
  for (int d = D0; d < D0 + Dp; ++d)
    for (int k = 0; k < 6; ++k) v[k] += scratch[NPS * (size_t)d + 2 + k];
  for (int j = J0; j < J0 + Jp; ++j) {
    v[6] += frame_part[NFS * (size_t)j + 2];
    v[7] += frame_part[NFS * (size_t)j + 3];
  }
  for (int k = 0; k < NRES; ++k) out[NRES * (size_t)i + k] = v[k];
}

hipError_t launch_residual_sums(const double* frame_part, int J, const double* tile_part, const int32_t* re_list,
                                const int32_t* re_first, int D, const int32_t* prob, int n, double* scratch,
                                double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_stats_reduce, dim3(D + 1), dim3(256), 0, s, frame_part, J, tile_part, re_list, re_first, D,
                     scratch);
  hipLaunchKernelGGL(k_residual_sums, dim3((n + 63) / 64), dim3(64), 0, s, scratch, frame_part, prob, n, out);
  return hipGetLastError();
}

__global__ void k_scale(float2* x, int64_t n, float f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = c_scale(x[i], f);
}

hipError_t launch_scale(float2* x, int64_t n, float f, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, f);
  return hipGetLastError();
}

// end of an iteration under a stopping rule (Sec. 4): per problem, its measures and the
// rule; problems already stopped keep their status
__global__ __launch_bounds__(256) void k_stop_check(StopArgs a) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  StopStatus* st = a.status + i;
  if (st->stopped) return;  // uniform over the workgroup
  const int J0 = a.prob[4 * i], J = a.prob[4 * i + 1], D0 = a.prob[4 * i + 2], D = a.prob[4 * i + 3];
  double s0 = 0.0, s1 = 0.0;
  for (int k = threadIdx.x; k < J; k += 256) {
    s0 += a.frame_part[NFS * (size_t)(J0 + k)];
    s1 += a.frame_part[NFS * (size_t)(J0 + k) + 1];
  }
  s0 = block_sum<256>(s0, sh);
  s1 = block_sum<256>(s1, sh);
  if (threadIdx.x != 0) return;
  double re = 0.0;
  for (int d = D0; d < D0 + D; ++d) {
    const double num = a.sub_sums[NPS * d], den = a.sub_sums[NPS * d + 1];
    re = fmax(re, den > 0.0 ? sqrt(num / den) : 0.0);
  }
  const double rf = s0 / a.sum_sf[(size_t)i * a.sum_sf_stride];
  const int it = st->iters + a.n_add;
  const double m = a.measure == 1 ? rf : re;
  const bool met = a.measure != 0 && m <= a.tol;   // false for NaN
  st->iters = it;
  st->rf = rf;
  st->re = re;
  st->g = s1;
  st->stopped = (met || (a.max_iter > 0 && it >= a.max_iter)) ? 1 : 0;
}

hipError_t launch_stop_check(const StopArgs& a, const double* tile_part, const int32_t* re_list,
                             const int32_t* re_first, int D, double* scratch, hipStream_t s) {
  // per-subdomain (|du|^2, |u|^2) into scratch (blocks [0, D) of the statistics reduction)
  hipLaunchKernelGGL(k_stats_reduce, dim3(D), dim3(256), 0, s, a.frame_part, 0, tile_part, re_list, re_first, D,
                     scratch);
  StopArgs b = a;
  b.sub_sums = scratch;
  hipLaunchKernelGGL(k_stop_check, dim3(a.n), dim3(256), 0, s, b);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// merge (Sec. 4): mean of the copies over each pixel, 1 where no subdomain
// ---------------------------------------------------------------------------
__global__ void k_merge(const float2* __restrict__ usub, const int32_t* __restrict__ rects,
                        const int64_t* __restrict__ uoff, int D, int H, int W, float2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)H * W) return;
  const int y = (int)(i / W), x = (int)(i % W);
  float sx = 0.f, sy = 0.f;
  int n = 0;
  for (int d = 0; d < D; ++d) {
    const int r0 = rects[4 * d], c0 = rects[4 * d + 1], r1 = rects[4 * d + 2], c1 = rects[4 * d + 3];
    if (y >= r0 && y < r1 && x >= c0 && x < c1) {
      const float2 v = usub[uoff[d] + (int64_t)(y - r0) * (c1 - c0) + (x - c0)];
      sx += v.x;
      sy += v.y;
      ++n;
    }
  }
  out[i] = n ? make_float2(sx / n, sy / n) : make_float2(1.f, 0.f);
}

hipError_t launch_merge(const float2* u_sub, const int32_t* rects, const int64_t* usub_off, int D, int H, int W,
                        float2* out, hipStream_t s) {
  const int64_t n = (int64_t)H * W;
  hipLaunchKernelGGL(k_merge, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, u_sub, rects, usub_off, D, H, W,
                     out);
  return hipGetLastError();
}

}  // namespace odp

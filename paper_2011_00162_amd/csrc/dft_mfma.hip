// dft_mfma.hip -- frame sweep with the 2-D DFT computed as dense products on MFMA.
//
// For p = 64 the unitary DFT of a frame is X^ = F X F with F[k][n] = exp(-2 pi i kn/64)/8
// (F is symmetric), and the inverse is conj(F) T conj(F).  Each complex product is
// four real products; every real product a*b is evaluated in split BF16 as
//     a_hi b_hi + a_hi b_lo + a_lo b_hi,   a_hi = bf16(a), a_lo = bf16(a - a_hi)
// (round-to-nearest-even), accumulated in FP32 by v_mfma_f32_16x16x32_bf16.  The
// dropped a_lo b_lo term is about 2^-16 of each product.  F's split parts come from
// a host FP64 table.
//
// Per frame one workgroup of 4 wavefronts; wavefront w owns output rows 16w..16w+15
// and keeps the matching rows of F (real, imaginary, negated imaginary; hi and lo) in
// registers as the A operand of every product.  Between the two products of each
// direction the intermediate goes through LDS as four bf16 planes (re hi, re lo,
// im hi, im lo), laid out so every B-operand fetch is one 128-bit read.
// MFMA operand layouts (wave64, checked on the device): A[m][k] lane l element i at
// m = l%16, k = 8(l/16)+i; B[k][n] at k = 8(l/16)+i, n = l%16; D[m][n] at
// m = 4(l/16)+i, n = l%16.
//
// The prox / Gamma update between the two directions is the same as in k_sweep.
#include <hip/hip_runtime.h>

#include "fft_frame.hpp"
#include "odp_internal.hpp"
#include "prox.hpp"
#include "reduce.hpp"

namespace odp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short shortx8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

namespace {

constexpr int DP = 64;              // frame size of this kernel
constexpr int LRB = DP + 8;         // LDS row stride in bf16 (144 bytes: conflict-free 16-lane reads)
constexpr int PLANE = DP * LRB;     // one bf16 plane

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 neg(bf16x8 v) {
  shortx8 s = __builtin_bit_cast(shortx8, v);
  s ^= (short)0x8000;
  return __builtin_bit_cast(bf16x8, s);
}

// store the split of complex v at (row, col) of the four planes
__device__ __forceinline__ void put(__bf16* lds, int row, int col, float2 v) {
  const __bf16 rh = (__bf16)v.x, ih = (__bf16)v.y;
  const __bf16 rl = (__bf16)(v.x - (float)rh), il = (__bf16)(v.y - (float)ih);
  const int o = row * LRB + col;
  lds[o] = rh;
  lds[PLANE + o] = rl;
  lds[2 * PLANE + o] = ih;
  lds[3 * PLANE + o] = il;
}

struct BOp {
  bf16x8 rh, rl, ih, il;
};

// B operand: 8 consecutive columns c0..c0+7 of plane row `row`
__device__ __forceinline__ BOp get(const __bf16* lds, int row, int c0) {
  const int o = row * LRB + c0;
  BOp b;
  b.rh = *reinterpret_cast<const bf16x8*>(lds + o);
  b.rl = *reinterpret_cast<const bf16x8*>(lds + PLANE + o);
  b.ih = *reinterpret_cast<const bf16x8*>(lds + 2 * PLANE + o);
  b.il = *reinterpret_cast<const bf16x8*>(lds + 3 * PLANE + o);
  return b;
}

struct FRows {  // rows 16w..16w+15 of F in A-operand layout, for the two K chunks
  bf16x8 rh[2], rl[2], ih[2], il[2], nih[2], nil[2];
};

// C = F_rows(w) * B (CONJ: conj(F_rows) * B) over K = 64 for the four 16-column tiles;
// B row n = 16 nt + l%16 of the LDS planes holds the K index along its columns.
// Each tile keeps six independent accumulator chains (one per split term of the real
// and of the imaginary part) so consecutive MFMAs do not wait on each other.
template <bool CONJ>
__device__ __forceinline__ void cgemm(const FRows& f, const __bf16* lds, int lane, floatx4 (&re)[4],
                                      floatx4 (&im)[4]) {
  const int g = lane >> 4, n0 = lane & 15;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const BOp b0 = get(lds, 16 * nt + n0, 8 * g);
    const BOp b1 = get(lds, 16 * nt + n0, 32 + 8 * g);
    floatx4 r0{0.f, 0.f, 0.f, 0.f}, r1 = r0, r2 = r0, i0 = r0, i1 = r0, i2 = r0;
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      const BOp& b = kc ? b1 : b0;
      // re: Fr Br -/+ Fi Bi ; im: Fr Bi +/- Fi Br   (each as hi*hi + hi*lo + lo*hi)
      const bf16x8& fi_h = CONJ ? f.ih[kc] : f.nih[kc];
      const bf16x8& fi_l = CONJ ? f.il[kc] : f.nil[kc];
      const bf16x8& gi_h = CONJ ? f.nih[kc] : f.ih[kc];
      const bf16x8& gi_l = CONJ ? f.nil[kc] : f.il[kc];
      r0 = mfma(f.rh[kc], b.rh, r0);
      i0 = mfma(f.rh[kc], b.ih, i0);
      r1 = mfma(f.rh[kc], b.rl, r1);
      i1 = mfma(f.rh[kc], b.il, i1);
      r2 = mfma(f.rl[kc], b.rh, r2);
      i2 = mfma(f.rl[kc], b.ih, i2);
      r0 = mfma(fi_h, b.ih, r0);
      i0 = mfma(gi_h, b.rh, i0);
      r1 = mfma(fi_h, b.il, r1);
      i1 = mfma(gi_h, b.rl, i1);
      r2 = mfma(fi_l, b.ih, r2);
      i2 = mfma(gi_l, b.rh, i2);
    }
    re[nt] = r0 + r1 + r2;
    im[nt] = i0 + i1 + i2;
  }
}

}  // namespace

template <bool BLIND, bool STATS>
__global__ __launch_bounds__(256) void k_sweep_dft64(SweepArgs a, DftTable dt, float eps, float thr, float ctr,
                                                     float ca, float cb) {
  __shared__ __bf16 lds[4 * PLANE];
  __shared__ double red[4];
  const int b = blockIdx.x;
  const int pos = a.xcd_slice ? (b % NXCD) * a.chunk + b / NXCD : b;
  if (pos >= a.J) return;  // uniform over the workgroup
  const int j = a.order[pos];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, g = lane >> 4, n0 = lane & 15;
  const FrameDesc fd = a.frames[j];
  const size_t woff = (size_t)(a.w_per_sub ? fd.sub : fd.probe) * DP * DP;
  const float2* wp = a.w + woff;

  // rows 16w + n0 of F, K chunks kc: columns 32 kc + 8 g .. + 7
  FRows f;
#pragma unroll
  for (int kc = 0; kc < 2; ++kc) {
    const int o = (16 * w + n0) * DP + 32 * kc + 8 * g;
    const __bf16* tf = reinterpret_cast<const __bf16*>(dt.f);
    f.rh[kc] = *reinterpret_cast<const bf16x8*>(tf + o);
    f.rl[kc] = *reinterpret_cast<const bf16x8*>(tf + DP * DP + o);
    f.ih[kc] = *reinterpret_cast<const bf16x8*>(tf + 2 * DP * DP + o);
    f.il[kc] = *reinterpret_cast<const bf16x8*>(tf + 3 * DP * DP + o);
    f.nih[kc] = neg(f.ih[kc]);
    f.nil[kc] = neg(f.il[kc]);
  }

  // gather w o S_j u, stored transposed (row = column of the frame)
  {
    const int c = t & 63;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int r = 4 * k + (t >> 6);
      const float2 x = c_mul(a.u[fd.base + (int64_t)r * fd.pitch + c], wp[r * DP + c]);
      put(lds, c, r, x);
    }
  }
  __syncthreads();
  floatx4 re[4], im[4];
  // Y = F X: D rows kr = 16w + 4g + i, columns c = 16 nt + n0
  cgemm<false>(f, lds, lane, re, im);
  __syncthreads();
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) put(lds, 16 * w + 4 * g + i, 16 * nt + n0, make_float2(re[nt][i], im[nt][i]));
  __syncthreads();
  // X^T = F Y^T: D rows kc = 16w + 4g + i, columns kr = 16 nt + n0
  cgemm<false>(f, lds, lane, re, im);

  // prox and Gamma update at (kr, kc); re/im become t = z - Gamma
  const ProxC pc{thr, ctr, ca, cb};
  double mis = 0.0, gsum = 0.0;
  const size_t fbase = (size_t)j * DP * DP;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kr = 16 * nt + n0, kc = 16 * w + 4 * g + i;
      const size_t idx = fbase + kr * DP + kc;
      const float2 X = make_float2(re[nt][i], im[nt][i]);
      const float sf = a.sqrt_f[idx];
      const float2 y = c_add(a.gamma[idx], X);
      const float2 z = prox_stagm(y, sf, pc);
      const float2 gm = c_sub(y, z);
      a.gamma[idx] = gm;
      const float2 tv = c_sub(z, gm);
      re[nt][i] = tv.x;
      im[nt][i] = tv.y;
      if (STATS) {
        const double ax = sqrt((double)X.x * X.x + (double)X.y * X.y);
        mis += fabs(ax - (double)sf);
        gsum += g_eps(ax, (double)sf, (double)eps);
      }
    }
  }
  if (STATS) {
    mis = block_sum<256>(mis, red);
    gsum = block_sum<256>(gsum, red);
    if (t == 0) {
      a.part[2 * j] = mis;
      a.part[2 * j + 1] = gsum;
    }
  }
  __syncthreads();
  // T^T into LDS (row = kc, column = kr)
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) put(lds, 16 * w + 4 * g + i, 16 * nt + n0, make_float2(re[nt][i], im[nt][i]));
  __syncthreads();
  // W = conj(F) T: D rows r = 16w + 4g + i, columns kc = 16 nt + n0
  cgemm<true>(f, lds, lane, re, im);
  __syncthreads();
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) put(lds, 16 * w + 4 * g + i, 16 * nt + n0, make_float2(re[nt][i], im[nt][i]));
  __syncthreads();
  // x^T = conj(F) W^T: D rows c = 16w + 4g + i, columns r = 16 nt + n0
  cgemm<true>(f, lds, lane, re, im);
  const float2* wo = a.w_out + woff;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * nt + n0, c = 16 * w + 4 * g + i;
      const float2 x = make_float2(re[nt][i], im[nt][i]);
      a.psi[fbase + r * DP + c] = BLIND ? x : c_mulc(x, wo[r * DP + c]);
    }
  }
}

hipError_t launch_sweep_dft(int p, const SweepArgs& a, const DftTable& dt, hipStream_t s) {
  if (p != DP) return hipErrorInvalidValue;
  const double eps = a.eps, lam = a.eta, kappa = (1.0 - eps) / eps;
  const float thr = (float)(eps - (1.0 - eps) / lam);
  const float ctr = lam > kappa ? (float)(lam / (lam - kappa)) : 0.0f;
  const float ca = (float)(1.0 / (1.0 + lam)), cb = (float)(lam / (1.0 + lam));
  const dim3 grid(NXCD * a.chunk), blk(256);
  const bool st = a.part != nullptr, bl = a.blind != 0;
  if (bl && st) hipLaunchKernelGGL((k_sweep_dft64<true, true>), grid, blk, 0, s, a, dt, a.eps, thr, ctr, ca, cb);
  else if (bl) hipLaunchKernelGGL((k_sweep_dft64<true, false>), grid, blk, 0, s, a, dt, a.eps, thr, ctr, ca, cb);
  else if (st) hipLaunchKernelGGL((k_sweep_dft64<false, true>), grid, blk, 0, s, a, dt, a.eps, thr, ctr, ca, cb);
  else hipLaunchKernelGGL((k_sweep_dft64<false, false>), grid, blk, 0, s, a, dt, a.eps, thr, ctr, ca, cb);
  return hipGetLastError();
}

}  // namespace odp

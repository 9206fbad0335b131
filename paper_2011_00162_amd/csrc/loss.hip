// loss.hip -- amplitude data term and its gradients (the frame model of Sec. 2).
//
//   L      = sum_j || |X_j| - sqrt(f_j) ||^2,  X_j = F(w o S_j u)  (F unitary)
//   g_j    = 2 (1 - sqrt(f_j)/|X_j|) X_j        (0 where X_j = 0)
//   dL/du  = sum_j S_j^T( conj(w) o F^{-1} g_j )
//   dL/dw  = sum_j conj(S_j u) o F^{-1} g_j
// Gradients are dL/dRe + i dL/dIm.  One workgroup per frame recomputes X_j and
// writes phi_j = F^{-1} g_j; the image gradient is pulled per pixel over the
// covering frames and the probe gradient is reduced over frames in FP64, both in
// a fixed order.
#include <hip/hip_runtime.h>

#include "fft_frame.hpp"
#include "odp_internal.hpp"
#include "pull.hpp"
#include "reduce.hpp"

namespace odp {

// Frame of this workgroup: workgroup b runs on XCD b % 8, and each XCD takes a contiguous
// slice of the frames (scan order), so neighbouring windows, which share image rows, are
// read through one L2.  The grid is 8 ceil(J / 8); -1 for the workgroups past J.
__device__ __forceinline__ int loss_frame(int J) {
  const int chunk = (J + NXCD - 1) / NXCD, b = blockIdx.x;
  const int j = (b % NXCD) * chunk + b / NXCD;
  return j < J ? j : -1;
}

// One element's loss term (|X| - sqrt f)^2 from the FP32 spectrum: |X| = |X|^2 / |X| by the
// hardware reciprocal square root (about an ulp), the difference and its square in FP32,
// added to the FP64 sum one element after the other (an empty asm on the sum keeps the
// scheduler from interleaving the temporaries of many elements, which spilled).  Returns
// 1/|X| (0 for X = 0), which the gradient uses.
__device__ __forceinline__ float loss_term(float2 X, float sf, double& loss) {
  const float a2 = X.x * X.x + X.y * X.y;
  const float inv = a2 > 0.0f ? __builtin_amdgcn_rsqf(a2) : 0.0f;
  const float d = a2 * inv - sf;
  loss += (double)(d * d);
  asm volatile("" : "+v"(loss));
  return inv;
}

template <int P, bool GRAD>
__global__ __launch_bounds__(Frame<P>::T) void k_loss(LossArgs a) {
  using F = Frame<P>;
  __shared__ __align__(16) float2 lds[F::LDS];
  __shared__ __align__(16) float2 twl[F::N2 * TWL];   // stage-B twiddles in LDS (no global-load waits)
  __shared__ double red[F::T / 64];
  const int j = loss_frame(a.J), t = threadIdx.x;
  if (j < 0) return;   // uniform over the workgroup
  const int col = F::a_col(t), r2 = F::a_r2(t);
  const int64_t base = (int64_t)a.offsets[2 * j] * a.W + a.offsets[2 * j + 1];
  const float inv_p = 1.0f / (float)P;
  float2 v[16];
#pragma unroll
  for (int r1 = 0; r1 < 16; ++r1) {
    const int row = F::N2 * r1 + r2;
    v[r1] = c_mul(a.u[base + (int64_t)row * a.W + col], a.w[row * P + col]);
  }
  // the stage-B twiddles go to LDS after the gather's loads are issued, so waiting for
  // this copy overlaps their latency; visible after the first barrier of forward_bc
  if (t < F::N2 * 16) twl[(t >> 4) * TWL + (t & 15)] = a.tw[t];
  F::forward_a(v, lds, a.tw, t);
  F::template forward_bc<TWL>(v, lds, twl, t);
  double loss = 0.0;
  const size_t fbase = (size_t)j * P * P;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    int kr, kc;
    F::freq(t, e, kr, kc);
    const float2 X = c_scale(v[e], inv_p);
    const float sf = a.sqrt_f[fbase + kr * P + kc];
    const float inv = loss_term(X, sf, loss);
    if (GRAD) {
      const float sc = inv > 0.0f ? 2.0f * (1.0f - sf * inv) : 0.0f;
      v[e] = c_scale(X, sc * inv_p);
    }
  }
  loss = block_sum<F::T>(loss, red);
  if (t == 0) a.frame_loss[j] = loss;
  if (!GRAD) return;
  __syncthreads();
  F::template inverse<TWL>(v, lds, twl, t);
#pragma unroll
  for (int r1 = 0; r1 < 16; ++r1) a.phi[fbase + (F::N2 * r1 + r2) * P + col] = v[r1];
}

// The same at p = 128 on the two-half transform (Half128: 512 threads, 77 KB of LDS,
// two frames per CU): each half's frequencies are scored, scaled and sent back
// through the inverse stages as soon as that half's forward stages end.
template <bool GRAD>
__global__ __launch_bounds__(Half128::T) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_loss128(LossArgs a) {
  using F = Half128;
  constexpr int P = 128;
  __shared__ __align__(16) float2 lds[F::LDS];
  __shared__ __align__(16) float2 twl[F::N2 * TWL];
  __shared__ double red[F::T / 64];
  const int j = loss_frame(a.J), t = threadIdx.x;
  if (j < 0) return;   // uniform over the workgroup
  const int col = F::a_col(t);
  const int64_t base = (int64_t)a.offsets[2 * j] * a.W + a.offsets[2 * j + 1];
  const float inv_p = 1.0f / (float)P;
  // per-frame scalar bases, 32-bit element offsets (a window spans 128 image rows)
  const char* ub = reinterpret_cast<const char*>(a.u + base);
  const size_t fbase = (size_t)j * P * P;
  const float* sb = a.sqrt_f + fbase;
  float2* phib = a.phi + fbase;
  float2 v[32];
#pragma unroll
  for (int l = 0; l < 2; ++l) {
#pragma unroll
    for (int r0 = 0; r0 < 16; r0 += 8) {
#pragma unroll
      for (int r1 = r0; r1 < r0 + 8; ++r1) {
        const int row = F::row_of(t, 16 * l + r1);
        const uint32_t ob = 8u * (uint32_t)(row * a.W + col);
        v[16 * l + r1] = c_mul(*reinterpret_cast<const float2*>(ub + ob), a.w[(uint32_t)(row * P + col)]);
      }
      if (l == 1) asm volatile("" ::: "memory");   // keep the next group's loads after these
    }
    if (l == 0 && t < F::N2 * 16) twl[(t >> 4) * TWL + (t & 15)] = a.tw[t];
    F::stage_a_fwd_line(v, a.tw, t, l);
#pragma unroll
    for (int k = 0; k < 16; ++k) pin(v[16 * l + k]);
    asm volatile("" ::: "memory");
  }
  double loss = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // leading barriers only where a thread's first LDS writes could meet another thread's
    // last accesses: before the second half when no inverse ran in between (the first
    // half's stage-C reads are other slots than the stage-A writes); the stage-A and
    // own_pair slots are thread-private otherwise (Half128::a_slot, own_pair)
    if (h == 1 && !GRAD) F::template half_fwd<TWL, true>(v, lds, twl, t, h);
    else F::template half_fwd<TWL, false>(v, lds, twl, t, h);
    // frequency offsets from an opaque copy of the thread index, computed here (hoisted
    // to the start of the kernel they would stay live across the transforms)
    int tq = t;
    asm volatile("" : "+v"(tq));
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {   // two groups of 8, each finished before the next
      float sfq[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        int kr, kc;
        F::freq(tq, 16 * qq + 8 * h + i, kr, kc);
        sfq[i] = sb[(uint32_t)(kr * P + kc)];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = 16 * qq + 8 * h + i;
        const float2 X = c_scale(v[e], inv_p);
        const float sf = sfq[i];
        const float inv = loss_term(X, sf, loss);
        if (GRAD) {
          const float sc = inv > 0.0f ? 2.0f * (1.0f - sf * inv) : 0.0f;
          v[e] = c_scale(X, sc * inv_p);
        }
        pin(v[e]);
      }
      asm volatile("" ::: "memory");
    }
    if (GRAD) F::template half_inv<TWL, false>(v, lds, twl, t, h);
  }
  loss = block_sum<F::T>(loss, red);
  if (t == 0) a.frame_loss[j] = loss;
  if (!GRAD) return;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    asm volatile("" ::: "memory");
    F::stage_a_inv_line(v, a.tw, t, l);
#pragma unroll
    for (int r1 = 0; r1 < 16; ++r1) phib[(uint32_t)(F::row_of(t, 16 * l + r1) * P + col)] = v[16 * l + r1];
  }
}

// dL/du on every subdomain tile: pull over all frames covering the pixel (every
// slot of the tile's cell holds a disjoint set of frames).  Pixels in no
// subdomain are covered by no frame and stay 0 (cleared by the caller).  The padded
// pull lists are read PULL_B records at a time for both of the thread's pixels, so
// their loads are in flight together; each pixel sums its frames in list order.
__device__ __forceinline__ void grad_u_tile(const LossGradArgs& a, int tile) {
  const TileDesc td = a.tiles[tile];
  const CellDesc* cd = a.cells + td.cell;
  const int p = a.p;
  // tiles partition the covered pixels, so each pixel is written by one thread; with
  // a.pairs the thread's two pixels are row neighbours (one 16-byte load per frame)
  int yi[NPX], xi[NPX];
  bool act[NPX];
  float2 g[NPX];
#pragma unroll
  for (int h = 0; h < NPX; ++h) {
    const int i = a.pairs ? 2 * (int)threadIdx.x + h : (int)threadIdx.x + 256 * h;
    const int tr = i / a.tile_cols, tc = i % a.tile_cols;
    act[h] = tr < td.nr && tc < td.nc;
    yi[h] = cd->r0 + td.r0 + tr;
    xi[h] = cd->c0 + td.c0 + tc;
    g[h] = make_float2(0.f, 0.f);
  }
  static_assert(NPX == 2, "pixel pairs");
  for (int s = 0; s < cd->m; ++s) {
    const int k0 = a.tf_first[tile * MAXS + s], k1 = a.tf_first[tile * MAXS + s + 1];
    if (a.pairs) {
      pull_pairs<true, false, false>(a.pull, k0, k1, a.phi, a.w, yi[0], xi[0], 8u * (uint32_t)(yi[0] * p + xi[0]),
                                     p, g, nullptr);
    } else {
      uint32_t pix8[NPX];
#pragma unroll
      for (int h = 0; h < NPX; ++h) pix8[h] = 8u * (uint32_t)(yi[h] * p + xi[h]);
      pull_pixels<true, false, false>(a.pull, k0, k1, a.phi, a.w, yi, xi, pix8, p, g, nullptr);
    }
  }
#pragma unroll
  for (int h = 0; h < NPX; ++h)
    if (act[h]) a.grad_u[(int64_t)yi[h] * a.W + xi[h]] = g[h];
}

// dL/dw partial sums over frame chunks (FP64; eight frames' loads in flight per step,
// summed in frame order), then a fixed-order final sum.  Block kb of chunk `chunk`.
__device__ __forceinline__ void grad_w_part_block(const LossGradArgs& a, int kb, int chunk) {
  constexpr int B = 8;
  const int p = a.p, k = kb * 256 + threadIdx.x;
  if (k >= p * p) return;
  const int ky = k / p, kx = k % p;
  const int j0 = chunk * a.frames_per_chunk;
  const int j1 = min(a.J, j0 + a.frames_per_chunk);
  double gx = 0.0, gy = 0.0;
  auto acc = [&](const float2 uu, const float2 ph) {
    gx += (double)uu.x * ph.x + (double)uu.y * ph.y;     // conj(u) * phi
    gy += (double)uu.x * ph.y - (double)uu.y * ph.x;
  };
  int j = j0;
  for (; j + B <= j1; j += B) {
    int oy[B], ox[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      oy[i] = a.offsets[2 * (j + i)];
      ox[i] = a.offsets[2 * (j + i) + 1];
    }
    float2 uu[B], ph[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      uu[i] = a.u[((int64_t)oy[i] + ky) * a.W + ox[i] + kx];
      ph[i] = a.phi[(size_t)(j + i) * p * p + k];
    }
#pragma unroll
    for (int i = 0; i < B; ++i) acc(uu[i], ph[i]);
  }
  for (; j < j1; ++j)
    acc(a.u[((int64_t)a.offsets[2 * j] + ky) * a.W + a.offsets[2 * j + 1] + kx], a.phi[(size_t)j * p * p + k]);
  a.wpart[2 * ((size_t)chunk * p * p + k)] = gx;
  a.wpart[2 * ((size_t)chunk * p * p + k) + 1] = gy;
}

// Both gradients' pulls in one launch (they are independent): workgroups [0, n_u) take
// the image tiles, the rest the probe-gradient partial sums (block kb of chunk c at
// n_u + c * nb + kb), so neither waits for the other's tail.
__global__ __launch_bounds__(256) void k_grad(LossGradArgs a, int n_u, int nb) {
  const int b = blockIdx.x;
  if (b < n_u) grad_u_tile(a, b);
  else grad_w_part_block(a, (b - n_u) % nb, (b - n_u) / nb);
}

// the frames' loss terms summed in a fixed order by one workgroup
__device__ __forceinline__ void loss_total_block(const double* frame_loss, int J, double* out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int j = threadIdx.x; j < J; j += 256) s += frame_loss[j];
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) out[0] = s;
}

// the chunks' partial sums per probe pixel: the four wavefronts of a workgroup take every
// fourth chunk for the same 64 pixels, added in wavefront order
// With a.loss_out set, one more workgroup (the last) sums the frames' loss terms instead.
__global__ __launch_bounds__(256) void k_grad_w_final(LossGradArgs a) {
  if (a.loss_out && blockIdx.x == gridDim.x - 1) {   // uniform over the workgroup
    loss_total_block(a.frame_loss, a.J, a.loss_out);
    return;
  }
  __shared__ double part[2][4][64];
  const int p = a.p, lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const bool ok = k < p * p;
  double gx = 0.0, gy = 0.0;
  if (ok)
    for (int c = grp; c < a.n_chunks; c += 4) {
      gx += a.wpart[2 * ((size_t)c * p * p + k)];
      gy += a.wpart[2 * ((size_t)c * p * p + k) + 1];
    }
  part[0][grp][lane] = gx;
  part[1][grp][lane] = gy;
  __syncthreads();
  if (grp != 0 || !ok) return;
  gx = ((part[0][0][lane] + part[0][1][lane]) + part[0][2][lane]) + part[0][3][lane];
  gy = ((part[1][0][lane] + part[1][1][lane]) + part[1][2][lane]) + part[1][3][lane];
  a.grad_w[k] = make_float2((float)gx, (float)gy);
}

__global__ __launch_bounds__(256) void k_loss_total(const double* frame_loss, int J, double* out) {
  loss_total_block(frame_loss, J, out);
}

hipError_t launch_loss(int p, const LossArgs& a, bool grad, hipStream_t s) {
  const dim3 grid(NXCD * ((a.J + NXCD - 1) / NXCD));   // see loss_frame
#define ODP_LOSS(PP)                                                                                   \
  if (p == PP) {                                                                                       \
    if (grad) hipLaunchKernelGGL((k_loss<PP, true>), grid, dim3(Frame<PP>::T), 0, s, a);                 \
    else hipLaunchKernelGGL((k_loss<PP, false>), grid, dim3(Frame<PP>::T), 0, s, a);                     \
    return hipGetLastError();                                                                          \
  }
  ODP_LOSS(32)
  ODP_LOSS(64)
  // p = 128 on the two-half transform (two frames per CU)
  if (p == 128) {
    if (grad) hipLaunchKernelGGL((k_loss128<true>), grid, dim3(Half128::T), 0, s, a);
    else hipLaunchKernelGGL((k_loss128<false>), grid, dim3(Half128::T), 0, s, a);
    return hipGetLastError();
  }
#undef ODP_LOSS
  return hipErrorInvalidValue;
}

hipError_t launch_loss_total(const double* frame_loss, int J, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, frame_loss, J, out);
  return hipGetLastError();
}

hipError_t launch_loss_grads(const LossGradArgs& a, hipStream_t s) {
  const int nb = (a.p * a.p + 255) / 256;
  const int n_u = a.grad_u ? a.n_tiles : 0, n_w = a.grad_w ? nb * a.n_chunks : 0;
  if (n_u + n_w > 0) hipLaunchKernelGGL(k_grad, dim3(n_u + n_w), dim3(256), 0, s, a, n_u, nb);
  if (a.grad_w)
    hipLaunchKernelGGL(k_grad_w_final, dim3((a.p * a.p + 63) / 64 + (a.loss_out ? 1 : 0)), dim3(256), 0, s, a);
  else if (a.loss_out)
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, a.frame_loss, a.J, a.loss_out);
  return hipGetLastError();
}

}  // namespace odp

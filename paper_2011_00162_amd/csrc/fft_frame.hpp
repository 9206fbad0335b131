// fft_frame.hpp -- 2-D unitary DFT of one p x p frame per workgroup, for gfx950.
//
// The frame transform F of the measurement model (Sec. 2 of the paper: the
// normalized 2-D DFT) is computed as a three-step Cooley-Tukey factorisation of
// each axis, p = 16 * N2:
//     row index r = N2*r1 + r2,  frequency kr = k1 + 16*k2   (same for columns)
//     F_p x (kr) = sum_r2 W_N2^{r2 k2} * W_p^{r2 k1} * [ sum_r1 W_16^{r1 k1} x(N2 r1 + r2) ]
// Stage A: radix-16 DFT over r1 of every (r2, column) line, in registers;
//          twiddle W_p^{r2 k1}; exchange through LDS.
// Stage B: the same over the column index c1, in place in LDS.
// Stage C: the N2 x N2 DFT over (r2, c2) of every (k1_row, k1_col) block.
// Each thread holds 16 complex values in every stage (T = p*p/16 threads).
// LDS layout (at()): the columns of a row sit in blocks of 16, block b starting 2b
// complex values late (p = 64 and 128), and the row pitch LP is chosen with it:
// the 128-bit stage-C accesses of every 8 lanes then start in 8 different 4-bank
// groups (unshifted rows give them 2-way conflicts at p = 64 and 4-way at
// p = 128), the 64-bit stage-B column accesses of every 16 lanes hit 32 different
// banks, and the row-contiguous stage-A accesses stay contiguous.
//
// The inverse runs the stages backwards with conjugated twiddles.  Neither
// direction scales; the caller applies 1/p per direction (unitary F).
// Twiddles come from a host-computed (FP64, rounded to FP32) table
// tw[i][k] = W_p^{i k}, i < N2, k < 16, shared by stages A and B.
#pragma once
#include <hip/hip_runtime.h>

namespace odp {

// Row stride of the stage-B twiddle table when copied to LDS: rows 18 complex
// values (36 banks) apart start in different 4-bank groups, so the 128-bit reads
// of the N2 different rows a wavefront needs do not conflict (16 would put every
// row on the same banks).
constexpr int TWL = 18;

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 c_mulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// Streaming accesses (non-temporal hint) for the frame arrays a sweep touches once
// (amplitudes, multipliers, the handoff) when they are far larger than the last-level
// cache: they then do not push the reused image windows out of L2.  When the frame
// arrays fit in the 256 MB Infinity Cache, they stay there from one iteration to the
// next with ordinary accesses, which the hint would defeat; ld_s / st_s pick by NT.
typedef float odp_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float2 ld_nt(const float2* p) {
  const odp_f2v x = __builtin_nontemporal_load(reinterpret_cast<const odp_f2v*>(p));
  return make_float2(x.x, x.y);
}
__device__ __forceinline__ void st_nt(float2* p, float2 v) {
  odp_f2v x;
  x.x = v.x;
  x.y = v.y;
  __builtin_nontemporal_store(x, reinterpret_cast<odp_f2v*>(p));
}
typedef float odp_f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_nt(const float4* p) {
  const odp_f4v x = __builtin_nontemporal_load(reinterpret_cast<const odp_f4v*>(p));
  return make_float4(x.x, x.y, x.z, x.w);
}
__device__ __forceinline__ void st_nt(float4* p, float4 v) {
  odp_f4v x;
  x.x = v.x;
  x.y = v.y;
  x.z = v.z;
  x.w = v.w;
  __builtin_nontemporal_store(x, reinterpret_cast<odp_f4v*>(p));
}
template <bool NT, class T>
__device__ __forceinline__ T ld_s(const T* p) {
  if constexpr (NT) return ld_nt(p);
  else return *p;
}
template <bool NT, class T>
__device__ __forceinline__ void st_s(T* p, T v) {
  if constexpr (NT) st_nt(p, v);
  else *p = v;
}
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 c_rot(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// multiply by W^m (forward, W = exp(-2 pi i/n)) or its conjugate (inverse), tw = W^m
template <bool INV>
__device__ __forceinline__ float2 c_tw(float2 a, float2 tw) {
  return INV ? c_mulc(a, tw) : c_mul(a, tw);
}

// cos(2 pi m / 16) and sin(2 pi m / 16), m = 0..15, from the closed forms
// cos(pi/8) = sqrt(2 + sqrt 2)/2, sin(pi/8) = sqrt(2 - sqrt 2)/2, cos(pi/4) = sqrt(2)/2.
#define ODP_C8 0.92387953251128675613f
#define ODP_S8 0.38268343236508977173f
#define ODP_R2 0.70710678118654752440f

__device__ __forceinline__ float2 w16(int m) {  // forward twiddle exp(-2 pi i m / 16)
  // m is a compile-time constant after unrolling
  const float c[16] = {1.f, ODP_C8, ODP_R2, ODP_S8, 0.f, -ODP_S8, -ODP_R2, -ODP_C8,
                       -1.f, -ODP_C8, -ODP_R2, -ODP_S8, 0.f, ODP_S8, ODP_R2, ODP_C8};
  const float s[16] = {0.f, ODP_S8, ODP_R2, ODP_C8, 1.f, ODP_C8, ODP_R2, ODP_S8,
                       0.f, -ODP_S8, -ODP_R2, -ODP_C8, -1.f, -ODP_C8, -ODP_R2, -ODP_S8};
  return make_float2(c[m & 15], -s[m & 15]);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = c_add(t, b);
  b = c_sub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  float2 s02 = c_add(x0, x2), d02 = c_sub(x0, x2);
  float2 s13 = c_add(x1, x3), d13 = c_rot<INV>(c_sub(x1, x3));
  x0 = c_add(s02, s13);
  x2 = c_sub(s02, s13);
  x1 = c_add(d02, d13);
  x3 = c_sub(d02, d13);
}

// In-place length-8 DFT, natural order in and out (8 = 4 x 2, n = 2 n1 + n2).
template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  dft4<INV>(v[0], v[2], v[4], v[6]);   // n2 = 0 -> a0[k1] at v[2 k1]
  dft4<INV>(v[1], v[3], v[5], v[7]);   // n2 = 1 -> a1[k1] at v[2 k1 + 1]
  // twiddle W8^{k1} on a1: W8^1 = (r, -r), W8^2 = -i, W8^3 = (-r, -r)
  v[3] = c_tw<INV>(v[3], make_float2(ODP_R2, -ODP_R2));
  v[5] = c_rot<INV>(v[5]);
  v[7] = c_tw<INV>(v[7], make_float2(-ODP_R2, -ODP_R2));
  float2 o[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a = v[2 * k1], b = v[2 * k1 + 1];
    o[k1] = c_add(a, b);       // k2 = 0
    o[k1 + 4] = c_sub(a, b);   // k2 = 1
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = o[k];
}

// In-place length-16 DFT, natural order in and out (16 = 4 x 4, n = 4 n1 + n2).
template <bool INV>
__device__ __forceinline__ void dft16(float2* v) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // now v[4 k1 + n2] = a[n2][k1]; twiddle W16^{n2 k1}
#pragma unroll
  for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)   // W16^4 = -i is a swap (a multiply by 0 would not fold away)
      v[4 * k1 + n2] = n2 * k1 == 4 ? c_rot<INV>(v[4 * k1 + n2]) : c_tw<INV>(v[4 * k1 + n2], w16(n2 * k1));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // v[4 k1 + k2] = X[k1 + 4 k2]: transpose to natural order
  float2 o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = o[k];
}

template <int P>
struct Frame {
  static constexpr int N2 = P / 16;      // second radix per axis
  static constexpr int T = P * N2;       // threads per frame = p*p/16
  static constexpr int LP = P == 128 ? 152 : P == 64 ? 76 : P + N2;  // LDS row pitch (complex)
  static constexpr int LDS = P * LP;     // LDS complex elements per frame
  static constexpr int NC = (N2 * N2 >= 16) ? 1 : 16 / (N2 * N2);  // stage-C blocks per thread
  static constexpr int SHIFT = P >= 64 ? 2 : 0;  // per 16-column block (complex values)
  static_assert(P + SHIFT * (P / 16 - 1) <= LP, "shifted row must fit the row pitch");

  // LDS index of (row, col): column block b = col / 16 starts SHIFT * b values late
  __device__ static __forceinline__ int at(int row, int col) { return row * LP + col + SHIFT * (col >> 4); }

  // Stage-A line of thread t: column and r2.  Value r1 sits at row N2*r1 + r2.
  __device__ static __forceinline__ int a_col(int t) { return t % P; }
  __device__ static __forceinline__ int a_r2(int t) { return t / P; }
  // r2 is constant over a wavefront when p >= 64: make that visible to the
  // compiler so the stage-A twiddle row is fetched with scalar loads.
  __device__ static __forceinline__ int uniform_r2(int t) {
    if constexpr (P >= 64) return __builtin_amdgcn_readfirstlane(t / P);
    return t / P;
  }

  // ---- forward ---------------------------------------------------------------
  // v: the 16 spatial values of this thread's stage-A line (already multiplied
  // by the probe).  On return v holds 16 frequencies, see freq().
  __device__ static void forward(float2* v, float2* lds, const float2* __restrict__ tw, int t) {
    forward_a(v, lds, tw, t);
    forward_bc(v, lds, tw, t);
  }

  // the two halves of forward(): stage A into LDS, then stages B and C back to v
  __device__ static __forceinline__ void forward_a(float2* v, float2* lds, const float2* __restrict__ tw, int t) {
    const int col = a_col(t), r2 = a_r2(t);
    const float2* ta = tw + 16 * uniform_r2(t);
    dft16<false>(v);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const float2 x = k == 0 ? v[k] : c_mul(v[k], ta[k]);
      lds[at(N2 * k + r2, col)] = x;
    }
  }

  // TS: row stride of the twiddle table tw (16 in global memory; TWL for the padded
  // copy in LDS)
  template <int TS = 16>
  __device__ static __forceinline__ void forward_bc(float2* v, float2* lds, const float2* __restrict__ tw, int t) {
    __syncthreads();
    stage_b<false, TS>(lds, tw, t);
    __syncthreads();
    stage_c_fwd(v, lds, t);
  }

  // ---- inverse ---------------------------------------------------------------
  // v: 16 frequencies in the freq() layout.  On return v holds the 16 spatial
  // values of this thread's stage-A line (unscaled inverse DFT).
  template <int TS = 16>
  __device__ static void inverse(float2* v, float2* lds, const float2* __restrict__ tw, int t) {
    stage_c_inv(v, lds, t);
    __syncthreads();
    stage_b<true, TS>(lds, tw, t);
    __syncthreads();
    const int col = a_col(t), r2 = a_r2(t);
    const float2* ta = tw + TS * uniform_r2(t);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const float2 x = lds[at(N2 * k + r2, col)];
      v[k] = k == 0 ? x : c_mulc(x, ta[k]);
    }
    dft16<true>(v);
  }

  template <bool INV, int TS>
  __device__ static __forceinline__ void stage_b(float2* lds, const float2* __restrict__ tw, int t) {
    const int c2 = t % N2, R = t / N2;
    const float4* tb4 = reinterpret_cast<const float4*>(tw + TS * c2);
    float2 v[16], w[16];
#pragma unroll
    for (int k = 0; k < 16; k += 2) {
      const float4 q = tb4[k / 2];
      w[k] = make_float2(q.x, q.y);
      w[k + 1] = make_float2(q.z, q.w);
    }
    if (INV) {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const float2 x = lds[at(R, c2 + N2 * k)];
        v[k] = k == 0 ? x : c_mulc(x, w[k]);
      }
      dft16<true>(v);
#pragma unroll
      for (int k = 0; k < 16; ++k) lds[at(R, c2 + N2 * k)] = v[k];
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = lds[at(R, c2 + N2 * k)];
      dft16<false>(v);
#pragma unroll
      for (int k = 0; k < 16; ++k) lds[at(R, c2 + N2 * k)] = k == 0 ? v[k] : c_mul(v[k], w[k]);
    }
  }

  // Natural frequency (kr, kc) of value e held by thread t after forward().
  __device__ static __forceinline__ void freq(int t, int e, int& kr, int& kc) {
    if constexpr (P == 32) {            // 4 blocks of 2x2 per thread
      const int b = t + 64 * (e >> 2);
      const int k1c = b & 15, k1r = b >> 4;
      const int k2r = (e >> 1) & 1, k2c = e & 1;
      kr = k1r + 16 * k2r;
      kc = k1c + 16 * k2c;
    } else if constexpr (P == 64) {     // one 4x4 block per thread
      const int k1c = t & 15, k1r = t >> 4;
      kr = k1r + 16 * (e >> 2);
      kc = k1c + 16 * (e & 3);
    } else {                            // P == 128: two lines of 8 per thread
      const int L = t + 1024 * (e >> 3);
      const int k1c = L & 15, k2r = (L >> 4) & 7, k1r = L >> 7;
      kr = k1r + 16 * k2r;
      kc = k1c + 16 * (e & 7);
    }
  }

  __device__ static __forceinline__ void stage_c_fwd(float2* v, float2* lds, int t) {
    if constexpr (P == 32) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = t + 64 * q, k1c = b & 15, k1r = b >> 4;
        float4 r0 = *reinterpret_cast<const float4*>(lds + at(2 * k1r, 2 * k1c));
        float4 r1 = *reinterpret_cast<const float4*>(lds + at(2 * k1r + 1, 2 * k1c));
        float2 a00 = make_float2(r0.x, r0.y), a01 = make_float2(r0.z, r0.w);
        float2 a10 = make_float2(r1.x, r1.y), a11 = make_float2(r1.z, r1.w);
        dft2<false>(a00, a10);
        dft2<false>(a01, a11);
        dft2<false>(a00, a01);
        dft2<false>(a10, a11);
        v[4 * q + 0] = a00; v[4 * q + 1] = a01; v[4 * q + 2] = a10; v[4 * q + 3] = a11;
      }
    } else if constexpr (P == 64) {
      const int k1c = t & 15, k1r = t >> 4;
      float2 a[16];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float4 lo = *reinterpret_cast<const float4*>(lds + at(4 * k1r + r, 4 * k1c));
        float4 hi = *reinterpret_cast<const float4*>(lds + at(4 * k1r + r, 4 * k1c + 2));
        a[4 * r + 0] = make_float2(lo.x, lo.y); a[4 * r + 1] = make_float2(lo.z, lo.w);
        a[4 * r + 2] = make_float2(hi.x, hi.y); a[4 * r + 3] = make_float2(hi.z, hi.w);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) dft4<false>(a[c], a[4 + c], a[8 + c], a[12 + c]);
#pragma unroll
      for (int r = 0; r < 4; ++r) dft4<false>(a[4 * r], a[4 * r + 1], a[4 * r + 2], a[4 * r + 3]);
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = a[e];
    } else {  // P == 128: DFT8 over r2 (lines k1r,k1c,c2), then DFT8 over c2 (lines k1r,k2r,k1c)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int L = t + 1024 * q;
        const int c2 = L & 7, k1c = (L >> 3) & 15, k1r = L >> 7;
        float2 a[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) a[r] = lds[at(8 * k1r + r, 8 * k1c + c2)];
        dft8<false>(a);
#pragma unroll
        for (int r = 0; r < 8; ++r) lds[at(8 * k1r + r, 8 * k1c + c2)] = a[r];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int L = t + 1024 * q;
        const int k1c = L & 15, k2r = (L >> 4) & 7, k1r = L >> 7;
        float2 a[8];
#pragma unroll
        for (int c = 0; c < 8; c += 2) {
          float4 x = *reinterpret_cast<const float4*>(lds + at(8 * k1r + k2r, 8 * k1c + c));
          a[c] = make_float2(x.x, x.y);
          a[c + 1] = make_float2(x.z, x.w);
        }
        dft8<false>(a);
#pragma unroll
        for (int c = 0; c < 8; ++c) v[8 * q + c] = a[c];
      }
    }
  }

  // Exact reverse of stage_c_fwd (inverse DFTs, results written back to LDS).
  __device__ static __forceinline__ void stage_c_inv(float2* v, float2* lds, int t) {
    if constexpr (P == 32) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = t + 64 * q, k1c = b & 15, k1r = b >> 4;
        float2 a00 = v[4 * q + 0], a01 = v[4 * q + 1], a10 = v[4 * q + 2], a11 = v[4 * q + 3];
        dft2<true>(a00, a01);
        dft2<true>(a10, a11);
        dft2<true>(a00, a10);
        dft2<true>(a01, a11);
        *reinterpret_cast<float4*>(lds + at(2 * k1r, 2 * k1c)) = make_float4(a00.x, a00.y, a01.x, a01.y);
        *reinterpret_cast<float4*>(lds + at(2 * k1r + 1, 2 * k1c)) = make_float4(a10.x, a10.y, a11.x, a11.y);
      }
    } else if constexpr (P == 64) {
      const int k1c = t & 15, k1r = t >> 4;
      float2 a[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) a[e] = v[e];
#pragma unroll
      for (int r = 0; r < 4; ++r) dft4<true>(a[4 * r], a[4 * r + 1], a[4 * r + 2], a[4 * r + 3]);
#pragma unroll
      for (int c = 0; c < 4; ++c) dft4<true>(a[c], a[4 + c], a[8 + c], a[12 + c]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        *reinterpret_cast<float4*>(lds + at(4 * k1r + r, 4 * k1c)) =
            make_float4(a[4 * r].x, a[4 * r].y, a[4 * r + 1].x, a[4 * r + 1].y);
        *reinterpret_cast<float4*>(lds + at(4 * k1r + r, 4 * k1c + 2)) =
            make_float4(a[4 * r + 2].x, a[4 * r + 2].y, a[4 * r + 3].x, a[4 * r + 3].y);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int L = t + 1024 * q;
        const int k1c = L & 15, k2r = (L >> 4) & 7, k1r = L >> 7;
        float2 a[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = v[8 * q + c];
        dft8<true>(a);
#pragma unroll
        for (int c = 0; c < 8; c += 2)
          *reinterpret_cast<float4*>(lds + at(8 * k1r + k2r, 8 * k1c + c)) =
              make_float4(a[c].x, a[c].y, a[c + 1].x, a[c + 1].y);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int L = t + 1024 * q;
        const int c2 = L & 7, k1c = (L >> 3) & 15, k1r = L >> 7;
        float2 a[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) a[r] = lds[at(8 * k1r + r, 8 * k1c + c2)];
        dft8<true>(a);
#pragma unroll
        for (int r = 0; r < 8; ++r) lds[at(8 * k1r + r, 8 * k1c + c2)] = a[r];
      }
    }
  }
};

}  // namespace odp

namespace odp {

// An empty instruction that takes x in registers and may change it: values computed
// before it cannot be recomputed or moved after it (used to keep the compiler from
// sinking a butterfly's tail past later phases, where its intermediates would spill).
__device__ __forceinline__ void pin(float2& x) { asm volatile("" : "+v"(x.x), "+v"(x.y)); }

// p = 128 with 512 threads and the LDS exchanges done one half of the frame at a time.
// The same factorisation as Frame<128> (radix 16 x 8 per axis), but each thread holds
// 32 values: two stage-A lines (column col = t % 128, r2 = g and g + 4, g = t / 128),
// and the frame passes through a 64-row LDS buffer in two halves (rows 64h .. 64h + 63
// hold the stage-A outputs k1 in [8h, 8h + 8)).  Stages B and C of one half need only
// that half, and the elementwise prox can run on a half's frequencies at once, so the
// sweep does forward B/C, prox and inverse C/B per half; only stage A (and its inverse)
// needs both halves, and it runs in registers.  77 KB of LDS per frame lets two frames
// share a CU, which overlaps one frame's memory phases with the other's arithmetic.
//
// Register slots v[0..31]:
//   spatial:   v[16 l + r1] = x(row 8 r1 + g + 4 l, col)            l = 0, 1
//   stage A:   v[16 l + k1] = line l after the radix-16 DFT and twiddle
//   frequency: v[16 q + 8 h + k2c] = X(kr, kc), see freq(); half h occupies the slots
//              its stage-A outputs left (8h .. 8h + 7 and 16 + 8h .. 16 + 8h + 7)
struct Half128 {
  static constexpr int P = 128, N2 = 8, T = 512;
  static constexpr int LP = 152;                   // row pitch (complex), as Frame<128>
  static constexpr int ROWS = 64;                  // rows per half
  static constexpr int LDS = ROWS * LP;
  __host__ __device__ static __forceinline__ int at(int row, int col) { return row * LP + col + 2 * (col >> 4); }
  __device__ static __forceinline__ int a_col(int t) { return t & 127; }
  __device__ static __forceinline__ int uniform_g(int t) { return __builtin_amdgcn_readfirstlane(t >> 7); }
  // image row of spatial slot e (column a_col(t))
  __device__ static __forceinline__ int row_of(int t, int e) { return 8 * (e & 15) + (t >> 7) + 4 * (e >> 4); }

  // natural frequency (kr, kc) of slot e after the forward transform
  __device__ static __forceinline__ void freq(int t, int e, int& kr, int& kc) {
    const int q = e >> 4, h = (e >> 3) & 1, k2c = e & 7;
    const int L = t + 512 * q;
    const int k1c = L & 15, k2r = (L >> 4) & 7, k1r = 8 * h + (L >> 7);
    kr = k1r + 16 * k2r;
    kc = k1c + 16 * k2c;
  }

  // stage A of line l in registers (tw: [8][16] table W_128^{i k}, global; the row
  // is wavefront-uniform, so the twiddles come through scalar loads)
  __device__ static __forceinline__ void stage_a_fwd_line(float2* v, const float2* __restrict__ tw, int t, int l) {
    const float2* ta = tw + 16 * (uniform_g(t) + 4 * l);
    dft16<false>(v + 16 * l);
#pragma unroll
    for (int k = 1; k < 16; ++k) v[16 * l + k] = c_mul(v[16 * l + k], ta[k]);
  }
  __device__ static __forceinline__ void stage_a_inv_line(float2* v, const float2* __restrict__ tw, int t, int l) {
    const float2* ta = tw + 16 * (uniform_g(t) + 4 * l);
#pragma unroll
    for (int k = 1; k < 16; ++k) v[16 * l + k] = c_mulc(v[16 * l + k], ta[k]);
    dft16<true>(v + 16 * l);
  }

  // LDS index of the k-th (k < 8) 128-bit pair of complex values that thread t reads in
  // the last stage-C pass of a half (see half_fwd).  These pairs partition the buffer
  // over the threads, so a thread may overwrite its own right after that pass without a
  // barrier.
  __host__ __device__ static __forceinline__ int own_pair(int t, int k) {
    const int L = t + 512 * (k >> 2);
    const int k1c = L & 15, k2r = (L >> 4) & 7, k1r = L >> 7;
    return at(8 * k1r + k2r, 8 * k1c + 2 * (k & 3));
  }
  // LDS index of stage-A output k (< 8) of line l of thread t in a half (its slot
  // 16 l + 8 h + k): written first in half_fwd, read last in half_inv
  __host__ __device__ static __forceinline__ int a_slot(int t, int k, int l) {
    return at(8 * k + (t >> 7) + 4 * l, t & 127);
  }

  // half h forward: stage-A outputs of the half into LDS, stages B and C, frequencies
  // back into the same slots.  Starts with a barrier (the LDS buffer may still be read
  // by the previous half) unless LEAD is false: a caller whose last LDS accesses before
  // it were this thread's own final reads of half_inv (the same slots as the first
  // writes here) needs none.  Ends after the stage-C reads (no barrier).
  template <int TS, bool LEAD = true>
  __device__ static __forceinline__ void half_fwd(float2* v, float2* lds, const float2* __restrict__ twl, int t,
                                                  int h) {
    if (LEAD) __syncthreads();
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
      for (int k = 0; k < 8; ++k) lds[a_slot(t, k, l)] = v[16 * l + 8 * h + k];
    __syncthreads();
    stage_b<false, TS>(lds, twl, t);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {   // stage C, DFT8 over r2 of lines (k1r, k1c, c2)
      const int L = t + 512 * q;
      const int c2 = L & 7, k1c = (L >> 3) & 15, k1r = L >> 7;
      float2 a[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) a[r] = lds[at(8 * k1r + r, 8 * k1c + c2)];
      dft8<false>(a);
#pragma unroll
      for (int r = 0; r < 8; ++r) lds[at(8 * k1r + r, 8 * k1c + c2)] = a[r];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {   // stage C, DFT8 over c2 of lines (k1r, k2r, k1c): own_pair
      float2 a[8];
#pragma unroll
      for (int c = 0; c < 8; c += 2) {
        const float4 x = *reinterpret_cast<const float4*>(lds + own_pair(t, 4 * q + c / 2));
        a[c] = make_float2(x.x, x.y);
        a[c + 1] = make_float2(x.z, x.w);
      }
      dft8<false>(a);
#pragma unroll
      for (int c = 0; c < 8; ++c) v[16 * q + 8 * h + c] = a[c];
    }
  }

  // half h inverse: the exact reverse, ending with the stage-A inputs of the half back
  // in their slots.  Starts with a barrier (the stage-C reads of the forward half) unless
  // LEAD is false: its first writes go to the thread's own_pair slots, which no other
  // thread reads in the last stage-C pass, so a caller that touched no other LDS since
  // then needs none.  Ends after the final LDS reads (no barrier).
  template <int TS, bool LEAD = true>
  __device__ static __forceinline__ void half_inv(float2* v, float2* lds, const float2* __restrict__ twl, int t,
                                                  int h) {
    if (LEAD) __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {   // inverse DFT8 over c2 of lines (k1r, k2r, k1c): own_pair
      float2 a[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) a[c] = v[16 * q + 8 * h + c];
      dft8<true>(a);
#pragma unroll
      for (int c = 0; c < 8; c += 2)
        *reinterpret_cast<float4*>(lds + own_pair(t, 4 * q + c / 2)) = make_float4(a[c].x, a[c].y, a[c + 1].x, a[c + 1].y);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int L = t + 512 * q;
      const int c2 = L & 7, k1c = (L >> 3) & 15, k1r = L >> 7;
      float2 a[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) a[r] = lds[at(8 * k1r + r, 8 * k1c + c2)];
      dft8<true>(a);
#pragma unroll
      for (int r = 0; r < 8; ++r) lds[at(8 * k1r + r, 8 * k1c + c2)] = a[r];
    }
    __syncthreads();
    stage_b<true, TS>(lds, twl, t);
    __syncthreads();
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
      for (int k = 0; k < 8; ++k) v[16 * l + 8 * h + k] = lds[a_slot(t, k, l)];
  }

  // stage B on the 64 rows of a half: thread t takes row t / 8 and c2 = t % 8 (the
  // same column lines as Frame<128>, twiddle rows TS apart).  The twiddles are read
  // where they are applied (after the DFT forward, before it inverse), so they never
  // sit in registers across the butterfly.  The twiddle row's offset comes from an
  // opaque copy of c2: shared between the four calls of a frame sweep, it would stay
  // live across the prox and spill.
  template <bool INV, int TS>
  __device__ static __forceinline__ void stage_b(float2* lds, const float2* __restrict__ tw, int t) {
    const int c2 = t & 7, R = t >> 3;
    int c2q = c2;
    asm volatile("" : "+v"(c2q));
    const float4* tb4 = reinterpret_cast<const float4*>(tw + TS * c2q);
    float2 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = lds[at(R, c2 + 8 * k)];
    if (INV) {
#pragma unroll
      for (int k = 0; k < 16; k += 2) {
        const float4 q = tb4[k / 2];
        if (k > 0) v[k] = c_mulc(v[k], make_float2(q.x, q.y));
        v[k + 1] = c_mulc(v[k + 1], make_float2(q.z, q.w));
      }
      dft16<true>(v);
#pragma unroll
      for (int k = 0; k < 16; ++k) lds[at(R, c2 + 8 * k)] = v[k];
    } else {
      dft16<false>(v);
#pragma unroll
      for (int k = 0; k < 16; k += 2) {
        const float4 q = tb4[k / 2];
        if (k > 0) v[k] = c_mul(v[k], make_float2(q.x, q.y));
        v[k + 1] = c_mul(v[k + 1], make_float2(q.z, q.w));
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) lds[at(R, c2 + 8 * k)] = v[k];
    }
  }
};

}  // namespace odp

// fft_mfma.hpp -- the p x p unitary DFT of fft_frame.hpp with its radix-16 stages on
// the matrix cores (split BF16, FP32 accumulation); p = 64 and 128.
//
// The factorisation is Frame<P>'s (p = 16 * N2 per axis, stages A, B, C), and so are
// the LDS layout and stage C (the N2 x N2 block DFTs, FP32 on the vector ALUs).
// Stages A and B are each a batch of 16-point DFTs followed by a twiddle that depends
// on the line's residue q (r2 in stage A, c2 in stage B) and on the output index k:
//     y = M_q x,   M_q[k][r] = W_p^{q k} W_16^{r k}      (inverse: x = M_q^H y)
// Every wavefront owns lines of one residue q, so the twiddle folds into the 16 x 16
// matrix, and the batch is a real product
//     [Re y; Im y] = [Re M  -Im M; Im M  Re M] [Re x; Im x]
// over a 32-wide contraction: one v_mfma_f32_16x16x32_bf16 per output part and term,
// each real factor split as a = a_hi + a_lo (bf16, round to nearest even) and
// a b = a_hi b_hi + a_hi b_lo + a_lo b_hi (the dropped a_lo b_lo is about 2^-16 of it).
// The M_q splits come from a host FP64 table.
//
// MFMA operand layouts (wave64; lane l, g = l / 16, n0 = l % 16):
//   A[m][k]  element i (0..7) at m = n0, k = 8g + i
//   B[k][n]  element i (0..7) at k = 8g + i, n = n0
//   D[m][n]  element i (0..3) at m = 4g + i, n = n0
// Contraction element k = 8g + 2s + c is input r = 4g + s, part c (0 real, 1 imag), so a
// lane's B operand is the interleaved complex values r = 4g .. 4g + 3 of line n0, and
// its D tiles hold outputs k = 4g .. 4g + 3 of the same line: input and output share
// one register layout.  A thread holds four line blocks: value e = 4 cb + s is r (or k)
// = 4g + s of line n0 of block cb, 16 values as in Frame<P>.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_frame.hpp"

namespace odp {
namespace mf {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A-operand rows of one M_q for one lane: real-output row (hi, lo), imaginary-output row
struct Tab {
  bf16x8 rh, rl, ih, il;
};

// Table layout (uint4 = 8 bf16): [set][dir (0 forward, 1 inverse)][q < N2][lane < 64][4]
// with the four parts in Tab order.  Set 0 has the natural index orders; set 1 (p = 128,
// for Half128MF's stage A) permutes the forward matrix's output rows and the inverse
// matrix's contraction columns by pi (see Half128MF).
constexpr int SET_WORDS = 2 * 64 * 4;   // uint4 per set and residue
__device__ __forceinline__ Tab load_tab(const uint4* __restrict__ tab, int n2, int inv, int q, int lane) {
  const uint4* p = tab + ((size_t)(inv * n2 + q) * 64 + lane) * 4;
  const uint4 a = p[0], b = p[1], c = p[2], d = p[3];
  return Tab{__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), __builtin_bit_cast(bf16x8, c),
             __builtin_bit_cast(bf16x8, d)};
}

// hi and lo parts of (x0, x1), two to a dword (element 0 in the low half):
// .x = bf16(x), .y = bf16(x - hi), both round to nearest even
__device__ __forceinline__ uint2 split2(float x0, float x1) {
  const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{x0, x1}, bf16x2));
  const float h0 = __builtin_bit_cast(float, h << 16), h1 = __builtin_bit_cast(float, h & 0xffff0000u);
  return make_uint2(h, __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{x0 - h0, x1 - h1}, bf16x2)));
}

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// The 16-point transforms (with the folded twiddle) of NB line blocks, in place:
// v[4 cb + s] = value 4g + s of line n0 of block cb, before and after.
template <int NB = 4>
__device__ __forceinline__ void radix16(float2* v, const Tab& A) {
  bf16x8 bh[NB], bl[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const uint2 s0 = split2(v[4 * cb].x, v[4 * cb].y), s1 = split2(v[4 * cb + 1].x, v[4 * cb + 1].y);
    const uint2 s2 = split2(v[4 * cb + 2].x, v[4 * cb + 2].y), s3 = split2(v[4 * cb + 3].x, v[4 * cb + 3].y);
    bh[cb] = __builtin_bit_cast(bf16x8, u32x4{s0.x, s1.x, s2.x, s3.x});
    bl[cb] = __builtin_bit_cast(bf16x8, u32x4{s0.y, s1.y, s2.y, s3.y});
  }
  floatx4 re[NB], im[NB];
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
  // three passes over the blocks, so consecutive products of one accumulator are 2 NB
  // instructions apart
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    re[cb] = mfma(A.rh, bh[cb], zero);
    im[cb] = mfma(A.ih, bh[cb], zero);
  }
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    re[cb] = mfma(A.rh, bl[cb], re[cb]);
    im[cb] = mfma(A.ih, bl[cb], im[cb]);
  }
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    re[cb] = mfma(A.rl, bh[cb], re[cb]);
    im[cb] = mfma(A.il, bh[cb], im[cb]);
  }
#pragma unroll
  for (int cb = 0; cb < NB; ++cb)
#pragma unroll
    for (int s = 0; s < 4; ++s) v[4 * cb + s] = make_float2(re[cb][s], im[cb][s]);
}

}  // namespace mf

template <int P>
struct FrameMF {
  static_assert(P == 64 || P == 128, "the MFMA stages are built for p = 64 and 128");
  using Base = Frame<P>;
  static constexpr int N2 = Base::N2, T = Base::T, LP = Base::LP, LDS = Base::LDS;

  __device__ static __forceinline__ int wave(int t) { return __builtin_amdgcn_readfirstlane(t >> 6); }
  // stage A: wavefront w takes the lines of residue r2 over 64 columns from c0
  __device__ static __forceinline__ int a_r2(int w) { return P == 64 ? w : w >> 1; }
  __device__ static __forceinline__ int a_c0(int w) { return P == 64 ? 0 : 64 * (w & 1); }
  // stage B: wavefront w takes the lines of residue c2 over 64 rows from R0
  __device__ static __forceinline__ int b_c2(int w) { return P == 64 ? w : w & 7; }
  __device__ static __forceinline__ int b_r0(int w) { return P == 64 ? 0 : 64 * (w >> 3); }

  // spatial position of value e of thread t (the gather before forward(), the output of
  // inverse())
  __device__ static __forceinline__ int row(int t, int e) {
    return N2 * (4 * ((t & 63) >> 4) + (e & 3)) + a_r2(wave(t));
  }
  __device__ static __forceinline__ int col(int t, int e) { return a_c0(wave(t)) + 16 * (e >> 2) + (t & 15); }

  __device__ static __forceinline__ void freq(int t, int e, int& kr, int& kc) { Base::freq(t, e, kr, kc); }

  // v: the 16 spatial values at row(t, e), col(t, e) (already multiplied by the probe).
  __device__ static __forceinline__ void forward_a(float2* v, float2* lds, const uint4* __restrict__ tab, int t) {
    const int w = wave(t), lane = t & 63;
    const mf::Tab A = mf::load_tab(tab, N2, 0, a_r2(w), lane);
    mf::radix16(v, A);
#pragma unroll
    for (int e = 0; e < 16; ++e) lds[Base::at(row(t, e), col(t, e))] = v[e];   // output k1 sits where r1 was
  }

  template <bool INV>
  __device__ static __forceinline__ void stage_b(float2* lds, const uint4* __restrict__ tab, int t) {
    const int w = wave(t), lane = t & 63, g = lane >> 4, n0 = lane & 15;
    const int c2 = b_c2(w), r0 = b_r0(w);
    const mf::Tab A = mf::load_tab(tab, N2, INV ? 1 : 0, c2, lane);
    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = lds[Base::at(r0 + 16 * (e >> 2) + n0, c2 + N2 * (4 * g + (e & 3)))];
    mf::radix16(v, A);
#pragma unroll
    for (int e = 0; e < 16; ++e) lds[Base::at(r0 + 16 * (e >> 2) + n0, c2 + N2 * (4 * g + (e & 3)))] = v[e];
  }

  // stages B and C: on return v holds 16 frequencies, see freq()
  __device__ static __forceinline__ void forward_bc(float2* v, float2* lds, const uint4* __restrict__ tab, int t) {
    __syncthreads();
    stage_b<false>(lds, tab, t);
    __syncthreads();
    Base::stage_c_fwd(v, lds, t);
  }

  // v: 16 frequencies in the freq() layout; on return the 16 spatial values at
  // row(t, e), col(t, e) (unscaled inverse DFT)
  __device__ static __forceinline__ void inverse(float2* v, float2* lds, const uint4* __restrict__ tab, int t) {
    Base::stage_c_inv(v, lds, t);
    __syncthreads();
    stage_b<true>(lds, tab, t);
    __syncthreads();
    const int w = wave(t), lane = t & 63;
    const mf::Tab A = mf::load_tab(tab, N2, 1, a_r2(w), lane);
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = lds[Base::at(row(t, e), col(t, e))];
    mf::radix16(v, A);
  }
};

// p = 128 on the two-half transform (Half128's LDS buffer of 64 rows, 512 threads, two
// frames per CU) with stages A and B on the matrix cores.
// Thread t: wavefront w = t / 64 (stage A residue r2 = w, stage B residue c2 = w),
// lane = 16 g + n0.  Register slots v[4 cb + i] (cb < 8, i < 4):
//   spatial:   x(row 8 (4g + i) + w, col 16 cb + n0)
//   stage A:   output k1 = pi(4g + i) of line (r2 = w, col 16 cb + n0), where
//              pi(4g + i) = 8 (i / 2) + 2g + i % 2, so slots with i / 2 = h hold half h
//              (k1 in [8h, 8h + 8)): 16 slots per half per thread, as in Half128
//   frequency: the 16 frequencies f = 8q + c of half h (Half128's slot 16q + 8h + c)
//              sit in slot 4 (f / 2) + 2h + f % 2, the ones half h's stage A left.
// The forward stage-A matrix produces its outputs in pi order (its A-operand rows are
// permuted) and the inverse contracts in pi order (its columns are), table set 1.
struct Half128MF {
  static constexpr int P = 128, N2 = 8, T = 512;
  static constexpr int LP = Half128::LP, ROWS = Half128::ROWS, LDS = Half128::LDS;
  __device__ static __forceinline__ int at(int row, int col) { return Half128::at(row, col); }
  // LDS index of the half's stage-A value (block cb < 8, jj < 2) of lane `lane` of
  // wavefront w: written first in half_fwd, read last in half_inv
  __host__ __device__ static __forceinline__ int a_slot(int w, int lane, int cb, int jj) {
    return Half128::at(8 * (2 * (lane >> 4) + jj) + w, 16 * cb + (lane & 15));
  }
  __device__ static __forceinline__ int wave(int t) { return __builtin_amdgcn_readfirstlane(t >> 6); }
  __device__ static __forceinline__ int row(int t, int e) { return 8 * (4 * ((t & 63) >> 4) + (e & 3)) + wave(t); }
  __device__ static __forceinline__ int col(int t, int e) { return 16 * (e >> 2) + (t & 15); }
  // slot of frequency i (< 8) of group qq of half h
  __device__ static __forceinline__ int fslot(int h, int qq, int i) {
    const int f = 8 * qq + i;
    return 4 * (f >> 1) + 2 * h + (f & 1);
  }
  __device__ static __forceinline__ void freq_hq(int t, int h, int qq, int i, int& kr, int& kc) {
    Half128::freq(t, 16 * qq + 8 * h + i, kr, kc);
  }

  // stage A (forward) of blocks 2 grp, 2 grp + 1 (slots 8 grp .. 8 grp + 7), in place
  __device__ static __forceinline__ void stage_a_fwd(float2* v, const mf::Tab& A, int grp) {
    mf::radix16<2>(v + 8 * grp, A);
  }
  __device__ static __forceinline__ void stage_a_inv(float2* v, const mf::Tab& A, int grp) {
    mf::radix16<2>(v + 8 * grp, A);
  }
  __device__ static __forceinline__ mf::Tab tab_a(const uint4* __restrict__ tab, int inv, int t) {
    return mf::load_tab(tab + mf::SET_WORDS * N2, N2, inv, wave(t), t & 63);
  }

  // stage B on the 64 rows of a half: wavefront w takes c2 = w, rows 16 cb + n0 (cb < 4),
  // two blocks at a time
  template <bool INV>
  __device__ static __forceinline__ void stage_b(float2* lds, const uint4* __restrict__ tab, int t) {
    const int c2 = wave(t), lane = t & 63, g = lane >> 4, n0 = lane & 15;
    const mf::Tab A = mf::load_tab(tab, N2, INV ? 1 : 0, c2, lane);
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
      float2 v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = lds[at(32 * grp + 16 * (e >> 2) + n0, c2 + N2 * (4 * g + (e & 3)))];
      mf::radix16<2>(v, A);
#pragma unroll
      for (int e = 0; e < 8; ++e) lds[at(32 * grp + 16 * (e >> 2) + n0, c2 + N2 * (4 * g + (e & 3)))] = v[e];
    }
  }

  // half h forward: the half's stage-A outputs into LDS, stage B, stage C (FP32, as
  // Half128), frequencies back into the half's slots.  Starts with a barrier unless LEAD
  // is false (as Half128::half_fwd: the first writes here are the slots of this thread's
  // final reads in half_inv); ends after the stage-C reads (no barrier).
  template <bool LEAD = true>
  __device__ static __forceinline__ void half_fwd(float2* v, float2* lds, const uint4* __restrict__ tab, int t,
                                                  int h) {
    const int w = wave(t), lane = t & 63;
    if (LEAD) __syncthreads();
#pragma unroll
    for (int cb = 0; cb < 8; ++cb)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) lds[a_slot(w, lane, cb, jj)] = v[4 * cb + 2 * h + jj];
    __syncthreads();
    stage_b<false>(lds, tab, t);
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
        const float4 x = *reinterpret_cast<const float4*>(lds + Half128::own_pair(t, 4 * q + c / 2));
        a[c] = make_float2(x.x, x.y);
        a[c + 1] = make_float2(x.z, x.w);
      }
      dft8<false>(a);
#pragma unroll
      for (int c = 0; c < 8; ++c) v[fslot(h, q, c)] = a[c];
    }
  }

  // half h inverse: the exact reverse, ending with the half's stage-A values back in their
  // slots.  Starts with a barrier unless LEAD is false (as Half128::half_inv: the first
  // writes go to the thread's own_pair slots); ends after the final LDS reads (no barrier).
  template <bool LEAD = true>
  __device__ static __forceinline__ void half_inv(float2* v, float2* lds, const uint4* __restrict__ tab, int t,
                                                  int h) {
    if (LEAD) __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {   // inverse DFT8 over c2 of lines (k1r, k2r, k1c): own_pair
      float2 a[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) a[c] = v[fslot(h, q, c)];
      dft8<true>(a);
#pragma unroll
      for (int c = 0; c < 8; c += 2)
        *reinterpret_cast<float4*>(lds + Half128::own_pair(t, 4 * q + c / 2)) =
            make_float4(a[c].x, a[c].y, a[c + 1].x, a[c + 1].y);
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
    stage_b<true>(lds, tab, t);
    __syncthreads();
    const int w = wave(t), lane = t & 63;
#pragma unroll
    for (int cb = 0; cb < 8; ++cb)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) v[4 * cb + 2 * h + jj] = lds[a_slot(w, lane, cb, jj)];
  }
};

}  // namespace odp

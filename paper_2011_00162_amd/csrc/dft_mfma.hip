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
// MFMA operand layouts (wave64, checked on the device), lane l, g = l/16, n0 = l%16:
//   A[m][k]  element i (0..7) at m = n0, k = 8g + i
//   B[k][n]  element i (0..7) at k = 8g + i, n = n0
//   D[m][n]  element i (0..3) at m = 4g + i, n = n0
// A contraction may visit k in any order as long as A and B agree on it.  Two
// stacked D tiles hold, in lane l, rows {4g..4g+3} and {16+4g..16+4g+3} of column
// n0: with the k order pi(8g + i) = i < 4 ? 4g + i : 16 + 4g + i - 4 (within each
// 32-wide chunk) they are already a B operand (contracting over those rows), or,
// read as column n0 of the transpose, an A operand.  So a product whose output rows
// are the next product's contraction index hands its result over in registers.
// Every product contracts in the pi order, and every LDS matrix (F, X^T, W^T) keeps
// its columns in that order -- column k = 16t + 4g + i at 32(t/2) + 8g + 4(t%2) + i
// -- so each operand is one 16-byte read of 8 consecutive bf16.
//
// One workgroup of 4 wavefronts works through frames in a loop; wavefront w owns
// the 16-wide band w of the frequency rows (and of the output rows of the inverse).
// Per frame:
//   gather    X^T into LDS as split planes (row c, contiguous r)       LDS exchange 1
//   product 1 Y^T = X^T F          (all c, kr in band w)
//   product 2 X^^T = F Y^T         (B = product 1's D tiles, pi order)
//   prox and Gamma update on X^^T (kr in band w)
//   product 3 W = T conj(F)        (A = the prox output, pi order)
//   W into LDS as split planes (row c', contiguous kr)                  LDS exchange 2
//   product 4 x = conj(F) W        (r' in band w)
//   psi_j = conj(w) o x
// Both exchanges use 8- or 16-byte LDS accesses.  The F table (32 KB of split
// planes, columns in the pi order) is copied into LDS once per workgroup.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "fft_frame.hpp"
#include "odp_internal.hpp"
#include "prox.hpp"
#include "reduce.hpp"

namespace odp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short shortx8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int DP = 64;              // frame size of this kernel
constexpr int LR = DP + 8;          // LDS row stride in bf16 (144 bytes)
constexpr int PL = DP * LR;         // one bf16 plane
constexpr int WGS_PER_CU = 2;       // two workgroups of 72 KB LDS share a CU

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 neg(bf16x8 v) {
  shortx8 s = __builtin_bit_cast(shortx8, v);
  s ^= (short)0x8000;
  return __builtin_bit_cast(bf16x8, s);
}

// split complex operand: real and imaginary parts, each as hi + lo
struct CS {
  bf16x8 rh, rl, ih, il;
};

// 8 consecutive bf16 of row `row` of a plane, from (stored) column col
__device__ __forceinline__ bf16x8 ld8(const __bf16* pl, int row, int col) {
  return *reinterpret_cast<const bf16x8*>(pl + row * LR + col);
}

__device__ __forceinline__ CS ld_cs(const __bf16* planes, int row, int col) {
  return CS{ld8(planes, row, col), ld8(planes + PL, row, col), ld8(planes + 2 * PL, row, col),
            ld8(planes + 3 * PL, row, col)};
}

// hi and lo parts of the pair (x0, x1), packed two to a dword (element 0 in the low
// half): hi = bf16(x), lo = bf16(x - hi), both round-to-nearest-even
// (returned as .x = hi, .y = lo)
__device__ __forceinline__ uint2 split2(float x0, float x1) {
  const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{x0, x1}, bf16x2));
  const float h0 = __builtin_bit_cast(float, h << 16), h1 = __builtin_bit_cast(float, h & 0xffff0000u);
  return make_uint2(h, __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{x0 - h0, x1 - h1}, bf16x2)));
}

// split two D tiles (rows 4g+i of tile a, then of tile b) into one pi-ordered operand part
__device__ __forceinline__ void split8(const floatx4& a, const floatx4& b, bf16x8& h, bf16x8& l) {
  const uint2 p0 = split2(a[0], a[1]), p1 = split2(a[2], a[3]), p2 = split2(b[0], b[1]), p3 = split2(b[2], b[3]);
  h = __builtin_bit_cast(bf16x8, u32x4{p0.x, p1.x, p2.x, p3.x});
  l = __builtin_bit_cast(bf16x8, u32x4{p0.y, p1.y, p2.y, p3.y});
}

// acc += x y over one 32-wide k chunk in split form: x_h y_h + x_h y_l + x_l y_h
__device__ __forceinline__ floatx4 prod3(const bf16x8& xh, const bf16x8& xl, const bf16x8& yh, const bf16x8& yl,
                                         floatx4 acc) {
  acc = mfma(xh, yh, acc);
  acc = mfma(xh, yl, acc);
  return mfma(xl, yh, acc);
}

// Complex products over one 32-wide k chunk, accumulated into (re, im).  The one
// subtracted real product of each form takes a negated operand (nh, nl):
//   MUL:    A B        re += Ar Br + Ai (-Bi),  im += Ar Bi + Ai Br     (nh, nl = -Bi)
//   CONJ_B: A conj(B)  re += Ar Br + Ai Bi,     im += Ai Br + (-Ar) Bi  (nh, nl = -Ar)
//   CONJ_A: conj(A) B  re += Ar Br + Ai Bi,     im += Ar Bi + (-Ai) Br  (nh, nl = -Ai)
enum { MUL, CONJ_B, CONJ_A };
template <int FORM>
__device__ __forceinline__ void cmma(floatx4& re, floatx4& im, const CS& a, const CS& b, const bf16x8& nh,
                                     const bf16x8& nl) {
  re = prod3(a.rh, a.rl, b.rh, b.rl, re);
  if (FORM == MUL) {
    im = prod3(a.rh, a.rl, b.ih, b.il, im);
    re = prod3(a.ih, a.il, nh, nl, re);
    im = prod3(a.ih, a.il, b.rh, b.rl, im);
  } else if (FORM == CONJ_B) {
    im = prod3(a.ih, a.il, b.rh, b.rl, im);
    re = prod3(a.ih, a.il, b.ih, b.il, re);
    im = prod3(nh, nl, b.ih, b.il, im);
  } else {
    im = prod3(a.rh, a.rl, b.ih, b.il, im);
    re = prod3(a.ih, a.il, b.ih, b.il, re);
    im = prod3(nh, nl, b.rh, b.rl, im);
  }
}

}  // namespace

// ST: 0 no statistics, 1 the iteration's measures, 2 also the frame residuals
template <bool BLIND, int ST, bool NT>
__global__ __launch_bounds__(256, WGS_PER_CU) void k_sweep_dft64(SweepArgs a, DftTable dt, ProxC pc) {
  constexpr bool STATS = ST > 0;
  __shared__ __attribute__((aligned(16))) __bf16 ft[4 * PL];   // F: re hi, re lo, im hi, im lo
  __shared__ __attribute__((aligned(16))) __bf16 xb[4 * PL];   // exchange planes, same order
  __shared__ double red[4];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, g = lane >> 4, n0 = lane & 15;

  // F into LDS (rows 16w + n0 in the natural k order are the B operand of product 1
  // and, with the imaginary part negated, the A operand of product 4)
  {
    const uint4* src = reinterpret_cast<const uint4*>(dt.f);
    for (int e = t; e < 4 * DP * DP / 8; e += 256) {
      const int pl = e / (DP * DP / 8), rem = e % (DP * DP / 8), row = rem / (DP / 8), c8 = rem % (DP / 8);
      *reinterpret_cast<uint4*>(ft + pl * PL + row * LR + 8 * c8) = src[e];
    }
  }
  __syncthreads();

  // frame positions of this workgroup (XCD-aware slices of the order, or strided)
  const int G = gridDim.x, b = blockIdx.x;
  int pos, pos_end, step;
  if (a.xcd_slice) {
    const int x = b % NXCD;
    pos = x * a.chunk + b / NXCD;
    pos_end = min((x + 1) * a.chunk, a.J);
    step = G / NXCD;
  } else {
    pos = b;
    pos_end = a.J;
    step = G;
  }

  for (; pos < pos_end; pos += step) {
    const FrameDesc fd = a.fpos[pos];
    if (a.stop && a.stop[fd.probe].stopped) continue;   // its problem met its stopping rule
    const int j = fd.j;
    const size_t woff = (size_t)(a.w_per_sub ? fd.sub : fd.probe) * DP * DP;
    const float2* wp = a.w + woff;
    const size_t fbase = (size_t)j * DP * DP;

    // gather X = w o S_j u into LDS as X^T (row c, columns r in the pi order), split:
    // thread (wave v, column c) takes rows 32h + 4v + (0..3) and 32h + 16 + 4v + (0..3),
    // stored at 32h + 8v .. +7
    __syncthreads();  // the previous frame's reads of xb are done
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      const int c = t & 63, v = t >> 6, r0 = 32 * rep + 4 * v;
      float2 x[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = r0 + (i < 4 ? i : 12 + i);
        x[i] = c_mul(a.u[fd.base + (int64_t)r * fd.pitch + c], wp[r * DP + c]);
      }
      uint2 pr[4], pi[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pr[q] = split2(x[2 * q].x, x[2 * q + 1].x);
        pi[q] = split2(x[2 * q].y, x[2 * q + 1].y);
      }
      const int o = c * LR + 32 * rep + 8 * v;
      *reinterpret_cast<u32x4*>(xb + o) = u32x4{pr[0].x, pr[1].x, pr[2].x, pr[3].x};
      *reinterpret_cast<u32x4*>(xb + PL + o) = u32x4{pr[0].y, pr[1].y, pr[2].y, pr[3].y};
      *reinterpret_cast<u32x4*>(xb + 2 * PL + o) = u32x4{pi[0].x, pi[1].x, pi[2].x, pi[3].x};
      *reinterpret_cast<u32x4*>(xb + 3 * PL + o) = u32x4{pi[0].y, pi[1].y, pi[2].y, pi[3].y};
    }
    __syncthreads();

    // product 1: Y^T[c][kr] = sum_r X^T[c][r] F[r][kr], c = 16 mt + 4g + i, kr = 16w + n0;
    // B = F rows 16w + n0
    floatx4 yr[4], yi[4];
    {
      CS fw[2];
      bf16x8 fn_h[2], fn_l[2];   // -Im of those rows
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) {
        fw[kc] = ld_cs(ft, 16 * w + n0, 32 * kc + 8 * g);
        fn_h[kc] = neg(fw[kc].ih);
        fn_l[kc] = neg(fw[kc].il);
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        yr[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
        yi[mt] = yr[mt];
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
          cmma<MUL>(yr[mt], yi[mt], ld_cs(xb, 16 * mt + n0, 32 * kc + 8 * g), fw[kc], fn_h[kc], fn_l[kc]);
      }
    }

    // this lane's multipliers and amplitudes (kr = 16w + n0, kc = 16 mt + 4g + 0..3),
    // fetched now so their latency overlaps product 2
    const size_t rowb = fbase + (size_t)(16 * w + n0) * DP + 4 * g;
    float4 sfq[4], gq0[4], gq1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      sfq[mt] = ld_s<NT>(reinterpret_cast<const float4*>(a.sqrt_f + rowb + 16 * mt));
      gq0[mt] = ld_s<NT>(reinterpret_cast<const float4*>(a.gamma + rowb + 16 * mt));
      gq1[mt] = ld_s<NT>(reinterpret_cast<const float4*>(a.gamma + rowb + 16 * mt) + 1);
    }

    // product 2: X^^T[kc][kr] = sum_c F[kc][c] Y^T[c][kr]; B = product 1's tiles (pi order)
    floatx4 xr[4], xi[4];
    {
      CS yb[2];
      bf16x8 ybn_h[2], ybn_l[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        split8(yr[2 * h], yr[2 * h + 1], yb[h].rh, yb[h].rl);
        split8(yi[2 * h], yi[2 * h + 1], yb[h].ih, yb[h].il);
        ybn_h[h] = neg(yb[h].ih);
        ybn_l[h] = neg(yb[h].il);
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        xr[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
        xi[mt] = xr[mt];
#pragma unroll
        for (int h = 0; h < 2; ++h)
          cmma<MUL>(xr[mt], xi[mt], ld_cs(ft, 16 * mt + n0, 32 * h + 8 * g), yb[h], ybn_h[h], ybn_l[h]);
      }
    }

    // prox and Gamma update at kr = 16w + n0, kc = 16 mt + 4g + i; xr/xi become t = z - Gamma
    double mis = 0.0, gsum = 0.0, gdel = 0.0, gnrm = 0.0;
      {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        float4* gp = reinterpret_cast<float4*>(a.gamma + rowb + 16 * mt);
        const float4 sf = sfq[mt], g01 = gq0[mt], g23 = gq1[mt];
        const float sfv[4] = {sf.x, sf.y, sf.z, sf.w};
        const float2 gv[4] = {make_float2(g01.x, g01.y), make_float2(g01.z, g01.w), make_float2(g23.x, g23.y),
                              make_float2(g23.z, g23.w)};
        float2 gn[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float2 X = make_float2(xr[mt][i], xi[mt][i]);
          const float2 y = c_add(gv[i], X);
          const float2 z = prox_stagm(y, sfv[i], pc);
          gn[i] = c_sub(y, z);
          const float2 tv = c_sub(z, gn[i]);
          xr[mt][i] = tv.x;
          xi[mt][i] = tv.y;
          if (STATS) {
            elem_measures(X, sfv[i], a.eps, a.gcoef, mis, gsum);
            if (ST > 1) frame_terms(gv[i], gn[i], gdel, gnrm);
          }
        }
        st_s<NT>(gp, make_float4(gn[0].x, gn[0].y, gn[1].x, gn[1].y));
        st_s<NT>(gp + 1, make_float4(gn[2].x, gn[2].y, gn[3].x, gn[3].y));
      }
    }
    if (STATS) frame_stats<256, (ST > 1)>(a.part + NFS * (size_t)j, mis, gsum, gdel, gnrm, red);

    // probe values of this lane's outputs (r' = 16w + 4g + i, c' = 16 nt + n0), fetched
    // before products 3 and 4
    const float2* wo = a.w_out + woff;
    float2 wq[4][4];
    if (!BLIND) {
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) wq[nt][i] = wo[(16 * w + 4 * g + i) * DP + 16 * nt + n0];
    }

    // product 3: W[kr][c'] = sum_kc T[kr][kc] conj F[kc][c']; A = the prox output
    // (pi order), B = F rows 16 nt + n0
    floatx4 wr[4], wi[4];
    {
      CS ta[2];
      bf16x8 tn_h[2], tn_l[2];   // -Re T
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        split8(xr[2 * h], xr[2 * h + 1], ta[h].rh, ta[h].rl);
        split8(xi[2 * h], xi[2 * h + 1], ta[h].ih, ta[h].il);
        tn_h[h] = neg(ta[h].rh);
        tn_l[h] = neg(ta[h].rl);
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        wr[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        wi[nt] = wr[nt];
#pragma unroll
        for (int h = 0; h < 2; ++h)
          cmma<CONJ_B>(wr[nt], wi[nt], ta[h], ld_cs(ft, 16 * nt + n0, 32 * h + 8 * g), tn_h[h], tn_l[h]);
      }
    }

    // W into LDS as W^T (row c', columns kr in the pi order): lane holds kr = 16w + 4g .. +3
    // of column c', stored at 32(w/2) + 8g + 4(w%2)
    __syncthreads();  // every wavefront's product-1 reads of xb are done
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const uint2 r0 = split2(wr[nt][0], wr[nt][1]), r1 = split2(wr[nt][2], wr[nt][3]);
      const uint2 i0 = split2(wi[nt][0], wi[nt][1]), i1 = split2(wi[nt][2], wi[nt][3]);
      const int o = (16 * nt + n0) * LR + 32 * (w >> 1) + 8 * g + 4 * (w & 1);
      *reinterpret_cast<uint2*>(xb + o) = make_uint2(r0.x, r1.x);
      *reinterpret_cast<uint2*>(xb + PL + o) = make_uint2(r0.y, r1.y);
      *reinterpret_cast<uint2*>(xb + 2 * PL + o) = make_uint2(i0.x, i1.x);
      *reinterpret_cast<uint2*>(xb + 3 * PL + o) = make_uint2(i0.y, i1.y);
    }
    __syncthreads();

    // product 4: x[r'][c'] = sum_kr conj F[r'][kr] W[kr][c'], r' = 16w + 4g + i, c' = 16 nt + n0;
    // A = conj of F rows 16w + n0
    CS fw[2];
    bf16x8 fn_h[2], fn_l[2];   // -Im of those rows
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      fw[kc] = ld_cs(ft, 16 * w + n0, 32 * kc + 8 * g);
      fn_h[kc] = neg(fw[kc].ih);
      fn_l[kc] = neg(fw[kc].il);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      floatx4 xre{0.f, 0.f, 0.f, 0.f}, xim = xre;
#pragma unroll
      for (int kc = 0; kc < 2; ++kc)
        cmma<CONJ_A>(xre, xim, fw[kc], ld_cs(xb, 16 * nt + n0, 32 * kc + 8 * g), fn_h[kc], fn_l[kc]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * w + 4 * g + i, c = 16 * nt + n0;
        const float2 x = make_float2(xre[i], xim[i]);
        st_s<NT>(a.psi + fbase + r * DP + c, BLIND ? x : c_mulc(x, wq[nt][i]));
      }
    }
  }
}

hipError_t launch_sweep_dft(int p, const SweepArgs& a, const DftTable& dt, hipStream_t s, hipEvent_t ev0,
                            hipEvent_t ev1) {
  if (p != DP) return hipErrorInvalidValue;
  if (a.J == 0) return hipSuccess;
  const ProxC pc = prox_coeffs(a.eps, a.eta);
  // persistent workgroups: two per CU (256 CUs), in whole XCD rounds
  constexpr int MAXG = WGS_PER_CU * 256;
  const int G = a.xcd_slice ? NXCD * std::min(MAXG / NXCD, (int)a.chunk) : std::min(MAXG, (int)a.J);
  const dim3 grid(G), blk(256);
  const bool bl = a.blind != 0;
  const int st = a.part == nullptr ? 0 : (a.frame_res && !bl ? 2 : 1);
  auto go = [&](auto nt) {
    constexpr bool NT = decltype(nt)::value;
    if (bl && st) hipExtLaunchKernelGGL((k_sweep_dft64<true, 1, NT>), grid, blk, 0, s, ev0, ev1, 0, a, dt, pc);
    else if (bl) hipExtLaunchKernelGGL((k_sweep_dft64<true, 0, NT>), grid, blk, 0, s, ev0, ev1, 0, a, dt, pc);
    else if (st == 2) hipExtLaunchKernelGGL((k_sweep_dft64<false, 2, NT>), grid, blk, 0, s, ev0, ev1, 0, a, dt, pc);
    else if (st) hipExtLaunchKernelGGL((k_sweep_dft64<false, 1, NT>), grid, blk, 0, s, ev0, ev1, 0, a, dt, pc);
    else hipExtLaunchKernelGGL((k_sweep_dft64<false, 0, NT>), grid, blk, 0, s, ev0, ev1, 0, a, dt, pc);
  };
  if (a.stream) go(std::true_type{});
  else go(std::false_type{});
  return hipGetLastError();
}

}  // namespace odp

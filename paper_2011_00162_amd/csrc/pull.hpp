// pull.hpp -- the pull of A_d* over a pixel tile: for each of a thread's two image
// pixels, the sum over the covering frames' records (in list order) of the frames' values
// at that pixel, multiplied by conj(w) at the pixel's window position when BLIND (the
// probe copy or the probe the caller passes as ws), with the FP64 sum of |w|^2 when DEN.
// Shared by the pixel update (A_d*(z - Gamma), Alg. 2 Step 3 and Alg. 3 Step 4) and the
// amplitude loss's image gradient (the same adjoint applied to F^{-1} g).
#pragma once
#include <hip/hip_runtime.h>

#include "fft_frame.hpp"
#include "odp_internal.hpp"

namespace odp {

// one 16-byte load per record, so the frame base is fetched with the window corner
__device__ __forceinline__ PullEntry load_entry(const PullEntry* e) {
  const int4 v = *reinterpret_cast<const int4*>(e);
  PullEntry o;
  o.base = (int64_t)(((uint64_t)(uint32_t)v.y << 32) | (uint32_t)v.x);
  o.r = v.z;
  o.c = v.w;
  return o;
}

// Sums of the covering frames' contributions at the thread's NPX image pixels, over
// the records [k0, k1) in order.  Every list is padded to a multiple of PULL_B
// records with records whose window contains no pixel, and PULL_B such records
// follow the last list, so the records are read PULL_B at a time with no clamping
// (scalar loads when the copy group spans whole wavefronts), and the next group is
// requested before this group's psi loads.  pix8[h] is the byte offset
// 8 (y p + x) of pixel h, so a psi address is a per-record scalar base plus a
// per-lane 32-bit offset.  Only lanes inside a window load; the others add 0, which
// leaves the sum unchanged (it never holds -0).
template <bool BLIND, bool NT, bool DEN = BLIND>
__device__ __forceinline__ void pull_pixels(const PullEntry* __restrict__ pull, int k0, int k1,
                                            const float2* __restrict__ psi, const float2* __restrict__ ws,
                                            const int* yi, const int* xi, const uint32_t* pix8, int p,
                                            float2* num, double* den) {
  constexpr int B = PULL_B;
  PullEntry e[B];
#pragma unroll
  for (int q = 0; q < B; ++q) e[q] = load_entry(pull + k0 + q);
  for (int k = k0; k < k1; k += B) {
    PullEntry en[B];
#pragma unroll
    for (int q = 0; q < B; ++q) en[q] = load_entry(pull + k + B + q);
    bool in[B][NPX];
    float2 ps[B][NPX], ww[B][NPX];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const char* fb = reinterpret_cast<const char*>(psi + e[q].base);
#pragma unroll
      for (int h = 0; h < NPX; ++h) {
        const int dy = yi[h] - e[q].r, dx = xi[h] - e[q].c;
        in[q][h] = (unsigned)dy < (unsigned)p && (unsigned)dx < (unsigned)p;
        ps[q][h] = make_float2(0.f, 0.f);
        ww[q][h] = make_float2(0.f, 0.f);
        if (in[q][h]) {
          ps[q][h] = ld_s<NT>(reinterpret_cast<const float2*>(fb + pix8[h]));
          if (BLIND) ww[q][h] = ws[dy * p + dx];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
      for (int h = 0; h < NPX; ++h) {
        if (BLIND) {
          const float2 c = c_mulc(ps[q][h], ww[q][h]);
          num[h] = in[q][h] ? c_add(num[h], c) : num[h];
          if (DEN) den[h] += in[q][h] ? (double)ww[q][h].x * ww[q][h].x + (double)ww[q][h].y * ww[q][h].y : 0.0;
        } else {
          num[h] = c_add(num[h], ps[q][h]);
        }
      }
#pragma unroll
    for (int q = 0; q < B; ++q) e[q] = en[q];
  }
}

// The same sums for a thread whose two pixels are row neighbours (xi, xi + 1), in a plan
// where every record's column origin has the parity of xi (PixelArgs::pairs): dx = xi - c
// is even, so both pixels are inside a window or both outside it (p is even), and one
// 16-byte load fetches the two (16-byte aligned: the frame offset is 8 (dy p + dx)).  Each
// pixel's sum runs over the same records in the same order as in pull_pixels.
template <bool BLIND, bool NT, bool DEN = BLIND>
__device__ __forceinline__ void pull_pairs(const PullEntry* __restrict__ pull, int k0, int k1,
                                           const float2* __restrict__ psi, const float2* __restrict__ ws, int yi,
                                           int xi, uint32_t pix8, int p, float2* num, double* den) {
  constexpr int B = PULL_B;
  PullEntry e[B];
#pragma unroll
  for (int q = 0; q < B; ++q) e[q] = load_entry(pull + k0 + q);
  for (int k = k0; k < k1; k += B) {
    PullEntry en[B];
#pragma unroll
    for (int q = 0; q < B; ++q) en[q] = load_entry(pull + k + B + q);
    bool in[B];
    float4 ps[B], ww[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const char* fb = reinterpret_cast<const char*>(psi + e[q].base);
      const int dy = yi - e[q].r, dx = xi - e[q].c;
      in[q] = (unsigned)dy < (unsigned)p && (unsigned)dx < (unsigned)p;
      ps[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      ww[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (in[q]) {
        ps[q] = ld_s<NT>(reinterpret_cast<const float4*>(fb + pix8));
        if (BLIND) ww[q] = *reinterpret_cast<const float4*>(ws + dy * p + dx);
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const float2 p0 = make_float2(ps[q].x, ps[q].y), p1 = make_float2(ps[q].z, ps[q].w);
      if (BLIND) {
        const float2 w0 = make_float2(ww[q].x, ww[q].y), w1 = make_float2(ww[q].z, ww[q].w);
        const float2 c0 = c_mulc(p0, w0), c1 = c_mulc(p1, w1);
        num[0] = in[q] ? c_add(num[0], c0) : num[0];
        num[1] = in[q] ? c_add(num[1], c1) : num[1];
        if (DEN) den[0] += in[q] ? (double)w0.x * w0.x + (double)w0.y * w0.y : 0.0;
        if (DEN) den[1] += in[q] ? (double)w1.x * w1.x + (double)w1.y * w1.y : 0.0;
      } else {
        num[0] = c_add(num[0], p0);
        num[1] = c_add(num[1], p1);
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q) e[q] = en[q];
  }
}

}  // namespace odp

// pixel.hip -- the pixel update (one kernel per iteration) and the illumination
// reciprocals it uses, over the pixel tiles of the plan.
#include <hip/hip_runtime.h>

#include "fft_frame.hpp"
#include "odp_internal.hpp"
#include "pull.hpp"

namespace odp {

// ---------------------------------------------------------------------------
// K3: pixel update (Alg. 2 Steps 1 (v), 3 (u) and 4 (Lam); Alg. 3 Step 4 (U)
// and the Lam half of Step 5) on one tile of a cell.
//   num_d   = sum_{j in d, window covers x} psi_j(x - o_j)    (A_d*(z - Gamma), fixed order)
//   v_{a,b} = (u_a + u_b + Lam_{a,b} + Lam_{b,a}) / 2        from the iterate n
//   u_d     = (eta num_d + r sum_{e != d} (v_{d,e} - Lam_{d,e}) + gamma u_d) / (eta den_d + r k + gamma)
//   Lam_{d,e} += u_d^{new} - v_{d,e}
// Blind: num_d and the FP64 illumination den_d = sum |w_d|^2 both use the new
// probe copy w_d, in the same pull.  Non-blind: the reciprocal comes from bind.
//
// Every thread owns two (pixel, subdomain copy) pairs of one copy: a cell with m
// copies per pixel has tiles of 512 / m' pixels (m' = m rounded up to a power of
// two); thread t takes copy s = t / (256 / m') and two tile pixels of that copy, i and
// i + 256 / m' (i = t % (256 / m')), or in k_pixel_uni, when the plan's records allow it
// (PixelArgs::pairs), the row neighbours 2i and 2i + 1; so every copy does one pull and
// all copies of a pixel sit in one workgroup.  u_d and Lam_{d,e} of a pixel are written only by the
// thread of copy d, after a barrier that follows every thread's reads of the
// iterate n, so each thread sees u^n and Lam^n of the other copies.  Pairs (a, b),
// a < b, of the cell's subdomain list are stored at index b(b-1)/2 + a.
// ---------------------------------------------------------------------------
// u^{n+1} of one pixel copy from its pull (num, den), u^n (uo), the reciprocal and,
// per partner copy o < m - 1, u^n (ut) and Lam^n of both orders (lo: own, lt: the
// partner's); dv[o] = v - Lam_{s,t} is kept for the multiplier update.
template <bool BLIND, int NO>
__device__ __forceinline__ float2 pixel_value(const PixelArgs& a, int m, float r, float2 num, double den, float2 uo,
                                              float rc, const float2* ut, const float2* lo, const float2* lt,
                                              float2* dv) {
  float2 acc = c_add(c_scale(num, a.eta), c_scale(uo, a.gamma));
  if (BLIND) {
    const double qd = (double)a.eta * den + (double)r * (double)(m - 1) + (double)a.gamma;
    rc = qd == 0.0 ? 0.0f : (float)(1.0 / qd);
  }
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    dv[o] = make_float2(0.f, 0.f);
    if (o < m - 1) {
      const float2 v = c_scale(c_add(c_add(uo, ut[o]), c_add(lo[o], lt[o])), 0.5f);
      dv[o] = c_sub(v, lo[o]);
      acc = c_add(acc, c_scale(dv[o], r));
    }
  }
  return rc == 0.0f ? uo : c_scale(acc, rc);
}

// per copy group, NPS sums over the thread's pixels (the per-copy |du|^2 and |u|^2, then
// the consensus residual terms over the copy's ordered pairs: |Lam^{n+1} - Lam^n|^2,
// (m-1)|du|^2, (m-1)|u^{n+1}|^2, |Lam^{n+1}|^2, then the frame constraint's terms
// den |u^n|^2 and den |du|^2), reduced in a fixed order into part[tile][s][NPS]
__device__ __forceinline__ void pixel_stats(const PixelArgs& a, int tile, int m, int tpg, double (&v)[NPS],
                                            double (*red)[MAXS]) {
  const int g = min(tpg, 64);                    // lanes of one group inside a wavefront
  for (int o = g >> 1; o > 0; o >>= 1)
#pragma unroll
    for (int k = 0; k < NPS; ++k) v[k] += __shfl_xor(v[k], o, 64);
  const int chunk = threadIdx.x / g;             // 256 / g <= MAXS chunks, tpg / g per group
  if ((threadIdx.x & (g - 1)) == 0)
#pragma unroll
    for (int k = 0; k < NPS; ++k) red[k][chunk] = v[k];
  __syncthreads();
  if (threadIdx.x < MAXS && (int)threadIdx.x < m) {
    const int per = tpg / g;
#pragma unroll
    for (int k = 0; k < NPS; ++k) {
      double acc = 0.0;
      for (int c = threadIdx.x * per; c < (int)(threadIdx.x + 1) * per; ++c) acc += red[k][c];
      a.part[((size_t)tile * MAXS + threadIdx.x) * NPS + k] = acc;
    }
  }
}

// residual terms of one pixel of copy s (pixel_stats' order; dd = its den)
template <int NO>
__device__ __forceinline__ void residual_terms(int m, float2 un, float2 uo, const float2* lo, const float2 (&dv)[NO],
                                               double dd, double (&v)[NPS]) {
#pragma unroll
  for (int o = 0; o < NO; ++o)
    if (o < m - 1) {
      const float2 ln = c_sub(un, dv[o]);       // Lam^{n+1}, as stored
      const double ix = (double)ln.x - lo[o].x, iy = (double)ln.y - lo[o].y;
      v[2] += ix * ix + iy * iy;
      v[5] += (double)ln.x * ln.x + (double)ln.y * ln.y;
    }
  const double ex = (double)un.x - uo.x, ey = (double)un.y - uo.y;
  v[0] += ex * ex + ey * ey;
  v[1] += (double)un.x * un.x + (double)un.y * un.y;
  v[3] += (double)(m - 1) * (ex * ex + ey * ey);
  v[4] += (double)(m - 1) * ((double)un.x * un.x + (double)un.y * un.y);
  v[6] += dd * ((double)uo.x * uo.x + (double)uo.y * uo.y);
  v[7] += dd * (ex * ex + ey * ey);
}

// Tiles of cells with at most four copies: each wavefront lies inside one copy group
// and takes its descriptor from its own WaveRec (scalar loads, one round trip).
// The non-blind kernel is held to 80 VGPRs: six workgroups per CU keep all tiles of
// a 512 x 512 problem with 4 x 4 subdomains resident at once.
template <bool STATS, bool BLIND, bool NT>
__global__ __launch_bounds__(256, BLIND ? 1 : 6) void k_pixel_uni(PixelArgs a) {
  __shared__ double red[NPS][MAXS];
  constexpr int NO = 3;                          // partner copies at most
  const int tile = blockIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const WaveRec w = a.waves[(size_t)tile * 4 + wv];
  if (a.stop && a.stop[w.prob].stopped) return;  // every wavefront of the tile: one problem
  const int p = a.p, s = w.s, m = w.m;
  const int tpg = 256 >> w.lg;                   // threads per copy group
  const int q = threadIdx.x & (tpg - 1);
  int tr[NPX], tc[NPX], yi[NPX], xi[NPX];
  bool act[NPX];
#pragma unroll
  for (int h = 0; h < NPX; ++h) {                // row neighbours 2q, 2q + 1 with pairs, else q, q + tpg
    const int i = a.pairs ? 2 * q + h : q + h * tpg;
    tr[h] = i >> w.lcw;
    tc[h] = i & ((1 << w.lcw) - 1);
    act[h] = s < m && tr[h] < w.nr && tc[h] < w.nc;
    yi[h] = w.yi0 + tr[h];
    xi[h] = w.xi0 + tc[h];
  }

  // reads of the iterate n, issued before the pull so their latency overlaps it
  float2 uo[NPX], lo_[NO][NPX], lt_[NO][NPX], ut_[NO][NPX];
  float rc[NPX];
  int64_t idx[NPX];
#pragma unroll
  for (int h = 0; h < NPX; ++h) {
    idx[h] = w.u0 + (int64_t)tr[h] * w.upitch + tc[h];
    uo[h] = make_float2(0.f, 0.f);
    rc[h] = 0.0f;
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (act[h] && o < m - 1) {
        lo_[o][h] = a.lam[w.lo0[o] + (int64_t)tr[h] * w.lpitch[o] + tc[h]];
        lt_[o][h] = a.lam[w.lt0[o] + (int64_t)tr[h] * w.lpitch[o] + tc[h]];
        ut_[o][h] = a.u[w.pu0[o] + (int64_t)tr[h] * w.pupitch[o] + tc[h]];
      }
    if (act[h]) {
      uo[h] = a.u[idx[h]];
      if (!BLIND) rc[h] = a.rcp[idx[h]];
    }
  }

  // A_d*(z - Gamma) at these pixels: the covering frames of subdomain sub[s]
  float2 num[NPX];
  double den[NPX];
#pragma unroll
  for (int h = 0; h < NPX; ++h) {
    num[h] = make_float2(0.f, 0.f);
    den[h] = 0.0;
  }
  const float2* ws = BLIND ? a.w_sub + (size_t)w.sub * p * p : nullptr;
  static_assert(NPX == 2, "pixel pairs");
  if (a.pairs) {
    pull_pairs<BLIND, NT>(a.pull, w.k0, w.k1, a.psi, ws, yi[0], xi[0], 8u * (uint32_t)(yi[0] * p + xi[0]), p, num,
                          den);
  } else {
    uint32_t pix8[NPX];
#pragma unroll
    for (int h = 0; h < NPX; ++h) pix8[h] = 8u * (uint32_t)(yi[h] * p + xi[h]);
    pull_pixels<BLIND, NT>(a.pull, w.k0, w.k1, a.psi, ws, yi, xi, pix8, p, num, den);
  }

  float2 un[NPX], dv[NPX][NO];
  double sv[NPS] = {};
#pragma unroll
  for (int h = 0; h < NPX; ++h) {
    float2 ut[NO], lo[NO], lt[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      ut[o] = ut_[o][h];
      lo[o] = lo_[o][h];
      lt[o] = lt_[o][h];
    }
    un[h] = pixel_value<BLIND, NO>(a, m, w.r, num[h], den[h], uo[h], rc[h], ut, lo, lt, dv[h]);
    if (STATS && act[h]) residual_terms<NO>(m, un[h], uo[h], lo, dv[h], BLIND ? den[h] : a.dend[idx[h]], sv);
  }
  __syncthreads();  // every copy's reads of u^n and Lam^n precede the writes below
#pragma unroll
  for (int h = 0; h < NPX; ++h)
    if (act[h]) {
      a.u[idx[h]] = un[h];
#pragma unroll
      for (int o = 0; o < NO; ++o)
        if (o < m - 1)   // Lam + u^{n+1} - v
          a.lam[w.lo0[o] + (int64_t)tr[h] * w.lpitch[o] + tc[h]] = c_sub(un[h], dv[h][o]);
    }
  if (STATS) pixel_stats(a, tile, m, tpg, sv, red);
}

// log2 of the copy groups of a cell with m copies (m rounded up to a power of two)
__device__ __forceinline__ int copy_groups_log2(int m) {
  return m <= 1 ? 0 : m <= 2 ? 1 : m <= 4 ? 2 : m <= 8 ? 3 : 4;
}

// Tiles of cells with five to MAXS copies: the copy index varies inside a wavefront, so
// the descriptors come from the cell, per lane.  A thread keeps v - Lam for each of its up
// to MC - 1 partners until the barrier; the partners' iterate n is read partner by
// partner.  MC = 8 runs the tiles [n_uni, n_mid) of cells with five to eight copies,
// MC = MAXS the rest (the partner arrays, and so the registers, are sized by MC).
template <bool STATS, bool BLIND, int MC, bool NT>
__global__ __launch_bounds__(256) void k_pixel(PixelArgs a) {
  __shared__ double red[NPS][MAXS];
  constexpr int NO = MC - 1;
  const int tile = (MC <= 8 ? a.n_uni : a.n_mid) + blockIdx.x;
  const TileDesc td = a.tiles[tile];
  const CellDesc* cd = a.cells + td.cell;
  if (a.stop && a.stop[cd->probe].stopped) return;  // its problem met its stopping rule
  const int p = a.p, m = cd->m;
  const float r = cd->r;
  const int lg = copy_groups_log2(m);
  const int tpg = 256 >> lg;                     // threads per copy group
  const int cw = min(a.tile_cols, NPX * tpg);    // tile width
  const int q = threadIdx.x & (tpg - 1);
  const int s = threadIdx.x >> (8 - lg);
  const int sc = min(s, m - 1);                  // idle groups (s >= m) read slot m - 1's descriptors
  int y[NPX], x[NPX], yi[NPX], xi[NPX];
  bool act[NPX];
#pragma unroll
  for (int h = 0; h < NPX; ++h) {
    const int i = q + h * tpg, tr = i / cw, tc = i % cw;
    act[h] = s < m && tr < td.nr && tc < td.nc;
    y[h] = td.r0 + tr;
    x[h] = td.c0 + tc;
    yi[h] = cd->r0 + y[h];
    xi[h] = cd->c0 + x[h];
  }
  float2 uo[NPX], un[NPX], dv[NPX][NO];
  double sv[NPS] = {};
  float rc[NPX];
  int64_t idx[NPX];
  float2 num[NPX];
  double den[NPX];
#pragma unroll
  for (int h = 0; h < NPX; ++h) {
    idx[h] = cd->ubase[sc] + (int64_t)y[h] * cd->upitch[sc] + x[h];
    uo[h] = act[h] ? a.u[idx[h]] : make_float2(0.f, 0.f);
    rc[h] = act[h] && !BLIND ? a.rcp[idx[h]] : 0.0f;
    num[h] = make_float2(0.f, 0.f);
    den[h] = 0.0;
  }
  const float2* ws = BLIND ? a.w_sub + (size_t)cd->sub[sc] * p * p : nullptr;
  uint32_t pix8[NPX];
#pragma unroll
  for (int h = 0; h < NPX; ++h) pix8[h] = 8u * (uint32_t)(yi[h] * p + xi[h]);
  pull_pixels<BLIND, NT>(a.pull, a.tf_first[tile * MAXS + s], a.tf_first[tile * MAXS + s + 1], a.psi, ws, yi, xi, pix8,
                     p, num, den);
  if constexpr (STATS) {
#pragma unroll
    for (int h = 0; h < NPX; ++h) {
      float2 ut[NO], lo[NO], lt[NO];
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        ut[o] = lo[o] = lt[o] = make_float2(0.f, 0.f);
        const int t = o + (o >= s);
        if (act[h] && o < m - 1) {
          const int pl = min(s, t), ph = max(s, t), pq = ph * (ph - 1) / 2 + pl;
          const int64_t li = cd->lbase[pq] + (int64_t)y[h] * cd->lpitch[pq] + x[h], lj = li + cd->lstride[pq];
          lo[o] = a.lam[s < t ? li : lj];
          lt[o] = a.lam[s < t ? lj : li];
          ut[o] = a.u[cd->ubase[t] + (int64_t)y[h] * cd->upitch[t] + x[h]];
        }
      }
      un[h] = pixel_value<BLIND, NO>(a, m, r, num[h], den[h], uo[h], rc[h], ut, lo, lt, dv[h]);
      if (act[h]) residual_terms<NO>(m, un[h], uo[h], lo, dv[h], BLIND ? den[h] : a.dend[idx[h]], sv);
    }
  } else {
    // pixel_value's arithmetic partner by partner: each partner's descriptors are read
    // once for both pixels and its iterate-n values are consumed as they arrive, so only
    // the v - Lam terms stay live until the writes (150 -> 100 VGPRs with 16 copies)
    float2 acc[NPX];
#pragma unroll
    for (int h = 0; h < NPX; ++h) {
      acc[h] = c_add(c_scale(num[h], a.eta), c_scale(uo[h], a.gamma));
      if (BLIND) {
        const double qd = (double)a.eta * den[h] + (double)r * (double)(m - 1) + (double)a.gamma;
        rc[h] = qd == 0.0 ? 0.0f : (float)(1.0 / qd);
      }
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) {
#pragma unroll
      for (int h = 0; h < NPX; ++h) dv[h][o] = make_float2(0.f, 0.f);
      if (o < m - 1) {
        const int t = o + (o >= s);
        const int pl = min(s, t), ph = max(s, t), pq = ph * (ph - 1) / 2 + pl;
        const int64_t lb = cd->lbase[pq], ls = cd->lstride[pq], ub = cd->ubase[t];
        const int lp = cd->lpitch[pq], up = cd->upitch[t];
#pragma unroll
        for (int h = 0; h < NPX; ++h) {
          const int64_t li = lb + (int64_t)y[h] * lp + x[h], lj = li + ls;
          float2 lo = make_float2(0.f, 0.f), lt = lo, ut = lo;
          if (act[h]) {
            lo = a.lam[s < t ? li : lj];
            lt = a.lam[s < t ? lj : li];
            ut = a.u[ub + (int64_t)y[h] * up + x[h]];
          }
          const float2 v = c_scale(c_add(c_add(uo[h], ut), c_add(lo, lt)), 0.5f);
          dv[h][o] = c_sub(v, lo);
          acc[h] = c_add(acc[h], c_scale(dv[h][o], r));
        }
      }
    }
#pragma unroll
    for (int h = 0; h < NPX; ++h) un[h] = rc[h] == 0.0f ? uo[h] : c_scale(acc[h], rc[h]);
  }
  __syncthreads();  // every copy's reads of u^n and Lam^n precede the writes below
#pragma unroll
  for (int h = 0; h < NPX; ++h)
    if (act[h]) {
      a.u[idx[h]] = un[h];
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        const int t = o + (o >= s);
        if (o < m - 1) {
          const int pl = min(s, t), ph = max(s, t), pq = ph * (ph - 1) / 2 + pl;
          const int64_t li = cd->lbase[pq] + (int64_t)y[h] * cd->lpitch[pq] + x[h];
          a.lam[s < t ? li : li + cd->lstride[pq]] = c_sub(un[h], dv[h][o]);   // Lam + u^{n+1} - v
        }
      }
    }
  if (STATS) pixel_stats(a, tile, m, tpg, sv, red);
}

template <bool ST, bool BL, bool NT>
static void go_pixel(const PixelArgs& a, hipStream_t s) {
  const dim3 b(256);
  if (a.n_uni > 0) hipLaunchKernelGGL((k_pixel_uni<ST, BL, NT>), dim3(a.n_uni), b, 0, s, a);
  if (a.n_mid > a.n_uni) hipLaunchKernelGGL((k_pixel<ST, BL, 8, NT>), dim3(a.n_mid - a.n_uni), b, 0, s, a);
  if (a.n_tiles > a.n_mid) hipLaunchKernelGGL((k_pixel<ST, BL, MAXS, NT>), dim3(a.n_tiles - a.n_mid), b, 0, s, a);
}

hipError_t launch_pixel(const PixelArgs& a, bool stats, bool blind, hipStream_t s) {
#define ODP_PIXEL(ST, BL) \
  { if (a.stream) go_pixel<ST, BL, true>(a, s); else go_pixel<ST, BL, false>(a, s); }
  if (blind) {
    if (stats) ODP_PIXEL(true, true)
    else ODP_PIXEL(false, true)
  } else {
    if (stats) ODP_PIXEL(true, false)
    else ODP_PIXEL(false, false)
  }
#undef ODP_PIXEL
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K0: illumination den_d = sum_{j in d} S_j^T |w|^2 (eq. AtA) in FP64, over the
// tile's frame list in a fixed order, and rcp = 1/(eta den + r k + gamma).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_illum(IllumArgs a) {
  const int tile = blockIdx.x;
  const TileDesc td = a.tiles[tile];
  const CellDesc* cd = a.cells + td.cell;
  const int m = cd->m, p = a.p;
  const float2* w = a.w + (size_t)cd->probe * p * p;
  for (int h = 0; h < NPX; ++h) {
    const int i = threadIdx.x + 256 * h, tr = i / a.tile_cols, tc = i % a.tile_cols;
    if (!(tr < td.nr && tc < td.nc)) continue;
    const int y = td.r0 + tr, x = td.c0 + tc;
    const int yi = cd->r0 + y, xi = cd->c0 + x;
    for (int s = 0; s < m; ++s) {
      const int64_t idx = cd->ubase[s] + (int64_t)y * cd->upitch[s] + x;
      double den;
      if (a.recompute_den) {
        den = 0.0;
        for (int k = a.tf_first[tile * MAXS + s]; k < a.tf_first[tile * MAXS + s + 1]; ++k) {
          const PullEntry pe = a.pull[k];
          const int dy = yi - pe.r, dx = xi - pe.c;
          if ((unsigned)dy < (unsigned)p && (unsigned)dx < (unsigned)p) {
            const float2 ww = w[dy * p + dx];
            den += (double)ww.x * ww.x + (double)ww.y * ww.y;
          }
        }
        a.den[idx] = den;
      } else {
        den = a.den[idx];
      }
      const double q = a.eta * den + (double)cd->r * (double)(m - 1) + a.gamma;
      a.rcp[idx] = q == 0.0 ? 0.0f : (float)(1.0 / q);
    }
  }
}

hipError_t launch_illum(const IllumArgs& a, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_illum, dim3(a.n_tiles), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace odp

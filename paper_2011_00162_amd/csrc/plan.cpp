// plan.cpp -- host side of the C ABI: validation, decomposition geometry,
// workspace/state layout and the entry points that launch the kernels.
//
// Geometry follows Sec. 2.1 and Sec. 3.1 of the paper: frames are partitioned
// first; subdomain d is the bounding rectangle of its frames' windows; the pair
// set holds every intersecting pair; k_d(x) (sum over pairs of pi^T pi) is the
// number of other subdomains containing x.  On one GPU the subdomains are index
// ranges of one launch, not separate processes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "odp.h"
#include "odp_internal.hpp"

using namespace odp;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define ODP_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return fail(ODP_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// float -> bf16 bit pattern, round to nearest even (finite inputs)
uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

constexpr int LOSS_CHUNKS = 32;   // frame chunks of the probe-gradient reduction

struct Pair {
  int32_t a, b, r0, c0, r1, c1;
  int64_t off;  // lam index of Lam_{a,b}; Lam_{b,a} follows after h*w
};

}  // namespace

struct odp_plan {
  int32_t H = 0, W = 0, p = 0, J = 0, D = 0;
  double eps = 0, eta = 0, r = 0, mu = 0, gamma = 0;
  int32_t transform = ODP_FFT_F32, blind = 0;
  std::vector<int32_t> offsets, frame_sub;
  std::vector<float> fmask;  // empty = no projection
  // geometry
  std::vector<int32_t> rects;  // [D][4]
  std::vector<int64_t> usub_off;
  int64_t p_sub = 0;
  std::vector<Pair> pairs;
  int64_t n_lam = 0;
  std::vector<CellDesc> cells;
  int32_t max_cover = 0;
  std::vector<FrameDesc> frames;
  std::vector<int32_t> order, sub_first;
  // pixel-update tilings (the autotuner picks one); the active one is tsets[ts]
  struct TileSet {
    int rows = 0, cols = 0;
    std::vector<TileDesc> tiles;             // cells with m <= 4 first: tiles [0, n_uni)
    int32_t n_uni = 0;                       // then 5 <= m <= 8: tiles [n_uni, n_mid)
    int32_t n_mid = 0;
    std::vector<int32_t> re_list, re_first;  // (tile, slot) entries per subdomain, for RE
    std::vector<int32_t> tf_first;           // per (tile, slot): range of pull records
    std::vector<PullEntry> pull;             // frames whose window meets the tile, ascending id
    bool pairs = false;                      // tiles [0, n_uni): every record's column origin has
                                             // the parity of the tile's left column
  };
  TileSet tsets[3];
  int64_t covered = 0;  // image pixels in some subdomain (the tiles partition them)
  int ts = 0;
  int32_t xcd_slice = 2;
  // stopping rule (Sec. 4) evaluated on the device after every iteration
  int32_t stop_measure = ODP_STOP_NONE, stop_max_iter = 0, stop_every = 1;
  double stop_tol = 0.0;
  bool stopping() const { return stop_measure != ODP_STOP_NONE || stop_max_iter > 0; }
  // iterations issued per state since the rule was set or the state initialised; the rule
  // is evaluated on every stop_every-th
  mutable std::unordered_map<const void*, int64_t> stop_count;
  bool stop_check(const void* state) const {
    if (!stopping()) return false;
    const auto it = stop_count.find(state);
    return ((it == stop_count.end() ? 0 : it->second) + 1) % stop_every == 0;
  }
  // overlap penalties by residual balancing (0 = off), host-driven every bal_period iterations
  int32_t bal_period = 0, bal_until = 0, bal_which = ODP_BALANCE_R;
  int64_t bal_count = 0;
  double bal_mu = 10.0, bal_tau = 2.0;
  bool balancing() const { return bal_period > 0; }
  std::vector<std::pair<hipEvent_t, hipEvent_t>> sweep_ev;   // kernel timing of the next sweeps
  size_t sweep_ev_next = 0, sweep_ev_stride = 1;
  // problems of a batch (one entry for a single problem)
  struct Entry {
    int32_t row0, col0, H, W, J0, J, D0, D;
    double r, illum_max;
  };
  std::vector<Entry> batch;
  std::vector<int32_t> sub_problem;        // [D] problem of each subdomain
  std::vector<float2> tw;
  std::vector<uint16_t> dft;               // split-BF16 DFT matrix planes (transform = DFT)
  std::vector<uint16_t> mft;               // split-BF16 radix-16 stage matrices (hybrid transform)
  int32_t chunk = 0;
  int32_t stream = 0;   // 1: non-temporal accesses to the frame arrays (set from their size)
  int32_t pairs_on = 1; // 0: the pixel update keeps one load per pixel even where pairs apply
  // workspace layout (byte offsets)
  struct {
    size_t tw, w, frames, fpos, order, sub_first, offsets, rects, usub_off, cells, tiles, waves, re_list, re_first,
        tf_first, pull, den, rcp, fpart, tpart, stat_scratch, misc, pmax, psi, fmask, wpart, dft, mft, prob, resid,
        bytes;
  } ws{};
  struct {
    size_t u_sub, gamma, lam, w, w_sub, delta, stop, bytes;
  } st{};
  // bumped by every call that rewrites launch arguments or device tables a captured graph
  // holds (penalties, reciprocals, tiling and placement, rebinding); graphs record it
  uint64_t gen = 0;
  // bound state
  char* wsp = nullptr;
  const float* sqrt_f = nullptr;
  double illum_max = 0.0;

  template <class T>
  T* W_(size_t off) const { return reinterpret_cast<T*>(wsp + off); }
  const TileSet& tset() const { return tsets[ts]; }
  int n_probes() const { return (int)batch.size(); }
};

namespace {

// The default cache policy of a plan's frame arrays: streaming when they (Gamma read and
// written, sqrt(f), the handoff written and read back: 28 B per frame pixel) exceed the
// 256 MiB Infinity Cache.
int32_t stream_by_size(const odp_plan* P) {
  return (double)P->J * P->p * P->p * 28.0 > 256.0 * (1 << 20) ? 1 : 0;
}

// Cut every cell into tiles and list, per (tile, subdomain slot), the slot's frames
// whose window meets the tile (ascending id).  A cell with m copies per pixel gets
// tiles of 512 / m' pixels (m' = m rounded up to a power of two, at most MAXS = 16: 32
// pixels), so one workgroup of 256 threads, two pixels per thread, holds every copy of
// its pixels: width min(cols, 512 / m'), height the rest (rows x cols = 512 is the shape
// for m = 1).
void build_tiles(const odp_plan* P, int rows, int cols, odp_plan::TileSet& T) {
  const int p = P->p, D = P->D;
  T.rows = rows;
  T.cols = cols;
  T.tiles.clear();
  // cells with up to four copies first (their pixel kernel runs with wavefront-uniform
  // copy indices), then those with five to eight, then the rest (the general kernel is
  // instantiated for each group's largest number of partner copies)
  for (int pass = 0; pass < 3; ++pass) {
    for (size_t c = 0; c < P->cells.size(); ++c) {
      const CellDesc& cd = P->cells[c];
      if ((cd.m <= 4 ? 0 : cd.m <= 8 ? 1 : 2) != pass) continue;
      int groups = 1;
      while (groups < cd.m) groups *= 2;
      const int ppt = rows * cols / groups, tw = std::min(cols, ppt), th = ppt / tw;
      const int r1 = cd.r0 + cd.nr, c1 = cd.c0 + cd.nc;
      for (int ty = 0; ty < r1 - cd.r0; ty += th)
        for (int tx = 0; tx < c1 - cd.c0; tx += tw) {
          TileDesc td;
          std::memset(&td, 0, sizeof(td));
          td.cell = (int32_t)c;
          td.r0 = ty;
          td.c0 = tx;
          td.nr = std::min(th, r1 - cd.r0 - ty);
          td.nc = std::min(tw, c1 - cd.c0 - tx);
          T.tiles.push_back(td);
        }
    }
    if (pass == 0) T.n_uni = (int32_t)T.tiles.size();
    if (pass == 1) T.n_mid = (int32_t)T.tiles.size();
  }
  std::vector<std::vector<int32_t>> per(D);
  for (size_t t = 0; t < T.tiles.size(); ++t) {
    const CellDesc& cd = P->cells[T.tiles[t].cell];
    for (int s = 0; s < cd.m; ++s) per[cd.sub[s]].push_back((int32_t)(t * MAXS + s));
  }
  T.re_first.assign(D + 1, 0);
  T.re_list.clear();
  for (int d = 0; d < D; ++d) {
    T.re_first[d] = (int32_t)T.re_list.size();
    T.re_list.insert(T.re_list.end(), per[d].begin(), per[d].end());
  }
  T.re_first[D] = (int32_t)T.re_list.size();
  std::vector<std::vector<int32_t>> by_sub(D);
  for (int j = 0; j < P->J; ++j) by_sub[P->frame_sub[j]].push_back(j);
  T.tf_first.assign(T.tiles.size() * MAXS + 1, 0);
  T.pull.clear();
  for (size_t t = 0; t < T.tiles.size(); ++t) {
    const TileDesc& td = T.tiles[t];
    const CellDesc& cd = P->cells[td.cell];
    const int y0 = cd.r0 + td.r0, y1 = y0 + td.nr, x0 = cd.c0 + td.c0, x1 = x0 + td.nc;
    for (int s = 0; s < MAXS; ++s) {
      T.tf_first[t * MAXS + s] = (int32_t)T.pull.size();
      if (s >= cd.m) continue;
      for (int j : by_sub[cd.sub[s]]) {
        const int r = P->offsets[2 * j], c = P->offsets[2 * j + 1];
        if (r < y1 && r + p > y0 && c < x1 && c + p > x0)
          T.pull.push_back(PullEntry{(int64_t)j * p * p - (int64_t)r * p - c, r, c});
      }
      while ((T.pull.size() - T.tf_first[t * MAXS + s]) % PULL_B) T.pull.push_back(PullEntry{0, PULL_NONE, PULL_NONE});
    }
  }
  T.tf_first[T.tiles.size() * MAXS] = (int32_t)T.pull.size();
  for (int q = 0; q < PULL_B; ++q) T.pull.push_back(PullEntry{0, PULL_NONE, PULL_NONE});  // read ahead of the last list
  // with every window column origin of a tile's parity, a window edge never falls between
  // the two row neighbours a thread of k_pixel_uni or of the loss's image gradient holds
  // (tile widths are even); every tile is checked, the loss pulls over all of them
  T.pairs = true;
  for (size_t t = 0; t < T.tiles.size() && T.pairs; ++t) {
    const TileDesc& td = T.tiles[t];
    const CellDesc& cd = P->cells[td.cell];
    const int x0 = cd.c0 + td.c0;
    for (int32_t k = T.tf_first[(size_t)t * MAXS]; k < T.tf_first[(size_t)t * MAXS + cd.m]; ++k)
      if (T.pull[k].r != PULL_NONE && ((T.pull[k].c - x0) & 1)) {
        T.pairs = false;
        break;
      }
  }
}

int build_geometry(odp_plan* P) {
  const int J = P->J, D = P->D, p = P->p, H = P->H, W = P->W;
  // rectangles
  P->rects.assign((size_t)D * 4, 0);
  std::vector<int> count(D, 0);
  for (int d = 0; d < D; ++d) {
    P->rects[4 * d] = H;
    P->rects[4 * d + 1] = W;
    P->rects[4 * d + 2] = 0;
    P->rects[4 * d + 3] = 0;
  }
  for (int j = 0; j < J; ++j) {
    const int d = P->frame_sub[j], r = P->offsets[2 * j], c = P->offsets[2 * j + 1];
    int32_t* R = &P->rects[4 * d];
    R[0] = std::min(R[0], r);
    R[1] = std::min(R[1], c);
    R[2] = std::max(R[2], r + p);
    R[3] = std::max(R[3], c + p);
    ++count[d];
  }
  for (int d = 0; d < D; ++d)
    if (count[d] == 0) return fail(ODP_EGEOM, "subdomain " + std::to_string(d) + " has no frames");
  P->usub_off.resize(D);
  int64_t off = 0;
  for (int d = 0; d < D; ++d) {
    P->usub_off[d] = off;
    off += (int64_t)(P->rects[4 * d + 2] - P->rects[4 * d]) * (P->rects[4 * d + 3] - P->rects[4 * d + 1]);
  }
  P->p_sub = off;
  // pairs (all intersecting, i1 < i2)
  P->pairs.clear();
  int64_t loff = 0;
  for (int a = 0; a < D; ++a)
    for (int b = a + 1; b < D; ++b) {
      const int32_t* A = &P->rects[4 * a];
      const int32_t* B = &P->rects[4 * b];
      const int r0 = std::max(A[0], B[0]), c0 = std::max(A[1], B[1]);
      const int r1 = std::min(A[2], B[2]), c1 = std::min(A[3], B[3]);
      if (r0 < r1 && c0 < c1) {
        P->pairs.push_back(Pair{a, b, r0, c0, r1, c1, loff});
        loff += 2LL * (r1 - r0) * (c1 - c0);
      }
    }
  P->n_lam = loff;
  // pair lookup
  std::vector<int> pair_of((size_t)D * D, -1);
  for (size_t q = 0; q < P->pairs.size(); ++q) {
    pair_of[(size_t)P->pairs[q].a * D + P->pairs[q].b] = (int)q;
  }
  // cells: each problem's region cut at its own rectangles' edges (a batch places its
  // problems side by side; cutting every problem at the others' edges too would split
  // each into thin strips)
  P->cells.clear();
  P->max_cover = 0;
  for (const odp_plan::Entry& e : P->batch) {
    std::vector<int> rc = {e.row0, e.row0 + e.H}, cc = {e.col0, e.col0 + e.W};
    for (int d = e.D0; d < e.D0 + e.D; ++d) {
      rc.push_back(P->rects[4 * d]);
      rc.push_back(P->rects[4 * d + 2]);
      cc.push_back(P->rects[4 * d + 1]);
      cc.push_back(P->rects[4 * d + 3]);
    }
    std::sort(rc.begin(), rc.end());
    rc.erase(std::unique(rc.begin(), rc.end()), rc.end());
    std::sort(cc.begin(), cc.end());
    cc.erase(std::unique(cc.begin(), cc.end()), cc.end());
    for (size_t yi = 0; yi + 1 < rc.size(); ++yi)
      for (size_t xi = 0; xi + 1 < cc.size(); ++xi) {
        const int r0 = rc[yi], r1 = rc[yi + 1], c0 = cc[xi], c1 = cc[xi + 1];
        std::vector<int> S;
        for (int d = e.D0; d < e.D0 + e.D; ++d) {
          const int32_t* R = &P->rects[4 * d];
          if (R[0] <= r0 && r1 <= R[2] && R[1] <= c0 && c1 <= R[3]) S.push_back(d);
        }
        if (S.empty()) continue;
        P->max_cover = std::max<int32_t>(P->max_cover, (int32_t)S.size());
        if ((int)S.size() > MAXS)
          return fail(ODP_EUNSUPPORTED, "more than " + std::to_string(MAXS) + " subdomains overlap one pixel");
        CellDesc cd;
        std::memset(&cd, 0, sizeof(cd));
        cd.m = (int32_t)S.size();
        cd.npair = cd.m * (cd.m - 1) / 2;
        cd.r0 = r0;
        cd.c0 = c0;
        cd.nr = r1 - r0;
        cd.nc = c1 - c0;
        for (int s = 0; s < cd.m; ++s) {
          const int d = S[s];
          const int32_t* R = &P->rects[4 * d];
          cd.sub[s] = d;
          cd.upitch[s] = R[3] - R[1];
          cd.ubase[s] = P->usub_off[d] + (int64_t)(r0 - R[0]) * (R[3] - R[1]) + (c0 - R[1]);
        }
        for (int t = 1; t < cd.m; ++t)
          for (int s = 0; s < t; ++s) {
            const int q = t * (t - 1) / 2 + s;
            const int pq = pair_of[(size_t)S[s] * D + S[t]];
            if (pq < 0) return fail(ODP_EGEOM, "internal: missing pair");
            const Pair& pr = P->pairs[pq];
            const int pw = pr.c1 - pr.c0, ph = pr.r1 - pr.r0;
            cd.lbase[q] = pr.off + (int64_t)(r0 - pr.r0) * pw + (c0 - pr.c0);
            cd.lstride[q] = (int64_t)ph * pw;
            cd.lpitch[q] = pw;
            cd.pa[q] = (int8_t)s;
            cd.pb[q] = (int8_t)t;
          }
        cd.r = (float)P->batch[P->sub_problem[S[0]]].r;
        cd.probe = P->sub_problem[S[0]];
        P->cells.push_back(cd);
      }
  }
  // frames: base index inside the owning subdomain; processing order grouped by subdomain
  P->frames.resize(J);
  for (int j = 0; j < J; ++j) {
    const int d = P->frame_sub[j];
    const int32_t* R = &P->rects[4 * d];
    FrameDesc fd;
    fd.pitch = R[3] - R[1];
    fd.base = P->usub_off[d] + (int64_t)(P->offsets[2 * j] - R[0]) * fd.pitch + (P->offsets[2 * j + 1] - R[1]);
    fd.sub = d;
    fd.probe = P->sub_problem[d];
    fd.j = j;
    P->frames[j] = fd;
  }
  P->order.resize(J);
  for (int j = 0; j < J; ++j) P->order[j] = j;
  std::stable_sort(P->order.begin(), P->order.end(),
                   [&](int a, int b) { return P->frame_sub[a] < P->frame_sub[b]; });
  P->sub_first.assign(D + 1, 0);
  for (int j = 0; j < J; ++j) P->sub_first[P->frame_sub[j] + 1]++;
  for (int d = 0; d < D; ++d) P->sub_first[d + 1] += P->sub_first[d];
  P->chunk = (J + NXCD - 1) / NXCD;
  // The frame arrays an iteration streams (Gamma read and written, sqrt(f), the handoff
  // written and read back: 28 B per frame pixel) are accessed with the non-temporal hint
  // when they exceed the 256 MiB Infinity Cache of an MI355X; smaller ones stay in that
  // cache from one iteration to the next with ordinary accesses.
  P->stream = stream_by_size(P);
  static const int shapes[3][2] = {{16, 32}, {8, 64}, {32, 16}};
  for (int k = 0; k < 3; ++k) build_tiles(P, shapes[k][0], shapes[k][1], P->tsets[k]);
  P->covered = 0;
  for (const TileDesc& td : P->tsets[0].tiles) P->covered += (int64_t)td.nr * td.nc;
  P->ts = 0;
  // twiddle table tw[i][k] = W_p^{i k} = exp(-2 pi i i k / p), i < p/16, k < 16, FP64 on the host
  const int n2 = p / 16;
  P->tw.resize((size_t)n2 * 16);
  for (int i = 0; i < n2; ++i)
    for (int k = 0; k < 16; ++k) {
      const double a = 2.0 * M_PI * (double)(i * k) / (double)p;
      P->tw[i * 16 + k] = make_float2((float)std::cos(a), (float)-std::sin(a));
    }
  // split-BF16 DFT matrix F[k][n] = exp(-2 pi i k n / p) / sqrt(p), FP64 on the host:
  // hi = bf16(F), lo = bf16(F - hi).  Columns are stored in the MFMA kernel's
  // contraction order: n = 16t + 4g + i sits at 32(t/2) + 8g + 4(t%2) + i.
  if (p == 64) {  // the autotuner may switch a p = 64 plan between the two transforms
    const size_t pp = (size_t)p * p;
    P->dft.assign(4 * pp, 0);
    const double s = 1.0 / std::sqrt((double)p);
    for (int k = 0; k < p; ++k)
      for (int n = 0; n < p; ++n) {
        const double a = 2.0 * M_PI * (double)((k * n) % p) / (double)p;
        const double re = s * std::cos(a), im = -s * std::sin(a);
        const int nt = n >> 4, ng = (n >> 2) & 3, ni = n & 3;
        const size_t o = (size_t)k * p + 32 * (nt >> 1) + 8 * ng + 4 * (nt & 1) + ni;
        const uint16_t rh = bf16_rne((float)re), ih = bf16_rne((float)im);
        P->dft[o] = rh;
        P->dft[pp + o] = bf16_rne((float)(re - bf16_value(rh)));
        P->dft[2 * pp + o] = ih;
        P->dft[3 * pp + o] = bf16_rne((float)(im - bf16_value(ih)));
      }
  }
  // hybrid transform (fft_mfma.hpp): for every residue q < p/16 the 16-point stage
  // matrix M_q[k][r] = W_p^{q k} W_16^{r k} (and its conjugate transpose for the
  // inverse), FP64 on the host, as MFMA A operands per lane l = 16 g + n0: row m = n0,
  // element e = 2 s + c at contraction index 4 g + s, part c; the real-output row holds
  // (Re M, -Im M) and the imaginary-output row (Im M, Re M); each split hi + lo.  Set 0
  // in natural order; set 1 (p = 128, the two-half transform's stage A) with the
  // forward output rows and the inverse contraction columns permuted by
  // pi(4g + i) = 8 (i / 2) + 2g + i % 2.
  if (p == 64 || p == 128) {
    const int nq = p / 16, nsets = p == 128 ? 2 : 1;
    auto pi = [](int x) { return 8 * ((x & 3) >> 1) + 2 * (x >> 2) + (x & 1); };
    P->mft.assign((size_t)nsets * 2 * nq * 64 * 4 * 8, 0);
    for (int set = 0; set < nsets; ++set)
      for (int dir = 0; dir < 2; ++dir)
        for (int q = 0; q < nq; ++q)
          for (int l = 0; l < 64; ++l) {
            const int g = l >> 4, m = l & 15;
            for (int e = 0; e < 8; ++e) {
              const int c = e & 1, x = 4 * g + (e >> 1);
              const int out = set == 1 && dir == 0 ? pi(m) : m, in = set == 1 && dir == 1 ? pi(x) : x;
              // forward M[out][in]; inverse M^H[out][in] = conj(M[in][out])
              const int kk = dir == 0 ? out : in, rr = dir == 0 ? in : out;
              const double a = -2.0 * M_PI * ((double)(q * kk) / (double)p + (double)((rr * kk) % 16) / 16.0);
              const double mr = std::cos(a), mi = dir == 0 ? std::sin(a) : -std::sin(a);
              const double vre = c == 0 ? mr : -mi, vim = c == 0 ? mi : mr;
              const size_t o = ((((size_t)(set * 2 + dir) * nq + q) * 64 + l) * 4) * 8 + e;
              const uint16_t h0 = bf16_rne((float)vre), h1 = bf16_rne((float)vim);
              P->mft[o] = h0;
              P->mft[o + 8] = bf16_rne((float)(vre - bf16_value(h0)));
              P->mft[o + 16] = h1;
              P->mft[o + 24] = bf16_rne((float)(vim - bf16_value(h1)));
            }
          }
  }
  return ODP_OK;
}

void layout(odp_plan* P) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t pp = (size_t)P->p * P->p;
  P->ws.tw = take(sizeof(float2) * P->tw.size());
  P->ws.w = take(sizeof(float2) * pp * P->n_probes());
  P->ws.frames = take(sizeof(FrameDesc) * P->J);
  P->ws.order = take(sizeof(int32_t) * P->J);
  P->ws.fpos = take(sizeof(FrameDesc) * P->J);
  P->ws.sub_first = take(sizeof(int32_t) * (P->D + 1));
  P->ws.offsets = take(sizeof(int32_t) * 2 * P->J);
  P->ws.rects = take(sizeof(int32_t) * 4 * P->D);
  P->ws.usub_off = take(sizeof(int64_t) * P->D);
  P->ws.cells = take(sizeof(CellDesc) * P->cells.size());
  size_t n_tiles = 1, n_uni = 1, n_re = 1, n_tf = 1, n_pull = 1;
  for (const auto& T : P->tsets) {
    n_tiles = std::max(n_tiles, T.tiles.size());
    n_uni = std::max(n_uni, (size_t)T.n_uni);
    n_re = std::max(n_re, T.re_list.size());
    n_tf = std::max(n_tf, T.tf_first.size());
    n_pull = std::max(n_pull, T.pull.size());
  }
  P->ws.tiles = take(sizeof(TileDesc) * n_tiles);
  P->ws.waves = take(sizeof(WaveRec) * 4 * n_uni);
  P->ws.re_list = take(sizeof(int32_t) * n_re);
  P->ws.re_first = take(sizeof(int32_t) * (P->D + 1));
  P->ws.tf_first = take(sizeof(int32_t) * n_tf);
  P->ws.pull = take(sizeof(PullEntry) * n_pull);
  P->ws.den = take(sizeof(double) * P->p_sub);
  P->ws.rcp = take(sizeof(float) * P->p_sub);
  P->ws.fpart = take(sizeof(double) * NFS * P->J);
  P->ws.tpart = take(sizeof(double) * NPS * MAXS * n_tiles);
  P->ws.stat_scratch = take(sizeof(double) * NPS * (P->D + 1));
  P->ws.misc = take(sizeof(double) * (2 + 2 * 1024 + 8));
  P->ws.pmax = take(sizeof(double) * (2 + 2 * 1024) * P->n_probes());
  P->ws.psi = take(sizeof(float2) * pp * P->J);
  P->ws.fmask = take(sizeof(float) * pp);
  P->ws.wpart = take(sizeof(double) * 2 * pp * LOSS_CHUNKS);
  P->ws.dft = take(sizeof(uint16_t) * P->dft.size() + 16);
  P->ws.mft = take(sizeof(uint16_t) * P->mft.size() + 16);
  P->ws.prob = take(sizeof(int32_t) * 4 * P->n_probes());
  P->ws.resid = take(sizeof(double) * NRES * P->n_probes());
  P->ws.bytes = o;
  size_t s = 0;
  auto stake = [&](size_t bytes) {
    const size_t at = s;
    s = align256(s + bytes);
    return at;
  };
  P->st.u_sub = stake(sizeof(float2) * P->p_sub);
  P->st.gamma = stake(sizeof(float2) * pp * P->J);
  P->st.lam = stake(sizeof(float2) * std::max<int64_t>(1, P->n_lam));
  P->st.w = P->blind ? stake(sizeof(float2) * pp) : 0;
  P->st.w_sub = P->blind ? stake(sizeof(float2) * pp * P->D) : 0;
  P->st.delta = P->blind ? stake(sizeof(float2) * pp * P->D) : 0;
  P->st.stop = stake(sizeof(StopStatus) * P->n_probes());
  P->st.bytes = s;
}

int check_params(double eps, double eta, double r, double mu, double gamma, int D, int blind) {
  if (!(eps > 0.0 && eps < 1.0)) return fail(ODP_EINVAL, "eps must lie in (0, 1)");
  if (!(eta > 0.0)) return fail(ODP_EINVAL, "eta must be positive");
  if (D > 1 && !(r > 0.0)) return fail(ODP_EINVAL, "r must be positive when D > 1");
  if (!(r >= 0.0)) return fail(ODP_EINVAL, "r must be non-negative");
  if (blind && !(mu > 0.0)) return fail(ODP_EINVAL, "mu must be positive for blind recovery");
  if (!(gamma >= 0.0)) return fail(ODP_EINVAL, "gamma must be non-negative");
  return ODP_OK;
}

IllumArgs illum_args(const odp_plan* P, const float2* w, int recompute) {
  IllumArgs a;
  a.w = w;
  a.tf_first = P->W_<int32_t>(P->ws.tf_first);
  a.pull = P->W_<PullEntry>(P->ws.pull);
  a.cells = P->W_<CellDesc>(P->ws.cells);
  a.tiles = P->W_<TileDesc>(P->ws.tiles);
  a.n_tiles = (int32_t)P->tset().tiles.size();
  a.p = P->p;
  a.tile_cols = P->tset().cols;
  a.den = P->W_<double>(P->ws.den);
  a.rcp = P->W_<float>(P->ws.rcp);
  a.eta = P->eta;
  a.gamma = P->gamma;
  a.recompute_den = recompute;
  return a;
}

// The active tiling's arrays in launch order.  With xcd_slice = 2 the tiles of cells
// with at most four copies are placed so that the tile at launch position i runs on
// XCD i mod 8 whenever that is the XCD whose frame slice holds the frames of the
// tile's first copy (its psi is then read back through that XCD's L2); the other
// XCDs' leftovers fill the remaining positions.  tf_first, the pull records and
// re_list follow the tiles (re_list keeps its order, so the statistics are summed
// in the same order under every placement), and every wavefront of those tiles
// gets its WaveRec.
struct DevTiles {
  std::vector<TileDesc> tiles;
  std::vector<int32_t> re_list, tf_first;
  std::vector<PullEntry> pull;
  std::vector<WaveRec> waves;
};

void device_tiles(const odp_plan* P, DevTiles& o) {
  const odp_plan::TileSet& T = P->tset();
  const size_t n = T.tiles.size(), nu = (size_t)T.n_uni;
  std::vector<int32_t> perm(n);   // launch position -> tile
  for (size_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  if (P->xcd_slice == 2 && P->chunk > 0) {
    std::vector<std::vector<int32_t>> q(NXCD);
    for (size_t t = 0; t < nu; ++t) {
      const int d = P->cells[T.tiles[t].cell].sub[0];
      const int mid = (P->sub_first[d] + P->sub_first[d + 1]) / 2;
      q[std::min(NXCD - 1, mid / P->chunk)].push_back((int32_t)t);
    }
    std::vector<size_t> h(NXCD, 0);
    for (size_t i = 0; i < nu; ++i) {
      int x = (int)(i % NXCD);
      if (h[x] >= q[x].size()) {  // XCD x has no tiles left: take from the longest queue
        size_t left = 0;
        for (int y = 0; y < NXCD; ++y)
          if (q[y].size() - h[y] > left) {
            left = q[y].size() - h[y];
            x = y;
          }
      }
      perm[i] = q[x][h[x]++];
    }
  }
  std::vector<int32_t> inv(n);
  for (size_t i = 0; i < n; ++i) inv[perm[i]] = (int32_t)i;
  o.tiles.resize(n);
  o.tf_first.assign(n * MAXS + 1, 0);
  o.pull.clear();
  o.pull.reserve(T.pull.size());
  for (size_t i = 0; i < n; ++i) {
    const int t = perm[i];
    o.tiles[i] = T.tiles[t];
    for (int sl = 0; sl < MAXS; ++sl) {
      o.tf_first[i * MAXS + sl] = (int32_t)o.pull.size();
      o.pull.insert(o.pull.end(), T.pull.begin() + T.tf_first[(size_t)t * MAXS + sl],
                    T.pull.begin() + T.tf_first[(size_t)t * MAXS + sl + 1]);
    }
  }
  o.tf_first[n * MAXS] = (int32_t)o.pull.size();
  for (int q = 0; q < PULL_B; ++q) o.pull.push_back(PullEntry{0, PULL_NONE, PULL_NONE});  // read ahead of the last list
  o.re_list.resize(T.re_list.size());
  for (size_t k = 0; k < T.re_list.size(); ++k) {
    const int32_t e = T.re_list[k];
    o.re_list[k] = inv[e / MAXS] * MAXS + e % MAXS;
  }
  o.waves.assign(nu * 4, WaveRec{});
  for (size_t i = 0; i < nu; ++i) {
    const TileDesc& td = o.tiles[i];
    const CellDesc& cd = P->cells[td.cell];
    int lg = 0;
    while ((1 << lg) < cd.m) ++lg;
    const int tpg = 256 >> lg, cw = std::min(T.cols, NPX * tpg);
    int lcw = 0;
    while ((1 << lcw) < cw) ++lcw;
    for (int wv = 0; wv < 4; ++wv) {
      WaveRec& r = o.waves[i * 4 + wv];
      const int sl = wv * 64 / tpg;
      r.s = sl;
      r.m = cd.m;
      r.lg = lg;
      r.lcw = lcw;
      r.nr = td.nr;
      r.nc = td.nc;
      r.yi0 = cd.r0 + td.r0;
      r.xi0 = cd.c0 + td.c0;
      r.r = cd.r;
      r.sub = cd.sub[std::min(sl, cd.m - 1)];
      r.prob = cd.probe;
      if (sl >= cd.m) continue;  // idle copy group: empty pull, no pixels
      r.u0 = cd.ubase[sl] + (int64_t)td.r0 * cd.upitch[sl] + td.c0;
      r.upitch = cd.upitch[sl];
      r.k0 = o.tf_first[i * MAXS + sl];
      r.k1 = o.tf_first[i * MAXS + sl + 1];
      for (int pt = 0; pt < cd.m - 1; ++pt) {
        const int t = pt + (pt >= sl), lo = std::min(sl, t), hi = std::max(sl, t), pq = hi * (hi - 1) / 2 + lo;
        const int64_t li = cd.lbase[pq] + (int64_t)td.r0 * cd.lpitch[pq] + td.c0, lj = li + cd.lstride[pq];
        r.lo0[pt] = sl < t ? li : lj;
        r.lt0[pt] = sl < t ? lj : li;
        r.lpitch[pt] = cd.lpitch[pq];
        r.pu0[pt] = cd.ubase[t] + (int64_t)td.r0 * cd.upitch[t] + td.c0;
        r.pupitch[pt] = cd.upitch[t];
      }
    }
  }
}

int upload_tiles(odp_plan* P, hipStream_t s) {
  DevTiles D;
  device_tiles(P, D);
  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(P->wsp + off, src, bytes, hipMemcpyHostToDevice, s);
  };
  ODP_HIP(up(P->ws.tiles, D.tiles.data(), sizeof(TileDesc) * D.tiles.size()));
  ODP_HIP(up(P->ws.waves, D.waves.data(), sizeof(WaveRec) * D.waves.size()));
  ODP_HIP(up(P->ws.re_list, D.re_list.data(), sizeof(int32_t) * D.re_list.size()));
  ODP_HIP(up(P->ws.re_first, P->tset().re_first.data(), sizeof(int32_t) * P->tset().re_first.size()));
  ODP_HIP(up(P->ws.tf_first, D.tf_first.data(), sizeof(int32_t) * D.tf_first.size()));
  ODP_HIP(up(P->ws.pull, D.pull.data(), sizeof(PullEntry) * D.pull.size()));
  // pageable host sources: finish before the vectors go out of scope
  ODP_HIP(hipStreamSynchronize(s));
  return ODP_OK;
}

// per-problem overlap penalties: cell descriptors carry r; reciprocals rebuilt
int set_penalties(odp_plan* P, const double* r, hipStream_t s) {
  ++P->gen;
  for (int i = 0; i < P->n_probes(); ++i) P->batch[i].r = r[i];
  for (CellDesc& cd : P->cells) cd.r = (float)P->batch[cd.probe].r;
  if (!P->wsp) return ODP_OK;
  ODP_HIP(hipMemcpyAsync(P->wsp + P->ws.cells, P->cells.data(), sizeof(CellDesc) * P->cells.size(),
                         hipMemcpyHostToDevice, s));
  const int rc = upload_tiles(P, s);   // the wave records carry r too
  if (rc) return rc;
  ODP_HIP(launch_illum(illum_args(P, P->W_<float2>(P->ws.w), 0), s));
  ODP_HIP(hipStreamSynchronize(s));
  return ODP_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* odp_last_error(void) { return g_err.c_str(); }
const char* odp_version(void) { return "odp 0.1 (gfx950)"; }

// The frame transforms a plan of probe size p can run.
static int check_transform(int32_t transform, int p) {
  if (transform != ODP_FFT_F32 && transform != ODP_DFT_SPLIT_BF16 && transform != ODP_HYBRID_MFMA)
    return fail(ODP_EINVAL, "unknown transform");
  if (transform == ODP_DFT_SPLIT_BF16 && p != 64)
    return fail(ODP_EUNSUPPORTED, "the split-BF16 DFT transform is built for p = 64");
  if (transform == ODP_HYBRID_MFMA && p != 64 && p != 128)
    return fail(ODP_EUNSUPPORTED, "the hybrid MFMA transform is built for p = 64 and 128");
  return ODP_OK;
}

static int validate_problem(const odp_problem* prob) {
  if (prob->p != 32 && prob->p != 64 && prob->p != 128)
    return fail(ODP_EUNSUPPORTED, "p must be 32, 64 or 128");
  if (prob->H < prob->p || prob->W < prob->p) return fail(ODP_EINVAL, "image smaller than the probe");
  if (prob->J < 1 || !prob->offsets || !prob->frame_sub) return fail(ODP_EINVAL, "no frames");
  if (prob->D < 1) return fail(ODP_EINVAL, "D must be >= 1");
  int rc = check_transform(prob->transform, prob->p);
  if (rc) return rc;
  rc = check_params(prob->eps, prob->eta, prob->r, prob->mu, prob->gamma, prob->D, prob->blind);
  if (rc) return rc;
  if ((int64_t)prob->H * prob->W >= (int64_t)1 << 31) return fail(ODP_EUNSUPPORTED, "image too large");
  for (int j = 0; j < prob->J; ++j) {
    const int r = prob->offsets[2 * j], c = prob->offsets[2 * j + 1];
    if (r < 0 || c < 0 || r + prob->p > prob->H || c + prob->p > prob->W)
      return fail(ODP_EGEOM, "window " + std::to_string(j) + " leaves the image");
    if (prob->frame_sub[j] < 0 || prob->frame_sub[j] >= prob->D)
      return fail(ODP_EGEOM, "frame_sub out of range at frame " + std::to_string(j));
  }
  return ODP_OK;
}

// Build a plan from a validated problem; `batch` describes the independent
// problems it packs (one entry for a single problem).
static int create_impl(const odp_problem* prob, std::vector<odp_plan::Entry> batch,
                       std::vector<int32_t> sub_problem, odp_plan** out) {
  odp_plan* P = new (std::nothrow) odp_plan();
  if (!P) return fail(ODP_ENOMEM, "host allocation failed");
  P->H = prob->H;
  P->W = prob->W;
  P->p = prob->p;
  P->J = prob->J;
  P->D = prob->D;
  P->eps = prob->eps;
  P->eta = prob->eta;
  P->r = prob->r;
  P->mu = prob->mu;
  P->gamma = prob->gamma;
  P->transform = prob->transform;
  P->blind = prob->blind ? 1 : 0;
  P->batch = std::move(batch);
  P->sub_problem = std::move(sub_problem);
  P->offsets.assign(prob->offsets, prob->offsets + 2 * (size_t)prob->J);
  P->frame_sub.assign(prob->frame_sub, prob->frame_sub + prob->J);
  if (prob->probe_fmask) {
    P->fmask.resize((size_t)prob->p * prob->p);
    for (size_t i = 0; i < P->fmask.size(); ++i) P->fmask[i] = prob->probe_fmask[i] ? 1.0f : 0.0f;
  }
  int rc;
  try {
    rc = build_geometry(P);
  } catch (const std::bad_alloc&) {
    rc = fail(ODP_ENOMEM, "host allocation failed");
  }
  if (rc) {
    delete P;
    return rc;
  }
  layout(P);
  *out = P;
  return ODP_OK;
}

int odp_plan_create(const odp_problem* prob, odp_plan** out) {
  if (!prob || !out) return fail(ODP_EINVAL, "null argument");
  *out = nullptr;
  int rc = validate_problem(prob);
  if (rc) return rc;
  std::vector<odp_plan::Entry> batch{{0, 0, prob->H, prob->W, 0, prob->J, 0, prob->D, prob->r, 0.0}};
  return create_impl(prob, std::move(batch), std::vector<int32_t>(prob->D, 0), out);
}

int odp_batch_plan_create(const odp_problem* probs, int32_t n, odp_plan** out) {
  if (!probs || !out || n < 1) return fail(ODP_EINVAL, "null argument or empty batch");
  *out = nullptr;
  const int p = probs[0].p;
  int64_t Wt = 0, Jt = 0, Dt = 0;
  int32_t Ht = 0;
  for (int i = 0; i < n; ++i) {
    const odp_problem& q = probs[i];
    int rc = validate_problem(&q);
    if (rc) return fail(rc, "problem " + std::to_string(i) + ": " + g_err);
    if (q.p != p || q.transform != probs[0].transform || q.eps != probs[0].eps || q.eta != probs[0].eta ||
        q.gamma != probs[0].gamma)
      return fail(ODP_EINVAL, "batched problems must share p, transform, eps, eta and gamma");
    if (q.blind) return fail(ODP_EUNSUPPORTED, "batches hold known-probe problems");
    if (q.probe_fmask) return fail(ODP_EINVAL, "batches take no probe mask");
    Ht = std::max(Ht, q.H);
    Wt += q.W + (i ? 1 : 0);   // one blank column between problems: their subdomains never meet
    Jt += q.J;
    Dt += q.D;
  }
  if ((int64_t)Ht * Wt >= (int64_t)1 << 31 || Jt >= (int64_t)1 << 31) return fail(ODP_EUNSUPPORTED, "batch too large");
  std::vector<int32_t> off((size_t)2 * Jt), sub((size_t)Jt), sub_problem((size_t)Dt);
  std::vector<odp_plan::Entry> batch;
  int32_t col = 0, J0 = 0, D0 = 0;
  for (int i = 0; i < n; ++i) {
    const odp_problem& q = probs[i];
    for (int j = 0; j < q.J; ++j) {
      off[2 * (size_t)(J0 + j)] = q.offsets[2 * j];
      off[2 * (size_t)(J0 + j) + 1] = q.offsets[2 * j + 1] + col;
      sub[J0 + j] = q.frame_sub[j] + D0;
    }
    for (int d = 0; d < q.D; ++d) sub_problem[D0 + d] = i;
    batch.push_back(odp_plan::Entry{0, col, q.H, q.W, J0, q.J, D0, q.D, q.r, 0.0});
    col += q.W + 1;
    J0 += q.J;
    D0 += q.D;
  }
  odp_problem all = probs[0];
  all.H = Ht;
  all.W = (int32_t)Wt;
  all.J = (int32_t)Jt;
  all.D = (int32_t)Dt;
  all.offsets = off.data();
  all.frame_sub = sub.data();
  all.r = 1.0;  // per problem (cells carry their own r)
  return create_impl(&all, std::move(batch), std::move(sub_problem), out);
}

int odp_batch_get_entry(const odp_plan* P, int32_t i, odp_batch_entry* o) {
  if (!P || !o) return fail(ODP_EINVAL, "null argument");
  if (i < 0 || i >= P->n_probes()) return fail(ODP_EINVAL, "batch index out of range");
  const odp_plan::Entry& e = P->batch[i];
  o->row0 = e.row0;
  o->col0 = e.col0;
  o->H = e.H;
  o->W = e.W;
  o->J0 = e.J0;
  o->J = e.J;
  o->D0 = e.D0;
  o->D = e.D;
  o->r = e.r;
  o->illum_max = e.illum_max;
  return ODP_OK;
}

void odp_plan_destroy(odp_plan* plan) { delete plan; }

int odp_plan_get_info(const odp_plan* P, odp_plan_info* o) {
  if (!P || !o) return fail(ODP_EINVAL, "null argument");
  o->H = P->H;
  o->W = P->W;
  o->p = P->p;
  o->J = P->J;
  o->D = P->D;
  o->n_pairs = (int32_t)P->pairs.size();
  o->max_cover = P->max_cover;
  o->n_cells = (int32_t)P->cells.size();
  o->n_tiles = (int32_t)P->tset().tiles.size();
  o->p_sub = P->p_sub;
  o->n_lam = P->n_lam;
  o->workspace_bytes = P->ws.bytes;
  o->state_bytes = P->st.bytes;
  return ODP_OK;
}

size_t odp_plan_workspace_bytes(const odp_plan* P) { return P ? P->ws.bytes : 0; }
double odp_plan_get_eta(const odp_plan* P) { return P ? P->eta : 0.0; }
size_t odp_state_bytes(const odp_plan* P) { return P ? P->st.bytes : 0; }

int odp_state_get_layout(const odp_plan* P, odp_state_layout* o) {
  if (!P || !o) return fail(ODP_EINVAL, "null argument");
  o->u_sub = P->st.u_sub;
  o->gamma = P->st.gamma;
  o->lam = P->st.lam;
  o->w = P->st.w;
  o->w_sub = P->st.w_sub;
  o->delta = P->st.delta;
  o->stop = P->st.stop;
  o->bytes = P->st.bytes;
  return ODP_OK;
}

int odp_plan_get_rects(const odp_plan* P, int32_t* rects, int64_t* usub_off) {
  if (!P || !rects) return fail(ODP_EINVAL, "null argument");
  std::memcpy(rects, P->rects.data(), sizeof(int32_t) * P->rects.size());
  if (usub_off) std::memcpy(usub_off, P->usub_off.data(), sizeof(int64_t) * P->usub_off.size());
  return ODP_OK;
}

int odp_plan_get_pairs(const odp_plan* P, int32_t* pairs, int64_t* lam_off) {
  if (!P || !pairs) return fail(ODP_EINVAL, "null argument");
  for (size_t q = 0; q < P->pairs.size(); ++q) {
    const Pair& pr = P->pairs[q];
    int32_t* o = pairs + 6 * q;
    o[0] = pr.a; o[1] = pr.b; o[2] = pr.r0; o[3] = pr.c0; o[4] = pr.r1; o[5] = pr.c1;
    if (lam_off) lam_off[q] = pr.off;
  }
  return ODP_OK;
}

int odp_plan_get_cover(const odp_plan* P, int32_t* cover) {
  if (!P || !cover) return fail(ODP_EINVAL, "null argument");
  std::fill(cover, cover + (size_t)P->H * P->W, 0);
  for (const TileDesc& td : P->tset().tiles) {
    const CellDesc& cd = P->cells[td.cell];
    for (int y = 0; y < td.nr; ++y)
      for (int x = 0; x < td.nc; ++x)
        cover[(size_t)(cd.r0 + td.r0 + y) * P->W + (cd.c0 + td.c0 + x)] = cd.m;
  }
  return ODP_OK;
}

int odp_plan_bind(odp_plan* P, void* dev_ws, const float* dev_sqrt_f, const odp_c32* dev_w, hipStream_t s) {
  if (!P || !dev_ws || !dev_sqrt_f || !dev_w) return fail(ODP_EINVAL, "null argument");
  if (reinterpret_cast<uintptr_t>(dev_ws) & 255) return fail(ODP_EINVAL, "workspace must be 256-byte aligned");
  ++P->gen;
  P->wsp = static_cast<char*>(dev_ws);
  P->sqrt_f = dev_sqrt_f;
  const size_t pp = (size_t)P->p * P->p;
  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(P->wsp + off, src, bytes, hipMemcpyHostToDevice, s);
  };
  ODP_HIP(up(P->ws.tw, P->tw.data(), sizeof(float2) * P->tw.size()));
  ODP_HIP(hipMemcpyAsync(P->wsp + P->ws.w, dev_w, sizeof(float2) * pp * P->n_probes(), hipMemcpyDeviceToDevice, s));
  ODP_HIP(up(P->ws.frames, P->frames.data(), sizeof(FrameDesc) * P->frames.size()));
  ODP_HIP(up(P->ws.order, P->order.data(), sizeof(int32_t) * P->order.size()));
  std::vector<FrameDesc> fpos(P->J);
  for (int q = 0; q < P->J; ++q) fpos[q] = P->frames[P->order[q]];
  ODP_HIP(up(P->ws.fpos, fpos.data(), sizeof(FrameDesc) * fpos.size()));
  ODP_HIP(up(P->ws.sub_first, P->sub_first.data(), sizeof(int32_t) * P->sub_first.size()));
  ODP_HIP(up(P->ws.offsets, P->offsets.data(), sizeof(int32_t) * P->offsets.size()));
  ODP_HIP(up(P->ws.rects, P->rects.data(), sizeof(int32_t) * P->rects.size()));
  ODP_HIP(up(P->ws.usub_off, P->usub_off.data(), sizeof(int64_t) * P->usub_off.size()));
  ODP_HIP(up(P->ws.cells, P->cells.data(), sizeof(CellDesc) * P->cells.size()));
  int rc = upload_tiles(P, s);
  if (rc) return rc;
  if (!P->fmask.empty()) ODP_HIP(up(P->ws.fmask, P->fmask.data(), sizeof(float) * pp));
  if (!P->dft.empty()) ODP_HIP(up(P->ws.dft, P->dft.data(), sizeof(uint16_t) * P->dft.size()));
  if (!P->mft.empty()) ODP_HIP(up(P->ws.mft, P->mft.data(), sizeof(uint16_t) * P->mft.size()));
  std::vector<int32_t> prob;
  for (const odp_plan::Entry& e : P->batch) prob.insert(prob.end(), {e.J0, e.J, e.D0, e.D});
  ODP_HIP(up(P->ws.prob, prob.data(), sizeof(int32_t) * prob.size()));
  ODP_HIP(launch_illum(illum_args(P, P->W_<float2>(P->ws.w), 1), s));
  double* misc = P->W_<double>(P->ws.misc);
  ODP_HIP(launch_sum_max(P->W_<double>(P->ws.den), P->p_sub, dev_sqrt_f, (int64_t)P->J * pp, misc, s));
  // the largest illumination of each problem (penalty scales are chosen from it) and
  // its sum of sqrt f (the denominator of its RF)
  const int nb = P->n_probes();
  double* pm = P->W_<double>(P->ws.pmax);
  for (int i = 0; i < nb; ++i) {
    const odp_plan::Entry& e = P->batch[i];
    const int64_t u0 = P->usub_off[e.D0];
    const int64_t u1 = e.D0 + e.D < P->D ? P->usub_off[e.D0 + e.D] : P->p_sub;
    ODP_HIP(launch_sum_max(P->W_<double>(P->ws.den) + u0, u1 - u0, dev_sqrt_f + (size_t)e.J0 * pp,
                           (int64_t)e.J * pp, pm + (size_t)i * (2 + 2048), s));
  }
  double host[2] = {0, 0};
  std::vector<double> hp((size_t)nb * (2 + 2048));
  ODP_HIP(hipMemcpyAsync(host, misc, sizeof(host), hipMemcpyDeviceToHost, s));
  ODP_HIP(hipMemcpyAsync(hp.data(), pm, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s));
  ODP_HIP(hipStreamSynchronize(s));
  P->illum_max = host[0];
  for (int i = 0; i < nb; ++i) P->batch[i].illum_max = hp[(size_t)i * (2 + 2048)];
  return ODP_OK;
}

int odp_plan_illum_max(const odp_plan* P, double* out) {
  if (!P || !out) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp) return fail(ODP_EINVAL, "plan is not bound");
  *out = P->illum_max;
  return ODP_OK;
}

int odp_plan_set_params(odp_plan* P, double eps, double eta, double r, double mu, double gamma, hipStream_t s) {
  if (!P) return fail(ODP_EINVAL, "null argument");
  int rc = check_params(eps, eta, r, mu, gamma, P->D, P->blind);
  if (rc) return rc;
  P->eps = eps;
  P->eta = eta;
  P->r = r;
  P->mu = mu;
  P->gamma = gamma;
  std::vector<double> rs(P->n_probes(), r);
  return set_penalties(P, rs.data(), s);
}

int odp_batch_set_penalties(odp_plan* P, const double* r, hipStream_t s) {
  if (!P || !r) return fail(ODP_EINVAL, "null argument");
  for (int i = 0; i < P->n_probes(); ++i)
    if (!(r[i] > 0.0) && P->batch[i].D > 1) return fail(ODP_EINVAL, "r must be positive when D > 1");
  return set_penalties(P, r, s);
}

int odp_forward(const odp_plan* P, const odp_c32* u, const odp_c32* w, odp_c32* out, hipStream_t s) {
  if (!P || !u || !w || !out) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp) return fail(ODP_EINVAL, "plan is not bound");
  ODP_HIP(launch_forward(P->p, reinterpret_cast<const float2*>(u), P->H, P->W, reinterpret_cast<const float2*>(w),
                         P->W_<float2>(P->ws.tw), P->W_<int32_t>(P->ws.offsets), P->J,
                         reinterpret_cast<float2*>(out), s));
  return ODP_OK;
}

int odp_adjoint(const odp_plan* P, const odp_c32* frames, const odp_c32* w, odp_c32* u_out, hipStream_t s) {
  if (!P || !frames || !w || !u_out) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp) return fail(ODP_EINVAL, "plan is not bound");
  ODP_HIP(launch_adjoint(P->p, reinterpret_cast<const float2*>(frames), reinterpret_cast<const float2*>(w),
                         P->W_<float2>(P->ws.tw), P->W_<int32_t>(P->ws.offsets), P->J,
                         reinterpret_cast<float2*>(u_out), P->H, P->W, s));
  return ODP_OK;
}

int odp_prox_stagm(const odp_c32* y, const float* sqrt_f, int64_t count, float eps, float lambda, odp_c32* z,
                   hipStream_t s) {
  if (count < 0) return fail(ODP_EINVAL, "negative count");
  if (count > 0 && (!y || !sqrt_f || !z)) return fail(ODP_EINVAL, "null argument");
  if (!(eps > 0.f && eps < 1.f)) return fail(ODP_EINVAL, "eps must lie in (0, 1)");
  if (!(lambda > 0.f)) return fail(ODP_EINVAL, "lambda must be positive");
  ODP_HIP(launch_prox(reinterpret_cast<const float2*>(y), sqrt_f, count, eps, lambda, reinterpret_cast<float2*>(z),
                      s));
  return ODP_OK;
}

int odp_state_init(const odp_plan* P, void* dev_state, const odp_c32* dev_w0, hipStream_t s) {
  if (!P || !dev_state) return fail(ODP_EINVAL, "null argument");
  if (P->blind && !dev_w0) return fail(ODP_EINVAL, "blind state needs an initial probe");
  char* b = static_cast<char*>(dev_state);
  const size_t pp = (size_t)P->p * P->p;
  ODP_HIP(launch_fill(reinterpret_cast<float2*>(b + P->st.u_sub), P->p_sub, make_float2(1.f, 0.f), s));
  ODP_HIP(launch_fill(reinterpret_cast<float2*>(b + P->st.gamma), (int64_t)pp * P->J, make_float2(0.f, 0.f), s));
  ODP_HIP(launch_fill(reinterpret_cast<float2*>(b + P->st.lam), P->n_lam, make_float2(0.f, 0.f), s));
  ODP_HIP(launch_fill(reinterpret_cast<float2*>(b + P->st.stop),
                      (int64_t)(sizeof(StopStatus) / sizeof(float2)) * P->n_probes(), make_float2(0.f, 0.f), s));
  P->stop_count.erase(dev_state);
  if (P->blind) {
    const float2* w0 = reinterpret_cast<const float2*>(dev_w0);
    ODP_HIP(launch_copy(reinterpret_cast<float2*>(b + P->st.w), w0, (int64_t)pp, s));
    for (int d = 0; d < P->D; ++d)
      ODP_HIP(launch_copy(reinterpret_cast<float2*>(b + P->st.w_sub) + d * pp, w0, (int64_t)pp, s));
    ODP_HIP(launch_fill(reinterpret_cast<float2*>(b + P->st.delta), (int64_t)pp * P->D, make_float2(0.f, 0.f), s));
  }
  return ODP_OK;
}

static SweepArgs sweep_args(const odp_plan* P, char* b, double* stats) {
  SweepArgs a;
  a.u = reinterpret_cast<const float2*>(b + P->st.u_sub);
  a.w = P->blind ? reinterpret_cast<const float2*>(b + P->st.w_sub) : P->W_<float2>(P->ws.w);
  a.w_out = a.w;
  a.w_per_sub = P->blind;
  a.tw = P->W_<float2>(P->ws.tw);
  a.mft = P->transform == ODP_HYBRID_MFMA ? P->W_<uint4>(P->ws.mft) : nullptr;
  a.gamma = reinterpret_cast<float2*>(b + P->st.gamma);
  a.sqrt_f = P->sqrt_f;
  a.frames = P->W_<FrameDesc>(P->ws.frames);
  a.order = P->W_<int32_t>(P->ws.order);
  a.fpos = P->W_<FrameDesc>(P->ws.fpos);
  a.J = P->J;
  a.chunk = P->chunk;
  a.xcd_slice = P->xcd_slice;
  a.eps = (float)P->eps;
  a.eta = (float)P->eta;
  a.gcoef = (float)(0.5 * (1.0 - P->eps) / P->eps);
  a.part = stats || P->balancing() || P->stop_check(b) ? P->W_<double>(P->ws.fpart) : nullptr;
  a.psi = P->W_<float2>(P->ws.psi);
  a.blind = P->blind;
  a.stop = P->stopping() ? reinterpret_cast<const StopStatus*>(b + P->st.stop) : nullptr;
  a.frame_res = P->balancing() && (P->bal_which & ODP_BALANCE_ETA) ? 1 : 0;
  a.stream = P->stream;
  return a;
}

static PixelArgs pixel_args(const odp_plan* P, char* b, double* stats) {
  PixelArgs a;
  a.u = reinterpret_cast<float2*>(b + P->st.u_sub);
  a.rcp = P->W_<float>(P->ws.rcp);
  a.lam = reinterpret_cast<float2*>(b + P->st.lam);
  a.cells = P->W_<CellDesc>(P->ws.cells);
  a.tiles = P->W_<TileDesc>(P->ws.tiles);
  a.waves = P->W_<WaveRec>(P->ws.waves);
  a.pairs = P->pairs_on && P->tset().pairs ? 1 : 0;
  a.n_tiles = (int32_t)P->tset().tiles.size();
  a.n_uni = P->tset().n_uni;
  a.n_mid = P->tset().n_mid;
  a.p = P->p;
  a.tile_cols = P->tset().cols;
  a.psi = P->W_<float2>(P->ws.psi);
  a.tf_first = P->W_<int32_t>(P->ws.tf_first);
  a.pull = P->W_<PullEntry>(P->ws.pull);
  a.w_sub = P->blind ? reinterpret_cast<const float2*>(b + P->st.w_sub) : nullptr;
  a.eta = (float)P->eta;
  a.gamma = (float)P->gamma;
  a.part = stats || P->balancing() || P->stop_check(b) ? P->W_<double>(P->ws.tpart) : nullptr;
  a.dend = P->W_<double>(P->ws.den);
  a.stop = P->stopping() ? reinterpret_cast<const StopStatus*>(b + P->st.stop) : nullptr;
  a.stream = P->stream;
  return a;
}

// Residual balancing of the penalties (He, Yang and Wang 2000; Boyd et al. 2011, Sec.
// 3.4.1) after the iteration just issued.  Overlap penalty r, per problem: the normalised
// primal consensus residual rp = ||pi u - v|| / ||pi u|| against the dual rd = ||pi du|| /
// ||Lam||.  Data penalty eta, for the whole plan: rp = ||Gamma^{n+1} - Gamma^n|| / ||A u^n||
// against rd = ||A du|| / ||Gamma^{n+1}|| (||A x||^2 = sum den |x|^2).  A penalty q becomes
// tau q when rp > mu rd and q / tau when rd > mu rp; its scaled multipliers (Lam or Gamma)
// are multiplied by q_old / q_new.  Reads the sums to the host (synchronises).
static int balance_penalties(odp_plan* P, char* b, hipStream_t s) {
  const int n = P->n_probes();
  const bool do_r = (P->bal_which & ODP_BALANCE_R) != 0, do_eta = (P->bal_which & ODP_BALANCE_ETA) != 0;
  bool any_pairs = false;
  for (const odp_plan::Entry& e : P->batch) any_pairs = any_pairs || e.D >= 2;
  if (!do_eta && !any_pairs) return ODP_OK;   // nothing to balance: no read, no synchronisation
  double* dev = P->W_<double>(P->ws.resid);
  ODP_HIP(launch_residual_sums(P->W_<double>(P->ws.fpart), P->J, P->W_<double>(P->ws.tpart),
                               P->W_<int32_t>(P->ws.re_list), P->W_<int32_t>(P->ws.re_first), P->D,
                               P->W_<int32_t>(P->ws.prob), n, P->W_<double>(P->ws.stat_scratch), dev, s));
  std::vector<double> h((size_t)NRES * n);
  ODP_HIP(hipMemcpyAsync(h.data(), dev, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  // a problem stopped by its rule (this iteration included) keeps its state: its penalty and
  // multipliers stay as they are, and its sums (stale once it skips iterations) are left out
  std::vector<StopStatus> stop(P->stopping() ? n : 0);
  if (!stop.empty())
    ODP_HIP(hipMemcpyAsync(stop.data(), b + P->st.stop, sizeof(StopStatus) * n, hipMemcpyDeviceToHost, s));
  ODP_HIP(hipStreamSynchronize(s));
  auto running = [&](int i) { return stop.empty() || !stop[i].stopped; };
  auto factor = [&](double Pr, double S, double U, double L) {
    if (!(U > 0.0 && L > 0.0)) return 1.0;
    const double rp = std::sqrt(Pr / U), rd = std::sqrt(S / L);
    if (rp > P->bal_mu * rd) return P->bal_tau;
    if (rd > P->bal_mu * rp) return 1.0 / P->bal_tau;
    return 1.0;
  };
  std::vector<double> r(n);
  bool changed = false;
  for (int i = 0; i < n; ++i) {
    const odp_plan::Entry& e = P->batch[i];
    const double* hi = &h[(size_t)NRES * i];
    r[i] = e.r;
    if (!do_r || e.D < 2 || !running(i)) continue;
    const double fac = factor(hi[0], hi[1], hi[2], hi[3]);
    if (fac == 1.0) continue;
    r[i] = e.r * fac;
    changed = true;
    // the problem's multipliers: its pairs are contiguous (pairs are ordered by their
    // first subdomain, and a problem's subdomains are contiguous)
    int64_t l0 = -1, l1 = -1;
    for (const Pair& q : P->pairs)
      if (q.a >= e.D0 && q.a < e.D0 + e.D) {
        if (l0 < 0) l0 = q.off;
        l1 = q.off + 2LL * (q.r1 - q.r0) * (q.c1 - q.c0);
      }
    if (l0 >= 0)
      ODP_HIP(launch_scale(reinterpret_cast<float2*>(b + P->st.lam) + l0, l1 - l0, (float)(1.0 / fac), s));
  }
  if (do_eta) {
    // eta is shared by the plan's problems: decided on the running ones' sums, applied to
    // the running ones' multipliers Gamma (a stopped problem keeps its Gamma; it reads eta
    // again only through a new state)
    double U = 0.0, S = 0.0, Pr = 0.0, L = 0.0;
    for (int i = 0; i < n; ++i) {
      if (!running(i)) continue;
      const double* hi = &h[(size_t)NRES * i];
      U += hi[4];
      S += hi[5];
      Pr += hi[6];
      L += hi[7];
    }
    const double fac = factor(Pr, S, U, L);
    if (fac != 1.0) {
      P->eta *= fac;
      const int64_t pp = (int64_t)P->p * P->p;
      for (int i = 0; i < n; ++i) {
        if (!running(i)) continue;
        const odp_plan::Entry& e = P->batch[i];
        // consecutive running problems share one launch
        int k = i;
        while (k + 1 < n && running(k + 1)) ++k;
        const int64_t j0 = e.J0, j1 = (int64_t)P->batch[k].J0 + P->batch[k].J;
        ODP_HIP(launch_scale(reinterpret_cast<float2*>(b + P->st.gamma) + j0 * pp, (j1 - j0) * pp,
                             (float)(1.0 / fac), s));
        i = k;
      }
      changed = true;
    }
  }
  if (!changed) return ODP_OK;
  return set_penalties(P, r.data(), s);   // the reciprocals follow eta and r
}

static int finish_stats(const odp_plan* P, double* stats, hipStream_t s) {
  ODP_HIP(launch_stats(P->W_<double>(P->ws.fpart), P->J, P->W_<double>(P->ws.tpart), P->W_<int32_t>(P->ws.re_list),
                       P->W_<int32_t>(P->ws.re_first), P->D, P->W_<double>(P->ws.misc) + 1, stats,
                       P->W_<double>(P->ws.stat_scratch), s));
  return ODP_OK;
}

int odp_frame_sweep(odp_plan* P, void* dev_state, double* dev_stats, hipStream_t s) {
  if (!P || !dev_state) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp) return fail(ODP_EINVAL, "plan is not bound");
  const SweepArgs a = sweep_args(P, static_cast<char*>(dev_state), dev_stats);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!P->sweep_ev.empty()) {
    const size_t c = P->sweep_ev_next++;
    if (c % P->sweep_ev_stride == 0) {
      e0 = P->sweep_ev[c / P->sweep_ev_stride].first;
      e1 = P->sweep_ev[c / P->sweep_ev_stride].second;
    }
    if (P->sweep_ev_next == P->sweep_ev.size() * P->sweep_ev_stride) {
      P->sweep_ev.clear();
      P->sweep_ev_next = 0;
    }
  }
  if (P->transform == ODP_DFT_SPLIT_BF16) {
    ODP_HIP(launch_sweep_dft(P->p, a, DftTable{P->W_<uint16_t>(P->ws.dft)}, s, e0, e1));
  } else {
    ODP_HIP(launch_sweep(P->p, a, s, e0, e1));
  }
  return ODP_OK;
}

int odp_plan_set_sweep_events(odp_plan* P, const hipEvent_t* start, const hipEvent_t* stop, int32_t n,
                              int32_t stride) {
  if (!P) return fail(ODP_EINVAL, "null argument");
  if (n < 0) return fail(ODP_EINVAL, "negative event count");
  if (stride < 1) return fail(ODP_EINVAL, "stride must be at least 1");
  if (n > 0 && (!start || !stop)) return fail(ODP_EINVAL, "null event array");
  for (int32_t i = 0; i < n; ++i)
    if (!start[i] || !stop[i]) return fail(ODP_EINVAL, "null event");
  P->sweep_ev.clear();
  for (int32_t i = 0; i < n; ++i) P->sweep_ev.emplace_back(start[i], stop[i]);
  P->sweep_ev_next = 0;
  P->sweep_ev_stride = (size_t)stride;
  return ODP_OK;
}

int odp_blind_initial_probe(const odp_plan* P, odp_c32* w_out, hipStream_t s) {
  if (!P || !w_out) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp || !P->sqrt_f) return fail(ODP_EINVAL, "plan is not bound");
  const size_t pp = (size_t)P->p * P->p;
  for (int i = 0; i < P->n_probes(); ++i) {
    const odp_plan::Entry& e = P->batch[i];
    InitProbeArgs a;
    a.sqrt_f = P->sqrt_f + (size_t)e.J0 * pp;
    a.J = e.J;
    a.p = P->p;
    a.n_chunks = std::min(LOSS_CHUNKS, std::max(1, e.J));
    a.frames_per_chunk = (e.J + a.n_chunks - 1) / a.n_chunks;
    a.n_chunks = (e.J + a.frames_per_chunk - 1) / a.frames_per_chunk;
    a.part = P->W_<double>(P->ws.wpart);   // 2 p^2 LOSS_CHUNKS doubles: room for every chunk
    a.w = reinterpret_cast<float2*>(w_out) + i * pp;
    a.tw = P->W_<float2>(P->ws.tw);
    ODP_HIP(launch_init_probe(a, s));
  }
  return ODP_OK;
}

int odp_blind_initial_probe_static(const float* dev_sqrt_f, int32_t J, int32_t p, odp_c32* w_out,
                                   hipStream_t s) {
  if (!dev_sqrt_f || !w_out) return fail(ODP_EINVAL, "null argument");
  if (J < 1) return fail(ODP_EINVAL, "J must be at least 1");
  if (p > STATIC_MAXP)
    return fail(ODP_ENOMEM, "p = " + std::to_string(p) + " exceeds the static scratch (p <= " +
                                std::to_string(STATIC_MAXP) + ")");
  if (p != 32 && p != 64 && p != 128) return fail(ODP_EUNSUPPORTED, "p must be 32, 64 or 128");
  if (!static_scratch_fits(J, p)) return fail(ODP_ENOMEM, "the problem exceeds the static scratch");
  ODP_HIP(launch_init_probe_static(dev_sqrt_f, J, p, reinterpret_cast<float2*>(w_out), s));
  return ODP_OK;
}

int odp_probe_update(odp_plan* P, void* dev_state, hipStream_t s) {
  if (!P || !dev_state) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp) return fail(ODP_EINVAL, "plan is not bound");
  if (!P->blind) return fail(ODP_EINVAL, "plan is not blind");
  char* b = static_cast<char*>(dev_state);
  ProbeArgs a;
  a.u = reinterpret_cast<const float2*>(b + P->st.u_sub);
  a.phi = P->W_<float2>(P->ws.psi);
  a.frames = P->W_<FrameDesc>(P->ws.frames);
  a.order = P->W_<int32_t>(P->ws.order);
  a.fpos = P->W_<FrameDesc>(P->ws.fpos);
  a.sub_first = P->W_<int32_t>(P->ws.sub_first);
  a.D = P->D;
  a.p = P->p;
  a.w = reinterpret_cast<float2*>(b + P->st.w);
  a.w_sub = reinterpret_cast<float2*>(b + P->st.w_sub);
  a.delta = reinterpret_cast<float2*>(b + P->st.delta);
  a.fmask = P->fmask.empty() ? nullptr : P->W_<float>(P->ws.fmask);
  a.tw = P->W_<float2>(P->ws.tw);
  a.eta = P->eta;
  a.mu = P->mu;
  a.stop = P->stopping() ? reinterpret_cast<const StopStatus*>(b + P->st.stop) : nullptr;
  a.stream = P->stream;
  ODP_HIP(launch_probe_update(a, s));
  return ODP_OK;
}

int odp_pixel_update(odp_plan* P, void* dev_state, double* dev_stats, hipStream_t s) {
  if (!P || !dev_state) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp) return fail(ODP_EINVAL, "plan is not bound");
  char* b = static_cast<char*>(dev_state);
  const PixelArgs pa = pixel_args(P, b, dev_stats);
  ODP_HIP(launch_pixel(pa, pa.part != nullptr, P->blind != 0, s));
  if (dev_stats) {
    int rc = finish_stats(P, dev_stats, s);
    if (rc) return rc;
  }
  if (P->stop_check(b)) {
    StopArgs sa;
    sa.n_add = P->stop_every;
    sa.frame_part = P->W_<double>(P->ws.fpart);
    sa.sub_sums = nullptr;
    sa.prob = P->W_<int32_t>(P->ws.prob);
    sa.sum_sf = P->W_<double>(P->ws.pmax) + 1;
    sa.sum_sf_stride = 2 + 2048;
    sa.n = P->n_probes();
    sa.measure = P->stop_measure;
    sa.max_iter = P->stop_max_iter;
    sa.tol = P->stop_tol;
    sa.status = reinterpret_cast<StopStatus*>(b + P->st.stop);
    ODP_HIP(launch_stop_check(sa, P->W_<double>(P->ws.tpart), P->W_<int32_t>(P->ws.re_list),
                              P->W_<int32_t>(P->ws.re_first), P->D, P->W_<double>(P->ws.stat_scratch), s));
  }
  if (P->stopping()) ++P->stop_count[b];
  return ODP_OK;
}

int odp_plan_set_balancing(odp_plan* P, double mu, double tau, int32_t period, int32_t until, int32_t which) {
  if (!P) return fail(ODP_EINVAL, "null argument");
  if (period < 0 || until < 0) return fail(ODP_EINVAL, "negative period or limit");
  if (period > 0 && !(mu >= 1.0 && tau > 1.0 && std::isfinite(tau)))
    return fail(ODP_EINVAL, "need mu >= 1 and a finite tau > 1");
  if (period > 0 && (which < 1 || which > (ODP_BALANCE_R | ODP_BALANCE_ETA)))
    return fail(ODP_EINVAL, "which must select r, eta or both");
  if (period > 0 && (which & ODP_BALANCE_ETA) && P->blind)
    return fail(ODP_EUNSUPPORTED, "eta balancing is for known-probe plans");
  P->bal_which = which;
  P->bal_period = period;
  P->bal_until = until;
  P->bal_mu = mu;
  P->bal_tau = tau;
  P->bal_count = 0;
  return ODP_OK;
}

int odp_plan_set_stopping(odp_plan* P, int32_t measure, double tol, int32_t max_iter, int32_t every) {
  if (!P) return fail(ODP_EINVAL, "null argument");
  if (measure < ODP_STOP_NONE || measure > ODP_STOP_RE) return fail(ODP_EINVAL, "unknown stopping measure");
  if (measure != ODP_STOP_NONE && !(tol >= 0.0)) return fail(ODP_EINVAL, "tolerance must be non-negative");
  if (max_iter < 0) return fail(ODP_EINVAL, "negative iteration cap");
  if (every < 1) return fail(ODP_EINVAL, "the check interval must be at least 1");
  P->stop_measure = measure;
  P->stop_tol = measure != ODP_STOP_NONE ? tol : 0.0;
  P->stop_max_iter = max_iter;
  P->stop_every = every;
  P->stop_count.clear();
  return ODP_OK;
}

int odp_state_get_stop_status(const odp_plan* P, const void* dev_state, odp_stop_status* out, hipStream_t s) {
  if (!P || !dev_state || !out) return fail(ODP_EINVAL, "null argument");
  static_assert(sizeof(odp_stop_status) == sizeof(StopStatus), "stop status layout");
  ODP_HIP(hipMemcpyAsync(out, static_cast<const char*>(dev_state) + P->st.stop,
                         sizeof(StopStatus) * P->n_probes(), hipMemcpyDeviceToHost, s));
  ODP_HIP(hipStreamSynchronize(s));
  return ODP_OK;
}

int odp_admm_iterate(odp_plan* P, void* dev_state, int32_t n_iter, double* dev_stats, hipStream_t s) {
  if (!P || !dev_state) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp) return fail(ODP_EINVAL, "plan is not bound");
  if (n_iter < 0) return fail(ODP_EINVAL, "negative iteration count");
  for (int it = 0; it < n_iter; ++it) {
    double* st = dev_stats ? dev_stats + 3 * (size_t)it : nullptr;
    int rc = odp_frame_sweep(P, dev_state, st, s);
    if (!rc && P->blind) rc = odp_probe_update(P, dev_state, s);
    if (!rc) rc = odp_pixel_update(P, dev_state, st, s);
    if (rc) return rc;
    if (P->balancing()) {
      ++P->bal_count;
      if (P->bal_count % P->bal_period == 0 && (P->bal_until == 0 || P->bal_count <= P->bal_until)) {
        rc = balance_penalties(P, static_cast<char*>(dev_state), s);
        if (rc) return rc;
      }
    }
  }
  return ODP_OK;
}

int odp_merge(const odp_plan* P, const void* dev_state, odp_c32* u_out, hipStream_t s) {
  if (!P || !dev_state || !u_out) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp) return fail(ODP_EINVAL, "plan is not bound");
  const char* b = static_cast<const char*>(dev_state);
  ODP_HIP(launch_merge(reinterpret_cast<const float2*>(b + P->st.u_sub), P->W_<int32_t>(P->ws.rects),
                       P->W_<int64_t>(P->ws.usub_off), P->D, P->H, P->W, reinterpret_cast<float2*>(u_out), s));
  return ODP_OK;
}

int odp_amp_loss(const odp_plan* P, const odp_c32* u, const odp_c32* w, double* loss_out, odp_c32* grad_u,
                 odp_c32* grad_w, hipStream_t s) {
  if (!P || !u || !w || !loss_out) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp) return fail(ODP_EINVAL, "plan is not bound");
  const bool grad = grad_u || grad_w;
  LossArgs la;
  la.u = reinterpret_cast<const float2*>(u);
  la.H = P->H;
  la.W = P->W;
  la.w = reinterpret_cast<const float2*>(w);
  la.tw = P->W_<float2>(P->ws.tw);
  la.sqrt_f = P->sqrt_f;
  la.offsets = P->W_<int32_t>(P->ws.offsets);
  la.J = P->J;
  la.frame_loss = P->W_<double>(P->ws.fpart);
  la.phi = P->W_<float2>(P->ws.psi);
  ODP_HIP(launch_loss(P->p, la, grad, s));
  if (!grad) {
    ODP_HIP(launch_loss_total(la.frame_loss, P->J, loss_out, s));
    return ODP_OK;
  }
  // pixels in no tile are covered by no frame: their gradient is 0 (the tiles write the rest)
  if (grad_u && P->covered < (int64_t)P->H * P->W)
    ODP_HIP(launch_fill(reinterpret_cast<float2*>(grad_u), (int64_t)P->H * P->W, make_float2(0.f, 0.f), s));
  LossGradArgs ga;
  ga.u = la.u;
  ga.W = P->W;
  ga.w = la.w;
  ga.phi = la.phi;
  ga.offsets = la.offsets;
  ga.J = P->J;
  ga.p = P->p;
  ga.cells = P->W_<CellDesc>(P->ws.cells);
  ga.tiles = P->W_<TileDesc>(P->ws.tiles);
  ga.n_tiles = (int32_t)P->tset().tiles.size();
  ga.tile_cols = P->tset().cols;
  ga.tf_first = P->W_<int32_t>(P->ws.tf_first);
  ga.pull = P->W_<PullEntry>(P->ws.pull);
  ga.pairs = P->pairs_on && P->tset().pairs ? 1 : 0;
  ga.grad_u = reinterpret_cast<float2*>(grad_u);
  ga.grad_w = reinterpret_cast<float2*>(grad_w);
  ga.wpart = P->W_<double>(P->ws.wpart);
  ga.frames_per_chunk = (P->J + LOSS_CHUNKS - 1) / LOSS_CHUNKS;
  ga.n_chunks = (P->J + ga.frames_per_chunk - 1) / ga.frames_per_chunk;
  ga.frame_loss = la.frame_loss;   // the loss total is summed with the probe gradient
  ga.loss_out = loss_out;
  ODP_HIP(launch_loss_grads(ga, s));
  return ODP_OK;
}

// ---- tuning -----------------------------------------------------------------

int odp_plan_get_tuning(const odp_plan* P, odp_tuning* o) {
  if (!P || !o) return fail(ODP_EINVAL, "null argument");
  o->transform = P->transform;
  o->xcd_slice = P->xcd_slice;
  o->tiling = P->ts;
  o->tile_rows = P->tset().rows;
  o->tile_cols = P->tset().cols;
  o->ms_per_iter = 0.0;
  o->n_tried = 0;
  o->pixel_pairs = P->pairs_on && P->tset().pairs ? 1 : 0;
  return ODP_OK;
}

int odp_plan_set_tuning(odp_plan* P, int32_t transform, int32_t xcd_slice, int32_t tiling, hipStream_t s) {
  if (!P) return fail(ODP_EINVAL, "null argument");
  const int rc = check_transform(transform, P->p);
  if (rc) return rc;
  if (tiling < 0 || tiling > 2) return fail(ODP_EINVAL, "tiling must be 0, 1 or 2");
  if (xcd_slice < 0 || xcd_slice > 2) return fail(ODP_EINVAL, "xcd_slice must be 0, 1 or 2");
  if (transform != P->transform || xcd_slice != P->xcd_slice || tiling != P->ts) ++P->gen;
  P->transform = transform;
  const bool moved = tiling != P->ts || (xcd_slice == 2) != (P->xcd_slice == 2);
  P->xcd_slice = xcd_slice;
  P->ts = tiling;
  if (moved && P->wsp) return upload_tiles(P, s);
  return ODP_OK;
}

int odp_plan_set_streaming(odp_plan* P, int32_t mode) {
  if (!P) return fail(ODP_EINVAL, "null argument");
  if (mode < -1 || mode > 1) return fail(ODP_EINVAL, "streaming mode must be -1, 0 or 1");
  const int32_t st = mode < 0 ? stream_by_size(P) : mode;
  if (st != P->stream) ++P->gen;
  P->stream = st;
  return ODP_OK;
}

int odp_plan_set_pixel_pairs(odp_plan* P, int32_t mode) {
  if (!P) return fail(ODP_EINVAL, "null argument");
  if (mode < 0 || mode > 1) return fail(ODP_EINVAL, "pixel pairs mode must be 0 or 1");
  if (mode != P->pairs_on) ++P->gen;
  P->pairs_on = mode;
  return ODP_OK;
}

int odp_plan_autotune(odp_plan* P, void* dev_scratch_state, int32_t iters, hipStream_t s, odp_tuning* best) {
  if (!P || !dev_scratch_state) return fail(ODP_EINVAL, "null argument");
  if (!P->wsp) return fail(ODP_EINVAL, "plan is not bound");
  if (iters < 1) iters = 1;
  std::vector<int> transforms = {P->transform};
  if (P->p == 64) transforms = {ODP_FFT_F32, ODP_DFT_SPLIT_BF16, ODP_HYBRID_MFMA};
  if (P->p == 128) transforms = {ODP_FFT_F32, ODP_HYBRID_MFMA};
  hipEvent_t e0, e1;
  ODP_HIP(hipEventCreate(&e0));
  ODP_HIP(hipEventCreate(&e1));
  double best_ms = 1e300;
  int bt = P->transform, bx = P->xcd_slice, bs = P->ts, tried = 0;
  int rc = ODP_OK;
  // time whole iterations: no problem of the scratch state may stop early
  const int32_t sm = P->stop_measure, smax = P->stop_max_iter, bp = P->bal_period;
  P->stop_measure = ODP_STOP_NONE;
  P->stop_max_iter = 0;
  P->bal_period = 0;
  for (int tr : transforms) {
    for (int xs = 2; xs >= 0 && !rc; --xs) {
      for (int ts = 0; ts < 3 && !rc; ++ts) {
        rc = odp_plan_set_tuning(P, tr, xs, ts, s);
        if (!rc) rc = odp_admm_iterate(P, dev_scratch_state, 2, nullptr, s);  // warm-up
        if (rc) break;
        if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(ODP_EHIP, "hipEventRecord"); break; }
        rc = odp_admm_iterate(P, dev_scratch_state, iters, nullptr, s);
        if (rc) break;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = fail(ODP_EHIP, "event timing failed");
          break;
        }
        ++tried;
        const double per = (double)ms / iters;
        // a later setting must be faster by more than the timing noise of a few
        // iterations (1 %): within it the earlier one is kept, so the choice is stable
        // and favours the XCD-aware placements (tried first), which read less from HBM
        if (per < best_ms * 0.99) {
          best_ms = per;
          bt = tr;
          bx = xs;
          bs = ts;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->stop_measure = sm;
  P->stop_max_iter = smax;
  P->bal_period = bp;
  if (rc) return rc;
  rc = odp_plan_set_tuning(P, bt, bx, bs, s);
  if (rc) return rc;
  if (best) {
    odp_plan_get_tuning(P, best);
    best->ms_per_iter = best_ms;
    best->n_tried = tried;
  }
  return ODP_OK;
}

// ---- graphs -------------------------------------------------------------------

}  // extern "C"

struct odp_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<std::pair<const odp_plan*, uint64_t>> plans;   // each plan's generation at capture
};

extern "C" {

int odp_graph_create(odp_plan* const* plans, void* const* states, int32_t n, int32_t n_iter, odp_graph** out) {
  if (!plans || !states || !out || n < 1 || n_iter < 1) return fail(ODP_EINVAL, "bad graph arguments");
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (!plans[i] || !states[i] || !plans[i]->wsp) return fail(ODP_EINVAL, "unbound plan or null state");
  for (int i = 0; i < n; ++i) {
    if (plans[i]->balancing())
      return fail(ODP_EUNSUPPORTED, "penalty balancing reads residuals on the host: not in a graph");
    if (plans[i]->stopping() && n_iter % plans[i]->stop_every != 0)
      return fail(ODP_EINVAL, "n_iter must be a multiple of the stopping check interval");
  }
  // One capture stream forks into one stream per distinct plan (pairs of one plan share
  // its workspace and stay on one branch, in the given order): distinct plans touch
  // disjoint memory, so the graph holds independent chains of n_iter iterations that the
  // runtime may run side by side, joined at the end.
  std::vector<int> branch(n);
  int nb = 0;
  for (int i = 0; i < n; ++i) {
    branch[i] = -1;
    for (int k = 0; k < i; ++k) {
      if (plans[k] == plans[i]) branch[i] = branch[k];
      else if (states[k] == states[i]) return fail(ODP_EINVAL, "two plans share one state");
      if (states[k] == states[i] && plans[k] == plans[i]) return fail(ODP_EINVAL, "repeated (plan, state) pair");
    }
    if (branch[i] < 0) branch[i] = nb++;
  }
  std::vector<hipStream_t> ss(nb + 1, nullptr);
  std::vector<hipEvent_t> ev(nb + 1, nullptr);
  auto cleanup = [&]() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t q : ss)
      if (q) (void)hipStreamDestroy(q);
  };
  for (int b = 0; b <= nb; ++b) {
    if (hipStreamCreateWithFlags(&ss[b], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev[b], hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return fail(ODP_EHIP, "stream or event creation failed");
    }
  }
  hipStream_t cs = ss[nb];
  int rc = ODP_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    cleanup();
    return fail(ODP_EHIP, "hipStreamBeginCapture failed");
  }
  if (hipEventRecord(ev[nb], cs) != hipSuccess) rc = fail(ODP_EHIP, "fork event failed");
  for (int b = 0; b < nb && !rc; ++b) {
    if (hipStreamWaitEvent(ss[b], ev[nb], 0) != hipSuccess) {
      rc = fail(ODP_EHIP, "fork wait failed");
      break;
    }
    for (int it = 0; it < n_iter && !rc; ++it)
      for (int i = 0; i < n && !rc; ++i)
        if (branch[i] == b) rc = odp_admm_iterate(plans[i], states[i], 1, nullptr, ss[b]);
    if (!rc && (hipEventRecord(ev[b], ss[b]) != hipSuccess || hipStreamWaitEvent(cs, ev[b], 0) != hipSuccess))
      rc = fail(ODP_EHIP, "join failed");
  }
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &g);
  cleanup();
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (ec != hipSuccess || !g) return fail(ODP_EHIP, "hipStreamEndCapture failed");
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(ODP_EHIP, "hipGraphInstantiate failed");
  }
  odp_graph* G = new (std::nothrow) odp_graph();
  if (!G) {
    (void)hipGraphExecDestroy(ex);
    (void)hipGraphDestroy(g);
    return fail(ODP_ENOMEM, "host allocation failed");
  }
  G->graph = g;
  G->exec = ex;
  for (int i = 0; i < n; ++i) G->plans.emplace_back(plans[i], plans[i]->gen);
  *out = G;
  return ODP_OK;
}

int odp_graph_launch(odp_graph* G, hipStream_t s) {
  if (!G) return fail(ODP_EINVAL, "null graph");
  for (const auto& pg : G->plans)
    if (pg.first->gen != pg.second)
      return fail(ODP_EINVAL, "stale graph: a plan's penalties, tuning or binding changed after capture; "
                              "create the graph again");
  ODP_HIP(hipGraphLaunch(G->exec, s));
  return ODP_OK;
}

void odp_graph_destroy(odp_graph* G) {
  if (!G) return;
  if (G->exec) (void)hipGraphExecDestroy(G->exec);
  if (G->graph) (void)hipGraphDestroy(G->graph);
  delete G;
}

}  // extern "C"

// odp_internal.hpp -- structures shared by the host plan code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace odp {

constexpr int MAXS = 16;                       // most subdomains over one pixel
constexpr int MAXP = MAXS * (MAXS - 1) / 2;    // most pairs over one pixel
constexpr int NPX = 2;                          // pixels per thread in the pixel-tile kernels
constexpr int PULL_B = 4;                       // pull records per group (lists padded to a multiple)
constexpr int NPS = 8;                          // pixel-update statistics per (tile, copy slot)
constexpr int NFS = 4;                          // frame-sweep statistics per frame
constexpr int NRES = 8;                         // penalty-rule residual sums per problem (launch_residual_sums)
constexpr int NXCD = 8;                        // MI355X accelerator complex dies

// A cell is a rectangle of image pixels covered by the same set of subdomains
// (the cuts are the subdomain rectangle edges).  k_d = m - 1 on the whole cell.
struct CellDesc {
  int32_t m;                 // number of subdomains covering the cell
  int32_t npair;             // m (m - 1) / 2
  int32_t r0, c0;            // top-left pixel in the image
  float r;                   // overlap penalty of the problem the cell belongs to
  int32_t probe;             // probe index of that problem
  int32_t nr, nc;            // extent (rows, columns)
  int32_t sub[MAXS];         // subdomain ids, ascending
  int32_t upitch[MAXS];      // row pitch of each subdomain array
  int64_t ubase[MAXS];       // u_sub index of the cell's top-left in each subdomain
  int64_t lbase[MAXP];       // lam index of the top-left in Lam_{a,b}; Lam_{b,a} is lstride later
  int64_t lstride[MAXP];
  int32_t lpitch[MAXP];
  int8_t pa[MAXP], pb[MAXP]; // positions in sub[] of the pair's subdomains (pa < pb)
};

struct TileDesc {
  int32_t cell;
  int32_t r0, c0;            // relative to the cell's top-left
  int32_t nr, nc;
  int32_t pad[3];
};

// One covering frame of a pixel tile: psi index of pixel (y, x) of the image is
// base + y*p + x (base = j*p*p - row_j*p - col_j); the window is rows
// [row_j, row_j + p) and columns [col_j, col_j + p).  Padding records have
// base 0 and r = c = PULL_NONE, a window that holds no pixel.
struct PullEntry {
  int64_t base;
  int32_t r, c;
};
constexpr int32_t PULL_NONE = -(1 << 29);

struct FrameDesc {
  int64_t base;              // u_sub index of the window's top-left inside its subdomain
  int32_t pitch;             // row pitch of that subdomain
  int32_t sub;               // subdomain id
  int32_t probe;             // probe index (one probe per problem of a batch)
  int32_t j;                 // frame id
};

// Per-problem progress under a stopping rule (Sec. 4), kept in the state buffer;
// layout identical to odp_stop_status.
struct StopStatus {
  int32_t iters;             // iterations run
  int32_t stopped;           // 1 once the rule or the iteration cap was met
  double rf, re, g;          // measures of the last iteration run
};
static_assert(sizeof(StopStatus) == 32, "StopStatus layout");

// ---------------------------------------------------------------- launch args
struct SweepArgs {
  int32_t stream;            // 1: non-temporal accesses to the frame arrays (see ld_s)
  const float2* u;           // u_sub
  const float2* w;           // probe [p][p] (non-blind) or copies [D][p][p] (blind)
  const float2* w_out;       // the same probe, read again for the output multiply
  int w_per_sub;             // 1: w indexed by subdomain (blind)
  const float2* tw;          // twiddle table W_p^{i k}, [p/16][16]
  const uint4* mft;          // hybrid transform: split-BF16 radix-16 matrices (fft_mfma.hpp), else null
  float2* gamma;             // [J][p][p]
  const float* sqrt_f;       // [J][p][p]
  const FrameDesc* frames;
  const int32_t* order;      // frame processing order (grouped by subdomain)
  const FrameDesc* fpos;     // frames[order[pos]] by position pos (one load per frame)
  int32_t J, chunk;          // frames, frames per XCD slice
  int32_t xcd_slice;         // 1: workgroup b takes slice b % 8 of the order; 0: order[b]
  float eps, eta;
  float gcoef;               // (1 - eps) / (2 eps), the measures' truncated g_eps branch
  double* part;              // [J][NFS] statistics (L1 misfit, G_eps, |Gamma^{n+1} - Gamma^n|^2,
                             //   |Gamma^{n+1}|^2) or null
  float2* psi;               // [J][p][p] per-frame output, natural spatial layout:
                             //   non-blind conj(w) o F^{-1}(z - Gamma), blind F^{-1}(z - Gamma)
  int blind;
  int frame_res;             // 1: the statistics also sum the frame residuals (penalty rule)
  const StopStatus* stop;    // [n_problems] or null: frames of stopped problems are skipped
};

// One wavefront's share of a pixel-update tile whose cell has at most four copies
// per pixel: its copy slot s and every index at the tile's top-left pixel (partner o
// is copy t = o + (o >= s)), so a wavefront reads its whole descriptor in one
// scalar round trip, with no loads that depend on other loads.
struct WaveRec {
  int32_t s, m, lg, lcw;     // slot, copies, log2 copy groups, log2 tile width
  int32_t nr, nc;            // tile extent
  int32_t yi0, xi0;          // image coordinates of the top-left
  int32_t k0, k1;            // pull records [k0, k1) of copy s
  int32_t sub;               // subdomain of copy s
  float r;                   // overlap penalty
  int64_t u0;                // u_sub index of the top-left, copy s
  int64_t pu0[3];            // ... partner copies
  int64_t lo0[3];            // Lam_{s,t} index of the top-left (written by this copy)
  int64_t lt0[3];            // Lam_{t,s} index of the top-left
  int32_t upitch, pupitch[3], lpitch[3];
  int32_t prob;              // problem of the tile (batch index; 0 for a single problem)
};
static_assert(sizeof(WaveRec) == 160, "WaveRec layout");

struct PixelArgs {
  int32_t stream;            // 1: non-temporal reads of the handoff
  float2* u;                 // u_sub (updated in place)
  const float* rcp;          // 1 / (eta den + r k + gamma); 0 = held pixel (non-blind)
  float2* lam;
  const CellDesc* cells;
  const TileDesc* tiles;
  int32_t n_tiles, p, tile_cols;
  int32_t n_uni;             // tiles [0, n_uni) belong to cells with at most 4 copies,
  int32_t n_mid;             // [n_uni, n_mid) to cells with 5 to 8, the rest to 9 to MAXS
  const WaveRec* waves;      // [n_uni][4]
  int32_t pairs;             // 1: in every tile [0, n_uni) the pull records' column origins
                             // have the parity of the tile's left column, so a thread's two
                             // row neighbours take one 16-byte load per record
  const float2* psi;         // per-frame outputs of the sweep
  const int32_t* tf_first;   // [n_tiles*MAXS + 1]: frames of slot s overlapping tile t
  const PullEntry* pull;     // their records, ascending frame id
  const float2* w_sub;       // blind: probe copies (the illumination is formed in the pull)
  float eta, gamma;          // (r is per cell)
  double* part;              // [n_tiles][MAXS][NPS] statistics (pixel_stats) or null
  const double* dend;        // [p_sub] den (non-blind; the statistics weight |u|^2 by it)
  const StopStatus* stop;    // [n_problems] or null: tiles of stopped problems are skipped
};

struct IllumArgs {           // den and rcp on every subdomain pixel
  const float2* w;           // probes [n_probes][p][p] (indexed by the cell's probe)
  const int32_t* tf_first;   // per-tile frame lists (as in PixelArgs)
  const PullEntry* pull;
  const CellDesc* cells;
  const TileDesc* tiles;
  int32_t n_tiles, p, tile_cols;
  double* den;               // [p_sub]
  float* rcp;                // [p_sub]
  double eta, gamma;         // (r is per cell)
  int recompute_den;         // 0: reuse den, only rebuild rcp
};

hipError_t launch_sweep(int p, const SweepArgs& a, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Split-BF16 DFT matrix for the MFMA sweep: planes [re hi, re lo, im hi, im lo] of
// F[k][n] = exp(-2 pi i k n / p) / sqrt(p), each [p][p] bf16 bit patterns.
struct DftTable {
  const uint16_t* f;
};
// ev0/ev1: if non-null, recorded at the kernel's start and end (hipExtLaunchKernelGGL)
hipError_t launch_sweep_dft(int p, const SweepArgs& a, const DftTable& dt, hipStream_t s, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr);
hipError_t launch_pixel(const PixelArgs& a, bool stats, bool blind, hipStream_t s);
hipError_t launch_illum(const IllumArgs& a, hipStream_t s);
hipError_t launch_forward(int p, const float2* u, int H, int W, const float2* w, const float2* tw,
                          const int32_t* offsets, int J, float2* out, hipStream_t s);
hipError_t launch_adjoint(int p, const float2* frames, const float2* w, const float2* tw,
                          const int32_t* offsets, int J, float2* u_out, int H, int W, hipStream_t s);
hipError_t launch_prox(const float2* y, const float* sf, int64_t n, float eps, float lam, float2* z,
                       hipStream_t s);
hipError_t launch_fill(float2* p, int64_t n, float2 value, hipStream_t s);
hipError_t launch_sum_max(const double* x, int64_t n, const float* y, int64_t ny, double* out,
                          hipStream_t s);
hipError_t launch_stats(const double* frame_part, int J, const double* tile_part,
                        const int32_t* re_list, const int32_t* re_first, int D, const double* sum_sf,
                        double* out3, double* scratch, hipStream_t s);
hipError_t launch_merge(const float2* u_sub, const int32_t* rects, const int64_t* usub_off, int D,
                        int H, int W, float2* out, hipStream_t s);
hipError_t launch_copy(float2* dst, const float2* src, int64_t n, hipStream_t s);

// blind (Alg. 3) probe steps
struct ProbeArgs {
  int32_t stream;            // 1: non-temporal reads of the handoff
  const float2* u;           // u_sub (iterate n)
  const float2* phi;         // F^{-1}(Z - Gamma) per frame
  const FrameDesc* frames;
  const int32_t* order;      // frames grouped by subdomain
  const FrameDesc* fpos;     // frames[order[q]] by position q (one load per frame)
  const int32_t* sub_first;  // [D+1]
  int32_t D, p;
  float2* w;                 // shared probe w (out: w^{n+1})
  float2* w_sub;             // copies [D][p][p] (in W^n, out W^{n+1})
  float2* delta;             // [D][p][p] (in Delta^n, out Delta^{n+1})
  const float* fmask;        // [p][p] support indicator or null
  const float2* tw;
  double eta, mu;
  const StopStatus* stop;    // [1] or null: nothing is done once the problem has stopped
};
hipError_t launch_probe_update(const ProbeArgs& a, hipStream_t s);

// One iteration's end under a stopping rule: per problem i (one workgroup each, skipped
// once stopped) RF_i from its frames' partials and its sum of sqrt f, RE_i as the max
// over its subdomains of sqrt(|du|^2 / |u|^2), G_i; then iters_i += 1 and the rule.
struct StopArgs {
  const double* frame_part;  // [J][NFS] of the sweep
  const double* sub_sums;    // [D][2] (|du|^2, |u|^2) per subdomain (k_stats_reduce)
  const int32_t* prob;       // [n][4] = (J0, J, D0, D)
  const double* sum_sf;      // problem i's sum of sqrt f at sum_sf[i * sum_sf_stride]
  int32_t sum_sf_stride, n;
  int32_t measure;           // 0 none, 1 RF, 2 RE
  int32_t max_iter;          // 0: no cap
  int32_t n_add;             // iterations since the previous check
  double tol;
  StopStatus* status;        // [n]
};
hipError_t launch_stop_check(const StopArgs& a, const double* tile_part, const int32_t* re_list,
                             const int32_t* re_first, int D, double* scratch, hipStream_t s);

// Residual sums for the penalty rule, NRES per problem: out[NRES i + k], k < 6 = the sums
// over problem i's subdomains (from the per-subdomain statistics reduction in scratch) of
// (|Lam^{n+1} - Lam^n|^2, (m-1)|du|^2, (m-1)|u^{n+1}|^2, |Lam^{n+1}|^2, den |u^n|^2,
// den |du|^2); k = 6, 7 = the sums over problem i's frames of |Gamma^{n+1} - Gamma^n|^2 and
// |Gamma^{n+1}|^2.  out holds NRES * n doubles.
hipError_t launch_residual_sums(const double* frame_part, int J, const double* tile_part, const int32_t* re_list,
                                const int32_t* re_first, int D, const int32_t* prob, int n, double* scratch,
                                double* out, hipStream_t s);
hipError_t launch_scale(float2* x, int64_t n, float f, hipStream_t s);

struct InitProbeArgs {       // w0 = (1/J) sum_j F^{-1}(sqrt f_j) of one problem
  const float* sqrt_f;       // [J][p][p] of the problem's frames
  int32_t J, p;
  int32_t frames_per_chunk, n_chunks;
  double* part;              // [n_chunks][p][p] partial sums
  float2* w;                 // [p][p] out
  const float2* tw;          // twiddle table of p
};
hipError_t launch_init_probe(const InitProbeArgs& a, hipStream_t s);

// The initial probe from the amplitudes alone, its scratch in a static device array:
// at most STATIC_CHUNKS frame chunks of p x p FP64 partial sums plus the twiddle table,
// for p <= STATIC_MAXP (4 MiB + 1 KiB per device).
constexpr int STATIC_CHUNKS = 32;
constexpr int STATIC_MAXP = 128;
constexpr size_t STATIC_SCRATCH_DOUBLES = (size_t)STATIC_CHUNKS * STATIC_MAXP * STATIC_MAXP + STATIC_MAXP;
bool static_scratch_fits(int J, int p);
hipError_t launch_init_probe_static(const float* sqrt_f, int J, int p, float2* w, hipStream_t s);

struct LossArgs {
  const float2* u;           // image [H][W]
  int32_t H, W;
  const float2* w;           // probe [p][p]
  const float2* tw;
  const float* sqrt_f;       // [J][p][p]
  const int32_t* offsets;    // [J][2]
  int32_t J;
  double* frame_loss;        // [J]
  float2* phi;               // [J][p][p] F^{-1} g_j, natural spatial layout
};

struct LossGradArgs {
  const float2* u;
  int32_t W;
  const float2* w;
  const float2* phi;
  const int32_t* offsets;
  int32_t J, p;
  const CellDesc* cells;
  const TileDesc* tiles;
  int32_t n_tiles, tile_cols;
  const int32_t* tf_first;
  const PullEntry* pull;
  int32_t pairs;             // 1: row-neighbour pixel pairs (as PixelArgs::pairs)
  float2* grad_u;            // [H][W] or null
  float2* grad_w;            // [p][p] or null
  double* wpart;             // [n_chunks][p][p][2]
  int32_t n_chunks, frames_per_chunk;
  const double* frame_loss;  // [J] per-frame loss terms, summed into loss_out by the last
  double* loss_out;          //   workgroup of the probe gradient's final sum (or null)
};

hipError_t launch_loss(int p, const LossArgs& a, bool grad, hipStream_t s);
hipError_t launch_loss_total(const double* frame_loss, int J, double* out, hipStream_t s);
hipError_t launch_loss_grads(const LossGradArgs& a, hipStream_t s);

}  // namespace odp

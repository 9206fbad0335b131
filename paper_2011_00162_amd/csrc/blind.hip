// blind.hip -- probe steps of OD2BP (Algorithm 3 of the paper, Sec. 3.2).
//
//  w^{n+1}   = P_O( (1/D) sum_d (w_d^n + Delta_d^n) )                  (eq. blind_w, 1/D for D copies)
//  w_d^{n+1} = (eta sum_{j in d} conj(S_j u_d^n) o phi_j + mu (w^{n+1} - Delta_d^n))
//              / (eta sum_{j in d} |S_j u_d^n|^2 + mu)                 (eq. blind_W)
//  Delta_d^{n+1} = Delta_d^n + w_d^{n+1} - w^{n+1}                     (eq. admm_Delta)
// with phi_j = F^{-1}(Z_j - Gamma_j) from the frame sweep and P_O = F^{-1} M F the
// projection onto probes whose spectrum vanishes off the support mask M.
// The frame sums run in FP64 in a fixed order (ascending over the frames of a subdomain),
// so repeated runs agree bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "fft_frame.hpp"
#include "odp_internal.hpp"

namespace odp {

// (1/D) sum_d (w_d + Delta_d) per probe pixel in FP64: the four wavefronts of a workgroup
// take every fourth copy (ascending within each) for the same 64 pixels, and their partial
// sums are added in wavefront order
__global__ __launch_bounds__(256) void k_probe_avg(ProbeArgs a) {
  __shared__ double part[2][4][64];
  if (a.stop && a.stop[0].stopped) return;  // uniform over the workgroup
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const bool ok = k < a.p * a.p;
  const size_t pp = (size_t)a.p * a.p;
  double sx = 0.0, sy = 0.0;
  if (ok) {
#pragma unroll 4
    for (int d = grp; d < a.D; d += 4) {
      const float2 ws = a.w_sub[d * pp + k], dl = a.delta[d * pp + k];
      sx += (double)ws.x + dl.x;
      sy += (double)ws.y + dl.y;
    }
  }
  part[0][grp][lane] = sx;
  part[1][grp][lane] = sy;
  __syncthreads();
  if (grp != 0 || !ok) return;
  sx = ((part[0][0][lane] + part[0][1][lane]) + part[0][2][lane]) + part[0][3][lane];
  sy = ((part[1][0][lane] + part[1][1][lane]) + part[1][2][lane]) + part[1][3][lane];
  const double invD = 1.0 / (double)a.D;
  a.w[k] = make_float2((float)(sx * invD), (float)(sy * invD));
}

// P_O = F^{-1} M F on the averaged probe, in place (one workgroup: every thread reads
// its 16 values before any is written)
template <int P>
__global__ __launch_bounds__(Frame<P>::T) void k_probe_project(ProbeArgs a) {
  using F = Frame<P>;
  __shared__ __align__(16) float2 lds[F::LDS];
  if (a.stop && a.stop[0].stopped) return;  // uniform over the workgroup
  const int t = threadIdx.x;
  const int col = F::a_col(t), r2 = F::a_r2(t);
  float2 v[16];
#pragma unroll
  for (int r1 = 0; r1 < 16; ++r1) v[r1] = a.w[(F::N2 * r1 + r2) * P + col];
  F::forward(v, lds, a.tw, t);
  const float s = 1.0f / (float)(P * P);   // both unitary factors
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    int kr, kc;
    F::freq(t, e, kr, kc);
    v[e] = c_scale(v[e], s * a.fmask[kr * P + kc]);
  }
  __syncthreads();
  F::inverse(v, lds, a.tw, t);
#pragma unroll
  for (int r1 = 0; r1 < 16; ++r1) a.w[(F::N2 * r1 + r2) * P + col] = v[r1];
}

// w_d and Delta_d for 256 probe pixels of subdomain d, one per thread: the sums run over
// the frames of d in ascending order in groups of eight, so that a workgroup reads 2 KB
// contiguous of each frame's phi and of its u window rows.  The next group's loads are
// issued before the current group is summed (two groups in registers), which keeps the
// loads in flight while the FP64 sums run.
template <bool NT>
__global__ __launch_bounds__(256) void k_probe_copies(ProbeArgs a) {
  if (a.stop && a.stop[0].stopped) return;  // uniform over the workgroup
  constexpr int B = 8;
  const int p = a.p, d = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  const bool ok = k < p * p;
  const int kk = ok ? k : 0;
  const int ky = kk / p, kx = kk % p;
  const size_t pp = (size_t)p * p;
  double nr = 0.0, ni = 0.0, den = 0.0;
  auto acc = [&](const float2 pu, const float2 ph) {
    nr += (double)pu.x * ph.x + (double)pu.y * ph.y;   // conj(S_j u) o phi
    ni += (double)pu.x * ph.y - (double)pu.y * ph.x;
    den += (double)pu.x * pu.x + (double)pu.y * pu.y;
  };
  // the loads of frames q .. q + B - 1 (workgroup-uniform descriptors: scalar loads)
  auto load = [&](int q, float2* pu, float2* ph) {
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const FrameDesc f = a.fpos[q + i];
      pu[i] = a.u[f.base + (int64_t)ky * f.pitch + kx];
      ph[i] = ld_s<NT>(a.phi + (size_t)f.j * pp + kk);   // read here and once more by the U-step
    }
  };
  const int q1 = a.sub_first[d + 1];
  int q = a.sub_first[d];
  float2 pu[2][B], ph[2][B];
  if (q + B <= q1) load(q, pu[0], ph[0]);
  for (; q + B <= q1; q += 2 * B) {
    if (q + 2 * B <= q1) load(q + B, pu[1], ph[1]);
#pragma unroll
    for (int i = 0; i < B; ++i) acc(pu[0][i], ph[0][i]);
    if (q + 2 * B > q1) {
      q += B;
      break;
    }
    if (q + 3 * B <= q1) load(q + 2 * B, pu[0], ph[0]);
#pragma unroll
    for (int i = 0; i < B; ++i) acc(pu[1][i], ph[1][i]);
  }
  for (; q < q1; ++q) {
    const FrameDesc fd = a.fpos[q];
    acc(a.u[fd.base + (int64_t)ky * fd.pitch + kx], ld_s<NT>(a.phi + (size_t)fd.j * pp + kk));
  }
  if (!ok) return;
  const size_t o = (size_t)d * pp + k;
  const float2 w = a.w[k], dl = a.delta[o];
  const double qd = a.eta * den + a.mu;
  const double wx = (a.eta * nr + a.mu * ((double)w.x - dl.x)) / qd;
  const double wy = (a.eta * ni + a.mu * ((double)w.y - dl.y)) / qd;
  a.w_sub[o] = make_float2((float)wx, (float)wy);
  a.delta[o] = make_float2((float)((double)dl.x + wx - w.x), (float)((double)dl.y + wy - w.y));
}

// Initial probe of a blind run (Sec. 4, extended tests): w0 = (1/J) sum_j F^{-1}(sqrt f_j).
// F^{-1} is linear, so the amplitudes are summed over the frames first (FP64, frames of a
// chunk in order, then the chunks in order) and one unitary inverse transform follows.
__global__ __launch_bounds__(256) void k_init_part(InitProbeArgs a) {
  const int pp = a.p * a.p, k = blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
  if (k >= pp) return;
  const int j0 = c * a.frames_per_chunk, j1 = min(a.J, j0 + a.frames_per_chunk);
  double s0 = 0.0, s1 = 0.0;   // two interleaved partial sums (even, odd frames), added in order
  int j = j0;
  for (; j + 1 < j1; j += 2) {
    s0 += (double)a.sqrt_f[(size_t)j * pp + k];
    s1 += (double)a.sqrt_f[(size_t)(j + 1) * pp + k];
  }
  if (j < j1) s0 += (double)a.sqrt_f[(size_t)j * pp + k];
  a.part[(size_t)c * pp + k] = s0 + s1;
}

__global__ __launch_bounds__(256) void k_init_final(InitProbeArgs a) {
  const int pp = a.p * a.p, k = blockIdx.x * 256 + threadIdx.x;
  if (k >= pp) return;
  double s = 0.0;
  for (int c = 0; c < a.n_chunks; ++c) s += a.part[(size_t)c * pp + k];
  a.w[k] = make_float2((float)(s / (double)a.J), 0.0f);
}

// in place on w: every thread reads its 16 frequencies before the first barrier of the
// inverse, and writes only after the last
template <int P>
__global__ __launch_bounds__(Frame<P>::T) void k_init_ifft(InitProbeArgs a) {
  using F = Frame<P>;
  __shared__ __align__(16) float2 lds[F::LDS];
  const int t = threadIdx.x;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    int kr, kc;
    F::freq(t, e, kr, kc);
    v[e] = a.w[kr * P + kc];
  }
  F::inverse(v, lds, a.tw, t);
  const int col = F::a_col(t), r2 = F::a_r2(t);
  const float s = 1.0f / (float)P;   // unitary inverse
#pragma unroll
  for (int r1 = 0; r1 < 16; ++r1) a.w[(F::N2 * r1 + r2) * P + col] = c_scale(v[r1], s);
}

hipError_t launch_init_probe(const InitProbeArgs& a, hipStream_t s) {
  const int pp = a.p * a.p;
  hipLaunchKernelGGL(k_init_part, dim3((pp + 255) / 256, a.n_chunks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_init_final, dim3((pp + 255) / 256), dim3(256), 0, s, a);
#define ODP_INIT(PP) \
  if (a.p == PP) hipLaunchKernelGGL((k_init_ifft<PP>), dim3(1), dim3(Frame<PP>::T), 0, s, a);
  ODP_INIT(32)
  ODP_INIT(64)
  ODP_INIT(128)
#undef ODP_INIT
  return hipGetLastError();
}

// ---- the initial probe with no plan and no workspace ------------------------------
// The chunk partial sums ([n_chunks][p][p] FP64) and the twiddle table of p ([p/16][16]
// float2) of launch_init_probe_static live in one file-scope device array.  Each device
// holds its own copy until the process ends; every call on a device shares it and
// leaves its contents behind (each call rewrites all it reads, so nothing needs clearing).
static __device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];

// tw[i][k] = exp(-2 pi i i k / p) for i < p/16, k < 16, from an FP64 sincospi
__global__ __launch_bounds__(128) void k_twiddles(float2* tw, int p) {
  const int t = threadIdx.x;
  if (t >= p) return;
  double s, c;
  sincospi(2.0 * (double)((t / 16) * (t % 16)) / (double)p, &s, &c);
  tw[t] = make_float2((float)c, (float)-s);
}

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device.  In host
// code the array's name is only a stand-in for the device symbol, never an address.
hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}
}  // namespace

bool static_scratch_fits(int J, int p) {
  if (J < 1 || p < 16 || p > STATIC_MAXP) return false;
  const int n_chunks = std::min(STATIC_CHUNKS, J);
  return (size_t)n_chunks * p * p + (size_t)p <= STATIC_SCRATCH_DOUBLES;
}

hipError_t launch_init_probe_static(const float* sqrt_f, int J, int p, float2* w, hipStream_t s) {
  double* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return e;
  InitProbeArgs a;
  a.sqrt_f = sqrt_f;
  a.J = J;
  a.p = p;
  // the same chunking as the plan's entry point, so both sum in the same order
  a.n_chunks = std::min(STATIC_CHUNKS, std::max(1, J));
  a.frames_per_chunk = (J + a.n_chunks - 1) / a.n_chunks;
  a.n_chunks = (J + a.frames_per_chunk - 1) / a.frames_per_chunk;
  a.part = base;
  float2* tw = reinterpret_cast<float2*>(base + (size_t)STATIC_CHUNKS * STATIC_MAXP * STATIC_MAXP);
  a.tw = tw;
  a.w = w;
  hipLaunchKernelGGL(k_twiddles, dim3(1), dim3(128), 0, s, tw, p);
  return launch_init_probe(a, s);
}

hipError_t launch_probe_update(const ProbeArgs& a, hipStream_t s) {
  const int pp = a.p * a.p;
  hipLaunchKernelGGL(k_probe_avg, dim3((pp + 63) / 64), dim3(256), 0, s, a);
  if (a.fmask) {
#define ODP_PROJ(PP) \
  if (a.p == PP) hipLaunchKernelGGL((k_probe_project<PP>), dim3(1), dim3(Frame<PP>::T), 0, s, a);
    ODP_PROJ(32)
    ODP_PROJ(64)
    ODP_PROJ(128)
#undef ODP_PROJ
  }
  if (a.stream) hipLaunchKernelGGL(k_probe_copies<true>, dim3((pp + 255) / 256, a.D), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_probe_copies<false>, dim3((pp + 255) / 256, a.D), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace odp

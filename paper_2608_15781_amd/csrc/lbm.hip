// C ABI of the MI355X reactive colour-gradient lattice Boltzmann step: context, workspace
// layout, initialisation kernels and launch sequences. The per-step kernels live in
// step_kernels.hpp. Build: hipcc --offload-arch=gfx950 (see the package's build module).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lbm.h"
#include "lattice.hpp"
#include "precision.hpp"
#include "step_kernels.hpp"
#include "adjoint_kernels.hpp"

using namespace lbm;

namespace {

constexpr int kRing = 1024;          // per-step reduction rows kept on the device
constexpr int kEvents = 5;           // profiling events per step: before k_colour, after each kernel
constexpr int kTimed = 4;            // kernels timed per step: colour, extrap, normal, collide
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Byte ranges [a, a + na) and [b, b + nb) of device memory overlap.
bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

size_t store_bytes(int precision) { return precision == LBM_FP64 ? 8 : (precision == LBM_FP32 ? 4 : 2); }
size_t real_bytes(int precision) { return precision == LBM_FP64 ? 8 : 4; }

struct Layout {
  size_t info, wet, rhoN, nst, state[2], partials, ring, lists[2], linfo[2], fid, counts, order, total;
  size_t f_off, a_off, g_off, c_off, state_bytes;  // within one state buffer
  size_t ps;  // elements between consecutive state (and adjoint) planes
  int nblocks;  // one thread per node, rounded up to a multiple of kXcd workgroups
};

// Upper bounds of the two launch lists: the fluid nodes (params.fluid_nodes when given, else
// every node) and the solid nodes next to fluid (at most the solid nodes).
size_t fluid_bound(const lbm_params& p) {
  const size_t N = size_t(p.nx) * p.ny * p.nz;
  return p.fluid_nodes > 0 ? size_t(p.fluid_nodes) : N;
}
size_t ext_bound(const lbm_params& p) {
  const size_t N = size_t(p.nx) * p.ny * p.nz;
  return p.fluid_nodes > 0 ? N - size_t(p.fluid_nodes) : N;
}

// Bytes of host inputs staged on the device during lbm_init: theta, rho_r0, rho_p0, c0 (doubles)
// and the solid and reactive masks (bytes), N each.
size_t stage_bytes(const lbm_params& p) { return 34 * size_t(p.nx) * p.ny * p.nz; }

// Plane stride of the state and adjoint planes, which are indexed by fluid id: at least the
// number of fluid nodes and an odd multiple of 256 bytes of storage, so that the same entry of
// different planes does not fall on one memory channel (a power-of-two count would put every
// plane on the same one).
size_t plane_stride(const lbm_params& p) {
  const size_t F = fluid_bound(p);
  const size_t unit = 256 / store_bytes(p.precision);
  size_t m = (F + unit - 1) / unit;
  if (m % 2 == 0) ++m;
  return m * unit;
}

Layout make_layout(const lbm_params& p) {
  Layout L{};
  const size_t N = size_t(p.nx) * p.ny * p.nz;
  const size_t F = fluid_bound(p), E = ext_bound(p);
  const size_t s = store_bytes(p.precision), r = real_bytes(p.precision);
  const size_t ps = plane_stride(p);
  L.ps = ps;
  L.f_off = 0;
  L.a_off = align_up(19 * s * ps);
  L.g_off = align_up(L.a_off + 4 * r * ps);
  // 2-byte storages: the species total of each node follows the 7 species planes
  const bool cplane = p.species && s == 2;
  L.c_off = align_up(L.g_off + (p.species ? 7 * s * ps : 0));
  L.state_bytes = align_up(L.c_off + (cplane ? r * ps : 0));
  int nb = int((N + kBlock - 1) / kBlock);
  nb = (nb + kXcd - 1) / kXcd * kXcd;
  L.nblocks = nb;
  size_t o = 0;
  L.info = o; o = align_up(o + 4 * N);      // per node
  L.wet = o; o = align_up(o + 4 * r * F);   // per fluid id
  L.rhoN = o; o = align_up(o + r * N);      // per node (read at solid nodes too)
  L.nst = o; o = align_up(o + 4 * r * F);   // per fluid id
  L.partials = o; o = align_up(o + 5 * sizeof(double) * size_t(nb));
  L.ring = o; o = align_up(o + 5 * sizeof(double) * kRing);
  L.lists[0] = o; o = align_up(o + 4 * F);  // fluid nodes
  L.lists[1] = o; o = align_up(o + 4 * E);  // solid nodes with extrapolated colour
  L.linfo[0] = o; o = align_up(o + 4 * F);  // info words of the list entries
  L.linfo[1] = o; o = align_up(o + 4 * E);
  L.fid = o; o = align_up(o + 4 * N);       // node -> fluid id
  L.counts = o; o = align_up(o + 4 * (size_t(nb) + 2));
  L.order = o; o = align_up(o + 4 * size_t(nb));  // launch order of the fluid-list tiles
  L.state[0] = o; o = align_up(o + L.state_bytes);
  // The second state buffer comes last: lbm_init stages the host inputs there and in whatever
  // lies beyond it, so the workspace extends to the larger of the two.
  L.state[1] = o; o = align_up(o + std::max(L.state_bytes, stage_bytes(p)));
  L.total = o;
  return L;
}

struct AdjLayout {
  size_t adj_bytes;                                                       // one adjoint state
  size_t lrn, lng, lHn, lG, lr2, lgo, rmv, nraw, partials, sum, total;  // scratch offsets
};

// Forward fields of one level, kept by lbm_step_fields for lbm_adjoint_step_fields: rho^N (dense),
// n* and |G| (per fluid id), the normal before realignment at wetting nodes (per fluid id),
// rho^m (dense).
struct FieldLayout {
  size_t rhoN, nst, nraw, rm, total;
};

FieldLayout make_field_layout(const lbm_params& p) {
  FieldLayout F{};
  const size_t N = size_t(p.nx) * p.ny * p.nz;
  const size_t r = real_bytes(p.precision);
  size_t o = 0;
  F.rhoN = o; o = align_up(o + r * N);
  F.nst = o; o = align_up(o + 4 * r * fluid_bound(p));
  F.nraw = o; o = align_up(o + 4 * r * fluid_bound(p));
  F.rm = o; o = align_up(o + r * N);
  F.total = o;
  return F;
}

AdjLayout make_adj_layout(const lbm_params& p) {
  AdjLayout A{};
  const size_t N = size_t(p.nx) * p.ny * p.nz;
  const size_t r = real_bytes(p.precision);
  A.adj_bytes = align_up(size_t(kAdjPlanes) * r * plane_stride(p));
  size_t o = 0;
  A.lrn = o; o = align_up(o + r * N);
  A.lng = o; o = align_up(o + 4 * r * fluid_bound(p));
  A.lHn = o; o = align_up(o + 4 * r * fluid_bound(p));
  A.lG = o; o = align_up(o + 3 * r * N);
  A.lr2 = o; o = align_up(o + 2 * r * N);
  A.lgo = o; o = align_up(o + r * N);
  A.rmv = o; o = align_up(o + r * N);
  A.nraw = o; o = align_up(o + 4 * r * fluid_bound(p));
  A.partials = o; o = align_up(o + 5 * sizeof(double) * size_t(make_layout(p).nblocks));
  A.sum = o; o = align_up(o + 5 * sizeof(double));
  A.total = o;
  return A;
}

}  // namespace

struct lbm_ctx {
  lbm_params p;
  int N;
  Layout L;
  char* ws;
  hipStream_t stream;
  int cur;  // index of the state buffer holding S_t
  int64_t steps;
  int nfluid, next;      // list lengths
  int nb_fluid, nb_ext;  // workgroups over each list (multiples of kXcd, 0 if empty)
  bool ordered;          // fluid-list tiles launched in the order stored at L.order
  void* static_scr;      // device address of the file-scope scratch array on this context's device
  char err[512];
  // Profiling: kEvents events per step of the current chunk (before the first kernel, after each).
  bool prof;
  std::vector<hipEvent_t> ev;
  double kernel_ms[kTimed];
  int64_t prof_steps;
};

namespace {

lbm_status fail(lbm_ctx* c, lbm_status s, const char* fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return s;
}

#define HIP_TRY(ctx, expr)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail((ctx), LBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Message of the last error of a call without a context (lbm_last_error(NULL)), per thread.
thread_local char g_err[512] = "";

// Scratch of the allocation-free adjoint step (lbm_adjoint_step_static): a fixed array in the code
// object, so each device the library runs on holds one copy until the process ends. In host code
// `scratch` names a host-side stand-in, not device memory: kernels and copies get the device
// address that hipGetSymbolAddress returns for the current device, resolved once per device by
// lbm_init (static_scratch below) and kept in the context.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
__device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved on the first call for a device), or
// NULL with `msg` set if it cannot be resolved.
void* static_scratch(char* msg, size_t len) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    snprintf(msg, len, "hipGetDevice: %s", e != hipSuccess ? hipGetErrorString(e) : "device index out of range");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      snprintf(msg, len, "hipGetSymbolAddress(scratch): %s", e != hipSuccess ? hipGetErrorString(e) : "null address");
      return nullptr;
    }
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

lbm_status check_params(const lbm_params* p, char* msg, size_t len) {
  if (!p) { snprintf(msg, len, "params is NULL"); return LBM_ERR_ARG; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) { snprintf(msg, len, "lattice size must be >= 1"); return LBM_ERR_ARG; }
  const double N = double(p->nx) * p->ny * p->nz;
  if (N >= 2147483647.0) { snprintf(msg, len, "nx*ny*nz must be < 2^31"); return LBM_ERR_ARG; }
  if (p->precision < LBM_FP64 || p->precision > LBM_BF16_DEV) { snprintf(msg, len, "unknown precision %d", p->precision); return LBM_ERR_ARG; }
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) { snprintf(msg, len, "tau must be finite and > 0.5"); return LBM_ERR_ARG; }
  if (p->species && (!(p->tau_species > 0.5) || !std::isfinite(p->tau_species))) { snprintf(msg, len, "tau_species must be finite and > 0.5"); return LBM_ERR_ARG; }
  if (!(p->sigma >= 0) || !std::isfinite(p->sigma)) { snprintf(msg, len, "sigma must be finite and >= 0"); return LBM_ERR_ARG; }
  if (!(p->beta >= 0) || !std::isfinite(p->beta)) { snprintf(msg, len, "beta must be finite and >= 0"); return LBM_ERR_ARG; }
  if (!(p->xi >= 0) || !std::isfinite(p->xi)) { snprintf(msg, len, "xi must be finite and >= 0"); return LBM_ERR_ARG; }
  if (!(p->grad_eps > 0) || !std::isfinite(p->grad_eps)) { snprintf(msg, len, "grad_eps must be finite and > 0"); return LBM_ERR_ARG; }
  for (int k = 0; k < 2; ++k)
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p->accel[k][a])) { snprintf(msg, len, "accel must be finite"); return LBM_ERR_ARG; }
  if (p->species && p->x_open && (!std::isfinite(p->c_inlet) || p->c_inlet < 0)) { snprintf(msg, len, "c_inlet must be finite and >= 0"); return LBM_ERR_ARG; }
  if (p->species && p->x_open && p->nx < 2) { snprintf(msg, len, "x_open needs nx >= 2 (inlet and outflow planes)"); return LBM_ERR_ARG; }
  if (p->precision == LBM_FP16_DEV && (p->fp16_scale_log2 < 0 || p->fp16_scale_log2 > 20)) { snprintf(msg, len, "fp16_scale_log2 must be in 0..20"); return LBM_ERR_ARG; }
  if (p->fluid_nodes < 0 || double(p->fluid_nodes) > N) {
    snprintf(msg, len, "fluid_nodes must be in 0..nx*ny*nz");
    return LBM_ERR_ARG;
  }
  if (p->species != 0 && p->species != 1) { snprintf(msg, len, "species must be 0 or 1"); return LBM_ERR_ARG; }
  return LBM_OK;
}

// ------------------------------------------------------------------------------------------
// Initialisation kernels
// ------------------------------------------------------------------------------------------

__device__ inline int wrap(int v, int n) { v %= n; return v < 0 ? v + n : v; }

// Flags, bounce-back links, NN(x) (eq. nearest_solid_neighbors), wetting set, r(x) NN(x).
__global__ void k_init_info(int nx, int ny, int nz, const uint8_t* solid, const uint8_t* reactive, int open,
                            uint32_t* info) {
  using D = D3Q19;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = nx * ny * nz;
  if (n >= N) return;
  const int x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
  auto at = [&](int dx, int dy, int dz) { return wrap(x + dx, nx) + nx * (wrap(y + dy, ny) + ny * wrap(z + dz, nz)); };
  uint32_t v = 0;
  if (solid[n]) {
    for (int i = 0; i < 18; ++i)
      if (!solid[at(D::cx[i], D::cy[i], D::cz[i])]) v |= (1u << i);
    if (v) v |= kExtrap;
  } else {
    int nn = 0;
    for (int i = 0; i < 18; ++i) {
      if (solid[at(-D::cx[i], -D::cy[i], -D::cz[i])]) v |= (1u << i);
      if (i < 6 && solid[at(D::cx[i], D::cy[i], D::cz[i])]) ++nn;
    }
    v |= kFluid;
    if (v & kLinkMask) v |= kWet;
    const bool r = reactive ? (reactive[n] != 0) : (nn > 0);
    if (r) v |= uint32_t(nn) << kRnnShift;
    if (open && x == 0) v |= kInlet;
    if (open && x == nx - 1) v |= kOutlet;
  }
  info[n] = v;
}

// Solid normal n_s at wetting nodes (eq. normal_vector_solid) over the 92-vector eighth-order
// stencil. The weights of eq. (eigth_order_weight_function) are multiples of 1/5040, so the
// sum is accumulated exactly in integers (5040 w = 448, 240, 96, 50, 16, 8, 1) and normalised
// once; a zero sum leaves n_s undefined (stored as 0). Also stores cos(theta).
template <class R>
__global__ void k_init_wet(int nx, int ny, int nz, const uint8_t* solid, const uint32_t* info, const int* fid,
                           const double* theta, double theta_uniform, R* wet) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = nx * ny * nz;
  if (n >= N || !(info[n] & kFluid)) return;
  const int x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
  const double th = theta ? theta[n] : theta_uniform;
  long sx = 0, sy = 0, sz = 0;
  if (info[n] & kWet) {
    for (int ez = -2; ez <= 2; ++ez)
      for (int ey = -2; ey <= 2; ++ey)
        for (int ex = -2; ex <= 2; ++ex) {
          const int e2 = ex * ex + ey * ey + ez * ez;
          int w = 0;
          switch (e2) {
            case 1: w = 448; break;
            case 2: w = 240; break;
            case 3: w = 96; break;
            case 4: w = 50; break;
            case 5: w = 16; break;
            case 6: w = 8; break;
            case 8: w = 1; break;
            default: w = 0;
          }
          if (w && solid[wrap(x + ex, nx) + nx * (wrap(y + ey, ny) + ny * wrap(z + ez, nz))]) {
            sx += w * ex; sy += w * ey; sz += w * ez;
          }
        }
  }
  double len = sqrt(double(sx * sx + sy * sy + sz * sz));
  double il = len > 0 ? 1.0 / len : 0.0;
  st4(wet, fid[n], R(sx * il), R(sy * il), R(sz * il), R(cos(th)));
}

// Dense copy (4 reals per node, node-major) of the per-fluid-id wetting data; zero at solids.
template <class R>
__global__ void k_wet_dense(int N, const int* fid, const R* wet, R* out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int f = fid[n];
  if (f >= 0) {
    const typename V4<R>::T v = ld4(wet, f);
    st4(out, n, v.x, v.y, v.z, v.w);
  } else {
    st4(out, n, R(0), R(0), R(0), R(0));
  }
}

// S_0 = f^eq(rho^k_0, 0) per colour: f^m = w (rho^r + rho^p), a = rho^r / rho^m, v = 0, g = w C_0.
template <int P>
__global__ void k_init_state(StepArgs<P> A, const double* rr0, const double* rp0, const double* c0) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.nfluid) return;
  const int n = A.fluid[t];
  const double rm = rr0[n] + rp0[n];
  for (int i = 0; i < 19; ++i) A.fout[size_t(i) * A.ps + t] = Prec<P>::st(R(D::w(i) * rm), R(D::w(i)), A.scale);
  st4(A.aout, t, R(pack_frac(rr0[n] / rm, rp0[n] / rm)), R(0), R(0), R(0));
  if (A.species) {
    const double c = c0 ? c0[n] : 1.0;
    if (P >= 2) A.cout[t] = R(c);  // deviations from w_q C: zero at rest
    for (int i = 0; i < 7; ++i)
      A.gout[size_t(i) * A.ps + t] = Prec<P>::st(R(D3Q7::w(i) * c), P >= 2 ? R(D3Q7::w(i)) * R(c) : R(D3Q7::w(i)), A.gscale);
  }
}

// Order-preserving stream compaction of the nodes whose info word has any bit of `mask`:
// per-workgroup counts, one-workgroup exclusive scan, scatter with wavefront ballots.
__global__ void k_flag_count(const uint32_t* info, int N, uint32_t mask, int* counts) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = __syncthreads_count(n < N && (info[n] & mask));
  if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

// First node of each tile of kBlock consecutive fluid ids.
__global__ void k_tile_heads(const int* fluid, int ntiles, int* heads) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ntiles) heads[k] = fluid[size_t(k) * kBlock];
}

__global__ void k_gather_info(const uint32_t* info, const int* list, int len, uint32_t* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < len) out[t] = info[list[t]];
}

// Fluid id of every node (-1 for solid): the inverse of the fluid list.
__global__ void k_fill_fid(const uint32_t* info, const int* list, int N, int nfluid, int* fid) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N && !(info[n] & kFluid)) fid[n] = -1;
  if (n < nfluid) fid[list[n]] = n;
}

__global__ void k_scan_counts(int* counts, int nb) {
  __shared__ int part[1024];
  const int chunk = (nb + 1023) / 1024;
  const int b0 = threadIdx.x * chunk, b1 = min(nb, b0 + chunk);
  int sum = 0;
  for (int b = b0; b < b1; ++b) sum += counts[b];
  part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < 1024; ++i) { const int v = part[i]; part[i] = run; run += v; }
    counts[nb] = run;
  }
  __syncthreads();
  int run = part[threadIdx.x];
  for (int b = b0; b < b1; ++b) { const int v = counts[b]; counts[b] = run; run += v; }
}

__global__ void k_flag_scatter(const uint32_t* info, int N, uint32_t mask, const int* offsets, int* list) {
  __shared__ int wsum[4];
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const bool f = n < N && (info[n] & mask);
  const unsigned long long bal = __ballot(f);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int pre = __popcll(bal & below);
  if (lane == 0) wsum[wave] = __popcll(bal);
  __syncthreads();
  int off = offsets[blockIdx.x];
  for (int w = 0; w < wave; ++w) off += wsum[w];
  if (f) list[off + pre] = n;
}

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((uint64_t(1) << s) < d) ++s;
  f.s = s;
  f.m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << s) - d)) / d + 1);
  return f;
}

int rounded_blocks(int n) {
  if (n <= 0) return 0;
  const int nb = (n + kBlock - 1) / kBlock;
  return (nb + kXcd - 1) / kXcd * kXcd;
}

// ------------------------------------------------------------------------------------------
// Launch helpers
// ------------------------------------------------------------------------------------------

template <int P>
StepArgs<P> make_args(lbm_ctx* c, int src_buf) {
  using S = typename Prec<P>::S;
  using R = typename Prec<P>::R;
  StepArgs<P> A{};
  const lbm_params& p = c->p;
  const Layout& L = c->L;
  A.nx = p.nx; A.ny = p.ny; A.nz = p.nz; A.N = c->N;
  A.ps = L.ps;
  A.geo.nx = p.nx; A.geo.ny = p.ny; A.geo.nz = p.nz;
  A.geo.fx = make_fastdiv(uint32_t(p.nx));
  A.geo.fy = make_fastdiv(uint32_t(p.ny));
  A.fluid = reinterpret_cast<const int*>(c->ws + L.lists[0]);
  A.finfo = reinterpret_cast<const uint32_t*>(c->ws + L.linfo[0]);
  A.nfluid = c->nfluid;
  A.ext = reinterpret_cast<const int*>(c->ws + L.lists[1]);
  A.einfo = reinterpret_cast<const uint32_t*>(c->ws + L.linfo[1]);
  A.fid = reinterpret_cast<const int*>(c->ws + L.fid);
  A.order = c->ordered ? reinterpret_cast<const int*>(c->ws + L.order) : nullptr;
  A.next = c->next;
  A.info = reinterpret_cast<const uint32_t*>(c->ws + L.info);
  char* sb = c->ws + L.state[src_buf];
  char* db = c->ws + L.state[1 - src_buf];
  A.fin = reinterpret_cast<const S*>(sb + L.f_off);
  A.ain = reinterpret_cast<const R*>(sb + L.a_off);
  A.gin = reinterpret_cast<const S*>(sb + L.g_off);
  A.cin = reinterpret_cast<const R*>(sb + L.c_off);
  A.fout = reinterpret_cast<S*>(db + L.f_off);
  A.aout = reinterpret_cast<R*>(db + L.a_off);
  A.gout = reinterpret_cast<S*>(db + L.g_off);
  A.cout = reinterpret_cast<R*>(db + L.c_off);
  A.rhoN = reinterpret_cast<R*>(c->ws + L.rhoN);
  A.nst = reinterpret_cast<R*>(c->ws + L.nst);
  A.wet = reinterpret_cast<const R*>(c->ws + L.wet);
  A.partials = reinterpret_cast<double*>(c->ws + L.partials);
  A.ring_row = reinterpret_cast<double*>(c->ws + L.ring);
  A.relax = R(1.0 - 1.0 / p.tau);
  A.inv_tau_c = p.species ? R(1.0 / p.tau_species) : R(1);
  A.sigma = R(p.sigma); A.beta = R(p.beta); A.xi = R(p.xi); A.c_in = R(p.c_inlet); A.eps = R(p.grad_eps);
  for (int k = 0; k < 2; ++k)
    for (int a = 0; a < 3; ++a) A.acc[k][a] = R(p.accel[k][a]);
  const int k2 = p.precision == LBM_FP16_DEV ? p.fp16_scale_log2 : 0;
  A.scale = R(std::ldexp(1.0, k2));
  A.inv_scale = R(std::ldexp(1.0, -k2));
  A.gscale = A.scale;
  A.inv_gscale = A.inv_scale;
  A.species = p.species;
  return A;
}

// The step's level-t fields (rho^N, n* with |G|, rho^m) go to a caller's buffer.
template <int P>
void use_fields(lbm_ctx* c, StepArgs<P>& A, void* fields) {
  using R = typename Prec<P>::R;
  const FieldLayout FL = make_field_layout(c->p);
  char* fb = static_cast<char*>(fields);
  A.rhoN = reinterpret_cast<R*>(fb + FL.rhoN);
  A.nst = reinterpret_cast<R*>(fb + FL.nst);
  A.nraw = reinterpret_cast<R*>(fb + FL.nraw);
  A.rm_out = reinterpret_cast<R*>(fb + FL.rm);
}

// The four kernels of one step, with optional events (kEvents) around them; without `collide`
// only the level-t fields (colour, extrapolation, normals).
template <int P>
lbm_status enqueue_step(lbm_ctx* c, const StepArgs<P>& A, hipEvent_t* ev, bool collide = true) {
  const dim3 block(kBlock), gf(c->nb_fluid), ge(c->nb_ext);
  if (ev) HIP_TRY(c, hipEventRecord(ev[0], c->stream));
  if (c->nb_fluid) hipLaunchKernelGGL(k_colour<P>, gf, block, 0, c->stream, A);
  if (ev) HIP_TRY(c, hipEventRecord(ev[1], c->stream));
  if (c->nb_ext) hipLaunchKernelGGL(k_extrap<P>, ge, block, 0, c->stream, A);
  if (ev) HIP_TRY(c, hipEventRecord(ev[2], c->stream));
  if (c->nb_fluid) hipLaunchKernelGGL(k_normal<P>, gf, block, 0, c->stream, A);
  if (ev) HIP_TRY(c, hipEventRecord(ev[3], c->stream));
  if (collide && c->nb_fluid) hipLaunchKernelGGL((k_collide<P, false>), gf, block, 0, c->stream, A);
  if (ev) HIP_TRY(c, hipEventRecord(ev[4], c->stream));
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}

template <int P>
lbm_status launch_step(lbm_ctx* c, int slot, bool timed = true, void* fields = nullptr) {
  StepArgs<P> A = make_args<P>(c, c->cur);
  if (fields) use_fields<P>(c, A, fields);
  double* ring = reinterpret_cast<double*>(c->ws + c->L.ring);
  A.ring_row = ring + 5 * size_t(slot);
  // The previous step's partials (one per k_collide workgroup) are summed by k_colour of this
  // step (its workgroup 0); the last step of a chunk is summed by launch_finish.
  A.red_in = A.partials;
  A.red_n = c->nb_fluid;
  A.red_out = slot > 0 ? ring + 5 * size_t(slot - 1) : nullptr;
  if (A.red_out && !c->nb_fluid)
    hipLaunchKernelGGL(k_finish_reduce, dim3(1), dim3(kBlock), 0, c->stream, A.partials, A.red_n, A.red_out);
  hipEvent_t* ev = (c->prof && timed) ? &c->ev[kEvents * size_t(slot)] : nullptr;
  const lbm_status s = enqueue_step<P>(c, A, ev);
  if (s != LBM_OK) return s;
  c->cur = 1 - c->cur;
  c->steps++;
  return LBM_OK;
}

// One step from a caller's state buffer into another; the context's state is not touched. The
// per-block partial sums are written to the workspace as in every step and never reduced.
template <int P>
lbm_status launch_step_from(lbm_ctx* c, const void* src, void* dst, void* fields) {
  using S = typename Prec<P>::S;
  using R = typename Prec<P>::R;
  StepArgs<P> A = make_args<P>(c, c->cur);
  const char* sb = static_cast<const char*>(src);
  char* db = static_cast<char*>(dst);
  A.fin = reinterpret_cast<const S*>(sb + c->L.f_off);
  A.ain = reinterpret_cast<const R*>(sb + c->L.a_off);
  A.gin = reinterpret_cast<const S*>(sb + c->L.g_off);
  A.cin = reinterpret_cast<const R*>(sb + c->L.c_off);
  A.fout = db ? reinterpret_cast<S*>(db + c->L.f_off) : nullptr;
  A.aout = db ? reinterpret_cast<R*>(db + c->L.a_off) : nullptr;
  A.gout = db ? reinterpret_cast<S*>(db + c->L.g_off) : nullptr;
  A.cout = db ? reinterpret_cast<R*>(db + c->L.c_off) : nullptr;
  if (fields) use_fields<P>(c, A, fields);
  A.ring_row = reinterpret_cast<double*>(c->ws + c->L.ring);
  A.red_out = nullptr;
  return enqueue_step<P>(c, A, nullptr, db != nullptr);  // no destination: the fields only
}

// Final reduction of the last step of a chunk (ring row `slot`).
lbm_status launch_finish(lbm_ctx* c, int slot) {
  double* ring = reinterpret_cast<double*>(c->ws + c->L.ring);
  hipLaunchKernelGGL(k_finish_reduce, dim3(1), dim3(kBlock), 0, c->stream,
                     reinterpret_cast<const double*>(c->ws + c->L.partials), c->nb_fluid, ring + 5 * size_t(slot));
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}

template <int P>
lbm_status launch_moments(lbm_ctx* c, void* rr, void* rp, void* rn, void* u, void* cc) {
  using R = typename Prec<P>::R;
  StepArgs<P> A = make_args<P>(c, c->cur);
  A.m_rr = static_cast<R*>(rr); A.m_rp = static_cast<R*>(rp); A.m_rn = static_cast<R*>(rn);
  A.m_u = static_cast<R*>(u); A.m_c = static_cast<R*>(cc);
  const size_t N = c->N;
  const size_t rb = sizeof(R);
  for (void* ptr : {rr, rp, rn, cc})
    if (ptr) HIP_TRY(c, hipMemsetAsync(ptr, 0, rb * N, c->stream));
  if (u) HIP_TRY(c, hipMemsetAsync(u, 0, 3 * rb * N, c->stream));
  const dim3 gf(c->nb_fluid), ge(c->nb_ext), block(kBlock);
  if (c->nb_fluid) hipLaunchKernelGGL(k_colour<P>, gf, block, 0, c->stream, A);
  if (c->nb_ext) hipLaunchKernelGGL(k_extrap<P>, ge, block, 0, c->stream, A);
  if (c->nb_fluid) hipLaunchKernelGGL(k_normal<P>, gf, block, 0, c->stream, A);
  if (c->nb_fluid) hipLaunchKernelGGL((k_collide<P, true>), gf, block, 0, c->stream, A);
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}

template <int P>
lbm_status launch_expand(lbm_ctx* c, void* fr, void* fp, void* g) {
  using R = typename Prec<P>::R;
  StepArgs<P> A = make_args<P>(c, c->cur);
  const dim3 grid(c->L.nblocks), block(kBlock);
  hipLaunchKernelGGL(k_expand<P>, grid, block, 0, c->stream, A, static_cast<R*>(fr), static_cast<R*>(fp),
                     static_cast<R*>(g));
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}

// Launch order of the tiles of the fluid list. Tiles are keyed by their first node: y-bands of
// kTileBand rows, each swept through z (x and y in order inside a band), and the XCD-aware
// launch index walks that order, so each XCD takes whole bands and the tiles that read each
// other's planes as neighbours run close together in time on one L2. The plain list order
// (each XCD a slab of whole planes) already keeps a tile's neighbours in the planes above and
// below in L2 while three planes of per-node data fit in it; the bands are used only when they
// do not (more than kOrderBytes, three quarters of one XCD's 4 MB L2). Measured: FP32 at 128^3
// (3.3 MB by the count below), FP64 at 128^3 and every 512^3 case gain 2-4% with the bands; FP16
// at 128^3 (2.1 MB) loses 3%.
// With bands at least ny rows deep the key would be the node index, the list order itself.
constexpr int kTileBand = 16;
constexpr double kOrderBytes = 3.0 * (1 << 20);

lbm_status build_tile_order(lbm_ctx* c) {
  c->ordered = false;
  const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
  const int ntiles = (c->nfluid + kBlock - 1) / kBlock;
  if (ntiles == 0 || kTileBand <= 0 || kTileBand >= ny) return LBM_OK;
  // per fluid node: the state (19 + 7 stored populations, 4 colour scalars) and the normal
  // pass's n* with |G| and rho^N
  const double s = double(store_bytes(c->p.precision)), r = double(real_bytes(c->p.precision));
  const double node_bytes = 26 * s + 4 * r + 5 * r;
  if (3.0 * double(c->nfluid) / nz * node_bytes <= kOrderBytes) return LBM_OK;
  int* d_order = reinterpret_cast<int*>(c->ws + c->L.order);
  hipLaunchKernelGGL(k_tile_heads, dim3((ntiles + kBlock - 1) / kBlock), dim3(kBlock), 0, c->stream,
                     reinterpret_cast<const int*>(c->ws + c->L.lists[0]), ntiles, d_order);
  HIP_TRY(c, hipGetLastError());
  std::vector<int> heads(ntiles);
  HIP_TRY(c, hipMemcpyAsync(heads.data(), d_order, sizeof(int) * size_t(ntiles), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::vector<int64_t> key(ntiles);
  for (int k = 0; k < ntiles; ++k) {
    const int64_t n = heads[k];
    const int64_t x = n % nx, r = n / nx, y = r % ny, z = r / ny;
    key[k] = (((y / kTileBand) * nz + z) * ny + y) * nx + x;
  }
  std::vector<int> order(c->nb_fluid);
  for (int k = 0; k < c->nb_fluid; ++k) order[k] = k;  // the padding workgroups keep their index
  std::stable_sort(order.begin(), order.begin() + ntiles, [&](int a, int b) { return key[a] < key[b]; });
  HIP_TRY(c, hipMemcpyAsync(d_order, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->ordered = true;
  return LBM_OK;
}

template <int P>
lbm_status launch_init(lbm_ctx* c, const uint8_t* d_solid, const uint8_t* d_react, const double* d_theta,
                       double theta_uniform, const double* d_rr, const double* d_rp, const double* d_c0) {
  using R = typename Prec<P>::R;
  const lbm_params& p = c->p;
  const int tb = 256, gb = (c->N + tb - 1) / tb;
  uint32_t* info = reinterpret_cast<uint32_t*>(c->ws + c->L.info);
  hipLaunchKernelGGL(k_init_info, dim3(gb), dim3(tb), 0, c->stream, p.nx, p.ny, p.nz, d_solid, d_react,
                     int(p.species && p.x_open), info);
  // Launch lists: fluid nodes and solid nodes with extrapolated colour, in node order.
  int* counts = reinterpret_cast<int*>(c->ws + c->L.counts);
  const uint32_t masks[2] = {kFluid, kExtrap};
  int lens[2] = {0, 0};
  for (int k = 0; k < 2; ++k) {
    int* list = reinterpret_cast<int*>(c->ws + c->L.lists[k]);
    hipLaunchKernelGGL(k_flag_count, dim3(gb), dim3(tb), 0, c->stream, info, c->N, masks[k], counts);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, c->stream, counts, gb);
    hipLaunchKernelGGL(k_flag_scatter, dim3(gb), dim3(tb), 0, c->stream, info, c->N, masks[k], counts, list);
    HIP_TRY(c, hipMemcpyAsync(&lens[k], counts + gb, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  c->nfluid = lens[0];
  c->next = lens[1];
  hipLaunchKernelGGL(k_fill_fid, dim3(gb), dim3(tb), 0, c->stream, info,
                     reinterpret_cast<const int*>(c->ws + c->L.lists[0]), c->N, c->nfluid,
                     reinterpret_cast<int*>(c->ws + c->L.fid));
  hipLaunchKernelGGL(k_init_wet<R>, dim3(gb), dim3(tb), 0, c->stream, p.nx, p.ny, p.nz, d_solid, info,
                     reinterpret_cast<const int*>(c->ws + c->L.fid), d_theta, theta_uniform,
                     reinterpret_cast<R*>(c->ws + c->L.wet));
  for (int k = 0; k < 2; ++k)
    if (lens[k] > 0)
      hipLaunchKernelGGL(k_gather_info, dim3((lens[k] + tb - 1) / tb), dim3(tb), 0, c->stream, info,
                         reinterpret_cast<const int*>(c->ws + c->L.lists[k]), lens[k],
                         reinterpret_cast<uint32_t*>(c->ws + c->L.linfo[k]));
  c->nb_fluid = rounded_blocks(c->nfluid);
  c->nb_ext = rounded_blocks(c->next);
  if (lbm_status s = build_tile_order(c); s != LBM_OK) return s;
  // The initial state goes into buffer 0 (make_args with src 1 writes buffer 0).
  StepArgs<P> A = make_args<P>(c, 1);
  if (c->nfluid > 0)
    hipLaunchKernelGGL(k_init_state<P>, dim3((c->nfluid + tb - 1) / tb), dim3(tb), 0, c->stream, A, d_rr, d_rp, d_c0);
  HIP_TRY(c, hipGetLastError());
  c->cur = 0;
  return LBM_OK;
}

template <int P>
StepArgs<P> make_args_from(lbm_ctx* c, const void* state) {
  using S = typename Prec<P>::S;
  using R = typename Prec<P>::R;
  StepArgs<P> A = make_args<P>(c, c->cur);
  const char* sb = static_cast<const char*>(state);
  A.fin = reinterpret_cast<const S*>(sb + c->L.f_off);
  A.ain = reinterpret_cast<const R*>(sb + c->L.a_off);
  A.gin = reinterpret_cast<const S*>(sb + c->L.g_off);
  A.cin = reinterpret_cast<const R*>(sb + c->L.c_off);
  A.fout = nullptr;
  A.aout = nullptr;
  A.gout = nullptr;
  A.cout = nullptr;
  return A;
}

// FP64 sums of a stored state into `out` (host, 5 doubles). The per-step partials and the first
// reduction-ring row are free between calls, so they serve here.
template <int P>
lbm_status launch_state_sums(lbm_ctx* c, const void* state, double* out) {
  StepArgs<P> A = state ? make_args_from<P>(c, state) : make_args<P>(c, c->cur);
  double* row = reinterpret_cast<double*>(c->ws + c->L.ring);
  if (c->nb_fluid)
    hipLaunchKernelGGL(k_state_sums<P>, dim3(c->nb_fluid), dim3(kBlock), 0, c->stream, A);
  hipLaunchKernelGGL(k_finish_reduce, dim3(1), dim3(kBlock), 0, c->stream, A.partials, c->nb_fluid, row);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipMemcpyAsync(out, row, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

template <int P>
lbm_status launch_adj_seed(lbm_ctx* c, const void* state, void* adj) {
  using R = typename Prec<P>::R;
  StepArgs<P> A = make_args_from<P>(c, state);
  const AdjLayout AL = make_adj_layout(c->p);
  HIP_TRY(c, hipMemsetAsync(adj, 0, AL.adj_bytes, c->stream));
  if (c->nb_fluid)
    hipLaunchKernelGGL(k_adj_seed<P>, dim3(c->nb_fluid), dim3(kBlock), 0, c->stream, A, static_cast<R*>(adj));
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}

template <int P>
lbm_status launch_adj_step(lbm_ctx* c, const void* state, const void* fields, const void* lin, void* lout,
                           void* scr, double* gth, double* gxi) {
  using R = typename Prec<P>::R;
  const AdjLayout AL = make_adj_layout(c->p);
  char* sc = static_cast<char*>(scr);
  StepArgs<P> A = make_args_from<P>(c, state);
  A.rm_out = reinterpret_cast<R*>(sc + AL.rmv);
  A.nraw = reinterpret_cast<R*>(sc + AL.nraw);
  if (fields)  // level-t fields kept by the forward step: no recomputation
    use_fields<P>(c, A, const_cast<void*>(fields));
  AdjArgs<R> J;
  J.lin = static_cast<const R*>(lin);
  J.lout = static_cast<R*>(lout);
  J.lrn = reinterpret_cast<R*>(sc + AL.lrn);
  J.lng = reinterpret_cast<R*>(sc + AL.lng);
  J.lHn = reinterpret_cast<R*>(sc + AL.lHn);
  J.lG = reinterpret_cast<R*>(sc + AL.lG);
  J.lr2 = reinterpret_cast<R*>(sc + AL.lr2);
  J.lgo = reinterpret_cast<R*>(sc + AL.lgo);
  J.rmv = A.rm_out;
  J.gtheta = gth;
  J.partials = reinterpret_cast<double*>(sc + AL.partials);
  J.nparts = c->nb_fluid;
  J.sum = reinterpret_cast<double*>(sc + AL.sum);
  J.gxi = gxi;
  const dim3 gf(c->nb_fluid), ge(c->nb_ext), block(kBlock);
  // Forward fields of level t.
  if (!fields) {
    if (c->nb_fluid) hipLaunchKernelGGL(k_colour<P>, gf, block, 0, c->stream, A);
    if (c->nb_ext) hipLaunchKernelGGL(k_extrap<P>, ge, block, 0, c->stream, A);
    if (c->nb_fluid) hipLaunchKernelGGL(k_normal<P>, gf, block, 0, c->stream, A);
  }
  // Reverse pass. Every entry of lout a fluid node owns is written (see k_adj_collide).
  if (c->nb_fluid) {
    hipLaunchKernelGGL(k_adj_collide<P>, gf, block, 0, c->stream, A, J);
    hipLaunchKernelGGL(k_adj_normal<P>, gf, block, 0, c->stream, A, J);
    if (c->nb_ext) hipLaunchKernelGGL(k_adj_grad_ext<P>, ge, block, 0, c->stream, A, J);
    hipLaunchKernelGGL(k_adj_colour<P>, gf, block, 0, c->stream, A, J);
    hipLaunchKernelGGL(k_adj_final<P>, gf, block, 0, c->stream, A, J);
  }
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}

// The buffers one adjoint step writes (adjoint output, scratch) must not overlap anything it
// reads or writes (state, fields, adjoint input, each other).
lbm_status check_adjoint_buffers(lbm_ctx* c, const void* state, const void* fields, const void* lin,
                                 const void* lout, const void* scr) {
  const AdjLayout AL = make_adj_layout(c->p);
  const size_t sb = c->L.state_bytes, ab = AL.adj_bytes, cb = AL.total;
  const size_t fb = make_field_layout(c->p).total;
  if (overlap(lin, ab, lout, ab)) return fail(c, LBM_ERR_ARG, "adjoint input and output overlap");
  if (overlap(lout, ab, state, sb) || overlap(scr, cb, state, sb))
    return fail(c, LBM_ERR_ARG, "an adjoint buffer overlaps the state");
  if (overlap(scr, cb, lin, ab) || overlap(scr, cb, lout, ab))
    return fail(c, LBM_ERR_ARG, "the scratch buffer overlaps an adjoint buffer");
  if (fields && (overlap(fields, fb, lout, ab) || overlap(fields, fb, scr, cb)))
    return fail(c, LBM_ERR_ARG, "the fields buffer overlaps an adjoint output");
  return LBM_OK;
}

#define DISPATCH(ctx, fn, ...)                                   \
  switch ((ctx)->p.precision) {                                  \
    case LBM_FP64: return fn<0>((ctx), __VA_ARGS__);             \
    case LBM_FP32: return fn<1>((ctx), __VA_ARGS__);             \
    case LBM_FP16_DEV: return fn<2>((ctx), __VA_ARGS__);         \
    default: return fn<3>((ctx), __VA_ARGS__);                   \
  }

}  // namespace

extern "C" {

const char* lbm_version(void) { return "lbm-mi355x 0.1 (gfx950)"; }

lbm_status lbm_workspace_bytes(const lbm_params* params, size_t* bytes) {
  lbm_status s = check_params(params, g_err, sizeof(g_err));
  if (s != LBM_OK) return s;
  if (!bytes) return LBM_ERR_ARG;
  *bytes = make_layout(*params).total;
  return LBM_OK;
}

lbm_status lbm_state_bytes(const lbm_params* params, size_t* bytes) {
  lbm_status s = check_params(params, g_err, sizeof(g_err));
  if (s != LBM_OK) return s;
  if (!bytes) return LBM_ERR_ARG;
  *bytes = make_layout(*params).state_bytes;
  return LBM_OK;
}

lbm_status lbm_init(const lbm_params* params, const uint8_t* solid, const double* theta, double theta_uniform,
                    const uint8_t* reactive, const double* rho_r0, const double* rho_p0, const double* c0,
                    void* d_workspace, size_t workspace_bytes, void* stream, lbm_ctx** out) {
  lbm_status s = check_params(params, g_err, sizeof(g_err));
  if (s != LBM_OK) return s;
  if (!out || !solid || !rho_r0 || !rho_p0 || !d_workspace) {
    snprintf(g_err, sizeof(g_err), "required pointer is NULL");
    return LBM_ERR_ARG;
  }
  const Layout L = make_layout(*params);
  if (workspace_bytes < L.total) {
    snprintf(g_err, sizeof(g_err), "workspace too small: %zu < %zu bytes", workspace_bytes, L.total);
    return LBM_ERR_ARG;
  }
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) {
    snprintf(g_err, sizeof(g_err), "workspace must be %zu-byte aligned", kAlign);
    return LBM_ERR_ARG;
  }
  const size_t N = size_t(params->nx) * params->ny * params->nz;
  // Host-side validation of the inputs.
  if (!theta && !(theta_uniform >= 0 && theta_uniform <= M_PI)) {
    snprintf(g_err, sizeof(g_err), "theta_uniform must be in [0, pi]");
    return LBM_ERR_ARG;
  }
  if (params->fluid_nodes > 0) {
    size_t nf = 0;
    for (size_t n = 0; n < N; ++n) nf += solid[n] ? 0 : 1;
    if (nf != size_t(params->fluid_nodes)) {
      snprintf(g_err, sizeof(g_err), "fluid_nodes = %d but the mask has %zu fluid nodes", params->fluid_nodes, nf);
      return LBM_ERR_ARG;
    }
  }
  for (size_t n = 0; n < N; ++n) {
    if (solid[n]) continue;
    const double a = rho_r0[n], b = rho_p0[n];
    if (!std::isfinite(a) || !std::isfinite(b) || a < 0 || b < 0 || !(a + b > 0)) {
      snprintf(g_err, sizeof(g_err), "initial densities at fluid node %zu must be finite, >= 0, with positive sum", n);
      return LBM_ERR_ARG;
    }
    if (theta && !(theta[n] >= 0 && theta[n] <= M_PI)) {
      snprintf(g_err, sizeof(g_err), "theta at fluid node %zu outside [0, pi]", n);
      return LBM_ERR_ARG;
    }
    if (c0 && params->species && (!std::isfinite(c0[n]) || c0[n] < 0)) {
      snprintf(g_err, sizeof(g_err), "c0 at fluid node %zu must be finite and >= 0", n);
      return LBM_ERR_ARG;
    }
  }
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ERR_ALLOC;
  c->p = *params;
  c->N = int(N);
  c->L = L;
  c->ws = static_cast<char*>(d_workspace);
  c->stream = static_cast<hipStream_t>(stream);
  c->steps = 0;
  c->err[0] = 0;
  c->prof = false;
  for (double& v : c->kernel_ms) v = 0.0;
  c->prof_steps = 0;
  // The allocation-free adjoint step's scratch on this (the current) device; a failure here only
  // disables that entry point, which reports it.
  c->static_scr = static_scratch(c->err, sizeof(c->err));
  c->err[0] = 0;
  // Stage the host inputs in the second state buffer (free until the first step).
  char* stage = c->ws + L.state[1];
  double* d_theta = reinterpret_cast<double*>(stage);
  double* d_rr = d_theta + N;
  double* d_rp = d_rr + N;
  double* d_c0 = d_rp + N;
  uint8_t* d_solid = reinterpret_cast<uint8_t*>(d_c0 + N);
  uint8_t* d_react = d_solid + N;
  auto bail = [&](lbm_status st) {
    snprintf(g_err, sizeof(g_err), "%s", c->err);
    delete c;
    return st;
  };
#define INIT_TRY(expr)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      fail(c, LBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));                     \
      return bail(LBM_ERR_HIP);                                                         \
    }                                                                                   \
  } while (0)
  INIT_TRY(hipMemsetAsync(c->ws, 0, L.total, c->stream));
  INIT_TRY(hipMemcpyAsync(d_solid, solid, N, hipMemcpyHostToDevice, c->stream));
  if (reactive) INIT_TRY(hipMemcpyAsync(d_react, reactive, N, hipMemcpyHostToDevice, c->stream));
  if (theta) INIT_TRY(hipMemcpyAsync(d_theta, theta, 8 * N, hipMemcpyHostToDevice, c->stream));
  INIT_TRY(hipMemcpyAsync(d_rr, rho_r0, 8 * N, hipMemcpyHostToDevice, c->stream));
  INIT_TRY(hipMemcpyAsync(d_rp, rho_p0, 8 * N, hipMemcpyHostToDevice, c->stream));
  if (c0) INIT_TRY(hipMemcpyAsync(d_c0, c0, 8 * N, hipMemcpyHostToDevice, c->stream));
  lbm_status st;
  switch (c->p.precision) {
    case LBM_FP64: st = launch_init<0>(c, d_solid, reactive ? d_react : nullptr, theta ? d_theta : nullptr, theta_uniform, d_rr, d_rp, c0 ? d_c0 : nullptr); break;
    case LBM_FP32: st = launch_init<1>(c, d_solid, reactive ? d_react : nullptr, theta ? d_theta : nullptr, theta_uniform, d_rr, d_rp, c0 ? d_c0 : nullptr); break;
    case LBM_FP16_DEV: st = launch_init<2>(c, d_solid, reactive ? d_react : nullptr, theta ? d_theta : nullptr, theta_uniform, d_rr, d_rp, c0 ? d_c0 : nullptr); break;
    default: st = launch_init<3>(c, d_solid, reactive ? d_react : nullptr, theta ? d_theta : nullptr, theta_uniform, d_rr, d_rp, c0 ? d_c0 : nullptr); break;
  }
  if (st != LBM_OK) return bail(st);
  // The host inputs are pageable memory; finish the copies before returning to the caller.
  INIT_TRY(hipStreamSynchronize(c->stream));
#undef INIT_TRY
  *out = c;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int32_t nsteps, lbm_reductions* per_step) {
  if (!c) return LBM_ERR_ARG;
  if (nsteps < 0) return fail(c, LBM_ERR_ARG, "nsteps must be >= 0");
  std::vector<double> rows;
  bool bad = false;
  int done = 0;
  while (done < nsteps) {
    const int chunk = std::min(kRing, nsteps - done);
    for (int t = 0; t < chunk; ++t) {
      lbm_status s;
      switch (c->p.precision) {
        case LBM_FP64: s = launch_step<0>(c, t); break;
        case LBM_FP32: s = launch_step<1>(c, t); break;
        case LBM_FP16_DEV: s = launch_step<2>(c, t); break;
        default: s = launch_step<3>(c, t); break;
      }
      if (s != LBM_OK) return s;
    }
    if (lbm_status s = launch_finish(c, chunk - 1); s != LBM_OK) return s;
    rows.resize(5 * size_t(chunk));
    HIP_TRY(c, hipMemcpyAsync(rows.data(), c->ws + c->L.ring, rows.size() * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->prof) {
      for (int t = 0; t < chunk; ++t)
        for (int k = 0; k < kTimed; ++k) {
          float ms = 0.f;
          HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[kEvents * size_t(t) + k], c->ev[kEvents * size_t(t) + k + 1]));
          c->kernel_ms[k] += ms;
        }
      c->prof_steps += chunk;
    }
    for (int t = 0; t < chunk; ++t) {
      if (rows[5 * t + 4] > 0) bad = true;
      if (per_step) {
        lbm_reductions& r = per_step[done + t];
        r.mass_r = rows[5 * t];
        r.mass_p = rows[5 * t + 1];
        r.conversion = rows[5 * t + 2];
        r.species_total = rows[5 * t + 3];
        r.nonfinite = rows[5 * t + 4];
      }
    }
    done += chunk;
  }
  if (bad) return fail(c, LBM_ERR_NONFINITE, "non-finite values after step %lld", (long long)c->steps);
  return LBM_OK;
}

lbm_status lbm_step_async(lbm_ctx* c, int32_t nsteps) {
  if (!c) return LBM_ERR_ARG;
  if (nsteps < 0) return fail(c, LBM_ERR_ARG, "nsteps must be >= 0");
  for (int t = 0; t < nsteps; ++t) {
    lbm_status s;
    const int slot = t % kRing;
    switch (c->p.precision) {
      case LBM_FP64: s = launch_step<0>(c, slot, false); break;
      case LBM_FP32: s = launch_step<1>(c, slot, false); break;
      case LBM_FP16_DEV: s = launch_step<2>(c, slot, false); break;
      default: s = launch_step<3>(c, slot, false); break;
    }
    if (s != LBM_OK) return s;
  }
  return LBM_OK;
}

lbm_status lbm_fields_bytes(const lbm_params* params, size_t* bytes) {
  lbm_status s = check_params(params, g_err, sizeof(g_err));
  if (s != LBM_OK) return s;
  if (bytes) *bytes = make_field_layout(*params).total;
  return LBM_OK;
}

lbm_status lbm_step_fields(lbm_ctx* c, void* d_fields) {
  if (!c) return LBM_ERR_ARG;
  if (!d_fields) return fail(c, LBM_ERR_ARG, "a fields buffer is required");
  switch (c->p.precision) {
    case LBM_FP64: return launch_step<0>(c, 0, false, d_fields);
    case LBM_FP32: return launch_step<1>(c, 0, false, d_fields);
    case LBM_FP16_DEV: return launch_step<2>(c, 0, false, d_fields);
    default: return launch_step<3>(c, 0, false, d_fields);
  }
}

lbm_status lbm_step_from(lbm_ctx* c, const void* d_src, void* d_dst, void* d_fields) {
  if (!c) return LBM_ERR_ARG;
  if (!d_src) return fail(c, LBM_ERR_ARG, "a source state is required");
  if (!d_dst && !d_fields) return fail(c, LBM_ERR_ARG, "a destination state or a fields buffer is required");
  const size_t sb = c->L.state_bytes;
  if (d_dst && overlap(d_src, sb, d_dst, sb)) return fail(c, LBM_ERR_ARG, "source and destination states overlap");
  if (d_fields) {
    const size_t fb = make_field_layout(c->p).total;
    if ((d_dst && overlap(d_fields, fb, d_dst, sb)) || overlap(d_fields, fb, d_src, sb))
      return fail(c, LBM_ERR_ARG, "the fields buffer overlaps a state");
  }
  DISPATCH(c, launch_step_from, d_src, d_dst, d_fields);
}

lbm_status lbm_moments(lbm_ctx* c, void* rr, void* rp, void* rn, void* u, void* cc) {
  if (!c) return LBM_ERR_ARG;
  DISPATCH(c, launch_moments, rr, rp, rn, u, cc);
}

lbm_status lbm_state_sums(lbm_ctx* c, const void* d_state, lbm_reductions* out) {
  if (!c) return LBM_ERR_ARG;
  if (!out) return fail(c, LBM_ERR_ARG, "out is NULL");
  double row[5] = {0, 0, 0, 0, 0};
  lbm_status s;
  switch (c->p.precision) {
    case LBM_FP64: s = launch_state_sums<0>(c, d_state, row); break;
    case LBM_FP32: s = launch_state_sums<1>(c, d_state, row); break;
    case LBM_FP16_DEV: s = launch_state_sums<2>(c, d_state, row); break;
    default: s = launch_state_sums<3>(c, d_state, row); break;
  }
  if (s != LBM_OK) return s;
  out->mass_r = row[0];
  out->mass_p = row[1];
  out->conversion = 0.0;
  out->species_total = row[3];
  out->nonfinite = row[4];
  return LBM_OK;
}

lbm_status lbm_populations(lbm_ctx* c, void* fr, void* fp, void* g) {
  if (!c) return LBM_ERR_ARG;
  if (!fr || !fp) return fail(c, LBM_ERR_ARG, "fr and fp are required");
  DISPATCH(c, launch_expand, fr, fp, g);
}

lbm_status lbm_geometry(lbm_ctx* c, void* d_info, void* d_wet) {
  if (!c) return LBM_ERR_ARG;
  const size_t N = c->N;
  if (d_info) HIP_TRY(c, hipMemcpyAsync(d_info, c->ws + c->L.info, 4 * N, hipMemcpyDeviceToDevice, c->stream));
  if (d_wet) {
    const int tb = 256, gb = int((N + tb - 1) / tb);
    const int* fid = reinterpret_cast<const int*>(c->ws + c->L.fid);
    if (c->p.precision == LBM_FP64)
      hipLaunchKernelGGL(k_wet_dense<double>, dim3(gb), dim3(tb), 0, c->stream, int(N), fid,
                         reinterpret_cast<const double*>(c->ws + c->L.wet), static_cast<double*>(d_wet));
    else
      hipLaunchKernelGGL(k_wet_dense<float>, dim3(gb), dim3(tb), 0, c->stream, int(N), fid,
                         reinterpret_cast<const float*>(c->ws + c->L.wet), static_cast<float*>(d_wet));
    HIP_TRY(c, hipGetLastError());
  }
  return LBM_OK;
}

lbm_status lbm_state_layout(const lbm_params* params, size_t* f_off, size_t* a_off, size_t* g_off,
                            size_t* plane_stride_out) {
  lbm_status s = check_params(params, g_err, sizeof(g_err));
  if (s != LBM_OK) return s;
  const Layout L = make_layout(*params);
  if (plane_stride_out) *plane_stride_out = L.ps;
  if (f_off) *f_off = L.f_off;
  if (a_off) *a_off = L.a_off;
  if (g_off) *g_off = L.g_off;
  return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx* c, void* d_dst) {
  if (!c) return LBM_ERR_ARG;
  if (!d_dst) return fail(c, LBM_ERR_ARG, "destination is NULL");
  HIP_TRY(c, hipMemcpyAsync(d_dst, c->ws + c->L.state[c->cur], c->L.state_bytes, hipMemcpyDeviceToDevice, c->stream));
  return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx* c, const void* d_src, int64_t steps_done) {
  if (!c) return LBM_ERR_ARG;
  if (!d_src) return fail(c, LBM_ERR_ARG, "source is NULL");
  if (steps_done < 0) return fail(c, LBM_ERR_ARG, "steps_done must be >= 0");
  HIP_TRY(c, hipMemcpyAsync(c->ws + c->L.state[c->cur], d_src, c->L.state_bytes, hipMemcpyDeviceToDevice, c->stream));
  c->steps = steps_done;
  return LBM_OK;
}

lbm_status lbm_set_profiling(lbm_ctx* c, int32_t enable) {
  if (!c) return LBM_ERR_ARG;
  if (enable && c->ev.empty()) {
    c->ev.resize(kEvents * size_t(kRing));
    for (auto& e : c->ev) HIP_TRY(c, hipEventCreate(&e));
  }
  c->prof = enable != 0;
  for (double& v : c->kernel_ms) v = 0.0;
  c->prof_steps = 0;
  return LBM_OK;
}

lbm_status lbm_kernel_times(lbm_ctx* c, double* kernel_ms, int64_t* steps) {
  if (!c || !kernel_ms) return LBM_ERR_ARG;
  for (int k = 0; k < kTimed; ++k) kernel_ms[k] = c->kernel_ms[k];
  if (steps) *steps = c->prof_steps;
  return LBM_OK;
}

lbm_status lbm_adjoint_bytes(const lbm_params* params, size_t* adj_bytes, size_t* scratch_bytes) {
  lbm_status s = check_params(params, g_err, sizeof(g_err));
  if (s != LBM_OK) return s;
  const AdjLayout AL = make_adj_layout(*params);
  if (adj_bytes) *adj_bytes = AL.adj_bytes;
  if (scratch_bytes) *scratch_bytes = AL.total;
  return LBM_OK;
}

lbm_status lbm_adjoint_seed(lbm_ctx* c, const void* d_state, void* d_adj) {
  if (!c) return LBM_ERR_ARG;
  if (!d_state || !d_adj) return fail(c, LBM_ERR_ARG, "state and adjoint buffers are required");
  DISPATCH(c, launch_adj_seed, d_state, d_adj);
}

lbm_status lbm_adjoint_step(lbm_ctx* c, const void* d_state, const void* d_adj_in, void* d_adj_out, void* d_scratch,
                            double* d_grad_theta, double* d_grad_xi) {
  if (!c) return LBM_ERR_ARG;
  if (!d_state || !d_adj_in || !d_adj_out || !d_scratch || !d_grad_theta || !d_grad_xi)
    return fail(c, LBM_ERR_ARG, "all buffers are required");
  const lbm_status chk = check_adjoint_buffers(c, d_state, nullptr, d_adj_in, d_adj_out, d_scratch);
  if (chk != LBM_OK) return chk;
  const void* no_fields = nullptr;
  DISPATCH(c, launch_adj_step, d_state, no_fields, d_adj_in, d_adj_out, d_scratch, d_grad_theta, d_grad_xi);
}

lbm_status lbm_adjoint_step_fields(lbm_ctx* c, const void* d_state, const void* d_fields, const void* d_adj_in,
                                   void* d_adj_out, void* d_scratch, double* d_grad_theta, double* d_grad_xi) {
  if (!c) return LBM_ERR_ARG;
  if (!d_state || !d_fields || !d_adj_in || !d_adj_out || !d_scratch || !d_grad_theta || !d_grad_xi)
    return fail(c, LBM_ERR_ARG, "all buffers are required");
  const lbm_status chk = check_adjoint_buffers(c, d_state, d_fields, d_adj_in, d_adj_out, d_scratch);
  if (chk != LBM_OK) return chk;
  DISPATCH(c, launch_adj_step, d_state, d_fields, d_adj_in, d_adj_out, d_scratch, d_grad_theta, d_grad_xi);
}

lbm_status lbm_adjoint_step_static(lbm_ctx* c, const void* d_state, const void* d_adj_in, void* d_adj_out,
                                   double* d_grad_theta, double* d_grad_xi) {
  if (!c) return LBM_ERR_ARG;
  if (!d_state || !d_adj_in || !d_adj_out || !d_grad_theta || !d_grad_xi)
    return fail(c, LBM_ERR_ARG, "all buffers are required");
  const size_t need = make_adj_layout(c->p).total;
  if (need > kStaticScratchBytes)
    return fail(c, LBM_ERR_ARG, "the adjoint step needs %zu bytes of scratch, more than the %zu of the static "
                "scratch; use lbm_adjoint_step with a caller-owned scratch buffer", need, kStaticScratchBytes);
  if (!c->static_scr) {
    c->static_scr = static_scratch(c->err, sizeof(c->err));
    if (!c->static_scr) return LBM_ERR_HIP;
  }
  void* scr = c->static_scr;
  const lbm_status chk = check_adjoint_buffers(c, d_state, nullptr, d_adj_in, d_adj_out, scr);
  if (chk != LBM_OK) return chk;
  const void* no_fields = nullptr;
  DISPATCH(c, launch_adj_step, d_state, no_fields, d_adj_in, d_adj_out, scr, d_grad_theta, d_grad_xi);
}

size_t lbm_adjoint_static_scratch_bytes(void) { return kStaticScratchBytes; }

int64_t lbm_steps_done(const lbm_ctx* c) { return c ? c->steps : -1; }

void lbm_free(lbm_ctx* c) {
  if (!c) return;
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err : g_err; }

}  // extern "C"

// Forward kernels of one time step (HIP, gfx950).
//
// Storage. The state arrays hold fluid nodes only, indexed by fluid id (the rank of the node
// among fluid nodes in node order, so rows stay contiguous); thread t of a launch is fluid node t
// and writes its own slot, which makes every store a full coalesced line. Pulls find the id of
// the source node through a dense node -> id map. The small per-node fields (rho^N, the info
// word, the id map) stay dense, because the stencils also read them at solid nodes.
//
// State representation. Under Latva-Kokko recolouring of the colour-blind post-collision
// populations (eq. operator_recoloring) followed by the proportional wall-reaction transfer,
// the two colours' post-collision populations at a node are always
//     f^r_i = a f^m_i + (w_i/|c_i|) c_i . v,     f^p_i = b f^m_i - (w_i/|c_i|) c_i . v,
// with a = (1 - phi) rho^r / rho^m, b = 1 - a and v = (1 - phi) beta (rho^r rho^p / rho^m) n*. The
// state is therefore stored exactly as the 19 colour-blind populations f^m (storage precision),
// the four per-node scalars (a or b, v) (arithmetic precision) and, with the species, 7
// populations g: 30 values per node instead of 45. Pulling f^r_i from node x - c_i reads f^m_i
// and the scalars there.
//
// Near-pure phases. Where one colour is a trace (gas nucleating at a wall, a liquid film inside
// a bubble), storing a next to 1 or rho^N next to +-1 would round the trace colour to the
// absolute precision of the arithmetic type (6e-8 in FP32), and the interface normal, which
// divides by a gradient that may be as small as 1e-6, would be noise. Both are therefore kept
// in a minority form (pack_frac, rn_diff below): the smaller member of each pair (a, b) and
// ((1 + rho^N)/2, (1 - rho^N)/2) is stored at full relative precision, the sign bit telling
// which one it is. Colour densities and gradients of rho^N are formed from those directly.
//
// Layout: structure of arrays, one plane per population, planes a padded stride ps (at least the
// number of fluid nodes) apart, fluid ids in node order (x fastest); the colour scalars (a, v) as
// one 4-vector per fluid node. Two state buffers are used alternately (pull from one, write the
// other), so no kernel reads what another thread of the same launch writes.
//
// One step is four launches (each one thread per node):
//   colour   pull f^m, a, v -> rho^N at fluid nodes             (eqs. moments_components, color_function)
//   extrap   rho^N into solid nodes next to fluid               (eq. color_lattice_weighted_average)
//   normal   isotropic gradient, unit normal, Akai realignment   (eqs. finite_difference_scheme,
//                                                                 color_gradient_normal, realigned_normal_vectors)
//   collide  pull, curvature, forcing, central-moment collision, recolouring, reaction,
//            species, store, FP64 reductions                     (remaining equations)
// The 3-hop dependency rho^N -> n -> curvature between neighbours is what forces the split.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "lattice.hpp"
#include "precision.hpp"

namespace lbm {

constexpr int kBlock = 256;
constexpr int kXcd = 8;


// Per-node 4-vectors (colour scalars a, v; realigned normal and |G|; wetting data) are stored
// together (16 or 32 bytes per node) so that one load brings all four: a gather's cost follows
// the cache lines it touches, so loading a subset of the four costs about as much as all four.
template <class R> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };
template <class R> struct V2;
template <> struct V2<float> { using T = float2; };
template <> struct V2<double> { using T = double2; };
template <class R>
__device__ inline typename V4<R>::T ld4(const R* p, size_t n) { return reinterpret_cast<const typename V4<R>::T*>(p)[n]; }
template <class R>
__device__ inline void st4(R* p, size_t n, R x, R y, R z, R w) {
  typename V4<R>::T v;
  v.x = x; v.y = y; v.z = z; v.w = w;
  reinterpret_cast<typename V4<R>::T*>(p)[n] = v;
}  // MI355X: 8 XCDs; workgroups are dealt round-robin across them

// A pair of colour fractions (a, b), a + b = 1, stored as one number that holds the smaller one
// to full relative precision: e = -|b| (sign bit set) when 0 <= b <= a or a < 0, else e = |a|.
// So e = -0 is the pure reactant (red) state and e = +0 the pure product (blue) state; values
// outside [0, 1] (a colour density that rounded below zero) keep their sign consistently.
template <class R>
__device__ inline R pack_frac(R a, R b) {
  const bool minor_b = (b <= a && b >= R(0)) || a < R(0);
  return minor_b ? -fabs(b) : fabs(a);
}
template <class R>
__device__ inline void unpack_frac(R e, R& a, R& b) {
  if (signbit(e)) {
    b = -e;
    a = R(1) - b;
  } else {
    a = e;
    b = R(1) - a;
  }
}
// rho^N = a - b is stored as q = rho^N - s with s = +1 if the sign bit of q is set (product
// colour in the minority, q = -2b) and s = -1 otherwise (q = 2a).
template <class R>
__device__ inline R rn_side(R q) { return signbit(q) ? R(1) : R(-1); }
template <class R>
__device__ inline R rn_value(R q) { return q + rn_side(q); }
// rho^N(x) - rho^N(y) without the cancellation of two values next to +-1.
template <class R>
__device__ inline R rn_diff(R qx, R qy) { return (qx - qy) + (rn_side(qx) - rn_side(qy)); }
// q from the colour densities (rm = rho^r + rho^p up to rounding).
template <class R>
__device__ inline R rn_pack(R rr, R rp, R irm) { return R(2) * pack_frac(rr * irm, rp * irm); }
// rho^r and rho^p at a node from q and rho^m, the minority one directly.
template <class R>
__device__ inline void rn_densities(R q, R rm, R& rr, R& rp) {
  if (signbit(q)) {
    rp = R(-0.5) * q * rm;
    rr = rm - rp;
  } else {
    rr = R(0.5) * q * rm;
    rp = rm - rr;
  }
}

// Maps the hardware workgroup id to a logical tile so that each XCD (with its own L2) works on
// one contiguous slab of the lattice; neighbouring rows then share that XCD's L2.
// gridDim.x is always a multiple of kXcd.
__device__ inline int logical_block() {
  int per_xcd = gridDim.x / kXcd;
  return (blockIdx.x % kXcd) * per_xcd + blockIdx.x / kXcd;
}

// The tile of kBlock consecutive fluid ids that this workgroup processes: its XCD-aware launch
// index, through the context's tile order when there is one (on large lattices the tiles are
// launched in y-bands swept through z, so that tiles whose nodes neighbour each other across
// planes are in flight on the same XCD and share its L2).
template <class SA>
__device__ inline int fluid_tile(const SA& A) {
  const int lb = logical_block();
  return A.order ? A.order[lb] : lb;
}

// Periodic neighbour offsets of one node.
struct Nbr {
  int n, x;
  int dxm, dxp, dym, dyp, dzm, dzp;
  __device__ inline int at(int cx, int cy, int cz) const {
    return n + (cx > 0 ? dxp : (cx < 0 ? dxm : 0)) + (cy > 0 ? dyp : (cy < 0 ? dym : 0)) +
           (cz > 0 ? dzp : (cz < 0 ? dzm : 0));
  }
};

// Division by a runtime constant d for 0 <= n < 2^31: q = (umulhi(n, m) + n) >> s with
// s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1 (computed on the host).
struct FastDiv {
  uint32_t d, m, s;
  __device__ inline uint32_t div(uint32_t n) const { return (__umulhi(n, m) + n) >> s; }
};

struct Geom {
  int nx, ny, nz;
  FastDiv fx, fy;
};

__device__ inline Nbr make_nbr(int n, const Geom& g) {
  Nbr b;
  b.n = n;
  const uint32_t t = g.fx.div(uint32_t(n));
  const int x = n - int(t) * g.nx;
  const int z = int(g.fy.div(t));
  const int y = int(t) - z * g.ny;
  const int nx = g.nx, ny = g.ny, nz = g.nz, nxy = nx * ny;
  b.x = x;
  b.dxm = (x == 0) ? nx - 1 : -1;
  b.dxp = (x == nx - 1) ? -(nx - 1) : 1;
  b.dym = (y == 0) ? (ny - 1) * nx : -nx;
  b.dyp = (y == ny - 1) ? -(ny - 1) * nx : nx;
  b.dzm = (z == 0) ? (nz - 1) * nxy : -nxy;
  b.dzp = (z == nz - 1) ? -(nz - 1) * nxy : nxy;
  return b;
}

// Direction with no x component and the same y and z components as direction i (-1 for the
// x axis, whose counterpart is the rest position).
constexpr int yz_partner(int i) {
  for (int j = 0; j < 18; ++j)
    if (D3Q19::cx[j] == 0 && D3Q19::cy[j] == D3Q19::cy[i] && D3Q19::cz[j] == D3Q19::cz[i]) return j;
  return -1;
}

// Fluid ids of the 18 pull sources x - c_i of fluid node t, the node's own id where the source is
// solid. Fluid ids are ranks in dense order, so two fluid nodes next to each other along x within
// a row (no periodic wrap) have ids one apart: a source x - c_i with c_ix != 0 takes the id of its
// partner (x, y - c_iy, z - c_iz) minus c_ix when the partner is fluid, and the id map is read only
// for the other sources. All of those reads are issued before any id is formed, so they are in
// flight together.
// x - cx (cx = +-1) is the next node along the row of x (no periodic wrap between them).
__device__ inline bool row_step(const Nbr& nb, int cx) { return cx > 0 ? nb.dxm == -1 : nb.dxp == 1; }

__device__ inline void pull_sources(const int* fid, const Nbr& nb, int t, uint32_t inf, int sid[18]) {
  using D = D3Q19;
  // Which ids follow from a neighbour's: known from the info bits alone, before any load.
  bool derived[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    const int m = yz_partner(i);
    const bool mfluid = (m < 0) || !((inf >> m) & 1u);
    derived[i] = (D::cx[i] != 0) && mfluid && row_step(nb, D::cx[i]);
  }
  // Every id-map read first, so that they are in flight together; only then the ids.
  int look[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    look[i] = 0;
    if (!((inf >> i) & 1u) && !derived[i]) look[i] = fid[nb.at(-D::cx[i], -D::cy[i], -D::cz[i])];
  }
#pragma unroll
  for (int i = 0; i < 18; ++i)
    if (D::cx[i] == 0) sid[i] = ((inf >> i) & 1u) ? t : look[i];
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    if (D::cx[i] == 0) continue;
    const int m = yz_partner(i);
    const int mid = (m < 0) ? t : sid[m];
    sid[i] = ((inf >> i) & 1u) ? t : (derived[i] ? mid - D::cx[i] : look[i]);
  }
}

// The same ids with fewer registers live: each id-map read is consumed as it arrives, so the reads
// are not all in flight at once. For the adjoint passes, whose other state leaves few registers
// (the batched form made them spill or lose a wave per SIMD).
__device__ inline void pull_sources_lean(const int* fid, const Nbr& nb, int t, uint32_t inf, int sid[18]) {
  using D = D3Q19;
#pragma unroll
  for (int i = 0; i < 18; ++i)
    if (D::cx[i] == 0) sid[i] = ((inf >> i) & 1u) ? t : fid[nb.at(0, -D::cy[i], -D::cz[i])];
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    if (D::cx[i] == 0) continue;
    const int m = yz_partner(i);
    const int mid = (m < 0) ? t : sid[m];
    const bool mfluid = (m < 0) || !((inf >> m) & 1u);
    sid[i] = ((inf >> i) & 1u) ? t : ((mfluid && row_step(nb, D::cx[i])) ? mid - D::cx[i] : fid[nb.at(-D::cx[i], -D::cy[i], -D::cz[i])]);
  }
}

// Cross-lane moves within the 64-wide wave (DPP wave shifts, one VALU move per 32-bit word): the
// value that lane l - 1 (from_below) or lane l + 1 (from_above) holds in the same register. The end
// lanes of the wave receive their own value; callers use the result only where the neighbouring
// lane is active and holds the wanted node.
__device__ inline int lane_from_below(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false); }
__device__ inline int lane_from_above(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false); }
template <int DIR>
__device__ inline float lane_move(float v) {
  const int b = __float_as_int(v);
  return __int_as_float(DIR < 0 ? lane_from_below(b) : lane_from_above(b));
}
template <int DIR>
__device__ inline double lane_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = int(uint32_t(b)), hi = int(uint32_t(uint64_t(b) >> 32));
  const int mlo = DIR < 0 ? lane_from_below(lo) : lane_from_above(lo);
  const int mhi = DIR < 0 ? lane_from_below(hi) : lane_from_above(hi);
  return __longlong_as_double((long long)((uint64_t(uint32_t(mhi)) << 32) | uint32_t(mlo)));
}
template <int DIR>
__device__ inline float2 lane_move(const float2& v) {
  return make_float2(lane_move<DIR>(v.x), lane_move<DIR>(v.y));
}
template <int DIR>
__device__ inline double2 lane_move(const double2& v) {
  return make_double2(lane_move<DIR>(v.x), lane_move<DIR>(v.y));
}
template <int DIR>
__device__ inline float4 lane_move(const float4& v) {
  return make_float4(lane_move<DIR>(v.x), lane_move<DIR>(v.y), lane_move<DIR>(v.z), lane_move<DIR>(v.w));
}
template <int DIR>
__device__ inline double4 lane_move(const double4& v) {
  return make_double4(lane_move<DIR>(v.x), lane_move<DIR>(v.y), lane_move<DIR>(v.z), lane_move<DIR>(v.w));
}

// Values of a per-node quantity at the 18 neighbours x - c_i of fluid node x (out[i]), fetched with
// one gather per row. The sources x - c_i with c_ix != 0 lie on the row of the source
// x - (0, c_iy, c_iz) of the partner direction, one node along x; when the node's own neighbour
// x - c_ix along the row is fluid, it is the next fluid id and lane l - c_ix of the same wave holds
// it, and that lane's partner value is exactly the one wanted. Those values are moved across lanes
// instead of gathered, so each row triple costs one gather; the other lanes (wave ends, periodic
// wrap, a solid neighbour along x) gather their own. ld(i) gathers the value of direction i; own is
// the node's own value (the source of the x-shifted directions of the node's own row). SOLID_OWN:
// where x - c_i is solid the node's own value stands in (state vectors, whose solid sources are
// bounce-back); otherwise every neighbour has a value of its own (rho^N, extrapolated into solids).
// Every 64 consecutive threads of a launch hold consecutive fluid ids.
template <bool SOLID_OWN, class T, class Load>
__device__ inline void row_shared(const Nbr& nb, uint32_t inf, const T& own, Load ld, T out[18]) {
  using D = D3Q19;
  const int lane = __lane_id();
  // lane l - 1 holds node x - 1 of this row (direction 0 pulls from x - 1), lane l + 1 node x + 1
  const bool below = !(inf & 1u) && nb.dxm == -1 && lane > 0;
  const bool above = !((inf >> 1) & 1u) && nb.dxp == 1 && lane < 63;
  // The gathers: partner directions (c_ix = 0) for every lane, x-shifted directions only where the
  // neighbouring lane cannot supply them, all issued before any cross-lane move.
  T gathered[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    const bool solid = SOLID_OWN && ((inf >> i) & 1u);
    if (D::cx[i] == 0) {
      out[i] = ld(i);
    } else if (!solid && !(D::cx[i] > 0 ? below : above)) {
      gathered[i] = ld(i);
    }
  }
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    if (D::cx[i] == 0) continue;
    const int m = yz_partner(i);
    const T base = (m < 0) ? own : out[m];
    const T moved = (D::cx[i] > 0) ? lane_move<-1>(base) : lane_move<+1>(base);
    const bool solid = SOLID_OWN && ((inf >> i) & 1u);
    out[i] = solid ? own : ((D::cx[i] > 0 ? below : above) ? moved : gathered[i]);
  }
}

template <int P>
struct StepArgs {
  using S = typename Prec<P>::S;
  using R = typename Prec<P>::R;
  int nx, ny, nz, N;
  size_t ps;              // plane stride of the state and adjoint planes (>= fluid nodes)
  Geom geo;
  const int* fluid;       // dense indices of the fluid nodes, in increasing order
  const uint32_t* finfo;  // their info words
  int nfluid;
  const int* ext;         // dense indices of the solid nodes whose colour is extrapolated
  const uint32_t* einfo;  // their info words
  int next;
  const int* fid;         // dense node -> fluid id (index into the state arrays), -1 for solid
  const int* order;       // optional launch order of the fluid-list tiles (null: list order)
  const uint32_t* info;
  // state in (pull source) and out
  const S* fin;  // 19 planes f^m
  const R* ain;  // per node 4-vector (e, vx, vy, vz), e = pack_frac(a, b)
  const S* gin;  // 7 planes species
  const R* cin;  // 2-byte storages: the species total of each node (deviation reference of gin)
  S* fout;
  R* aout;
  S* gout;
  R* cout;
  R* rhoN;       // 1 plane, rho^N in the form of rn_value
  R* rm_out;     // optional: rho^m of each fluid node (adjoint recompute)
  R* nst;        // per fluid id 4-vector (n*_x, n*_y, n*_z, |grad rho^N|)
  R* nraw;       // optional: per fluid id, the unit normal before the wetting realignment at
                 // wetting nodes (kept for the adjoint; elsewhere it equals n*)
  const R* wet;  // per fluid id 4-vector (n_s, cos(theta))
  double* partials;
  double* ring_row;  // 5 doubles of this step
  // Deferred final reduction of the previous step, done by workgroup 0 of the step's first pass
  // (null: none)
  const double* red_in;
  int red_n;
  double* red_out;
  R relax;           // 1 - 1/tau
  R inv_tau_c;
  R sigma, beta, xi, c_in, eps;
  R acc[2][3];
  R scale, inv_scale;
  R gscale, inv_gscale;
  int species;
  // moments mode outputs (may be null)
  R* m_rr;
  R* m_rp;
  R* m_rn;
  R* m_u;
  R* m_c;
};

// Species storage. FP32 and FP64 hold the populations g_q themselves. The 2-byte storages hold
// each node's post-collision species total C (arithmetic type, plane cin/cout) and the
// populations as deviations (g_q - w_q C) 2^k from the equilibrium at rest of that total: those
// are small (advection and non-equilibrium parts only) wherever C lies in [0, 1], so the 11 or 8
// significant bits of the storage apply to them and not to C itself. Population q of the node with
// fluid id src:
template <int P>
__device__ inline typename Prec<P>::R ld_species(const StepArgs<P>& A, int q, int src) {
  using R = typename Prec<P>::R;
  const R w = R(D3Q7::w(q));
  return Prec<P>::ld(A.gin[size_t(q) * A.ps + src], P >= 2 ? w * A.cin[src] : w, A.inv_gscale);
}

// Sum of the per-workgroup partials (5 planes of nparts) by one workgroup of kBlock threads, in
// a fixed order: strided per-thread sums, then wavefront shuffles, then the waves in order. Every
// caller uses this one routine with the same thread count, so a step's sums do not depend on
// where the reduction ran.
__device__ inline void reduce_partials(const double* partials, int nparts, double* out) {
  __shared__ double red[kBlock / 64][5];
  double t[5] = {0, 0, 0, 0, 0};
  int b = threadIdx.x;
  for (; b + 3 * kBlock < nparts; b += 4 * kBlock) {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const double* p = partials + size_t(j) * nparts;
      t[j] += ((p[b] + p[b + kBlock]) + (p[b + 2 * kBlock] + p[b + 3 * kBlock]));
    }
  }
  for (; b < nparts; b += kBlock) {
#pragma unroll
    for (int j = 0; j < 5; ++j) t[j] += partials[size_t(j) * nparts + b];
  }
#pragma unroll
  for (int j = 0; j < 5; ++j) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t[j] += __shfl_xor(t[j], off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < 5; ++j) red[wave][j] = t[j];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      double v = red[0][j];
#pragma unroll
      for (int w = 1; w < kBlock / 64; ++w) v += red[w][j];
      out[j] = v;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_finish_reduce(const double* partials, int nparts, double* out) {
  reduce_partials(partials, nparts, out);
}

// ---------------------------------------------------------------------------------------------
// colour: rho^N = (rho^r - rho^p)/rho^m from the pulled populations. The pull-source ids come
// from pull_sources (most of them derived from a neighbour's rank) and the sources' colour
// scalars from row_shared (one gather per row triple); the pass is bound by its gathers' address
// and cache-line work, not by its bytes (102 VGPRs, four waves per SIMD).
// ---------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void k_colour(StepArgs<P> A) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  if (A.red_out && blockIdx.x == 0) reduce_partials(A.red_in, A.red_n, A.red_out);
  const int t = fluid_tile(A) * kBlock + threadIdx.x;
  if (t >= A.nfluid) return;
  const int n = A.fluid[t];
  const uint32_t inf = A.finfo[t];
  const Nbr nb = make_nbr(n, A.geo);
  int sid[18];
  pull_sources(A.fid, nb, t, inf, sid);
  const typename V4<R>::T own = ld4(A.ain, t);
  typename V4<R>::T avs[18];  // (e, v) at the sources (own where solid: bounce-back)
  row_shared<true>(nb, inf, own, [&](int i) { return ld4(A.ain, sid[i]); }, avs);
  R rm = 0, rr = 0, rp = 0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const bool bb = (i < 18) && ((inf >> i) & 1u);
    const int src = (i == 18) ? t : sid[i];
    const int q = bb ? D::opp[i] : i;
    const R sgn = bb ? R(-1) : R(1);  // c_q = sgn * c_i
    const R fm = Prec<P>::ld(A.fin[size_t(q) * A.ps + src], R(D::w(i)), A.inv_scale);
    const typename V4<R>::T av = (i == 18) ? own : avs[i];
    const R cv = R(D::cx[i]) * av.y + R(D::cy[i]) * av.z + R(D::cz[i]) * av.w;
    R a, b;
    unpack_frac(av.x, a, b);
    const R kv = R(D::w_over_len(i)) * sgn * cv;
    rm += fm;
    rr += a * fm + kv;
    rp += b * fm - kv;
  }
  A.rhoN[n] = rn_pack(rr, rp, R(1) / rm);
  if (A.rm_out) A.rm_out[n] = rm;
}

// ---------------------------------------------------------------------------------------------
// extrap: colour of solid nodes next to fluid, lattice-weighted average of fluid neighbours.
// ---------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void k_extrap(StepArgs<P> A) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int t = logical_block() * kBlock + threadIdx.x;
  if (t >= A.next) return;
  const int n = A.ext[t];
  const uint32_t inf = A.einfo[t];
  const Nbr nb = make_nbr(n, A.geo);
  // All 18 loads are issued before any is used, so their latencies overlap; a direction without a
  // fluid neighbour loads nothing (its lanes are masked off, which spares the address units; reading
  // the node's own entry instead made the pass 11% slower at 128^3).
  R qv[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    qv[i] = R(0);
    if ((inf >> i) & 1u) qv[i] = A.rhoN[nb.at(D::cx[i], D::cy[i], D::cz[i])];
  }
  // Weighted sums of the offsets q and of the sides s separately; -0 as the start keeps the
  // sign of an all-(-0) sum.
  R nq = R(-0.0), ns = 0, den = 0;
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    const bool use = (inf >> i) & 1u;
    nq = use ? nq + R(D::w(i)) * qv[i] : nq;
    ns = use ? ns + R(D::w(i)) * rn_side(qv[i]) : ns;
    den = use ? den + R(D::w(i)) : den;
  }
  if (ns == den || ns == -den) {
    A.rhoN[n] = nq / den;  // all neighbours on one side: the average keeps that side
  } else {
    const R v = (ns + nq) / den;
    A.rhoN[n] = R(2) * pack_frac(R(0.5) * (R(1) + v), R(0.5) * (R(1) - v));
  }
}

// ---------------------------------------------------------------------------------------------
// normal: G = 3 sum_i w_i c_i rho^N(x + c_i) as pair differences (a uniform field gives exactly
// zero), n = +G/|G| (the opposite of the sign printed in eq. color_gradient_normal: with +G the
// force, curvature, recolouring and wetting angle all act with the physical sign, theta measured
// through the reactant colour), and at wetting nodes the Akai realignment
// n* = n+ (n+ is always at least as close to n as n-: n+.n - n-.n = 2 sin(theta) sin(theta')).
// ---------------------------------------------------------------------------------------------
// The normal of one fluid node from the nine pair differences d_j = rho^N(x + c_p) - rho^N(x - c_p),
// p = half[j], of its neighbours' colour (rn_diff form): G, |G|, n = G/|G|, and at wetting nodes
// the Akai realignment with wv = (n_s, cos(theta)). raw: the unit normal before realignment, set
// (and raw_set true) at wetting nodes with |G| > eps. Every pass that forms a normal calls this.
template <class R>
__device__ inline void normal_from_pairs(const R d[9], uint32_t inf, const typename V4<R>::T& wv, R eps, R nv[3],
                                         R& len, R raw[3], bool& raw_set) {
  using D = D3Q19;
  R g[3] = {0, 0, 0};
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const int p = D::half[j];
    const R c3w = R(3.0 * D::w(p));
    if (D::cx[p]) g[0] += c3w * R(D::cx[p]) * d[j];
    if (D::cy[p]) g[1] += c3w * R(D::cy[p]) * d[j];
    if (D::cz[p]) g[2] += c3w * R(D::cz[p]) * d[j];
  }
  len = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  nv[0] = nv[1] = nv[2] = R(0);
  raw_set = false;
  if (len > eps) {
    const R il = R(1) / len;
    nv[0] = g[0] * il; nv[1] = g[1] * il; nv[2] = g[2] * il;
    if (inf & kWet) {
      raw[0] = nv[0]; raw[1] = nv[1]; raw[2] = nv[2];
      raw_set = true;
      const R sx = wv.x, sy = wv.y, sz = wv.z;
      if (sx * sx + sy * sy + sz * sz > R(0.5)) {
        const R ct = wv.w;
        const R st = sqrt(fmax(R(0), (R(1) - ct) * (R(1) + ct)));
        // cos and sin of theta' from the dot and cross products (accurate next to +-n_s).
        const R cp = sx * nv[0] + sy * nv[1] + sz * nv[2];
        const R q0 = nv[1] * sz - nv[2] * sy, q1 = nv[2] * sx - nv[0] * sz, q2 = nv[0] * sy - nv[1] * sx;
        const R sp = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
        // n+ = cos(theta) n_s + sin(theta) t, t = (n - cos(theta') n_s)/sin(theta'): n rotated in
        // the plane of n and n_s to the angle theta. Within sin(theta') < 1e-2 of +-n_s that plane
        // is not defined by n (an interface parallel to the wall) and n is kept; this also caps
        // the 1/sin(theta') amplification of rounding at 100.
        if (sp >= R(1e-2)) {
          const R b = st / sp;
          const R a = ct - b * cp;
          nv[0] = a * sx + b * nv[0];
          nv[1] = a * sy + b * nv[1];
          nv[2] = a * sz + b * nv[2];
        }
      }
    }
  }
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_normal(StepArgs<P> A) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int t = logical_block() * kBlock + threadIdx.x;
  if (t >= A.nfluid) return;
  const int n = A.fluid[t];
  const uint32_t inf = A.finfo[t];
  const Nbr nb = make_nbr(n, A.geo);
  // The wetting data of a wetting node is loaded with the neighbours' colours, not after the
  // gradient: one memory round trip for the node instead of two.
  typename V4<R>::T wv;
  wv.x = wv.y = wv.z = wv.w = R(0);
  if (inf & kWet) wv = ld4(A.wet, t);
  R src[18];  // rho^N at x - c_i (solid neighbours hold their extrapolated colour)
  row_shared<false>(nb, inf, A.rhoN[n], [&](int i) { return A.rhoN[nb.at(-D::cx[i], -D::cy[i], -D::cz[i])]; }, src);
  R d[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const int p = D::half[j];
    d[j] = rn_diff(src[D::opp[p]], src[p]);  // x + c_p is the source of opp(p)
  }
  R nv[3], len, raw[3];
  bool raw_set;
  normal_from_pairs<R>(d, inf, wv, A.eps, nv, len, raw, raw_set);
  if (raw_set && A.nraw) st4(A.nraw, t, raw[0], raw[1], raw[2], R(0));
  st4(A.nst, t, nv[0], nv[1], nv[2], len);
}

// T^{-1} k* of Appendix A (eq. back_transformation_vector), regrouped with common
// subexpressions: for a move along +-x, q_x = u_x^2 +- u_x, and similarly for y, z.
template <class R>
__device__ inline void cm_back(R ux, R uy, R uz, R k5, R k6, R k7, R k8, R k9, R d[19]) {
  const R x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
  const R pxp = x2 + ux, pxm = x2 - ux, pyp = y2 + uy, pym = y2 - uy, pzp = z2 + uz, pzm = z2 - uz;
  const R ax = k5 * R(1.0 / 3.0) + k6 * R(1.0 / 6.0);
  const R ay = (k6 - k5) * R(1.0 / 6.0);
  const R az = -(k5 * R(1.0 / 6.0) + k6 * R(1.0 / 3.0));
  const R tx = uy * k7 + uz * k8, ty = ux * k7 + uz * k9, tz = ux * k8 + uy * k9;
  const R ux2 = ux + ux, uy2 = uy + uy, uz2 = uz + uz;
  d[0] = (pxp - y2 - z2 + R(1)) * ax - (ux2 + R(1)) * tx;
  d[1] = (pxm - y2 - z2 + R(1)) * ax - (ux2 - R(1)) * tx;
  d[2] = (pyp - x2 - z2 + R(1)) * ay - (uy2 + R(1)) * ty;
  d[3] = (pym - x2 - z2 + R(1)) * ay - (uy2 - R(1)) * ty;
  d[4] = (pzp - x2 - y2 + R(1)) * az - (uz2 + R(1)) * tz;
  d[5] = (pzm - x2 - y2 + R(1)) * az - (uz2 - R(1)) * tz;
  const R c12 = R(1.0 / 12.0), c4 = R(0.25);
  // xy plane: (-q_x + 2 q_y) k5 + (q_x + q_y) k6 + 3 (2u_x + s_x)(2u_y + s_y) k7, all / 12
  d[6] = ((pyp + pyp - pxp) * k5 + (pxp + pyp) * k6) * c12 + (ux2 + R(1)) * (uy2 + R(1)) * k7 * c4;
  d[7] = ((pym + pym - pxp) * k5 + (pxp + pym) * k6) * c12 + (ux2 + R(1)) * (uy2 - R(1)) * k7 * c4;
  d[10] = ((pyp + pyp - pxm) * k5 + (pxm + pyp) * k6) * c12 + (ux2 - R(1)) * (uy2 + R(1)) * k7 * c4;
  d[11] = ((pym + pym - pxm) * k5 + (pxm + pym) * k6) * c12 + (ux2 - R(1)) * (uy2 - R(1)) * k7 * c4;
  // xz plane: (-q_x + 2 q_z) k5 + (-2 q_x + q_z) k6 + 3 (2u_x + s_x)(2u_z + s_z) k8
  d[8] = ((pzp + pzp - pxp) * k5 + (pzp - pxp - pxp) * k6) * c12 + (ux2 + R(1)) * (uz2 + R(1)) * k8 * c4;
  d[9] = ((pzm + pzm - pxp) * k5 + (pzm - pxp - pxp) * k6) * c12 + (ux2 + R(1)) * (uz2 - R(1)) * k8 * c4;
  d[12] = ((pzp + pzp - pxm) * k5 + (pzp - pxm - pxm) * k6) * c12 + (ux2 - R(1)) * (uz2 + R(1)) * k8 * c4;
  d[13] = ((pzm + pzm - pxm) * k5 + (pzm - pxm - pxm) * k6) * c12 + (ux2 - R(1)) * (uz2 - R(1)) * k8 * c4;
  // yz plane: (-q_y - q_z) k5 + (-2 q_y + q_z) k6 + 3 (2u_y + s_y)(2u_z + s_z) k9
  d[14] = (-(pyp + pzp) * k5 + (pzp - pyp - pyp) * k6) * c12 + (uy2 + R(1)) * (uz2 + R(1)) * k9 * c4;
  d[15] = (-(pyp + pzm) * k5 + (pzm - pyp - pyp) * k6) * c12 + (uy2 + R(1)) * (uz2 - R(1)) * k9 * c4;
  d[16] = (-(pym + pzp) * k5 + (pzp - pym - pym) * k6) * c12 + (uy2 - R(1)) * (uz2 + R(1)) * k9 * c4;
  d[17] = (-(pym + pzm) * k5 + (pzm - pym - pym) * k6) * c12 + (uy2 - R(1)) * (uz2 - R(1)) * k9 * c4;
  d[18] = ((y2 + z2 - x2 - x2) * k5 + (z2 + z2 - x2 - y2) * k6) * R(1.0 / 3.0) +
          R(4) * (ux * uy * k7 + ux * uz * k8 + uy * uz * k9);
}

template <class R>
__device__ inline bool finite(R v) {
  return isfinite(v);
}

// Deterministic FP64 reduction of 5 sums over a workgroup of NT threads: wavefront shuffles, then
// the workgroup's waves in fixed order; one partial per workgroup (plain stores, no fences or
// atomics). The sums are finished by reduce_partials, after the grid, in workgroup order.
template <int NT>
__device__ inline void block_reduce5_n(double s[5], double* partials) {
  __shared__ double red[NT / 64][5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s[j] += __shfl_xor(s[j], off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < 5; ++j) red[wave][j] = s[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int lb = logical_block();
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      double t = red[0][j];
#pragma unroll
      for (int w = 1; w < NT / 64; ++w) t += red[w][j];
      partials[size_t(j) * gridDim.x + lb] = t;
    }
  }
}

__device__ inline void block_reduce5(double s[5], double* partials) { block_reduce5_n<kBlock>(s, partials); }

// Pull of fluid node t with halfway bounce-back: f^m_i from S_t at x - c_i, or S_t,opp(i) at x
// where x - c_i is solid (sid: the sources' fluid ids, t for bounce-back), and likewise the species
// (the outflow plane takes its own S_1: zero gradient).
template <int P>
__device__ inline void pull_node(const StepArgs<P>& A, int t, uint32_t inf, const int sid[18],
                                 typename Prec<P>::R f[19], typename Prec<P>::R g[7]) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const bool bb = (i < 18) && ((inf >> i) & 1u);
    const int src = (i < 18) ? sid[i] : t;
    const int q = bb ? D::opp[i] : i;
    f[i] = Prec<P>::ld(A.fin[size_t(q) * A.ps + src], R(D::w(i)), A.inv_scale);
  }
#pragma unroll
  for (int i = 0; i < 7; ++i) g[i] = R(0);
  if (A.species) {
    const bool outlet = inf & kOutlet;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const bool own = (i == 1 && outlet);  // zero-gradient outflow: the node's own S_1
      const bool bb = !own && ((inf >> i) & 1u);
      const int src = own ? t : sid[i];
      const int q = own ? 1 : (bb ? D3Q7::opp[i] : i);
      g[i] = ld_species(A, q, src);
    }
    g[6] = ld_species(A, 6, t);
  }
}

// H |G| at fluid node x: the curvature H = -(tr J - n.J.n) (eq. interface_curvature) with
// J_ab = 3 sum_i w_i c_ib n*_a(x + c_i), times the gradient magnitude |G| of x; zero where
// |G| <= eps (no normal). nsv: (n*, |G|) of x; nbr(i): (n*, |G|) at x + c_i, or of x itself where
// x + c_i is solid (the value the curvature takes for a solid neighbour). Every pass that forms
// the curvature calls this.
template <class R, class NbrN>
__device__ inline R curvature_hg(const typename V4<R>::T& nsv, R eps, NbrN nbr) {
  using D = D3Q19;
  R J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    const typename V4<R>::T nbi = nbr(i);
    const R a0 = nbi.x, a1 = nbi.y, a2 = nbi.z;
    const R w3 = R(3.0 * D::w(i));
    if (D::cx[i]) { J[0][0] += w3 * R(D::cx[i]) * a0; J[1][0] += w3 * R(D::cx[i]) * a1; J[2][0] += w3 * R(D::cx[i]) * a2; }
    if (D::cy[i]) { J[0][1] += w3 * R(D::cy[i]) * a0; J[1][1] += w3 * R(D::cy[i]) * a1; J[2][1] += w3 * R(D::cy[i]) * a2; }
    if (D::cz[i]) { J[0][2] += w3 * R(D::cz[i]) * a0; J[1][2] += w3 * R(D::cz[i]) * a1; J[2][2] += w3 * R(D::cz[i]) * a2; }
  }
  const R glen = nsv.w;
  R H = 0;
  if (glen > eps) {
    const R nn[3] = {nsv.x, nsv.y, nsv.z};
    R nJn = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) nJn += nn[a] * nn[b] * J[a][b];
    H = -((J[0][0] + J[1][1] + J[2][2]) - nJn);
  }
  return H * glen;
}

// The collision and the rest of the step at one fluid node x (fluid id t, node n, info word inf):
// moments, forcing, central-moment collision, recolouring, reaction, species, store, and the
// node's contribution to the FP64 sums (added to red5). f, g: the pulled populations; rn: rho^N(x)
// (rn_value form); cur: (n*, H |G|) of x (n* = 0 where x has no normal). MOM writes the level-t
// fields instead.
template <int P, bool MOM>
__device__ inline void collide_node(const StepArgs<P>& A, int t, int n, uint32_t inf,
                                    const typename Prec<P>::R f[19], const typename Prec<P>::R g[7],
                                    typename Prec<P>::R rn, const typename V4<typename Prec<P>::R>::T& cur,
                                    double red5[5]) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const size_t N = A.N;
  // Moments (same summation order as k_colour, so rho^m agrees bit for bit).
  R rm = 0;
#pragma unroll
  for (int i = 0; i < 19; ++i) rm += f[i];
  R mx = 0, my = 0, mz = 0, pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    if (D::cx[i]) { mx += R(D::cx[i]) * f[i]; pxx += f[i]; }
    if (D::cy[i]) { my += R(D::cy[i]) * f[i]; pyy += f[i]; }
    if (D::cz[i]) { mz += R(D::cz[i]) * f[i]; pzz += f[i]; }
    if (D::cx[i] && D::cy[i]) pxy += R(D::cx[i] * D::cy[i]) * f[i];
    if (D::cx[i] && D::cz[i]) pxz += R(D::cx[i] * D::cz[i]) * f[i];
    if (D::cy[i] && D::cz[i]) pyz += R(D::cy[i] * D::cz[i]) * f[i];
  }
  const R irm = R(1) / rm;
  const R ux = mx * irm, uy = my * irm, uz = mz * irm;
  R rr, rp;
  rn_densities(rn, rm, rr, rp);

  // Realigned unit normal (zero where the node has no normal: a unit vector otherwise) and the
  // exact-difference forcing du^k = F^k / rho^k = (1/2) sigma H |G| n* / rho^m + a^k.
  const R n0 = cur.x, n1 = cur.y, n2 = cur.z;
  const bool has_n = n0 != R(0) || n1 != R(0) || n2 != R(0);
  const R fc = R(0.5) * A.sigma * cur.w * irm;
  const R dur[3] = {fc * n0 + A.acc[0][0], fc * n1 + A.acc[0][1], fc * n2 + A.acc[0][2]};
  const R dup[3] = {fc * n0 + A.acc[1][0], fc * n1 + A.acc[1][1], fc * n2 + A.acc[1][2]};
  const R upx = ux + R(0.5) * (rr * dur[0] + rp * dup[0]) * irm;
  const R upy = uy + R(0.5) * (rr * dur[1] + rp * dup[1]) * irm;
  const R upz = uz + R(0.5) * (rr * dur[2] + rp * dup[2]) * irm;

  R C = R(1);
  if (A.species) {
    C = 0;
#pragma unroll
    for (int i = 0; i < 7; ++i) C += g[i];
    if (inf & kInlet) C = A.c_in;
  }

  if (MOM) {
    if (A.m_rr) A.m_rr[n] = rr;
    if (A.m_rp) A.m_rp[n] = rp;
    if (A.m_rn) A.m_rn[n] = rn_value(rn);
    if (A.m_u) { A.m_u[n] = upx; A.m_u[N + n] = upy; A.m_u[2 * N + n] = upz; }
    if (A.m_c) A.m_c[n] = C;
  } else {
    // Central shear moments k5..k9 about the bare velocity, relaxed by (1 - 1/tau).
    const R cxx = pxx - rm * ux * ux, cyy = pyy - rm * uy * uy, czz = pzz - rm * uz * uz;
    const R k5 = A.relax * (cxx - cyy), k6 = A.relax * (cyy - czz);
    const R k7 = A.relax * (pxy - rm * ux * uy), k8 = A.relax * (pxz - rm * ux * uz), k9 = A.relax * (pyz - rm * uy * uz);
    R d[19];
    cm_back(ux, uy, uz, k5, k6, k7, k8, k9, d);
    // f^{m,*} = f^eq(rho^r, u + du^r) + f^eq(rho^p, u + du^p) + T^{-1} k*: the sum of both
    // colours' equilibria needs only M = sum_k rho^k U^k and Pi = sum_k rho^k U^k U^k.
    const R Ur[3] = {ux + dur[0], uy + dur[1], uz + dur[2]};
    const R Up[3] = {ux + dup[0], uy + dup[1], uz + dup[2]};
    const R M0 = rr * Ur[0] + rp * Up[0], M1 = rr * Ur[1] + rp * Up[1], M2 = rr * Ur[2] + rp * Up[2];
    const R Pxx = rr * Ur[0] * Ur[0] + rp * Up[0] * Up[0];
    const R Pyy = rr * Ur[1] * Ur[1] + rp * Up[1] * Up[1];
    const R Pzz = rr * Ur[2] * Ur[2] + rp * Up[2] * Up[2];
    const R Pxy = rr * Ur[0] * Ur[1] + rp * Up[0] * Up[1];
    const R Pxz = rr * Ur[0] * Ur[2] + rp * Up[0] * Up[2];
    const R Pyz = rr * Ur[1] * Ur[2] + rp * Up[1] * Up[2];
    const R base = rm - R(1.5) * (Pxx + Pyy + Pzz);
    R fs[19];
    R fsum = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const int cx = D::cx[i], cy = D::cy[i], cz = D::cz[i];
      R cM = 0, cPc = 0;
      if (cx) { cM += R(cx) * M0; cPc += Pxx; }
      if (cy) { cM += R(cy) * M1; cPc += Pyy; }
      if (cz) { cM += R(cz) * M2; cPc += Pzz; }
      if (cx && cy) cPc += R(2 * cx * cy) * Pxy;
      if (cx && cz) cPc += R(2 * cx * cz) * Pxz;
      if (cy && cz) cPc += R(2 * cy * cz) * Pyz;
      fs[i] = R(D::w(i)) * (base + R(3) * cM + R(4.5) * cPc) + d[i];
      fsum += fs[i];
    }
    // Wall reaction with level-t densities, capped at full conversion.
    const int rnn = int((inf & kRnnMask) >> kRnnShift);
    R delta = 0;
    if (rnn > 0 && rr > R(0)) {
      if (A.species) {
        if (C > R(0)) {
          const R rate = A.xi * R(rnn) * rr * C;
          const R cap = fmin(rr, C);
          delta = fmin(rate, cap);
        }
      } else {
        delta = fmin(A.xi * R(rnn), R(1)) * rr;
      }
    }
    const R keep = (delta != R(0)) ? R(1) - delta / rr : R(1);
    // Compact recoloured state: a = (rho^r - delta)/rho^m, b = (rho^p + delta)/rho^m,
    // v = keep beta rho^r rho^p/rho^m n* with keep = 1 - delta/rho^r.
    const R aout = pack_frac((rr - delta) * irm, (rp + delta) * irm);
    const R vc = keep * A.beta * rr * rp * irm;
    const R v0 = has_n ? vc * n0 : R(0), v1 = has_n ? vc * n1 : R(0), v2 = has_n ? vc * n2 : R(0);
#pragma unroll
    for (int i = 0; i < 19; ++i) A.fout[size_t(i) * A.ps + t] = Prec<P>::st(fs[i], R(D::w(i)), A.scale);
    st4(A.aout, t, aout, v0, v1, v2);
    bool ok = finite(fsum) && finite(aout) && finite(v0 + v1 + v2) && finite(rr) && finite(rp);
    if (A.species) {
      // BGK towards g^eq = w C (1 + 4 c.u_phys); at the inlet the populations are replaced by
      // the equilibrium at C_in; then the reaction sink.
      const bool inlet = inf & kInlet;
      const R sink = (delta != R(0)) ? R(1) - delta / C : R(1);
      const R cu[7] = {upx, -upx, upy, -upy, upz, -upz, R(0)};
      R go[7];
      R gs = 0;
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        const R geq = R(D3Q7::w(i)) * C * (R(1) + R(4) * cu[i]);
        const R gi = inlet ? geq : g[i];
        go[i] = (gi + (geq - gi) * A.inv_tau_c) * sink;
        gs += go[i];
      }
      if (P >= 2) A.cout[t] = gs;  // the deviation reference of the stored populations
#pragma unroll
      for (int i = 0; i < 7; ++i)
        A.gout[size_t(i) * A.ps + t] = Prec<P>::st(go[i], P >= 2 ? R(D3Q7::w(i)) * gs : R(D3Q7::w(i)), A.gscale);
      ok = ok && finite(gs);
    }
    red5[0] += double(rr);
    red5[1] += double(rp);
    red5[2] += double(delta);
    red5[3] += double(C);
    red5[4] += ok ? 0.0 : 1.0;
  }
}

// ---------------------------------------------------------------------------------------------
// collide: the rest of the step at every fluid node. MOM = true writes the level-t fields
// instead (lbm_moments) and leaves the state untouched. Four waves per SIMD in FP32, FP16 and BF16
// (at most 128 VGPRs, no spills; a five-wave bound made the 2-byte storages spill and run 11%
// slower at 512^3); FP64 runs fewer.
// ---------------------------------------------------------------------------------------------
template <int P, bool MOM>
__global__ __launch_bounds__(kBlock) void k_collide(StepArgs<P> A) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int t = fluid_tile(A) * kBlock + threadIdx.x;
  double red5[5] = {0, 0, 0, 0, 0};
  const int n = (t < A.nfluid) ? A.fluid[t] : 0;
  const uint32_t inf = (t < A.nfluid) ? A.finfo[t] : 0u;
  if (inf & kFluid) {
    const Nbr nb = make_nbr(n, A.geo);
    // All loads of the node first (pull of f^m and g with halfway bounce-back, rho^N, the node's
    // and its neighbours' realigned normals), so that one memory round trip covers them.
    int sid[18];  // fluid ids of the pull sources (own id for bounce-back)
    pull_sources(A.fid, nb, t, inf, sid);
    R f[19], g[7];
    pull_node(A, t, inf, sid, f, g);
    const R rn = A.rhoN[n];
    // The node's and its neighbours' realigned normals; x + c_i is the pull source of direction
    // opp(i), the node's own id where it is solid, which is the value the curvature takes for a
    // solid neighbour.
    const typename V4<R>::T nsv = ld4(A.nst, t);
    typename V4<R>::T srcv[18];
    row_shared<true>(nb, inf, nsv, [&](int i) { return ld4(A.nst, sid[i]); }, srcv);
    typename V4<R>::T cur = nsv;
    cur.w = curvature_hg<R>(nsv, A.eps, [&](int i) { return srcv[D::opp[i]]; });
    collide_node<P, MOM>(A, t, n, inf, f, g, rn, cur, red5);
  }
  if (!MOM) block_reduce5(red5, A.partials);
}

// ---------------------------------------------------------------------------------------------
// FP64 sums of a stored state S_t: m^r = sum a rho_s, m^p = sum b rho_s (eqs. reactant_mass,
// product_mass), sum C_s and the non-finite count, with rho_s = sum_i f^m_i and C_s = sum_i g_i
// the node's stored totals. Every stored population is pulled exactly once (by its neighbour,
// or by the node itself through bounce-back), and the recolouring terms of a node cancel in
// opposite pairs, so these are the colour masses and species total of level t. Slot 2
// (conversion) is zero. One partial per workgroup, summed by k_finish_reduce.
// ---------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void k_state_sums(StepArgs<P> A) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int t = logical_block() * kBlock + threadIdx.x;
  double red5[5] = {0, 0, 0, 0, 0};
  if (t < A.nfluid) {
    R a, b;
    unpack_frac(ld4(A.ain, t).x, a, b);
    R s = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i) s += Prec<P>::ld(A.fin[size_t(i) * A.ps + t], R(D::w(i)), A.inv_scale);
    R C = 0;
    if (A.species)
#pragma unroll
      for (int i = 0; i < 7; ++i) C += ld_species(A, i, t);
    red5[0] = double(a) * double(s);
    red5[1] = double(b) * double(s);
    red5[3] = double(C);
    red5[4] = (finite(s) && finite(a) && finite(C)) ? 0.0 : 1.0;
  }
  block_reduce5(red5, A.partials);
}

// ---------------------------------------------------------------------------------------------
// Expansion of the stored state to per-colour populations (lbm_populations).
// ---------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void k_expand(StepArgs<P> A, typename Prec<P>::R* fr,
                                                   typename Prec<P>::R* fp, typename Prec<P>::R* go) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int n = logical_block() * kBlock + threadIdx.x;
  if (n >= A.N) return;
  const size_t N = A.N;
  const int fi = A.fid[n];
  const bool fluid = fi >= 0;
  typename V4<R>::T av;
  av.x = av.y = av.z = av.w = R(0);
  if (fluid) av = ld4(A.ain, fi);
  const R v0 = av.y, v1 = av.z, v2 = av.w;
  R a, b;
  unpack_frac(av.x, a, b);
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const R fm = fluid ? Prec<P>::ld(A.fin[size_t(i) * A.ps + fi], R(D::w(i)), A.inv_scale) : R(0);
    const R kv = R(D::w_over_len(i)) * (R(D::cx[i]) * v0 + R(D::cy[i]) * v1 + R(D::cz[i]) * v2);
    fr[size_t(i) * N + n] = fluid ? a * fm + kv : R(0);
    fp[size_t(i) * N + n] = fluid ? b * fm - kv : R(0);
  }
  if (go) {
#pragma unroll
    for (int i = 0; i < 7; ++i)
      go[size_t(i) * N + n] = (fluid && A.species) ? ld_species(A, i, fi) : R(0);
  }
}

}  // namespace lbm

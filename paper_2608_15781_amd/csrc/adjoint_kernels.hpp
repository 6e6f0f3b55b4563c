// Discrete adjoint of one time step (reverse mode, HIP, gfx950).
//
// For the step map S_{t+1} = Phi(S_t; theta, xi) of step_kernels.hpp, one adjoint step turns
// lambda_{t+1} = dL/dS_{t+1} into lambda_t = (dPhi/dS_t)^T lambda_{t+1} and accumulates
// (dPhi/dtheta)^T lambda_{t+1} per node and (dPhi/dxi)^T lambda_{t+1}. The forward fields of
// level t (rho^N, rho^m, n*, |G|, and the normal before realignment at wetting nodes) come from
// the forward colour, extrapolation and normal kernels, run on S_t here or kept by the
// recomputing step; the reverse pass then runs
//   k_adj_collide   reverse of the collide kernel at each fluid node; the pull transposes to a
//                   scatter that is a bijection on (node, direction), so every adjoint population
//                   is written exactly once, without atomics (and the output needs no clearing;
//                   the two species entries without a reader, at the inlet and outflow planes,
//                   are zeroed by k_adj_final)
//   k_adj_normal    curvature transpose (gather of the neighbours' dH/dn*), then the normal and
//                   Akai realignment reversed to d/dG; accumulates dL/dtheta
//   k_adj_grad_ext  transpose of the isotropic gradient stencil (gather) at solid nodes
//   k_adj_colour    the same transpose at fluid nodes, the colour extrapolation into solids
//                   transposed, then d rho^N -> d rho^r, d rho^m
//   k_adj_final     the colour pass's dependence on f^m, a and v of each pull source (gather)
// Non-smooth points (the minimum in the reaction cap, the |G| and wetting-cone guards) take the
// derivative of the branch the forward step took. Gradients are accumulated in FP64.
#pragma once

#include "step_kernels.hpp"

namespace lbm {

// Adjoint-state layout: 30 planes of reals, the state's plane stride apart and indexed by fluid
// id like the state (19 f^m, a, v_x, v_y, v_z, 7 species).
constexpr int kAdjPlanes = 30;
constexpr int kAdjA = 19, kAdjV = 20, kAdjG = 23;

template <class R>
struct AdjArgs {
  const R* lin;      // lambda_{t+1}
  R* lout;           // lambda_t
  R* lrn;            // d/d rho^N: the collide part at fluid nodes; d/d rho^N / den at extrapolated solids
  R* lng;            // per fluid id 4-vector from the collide: d/d n* (including the node's own
                     // curvature terms) and d/d |G|
  R* lHn;            // per fluid id 4-vector (d/d H, n*): what the curvature transpose gathers
  R* lG;             // 3 planes: d/d G
  R* lr2;            // per node 2-vector (d/d rho^r, d/d rho^m) of the colour pass: read together,
                     // one load per pull reader
  R* lgo;            // species outflow nodes: d/d S_1(x) through their own pull
  const R* rmv;      // rho^m of level t (forward recompute)
  double* gtheta;    // dL/dtheta per node (accumulated)
  double* partials;  // dL/dxi per workgroup (5 planes of workgroup sums, slot 0 used)
  int nparts;        // number of workgroups of k_adj_collide
  double* sum;       // 5 doubles: the reduced partials
  double* gxi;       // dL/dxi (accumulated)
};

// Vector-Jacobian product of the closed-form back transform (cm_back): given ld_i, the
// derivatives of sum_i ld_i d_i(u, k) with respect to (u_x, u_y, u_z, k5..k9), written out from
// the same regrouped expressions (q_x = u_x^2 + s_x u_x for a move with x component s_x, and so
// on; e_x = 2 u_x + s_x = dq_x/du_x).
template <class R>
__device__ inline void cm_back_vjp(const R in[8], const R ld[19], R out[8]) {
  const R ux = in[0], uy = in[1], uz = in[2], k5 = in[3], k6 = in[4], k7 = in[5], k8 = in[6], k9 = in[7];
  const R x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
  const R ax = k5 * R(1.0 / 3.0) + k6 * R(1.0 / 6.0);
  const R ay = (k6 - k5) * R(1.0 / 6.0);
  const R az = -(k5 * R(1.0 / 6.0) + k6 * R(1.0 / 3.0));
  const R tx = uy * k7 + uz * k8, ty = ux * k7 + uz * k9, tz = ux * k8 + uy * k9;
  R gux = 0, guy = 0, guz = 0, g5 = 0, g6 = 0, g7 = 0, g8 = 0, g9 = 0;
  // moves along one axis: d = (q_a - (other squares) + 1) a_a - e_a t_a
  {
    const R lp = ld[0], lm = ld[1], ls = lp + lm;
    const R ep = ux + ux + R(1), em = ux + ux - R(1);
    const R lax = lp * (x2 + ux - y2 - z2 + R(1)) + lm * (x2 - ux - y2 - z2 + R(1));
    const R ltx = -(lp * ep + lm * em);
    gux += ax * (lp * ep + lm * em) - R(2) * tx * ls;
    guy += -R(2) * uy * ax * ls + ltx * k7;
    guz += -R(2) * uz * ax * ls + ltx * k8;
    g7 += ltx * uy;
    g8 += ltx * uz;
    g5 += lax * R(1.0 / 3.0);
    g6 += lax * R(1.0 / 6.0);
  }
  {
    const R lp = ld[2], lm = ld[3], ls = lp + lm;
    const R ep = uy + uy + R(1), em = uy + uy - R(1);
    const R lay = lp * (y2 + uy - x2 - z2 + R(1)) + lm * (y2 - uy - x2 - z2 + R(1));
    const R lty = -(lp * ep + lm * em);
    guy += ay * (lp * ep + lm * em) - R(2) * ty * ls;
    gux += -R(2) * ux * ay * ls + lty * k7;
    guz += -R(2) * uz * ay * ls + lty * k9;
    g7 += lty * ux;
    g9 += lty * uz;
    g5 -= lay * R(1.0 / 6.0);
    g6 += lay * R(1.0 / 6.0);
  }
  {
    const R lp = ld[4], lm = ld[5], ls = lp + lm;
    const R ep = uz + uz + R(1), em = uz + uz - R(1);
    const R laz = lp * (z2 + uz - x2 - y2 + R(1)) + lm * (z2 - uz - x2 - y2 + R(1));
    const R ltz = -(lp * ep + lm * em);
    guz += az * (lp * ep + lm * em) - R(2) * tz * ls;
    gux += -R(2) * ux * az * ls + ltz * k8;
    guy += -R(2) * uy * az * ls + ltz * k9;
    g8 += ltz * ux;
    g9 += ltz * uy;
    g5 -= laz * R(1.0 / 6.0);
    g6 -= laz * R(1.0 / 3.0);
  }
  // diagonal moves, (d index, sign of the first axis, sign of the second axis)
  const int xy[4][3] = {{6, 1, 1}, {7, 1, -1}, {10, -1, 1}, {11, -1, -1}};
  const int xz[4][3] = {{8, 1, 1}, {9, 1, -1}, {12, -1, 1}, {13, -1, -1}};
  const int yz[4][3] = {{14, 1, 1}, {15, 1, -1}, {16, -1, 1}, {17, -1, -1}};
  const R c12 = R(1.0 / 12.0);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    // xy plane: ((2 q_y - q_x) k5 + (q_x + q_y) k6)/12 + e_x e_y k7/4
    const R l = ld[xy[m][0]];
    const R sx = R(xy[m][1]), sy = R(xy[m][2]);
    const R qx = x2 + sx * ux, qy = y2 + sy * uy, ex = ux + ux + sx, ey = uy + uy + sy;
    gux += l * ((k6 - k5) * c12 * ex + R(0.5) * ey * k7);
    guy += l * ((k5 + k5 + k6) * c12 * ey + R(0.5) * ex * k7);
    g5 += l * (qy + qy - qx) * c12;
    g6 += l * (qx + qy) * c12;
    g7 += l * R(0.25) * ex * ey;
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    // xz plane: ((2 q_z - q_x) k5 + (q_z - 2 q_x) k6)/12 + e_x e_z k8/4
    const R l = ld[xz[m][0]];
    const R sx = R(xz[m][1]), sz = R(xz[m][2]);
    const R qx = x2 + sx * ux, qz = z2 + sz * uz, ex = ux + ux + sx, ez = uz + uz + sz;
    gux += l * (-(k5 + k6 + k6) * c12 * ex + R(0.5) * ez * k8);
    guz += l * ((k5 + k5 + k6) * c12 * ez + R(0.5) * ex * k8);
    g5 += l * (qz + qz - qx) * c12;
    g6 += l * (qz - qx - qx) * c12;
    g8 += l * R(0.25) * ex * ez;
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    // yz plane: (-(q_y + q_z) k5 + (q_z - 2 q_y) k6)/12 + e_y e_z k9/4
    const R l = ld[yz[m][0]];
    const R sy = R(yz[m][1]), sz = R(yz[m][2]);
    const R qy = y2 + sy * uy, qz = z2 + sz * uz, ey = uy + uy + sy, ez = uz + uz + sz;
    guy += l * (-(k5 + k6 + k6) * c12 * ey + R(0.5) * ez * k9);
    guz += l * ((k6 - k5) * c12 * ez + R(0.5) * ey * k9);
    g5 -= l * (qy + qz) * c12;
    g6 += l * (qz - qy - qy) * c12;
    g9 += l * R(0.25) * ey * ez;
  }
  {
    // rest: ((y2 + z2 - 2 x2) k5 + (2 z2 - x2 - y2) k6)/3 + 4 (ux uy k7 + ux uz k8 + uy uz k9)
    const R l = ld[18];
    gux += l * (-(R(4) * k5 + R(2) * k6) * ux * R(1.0 / 3.0) + R(4) * (uy * k7 + uz * k8));
    guy += l * ((R(2) * k5 - R(2) * k6) * uy * R(1.0 / 3.0) + R(4) * (ux * k7 + uz * k9));
    guz += l * ((R(2) * k5 + R(4) * k6) * uz * R(1.0 / 3.0) + R(4) * (ux * k8 + uy * k9));
    g5 += l * (y2 + z2 - x2 - x2) * R(1.0 / 3.0);
    g6 += l * (z2 + z2 - x2 - y2) * R(1.0 / 3.0);
    g7 += l * R(4) * ux * uy;
    g8 += l * R(4) * ux * uz;
    g9 += l * R(4) * uy * uz;
  }
  out[0] = gux; out[1] = guy; out[2] = guz;
  out[3] = g5; out[4] = g6; out[5] = g7; out[6] = g8; out[7] = g9;
}

// ---------------------------------------------------------------------------------------------
// Seed for L = m^p(T) = sum over fluid nodes and directions of the product populations of S_T:
// sum_i S^p_i = b sum_i f^m_i with b = 1 - a (the v term cancels by lattice symmetry).
// ---------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_seed(StepArgs<P> A, typename Prec<P>::R* lout) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int t = fluid_tile(A) * kBlock + threadIdx.x;
  if (t >= A.nfluid) return;
  R a, b;
  unpack_frac(ld4(A.ain, t).x, a, b);
  R s = 0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    s += Prec<P>::ld(A.fin[size_t(i) * A.ps + t], R(D::w(i)), A.inv_scale);
    lout[size_t(i) * A.ps + t] = b;
  }
  lout[size_t(kAdjA) * A.ps + t] = -s;
}

// ---------------------------------------------------------------------------------------------
// Reverse of the collide kernel at one fluid node (forward arithmetic recomputed as in k_collide).
// Register budget: the pull sources and the species populations, needed again only at the end,
// wait in LDS (25 KB per workgroup in FP32), which brings the FP32/FP16/BF16 kernels to 165
// VGPRs and three waves per SIMD (requested below) without spills; FP64 keeps one wave.
// ---------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock, P == 0 ? 1 : 3) void k_adj_collide(StepArgs<P> A, AdjArgs<typename Prec<P>::R> J) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int t = fluid_tile(A) * kBlock + threadIdx.x;
  double gxi = 0.0;
  const int n = (t < A.nfluid) ? A.fluid[t] : 0;
  const uint32_t inf = (t < A.nfluid) ? A.finfo[t] : 0u;
  if (inf & kFluid) {
    const Nbr nb = make_nbr(n, A.geo);
    // ---------------- forward recompute ----------------
    // The pull sources are needed again by the final scatter; they wait in LDS meanwhile.
    __shared__ int sid_lds[18][kBlock];
    int sid[18];
    pull_sources_lean(A.fid, nb, t, inf, sid);
#pragma unroll
    for (int i = 0; i < 18; ++i) sid_lds[i][threadIdx.x] = sid[i];
    R f[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const bool bb = (i < 18) && ((inf >> i) & 1u);
      const int src = (i < 18) ? sid[i] : t;
      const int q = bb ? D::opp[i] : i;
      f[i] = Prec<P>::ld(A.fin[size_t(q) * A.ps + src], R(D::w(i)), A.inv_scale);
    }
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
    rn_densities(A.rhoN[n], rm, rr, rp);
    const typename V4<R>::T nsv = ld4(A.nst, t);
    const R nn[3] = {nsv.x, nsv.y, nsv.z};
    const R glen = nsv.w;
    const bool has_n = glen > A.eps;
    R H = 0;
    R Js[3] = {0, 0, 0};  // sum_b n*_b (J_ab + J_ba), the only part of J the reverse needs
    if (has_n) {
      R Jm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
      for (int i = 0; i < 18; ++i) {
        const typename V4<R>::T mv = ld4(A.nst, sid[D::opp[i]]);  // own id where x + c_i is solid
        const R a0 = mv.x, a1 = mv.y, a2 = mv.z;
        const R w3 = R(3.0 * D::w(i));
        if (D::cx[i]) { Jm[0][0] += w3 * R(D::cx[i]) * a0; Jm[1][0] += w3 * R(D::cx[i]) * a1; Jm[2][0] += w3 * R(D::cx[i]) * a2; }
        if (D::cy[i]) { Jm[0][1] += w3 * R(D::cy[i]) * a0; Jm[1][1] += w3 * R(D::cy[i]) * a1; Jm[2][1] += w3 * R(D::cy[i]) * a2; }
        if (D::cz[i]) { Jm[0][2] += w3 * R(D::cz[i]) * a0; Jm[1][2] += w3 * R(D::cz[i]) * a1; Jm[2][2] += w3 * R(D::cz[i]) * a2; }
      }
      R nJn = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) nJn += nn[a] * nn[b] * Jm[a][b];
      H = -((Jm[0][0] + Jm[1][1] + Jm[2][2]) - nJn);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        R s = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) s += nn[b] * (Jm[a][b] + Jm[b][a]);
        Js[a] = s;
      }
    }
    const R fc = R(0.5) * A.sigma * H * glen * irm;
    R dur[3], dup[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) { dur[a] = fc * nn[a] + A.acc[0][a]; dup[a] = fc * nn[a] + A.acc[1][a]; }
    const R up[3] = {ux + R(0.5) * (rr * dur[0] + rp * dup[0]) * irm, uy + R(0.5) * (rr * dur[1] + rp * dup[1]) * irm,
                     uz + R(0.5) * (rr * dur[2] + rp * dup[2]) * irm};
    __shared__ R g_lds[7][kBlock];
    R g[7] = {0, 0, 0, 0, 0, 0, 0};
    R C = R(1);
    const bool inlet = A.species && (inf & kInlet);
    const bool outlet = A.species && (inf & kOutlet);
    if (A.species) {
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        if (i == 1 && outlet) {
          g[i] = ld_species(A, 1, t);
        } else {
          const bool bb = (inf >> i) & 1u;
          const int q = bb ? D3Q7::opp[i] : i;
          g[i] = ld_species(A, q, sid[i]);
        }
      }
      g[6] = ld_species(A, 6, t);
      C = 0;
#pragma unroll
      for (int i = 0; i < 7; ++i) C += g[i];
#pragma unroll
      for (int i = 0; i < 7; ++i) g_lds[i][threadIdx.x] = g[i];
      if (inlet) C = A.c_in;
    }
    const R Ur[3] = {ux + dur[0], uy + dur[1], uz + dur[2]};
    const R Upv[3] = {ux + dup[0], uy + dup[1], uz + dup[2]};
    const int rnn = int((inf & kRnnMask) >> kRnnShift);
    R delta = 0;
    int branch = 0;  // 0: no reaction, 1: rate, 2: cap = rho^r, 3: cap = C, 4: paper rate, 5: paper full
    if (rnn > 0 && rr > R(0)) {
      if (A.species) {
        if (C > R(0)) {
          const R rate = A.xi * R(rnn) * rr * C;
          const R cap = fmin(rr, C);
          delta = fmin(rate, cap);
          branch = (rate < cap) ? 1 : (rr < C ? 2 : 3);
        }
      } else {
        const R frac = A.xi * R(rnn);
        delta = fmin(frac, R(1)) * rr;
        branch = (frac < R(1)) ? 4 : 5;
      }
    }
    const bool reacts = delta != R(0);
    const R keep = reacts ? R(1) - delta / rr : R(1);
    const R vc = keep * A.beta * rr * rp * irm;

    // ---------------- reverse ----------------
    R lf[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) lf[i] = J.lin[size_t(i) * A.ps + t];
    const R la = J.lin[size_t(kAdjA) * A.ps + t];
    const R lv[3] = {J.lin[size_t(kAdjV) * A.ps + t], J.lin[size_t(kAdjV + 1) * A.ps + t], J.lin[size_t(kAdjV + 2) * A.ps + t]};
    R l_C = 0, l_delta = 0, l_up[3] = {0, 0, 0};
    R l_g[7] = {0, 0, 0, 0, 0, 0, 0};
    if (A.species) {
      asm volatile("" ::: "memory");  // read LDS back: no store-to-load forwarding into registers
#pragma unroll
      for (int i = 0; i < 7; ++i) g[i] = g_lds[i][threadIdx.x];
      const R sink = reacts ? R(1) - delta / C : R(1);
      R l_sink = 0;
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        const R cu = (i == 0) ? up[0] : (i == 1) ? -up[0] : (i == 2) ? up[1] : (i == 3) ? -up[1] : (i == 4) ? up[2] : (i == 5) ? -up[2] : R(0);
        const R wc = R(D3Q7::w(i));
        const R geq = wc * C * (R(1) + R(4) * cu);
        const R gi = inlet ? geq : g[i];
        const R pre = gi + (geq - gi) * A.inv_tau_c;
        const R lgo = J.lin[size_t(kAdjG + i) * A.ps + t];
        const R l_pre = lgo * sink;
        l_sink += lgo * pre;
        R l_geq = l_pre * A.inv_tau_c;
        const R l_gi = l_pre * (R(1) - A.inv_tau_c);
        if (inlet) l_geq += l_gi;
        else l_g[i] = l_gi;
        l_C += l_geq * wc * (R(1) + R(4) * cu);
        const R l_cu = l_geq * wc * C * R(4);
        if (i == 0) l_up[0] += l_cu;
        if (i == 1) l_up[0] -= l_cu;
        if (i == 2) l_up[1] += l_cu;
        if (i == 3) l_up[1] -= l_cu;
        if (i == 4) l_up[2] += l_cu;
        if (i == 5) l_up[2] -= l_cu;
      }
      if (reacts) {
        l_delta += -l_sink / C;
        l_C += l_sink * delta / (C * C);
      }
    }
    // a = keep rho^r / rho^m; v = vc n* with vc = keep beta rho^r rho^p / rho^m.
    R l_keep = la * rr * irm, l_rr = la * keep * irm, l_rp = 0, l_rm = -la * keep * rr * irm * irm;
    R l_n[3] = {0, 0, 0};
    if (has_n) {
      const R l_vc = lv[0] * nn[0] + lv[1] * nn[1] + lv[2] * nn[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) l_n[a] += vc * lv[a];
      l_keep += l_vc * A.beta * rr * rp * irm;
      l_rr += l_vc * keep * A.beta * rp * irm;
      l_rp += l_vc * keep * A.beta * rr * irm;
      l_rm += -l_vc * vc * irm;
    }
    if (reacts) {
      l_delta += -l_keep / rr;
      l_rr += l_keep * delta / (rr * rr);
    }
    switch (branch) {
      case 1:
        gxi += double(l_delta * R(rnn) * rr * C);
        l_rr += l_delta * A.xi * R(rnn) * C;
        l_C += l_delta * A.xi * R(rnn) * rr;
        break;
      case 2: l_rr += l_delta; break;
      case 3: l_C += l_delta; break;
      case 4:
        gxi += double(l_delta * R(rnn) * rr);
        l_rr += l_delta * A.xi * R(rnn);
        break;
      case 5: l_rr += l_delta; break;
      default: break;
    }
    // f^{m,*}_i = w_i (base + 3 c.M + 4.5 c.Pi.c) + d_i
    R l_base = 0, l_M[3] = {0, 0, 0}, l_Pxx = 0, l_Pyy = 0, l_Pzz = 0, l_Pxy = 0, l_Pxz = 0, l_Pyz = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const int cx = D::cx[i], cy = D::cy[i], cz = D::cz[i];
      const R wl = R(D::w(i)) * lf[i];
      l_base += wl;
      if (cx) { l_M[0] += R(3 * cx) * wl; l_Pxx += R(4.5) * wl; }
      if (cy) { l_M[1] += R(3 * cy) * wl; l_Pyy += R(4.5) * wl; }
      if (cz) { l_M[2] += R(3 * cz) * wl; l_Pzz += R(4.5) * wl; }
      if (cx && cy) l_Pxy += R(9 * cx * cy) * wl;
      if (cx && cz) l_Pxz += R(9 * cx * cz) * wl;
      if (cy && cz) l_Pyz += R(9 * cy * cz) * wl;
    }
    l_rm += l_base;
    l_Pxx += R(-1.5) * l_base;
    l_Pyy += R(-1.5) * l_base;
    l_Pzz += R(-1.5) * l_base;
    l_rr += l_M[0] * Ur[0] + l_M[1] * Ur[1] + l_M[2] * Ur[2];
    l_rp += l_M[0] * Upv[0] + l_M[1] * Upv[1] + l_M[2] * Upv[2];
    l_rr += l_Pxx * Ur[0] * Ur[0] + l_Pyy * Ur[1] * Ur[1] + l_Pzz * Ur[2] * Ur[2] + l_Pxy * Ur[0] * Ur[1] +
            l_Pxz * Ur[0] * Ur[2] + l_Pyz * Ur[1] * Ur[2];
    l_rp += l_Pxx * Upv[0] * Upv[0] + l_Pyy * Upv[1] * Upv[1] + l_Pzz * Upv[2] * Upv[2] + l_Pxy * Upv[0] * Upv[1] +
            l_Pxz * Upv[0] * Upv[2] + l_Pyz * Upv[1] * Upv[2];
    R l_Ur[3], l_Up[3];
    l_Ur[0] = rr * (l_M[0] + R(2) * l_Pxx * Ur[0] + l_Pxy * Ur[1] + l_Pxz * Ur[2]);
    l_Ur[1] = rr * (l_M[1] + R(2) * l_Pyy * Ur[1] + l_Pxy * Ur[0] + l_Pyz * Ur[2]);
    l_Ur[2] = rr * (l_M[2] + R(2) * l_Pzz * Ur[2] + l_Pxz * Ur[0] + l_Pyz * Ur[1]);
    l_Up[0] = rp * (l_M[0] + R(2) * l_Pxx * Upv[0] + l_Pxy * Upv[1] + l_Pxz * Upv[2]);
    l_Up[1] = rp * (l_M[1] + R(2) * l_Pyy * Upv[1] + l_Pxy * Upv[0] + l_Pyz * Upv[2]);
    l_Up[2] = rp * (l_M[2] + R(2) * l_Pzz * Upv[2] + l_Pxz * Upv[0] + l_Pyz * Upv[1]);
    R l_u[3], l_dur[3], l_dup[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) { l_u[a] = l_Ur[a] + l_Up[a]; l_dur[a] = l_Ur[a]; l_dup[a] = l_Up[a]; }
    // T^{-1} k* and the relaxed central moments.
    const R cxx = pxx - rm * ux * ux, cyy = pyy - rm * uy * uy, czz = pzz - rm * uz * uz;
    const R kin[8] = {ux, uy, uz, A.relax * (cxx - cyy), A.relax * (cyy - czz), A.relax * (pxy - rm * ux * uy),
                      A.relax * (pxz - rm * ux * uz), A.relax * (pyz - rm * uy * uz)};
    R kv[8];
    cm_back_vjp(kin, lf, kv);
    l_u[0] += kv[0];
    l_u[1] += kv[1];
    l_u[2] += kv[2];
    const R l_cxx = A.relax * kv[3], l_cyy = A.relax * (kv[4] - kv[3]), l_czz = -A.relax * kv[4];
    const R l_c7 = A.relax * kv[5], l_c8 = A.relax * kv[6], l_c9 = A.relax * kv[7];
    const R l_pxx = l_cxx, l_pyy = l_cyy, l_pzz = l_czz, l_pxy = l_c7, l_pxz = l_c8, l_pyz = l_c9;
    l_rm += -(l_cxx * ux * ux + l_cyy * uy * uy + l_czz * uz * uz + l_c7 * ux * uy + l_c8 * ux * uz + l_c9 * uy * uz);
    l_u[0] += -rm * (R(2) * l_cxx * ux + l_c7 * uy + l_c8 * uz);
    l_u[1] += -rm * (R(2) * l_cyy * uy + l_c7 * ux + l_c9 * uz);
    l_u[2] += -rm * (R(2) * l_czz * uz + l_c8 * ux + l_c9 * uy);
    // u_phys = u + (rr du^r + rp du^p) / (2 rm)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      l_u[a] += l_up[a];
      l_rr += R(0.5) * l_up[a] * dur[a] * irm;
      l_rp += R(0.5) * l_up[a] * dup[a] * irm;
      l_dur[a] += R(0.5) * rr * irm * l_up[a];
      l_dup[a] += R(0.5) * rp * irm * l_up[a];
      l_rm += -R(0.5) * l_up[a] * (rr * dur[a] + rp * dup[a]) * irm * irm;
    }
    // du^k = fc n* + a^k,  fc = sigma H |G| / (2 rm)
    R l_fc = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      l_fc += (l_dur[a] + l_dup[a]) * nn[a];
      l_n[a] += fc * (l_dur[a] + l_dup[a]);
    }
    const R l_H = l_fc * R(0.5) * A.sigma * glen * irm;
    const R l_glen = l_fc * R(0.5) * A.sigma * H * irm;
    l_rm += -l_fc * fc * irm;
    if (has_n) {
      // H = -(tr J - n.J.n): dependence on the centre normal, including solid neighbours' copies.
#pragma unroll
      for (int a = 0; a < 3; ++a) l_n[a] += l_H * Js[a];
#pragma unroll
      for (int i = 0; i < 18; ++i) {
        if ((inf >> D::opp[i]) & 1u) {
          const R cn = R(D::cx[i]) * nn[0] + R(D::cy[i]) * nn[1] + R(D::cz[i]) * nn[2];
          const R w3 = R(-3.0 * D::w(i)) * l_H;
          l_n[0] += w3 * (R(D::cx[i]) - nn[0] * cn);
          l_n[1] += w3 * (R(D::cy[i]) - nn[1] * cn);
          l_n[2] += w3 * (R(D::cz[i]) - nn[2] * cn);
        }
      }
    }
    // u = m / rm
    R l_m[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) l_m[a] = l_u[a] * irm;
    l_rm += -(l_u[0] * ux + l_u[1] * uy + l_u[2] * uz) * irm;
    // rho^r = rho^m (1 + rho^N)/2, rho^p = rho^m (1 - rho^N)/2
    l_rm += rr * irm * l_rr + rp * irm * l_rp;
    const R l_rn = R(0.5) * rm * (l_rr - l_rp);
    if (A.species && !inlet)
#pragma unroll
      for (int i = 0; i < 7; ++i) l_g[i] += l_C;
    // pulled populations: rm = sum f, m = sum f c, second moments
    asm volatile("" ::: "memory");  // read LDS back: no store-to-load forwarding into registers
#pragma unroll
    for (int i = 0; i < 18; ++i) sid[i] = sid_lds[i][threadIdx.x];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const int cx = D::cx[i], cy = D::cy[i], cz = D::cz[i];
      R v = l_rm;
      if (cx) v += R(cx) * l_m[0] + l_pxx;
      if (cy) v += R(cy) * l_m[1] + l_pyy;
      if (cz) v += R(cz) * l_m[2] + l_pzz;
      if (cx && cy) v += R(cx * cy) * l_pxy;
      if (cx && cz) v += R(cx * cz) * l_pxz;
      if (cy && cz) v += R(cy * cz) * l_pyz;
      // transpose of the pull: the population S_q(src) read by this node as direction i
      const bool bb = (i < 18) && ((inf >> i) & 1u);
      const int src = (i < 18) ? sid[i] : t;
      const int q = bb ? D::opp[i] : i;
      J.lout[size_t(q) * A.ps + src] = v;
    }
    if (A.species) {
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        if (i == 1 && outlet) {
          J.lgo[n] = l_g[1];
        } else {
          const bool bb = (inf >> i) & 1u;
          const int q = bb ? D3Q7::opp[i] : i;
          J.lout[size_t(kAdjG + q) * A.ps + sid[i]] = l_g[i];
        }
      }
      J.lout[size_t(kAdjG + 6) * A.ps + t] = l_g[6];
    }
    J.lrn[n] = l_rn;
    st4(J.lng, t, l_n[0], l_n[1], l_n[2], l_glen);
    st4(J.lHn, t, has_n ? l_H : R(0), nn[0], nn[1], nn[2]);
  }
  double s5[5] = {gxi, 0, 0, 0, 0};
  block_reduce5(s5, J.partials);
}

// ---------------------------------------------------------------------------------------------
// Curvature transpose and the normal / wetting reverse at each fluid node.
// ---------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_normal(StepArgs<P> A, AdjArgs<typename Prec<P>::R> J) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  // Workgroup 0 first finishes the xi sum of k_adj_collide and adds it to dL/dxi.
  if (blockIdx.x == 0) {
    reduce_partials(J.partials, J.nparts, J.sum);
    if (threadIdx.x == 0) *J.gxi += J.sum[0];
  }
  const int t = fluid_tile(A) * kBlock + threadIdx.x;
  if (t >= A.nfluid) return;
  const int n = A.fluid[t];
  const uint32_t inf = A.finfo[t];
  const Nbr nb = make_nbr(n, A.geo);
  const size_t N = A.N;
  // Every load of this node's own entries is issued here, before any is needed, so that they
  // share one memory round trip with the neighbours' ids (the wetting entries are read at every
  // node and used only at wetting nodes): the forward normal pass's n* and |G|, the normal
  // before realignment, the wetting data, dL/dn* and dL/d|G|, and the running dL/dtheta.
  const typename V4<R>::T nsv = ld4(A.nst, t);
  const typename V4<R>::T rv = ld4(A.nraw, t);
  const typename V4<R>::T wv = ld4(A.wet, t);
  const typename V4<R>::T lgv = ld4(J.lng, t);
  const R lgl = lgv.w;
  const double gth0 = J.gtheta[n];
  R mu[3] = {lgv.x, lgv.y, lgv.z};
  // H(x) at each fluid neighbour x = y - c_i used n*(x + c_i) = n*(y):
  // dH(x)/dn*_a(y) = -3 w_i (c_ia - n_a(x) (n(x).c_i)). The fluid ids of all 18 neighbours
  // first, then one gather of (dL/dH, n*) each; a solid y - c_i reads this node's own entry
  // and is discarded.
  int mid[18];
  pull_sources_lean(A.fid, nb, t, inf, mid);
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    const typename V4<R>::T qv = ld4(J.lHn, mid[i]);
    const R lh = qv.x, q0 = qv.y, q1 = qv.z, q2 = qv.w;
    const bool use = !((inf >> i) & 1u) && lh != R(0);
    const R cn = R(D::cx[i]) * q0 + R(D::cy[i]) * q1 + R(D::cz[i]) * q2;
    const R w3 = R(-3.0 * D::w(i)) * lh;
    mu[0] = use ? mu[0] + w3 * (R(D::cx[i]) - q0 * cn) : mu[0];
    mu[1] = use ? mu[1] + w3 * (R(D::cy[i]) - q1 * cn) : mu[1];
    mu[2] = use ? mu[2] + w3 * (R(D::cz[i]) - q2 * cn) : mu[2];
  }
  // The unit normal of this node: n* unless the wetting realignment changed it, in which case
  // the normal pass kept the one before realignment.
  const R len = nsv.w;
  R lG[3] = {0, 0, 0};
  if (len > A.eps) {
    const R il = R(1) / len;
    R nv[3] = {nsv.x, nsv.y, nsv.z};
    R ln[3] = {mu[0], mu[1], mu[2]};
    if (inf & kWet) {
      nv[0] = rv.x; nv[1] = rv.y; nv[2] = rv.z;
      const R sx = wv.x, sy = wv.y, sz = wv.z;
      if (sx * sx + sy * sy + sz * sz > R(0.5)) {
        const R ct = wv.w;
        const R st = sqrt(fmax(R(0), (R(1) - ct) * (R(1) + ct)));
        const R cp = sx * nv[0] + sy * nv[1] + sz * nv[2];
        const R c0 = nv[1] * sz - nv[2] * sy, c1 = nv[2] * sx - nv[0] * sz, c2 = nv[0] * sy - nv[1] * sx;
        const R sp = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        if (sp >= R(1e-2)) {
          // n* = a n_s + b n, b = sin(theta)/sin(theta'), a = cos(theta) - b cos(theta')
          const R b = st / sp;
          const R ns[3] = {sx, sy, sz};
          const R tv[3] = {(nv[0] - cp * sx) / sp, (nv[1] - cp * sy) / sp, (nv[2] - cp * sz) / sp};
          const R mns = mu[0] * sx + mu[1] * sy + mu[2] * sz;
          const R mn = mu[0] * nv[0] + mu[1] * nv[1] + mu[2] * nv[2];
#pragma unroll
          for (int a = 0; a < 3; ++a) ln[a] = b * mu[a] + mns * (b * cp / sp * tv[a] - b * ns[a]) - mn * (b / sp) * tv[a];
          // d n*/d theta = (-sin(theta) - cos(theta) cos(theta')/sin(theta')) n_s + (cos(theta)/sin(theta')) n
          J.gtheta[n] = gth0 + double(mns * (-st - ct * cp / sp) + mn * (ct / sp));
        }
      }
    }
    const R lnn = ln[0] * nv[0] + ln[1] * nv[1] + ln[2] * nv[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) lG[a] = (ln[a] - lnn * nv[a]) * il + lgl * nv[a];
  }
  J.lG[n] = lG[0];
  J.lG[N + n] = lG[1];
  J.lG[2 * N + n] = lG[2];
}

// ---------------------------------------------------------------------------------------------
// Transpose of G(x) = 3 sum_i w_i c_i rho^N(x + c_i): d/d rho^N(y) gathers 3 w_i c_i . lG(y - c_i)
// over fluid nodes y - c_i. EXT: y is a solid node with extrapolated colour; k_adj_grad_ext stores
// d/d rho^N(y) / den(y), den(y) = sum of w_k over the fluid nodes y + c_k (the extrapolation's
// weight sum, the only form in which its transpose uses it). For a fluid y, k_adj_colour adds
// the sum to the collide part of d/d rho^N itself.
// ---------------------------------------------------------------------------------------------
template <int P, bool EXT>
__device__ inline typename Prec<P>::R grad_transpose(const StepArgs<P>& A, const AdjArgs<typename Prec<P>::R>& J,
                                                     int n, uint32_t inf, const Nbr& nb) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const size_t N = A.N;
  // Every load is issued before any is used; a direction whose source is solid reads this
  // node's own entries and is discarded.
  R gx[18], gy[18], gz[18];
  if (EXT) {
#pragma unroll
    for (int i = 0; i < 18; ++i) {
      // solid y: bit opp(i) set means y - c_i is fluid
      const bool src_fluid = (inf >> D::opp[i]) & 1u;
      const int m = src_fluid ? nb.at(-D::cx[i], -D::cy[i], -D::cz[i]) : n;
      gx[i] = D::cx[i] ? J.lG[m] : R(0);
      gy[i] = D::cy[i] ? J.lG[N + m] : R(0);
      gz[i] = D::cz[i] ? J.lG[2 * N + m] : R(0);
    }
  } else {
    // Fluid y (bit i set: y - c_i is solid, read as y and discarded): each component plane with
    // one gather per row triple. A component is read where c_i has it, and at the row centres
    // whose x-neighbours need it.
    auto plane = [&](const R* g, int a, R out[18]) {
      row_shared<true>(nb, inf, g[n], [&](int i) {
        const int c = a == 0 ? D::cx[i] : (a == 1 ? D::cy[i] : D::cz[i]);
        const bool centre = D::cx[i] == 0 && (D::cy[i] == 0 || D::cz[i] == 0);
        const bool need = c != 0 || (a == 0 && centre);
        return need ? g[((inf >> i) & 1u) ? n : nb.at(-D::cx[i], -D::cy[i], -D::cz[i])] : R(0);
      }, out);
    };
    plane(J.lG, 0, gx);
    plane(J.lG + N, 1, gy);
    plane(J.lG + 2 * N, 2, gz);
  }
  R s = 0;
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    const bool src_fluid = EXT ? ((inf >> D::opp[i]) & 1u) : !((inf >> i) & 1u);
    R v = 0;
    if (D::cx[i]) v += R(D::cx[i]) * gx[i];
    if (D::cy[i]) v += R(D::cy[i]) * gy[i];
    if (D::cz[i]) v += R(D::cz[i]) * gz[i];
    s = src_fluid ? s + R(3.0 * D::w(i)) * v : s;
  }
  return s;
}

// The solid nodes with extrapolated colour (the fluid nodes' part is taken by k_adj_colour).
template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_grad_ext(StepArgs<P> A, AdjArgs<typename Prec<P>::R> J) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int t = logical_block() * kBlock + threadIdx.x;
  if (t >= A.next) return;
  const int n = A.ext[t];
  const uint32_t inf = A.einfo[t];
  const Nbr nb = make_nbr(n, A.geo);
  const R s = grad_transpose<P, true>(A, J, n, inf, nb);
  R den = 0;  // > 0: a solid node on this list has a fluid neighbour
#pragma unroll
  for (int k = 0; k < 18; ++k) den = ((inf >> k) & 1u) ? den + R(D::w(k)) : den;
  J.lrn[n] = s / den;
}

// ---------------------------------------------------------------------------------------------
// Transpose of the extrapolation rho^N(y) = sum_j w_j rho^N(y + c_j) / den(y) into the fluid node
// z = y + c_j, then rho^N = (2 rho^r - rho^m)/rho^m reversed to d/d rho^r and d/d rho^m (the
// colour pass forms rho^N from rho^r and rho^p = rho^m - rho^r separately; the same function).
// ---------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_colour(StepArgs<P> A, AdjArgs<typename Prec<P>::R> J) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int t = fluid_tile(A) * kBlock + threadIdx.x;
  if (t >= A.nfluid) return;
  const int n = A.fluid[t];
  const uint32_t inf = A.finfo[t];
  const Nbr nb = make_nbr(n, A.geo);
  // At a solid y the adjoint is stored already divided by den(y) (k_adj_grad_ext). Loads for all
  // directions first (a fluid z - c_j reads this node's own entry, discarded).
  R ly[18];
#pragma unroll
  for (int j = 0; j < 18; ++j) ly[j] = J.lrn[((inf >> j) & 1u) ? nb.at(-D::cx[j], -D::cy[j], -D::cz[j]) : n];
  // d/d rho^N of this fluid node: the collide part plus the gradient stencil's transpose
  R l = J.lrn[n] + grad_transpose<P, false>(A, J, n, inf, nb);
#pragma unroll
  for (int j = 0; j < 18; ++j) l = ((inf >> j) & 1u) ? l + R(D::w(j)) * ly[j] : l;  // z - c_j is solid
  const R rm = J.rmv[n];
  const R q = A.rhoN[n];
  const R one_plus_rn = signbit(q) ? R(2) + q : q;  // 1 + rho^N = 2 rho^r / rho^m
  typename V2<R>::T v;
  v.x = R(2) * l / rm;
  v.y = -one_plus_rn * l / rm;
  reinterpret_cast<typename V2<R>::T*>(J.lr2)[n] = v;
}

// ---------------------------------------------------------------------------------------------
// The colour pass read f^m_q, a and v of each pull source: add those terms to lambda_t at the
// source y. The reader of S_q(y) is y + c_q if that node is fluid, else y itself (bounce-back),
// and y itself for the rest population.
// ---------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_final(StepArgs<P> A, AdjArgs<typename Prec<P>::R> J) {
  using R = typename Prec<P>::R;
  using D = D3Q19;
  const int t = fluid_tile(A) * kBlock + threadIdx.x;
  if (t >= A.nfluid) return;
  const int n = A.fluid[t];
  const uint32_t inf = A.finfo[t];
  const Nbr nb = make_nbr(n, A.geo);
  R a, b;
  unpack_frac(ld4(A.ain, t).x, a, b);
  R la = 0, lv[3] = {0, 0, 0};
  // The readers' pairs: y + c_q is the neighbour y - c_opp(q); where it is solid the reader is y
  // itself (bounce-back), and y for the rest population.
  using V2R = typename V2<R>::T;
  const V2R* lr2 = reinterpret_cast<const V2R*>(J.lr2);
  const V2R own2 = lr2[n];
  V2R rdv[18];
  row_shared<true>(nb, inf, own2,
                   [&](int i) { return lr2[((inf >> i) & 1u) ? n : nb.at(-D::cx[i], -D::cy[i], -D::cz[i])]; }, rdv);
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const V2R lv2 = (q == 18) ? own2 : rdv[D::opp[q]];
    const R lr = lv2.x, lm = lv2.y;
    const R fq = Prec<P>::ld(A.fin[size_t(q) * A.ps + t], R(D::w(q)), A.inv_scale);
    J.lout[size_t(q) * A.ps + t] += lr * a + lm;
    la += lr * fq;
    const R wl = R(D::w_over_len(q)) * lr;
    lv[0] += wl * R(D::cx[q]);
    lv[1] += wl * R(D::cy[q]);
    lv[2] += wl * R(D::cz[q]);
  }
  J.lout[size_t(kAdjA) * A.ps + t] = la;
  J.lout[size_t(kAdjV) * A.ps + t] = lv[0];
  J.lout[size_t(kAdjV + 1) * A.ps + t] = lv[1];
  J.lout[size_t(kAdjV + 2) * A.ps + t] = lv[2];
  if (A.species && (inf & kOutlet)) J.lout[size_t(kAdjG + 1) * A.ps + t] += J.lgo[n];
  // Species populations without a reader, which the scatter of k_adj_collide left untouched:
  // their adjoint is zero. An outflow node takes its own S_1 instead of the one from its periodic
  // +x image, so S_1 of an inlet node whose -x image is an outflow node is unread, and S_0 of an
  // outflow node whose +x image is solid is unread (bounce-back would have read it).
  if (A.species && (inf & kInlet) && !(inf & 1u)) J.lout[size_t(kAdjG + 1) * A.ps + t] = R(0);
  if (A.species && (inf & kOutlet) && (inf & 2u)) J.lout[size_t(kAdjG + 0) * A.ps + t] = R(0);
}


}  // namespace lbm

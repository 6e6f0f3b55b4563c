// Plain FP64 CPU oracle of the two-colour colour-gradient lattice Boltzmann time step
// (Beunen & Harting, "Gas-generating reactive flows in bicontinuous catalyst support
// structures": Sec. II "Numerical method" and Appendix A "Generalized central moments
// collision operator"), plus the D3Q7 reacting species that the wall reaction couples to.
//
// TEST INFRASTRUCTURE ONLY. This is the slow, obviously-correct reference the HIP library is
// checked against. Only the test suite, the smoke check and the CPU-baseline leg of the
// benchmark may load it. It shares no code, header, table or helper with the HIP library.
//
// Every step below follows the paper's equations in the paper's order and notation, with
// per-colour populations f^r, f^p stored in full (2 x 19 values per node). The few places
// where the paper is silent, ambiguous or self-contradictory take the following readings
// (each is repeated where it is used):
//   * normal sign: n = +grad(rho^N)/|grad(rho^N)|. With the printed minus sign the CSF force
//     of eq. (continuum_surface_force), the curvature of eq. (interface_curvature) and the
//     recolouring of eq. (operator_recoloring) all act with the wrong sign (a droplet is
//     pushed outward and the colours mix); the plus sign makes all four consistent.
//   * recolouring acts on the colour-blind post-collision population (Latva-Kokko form):
//     f^k_post = (rho^k/rho^m) f^{m,*} +/- beta (rho^r rho^p / rho^m) w_i (c_i.n)/|c_i|.
//   * the reaction of eqs. (reactive_boundary_condition_*) is applied after recolouring as a
//     proportional transfer of red populations into product populations, explicit in time,
//     capped at full conversion.
//   * velocity: the transform T and the equilibria use the bare mixture velocity
//     u = sum_i f^m_i c_i / rho^m; the reported velocity adds half the force (u + F/(2 rho)).
//   * a gradient with |G| <= eps_G gives n = 0 and H = 0.
//   * the D3Q7 species is not in the paper: BGK advection-diffusion with
//     g^eq_i = w_i C (1 + 4 c_i.u), bounce-back at solids, optional inlet/outlet along x, and
//     the same wall reaction consuming species and red colour at the same rate.
//
// The closed form for T^{-1} k* is the one printed in Appendix A (eq. back_transformation_vector);
// the tests check it against a numerical solve of T d = k* with T built from the moment
// definitions of eq. (forward_transformation_vector).
//
// The step is written once as a template on the scalar type. Instantiated with double it is the
// oracle; instantiated with a forward-mode dual number it gives exact directional derivatives
// of the gas production with respect to the contact angles and the reaction rate.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdlib>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

// ---------------------------------------------------------------------------------------------
// Forward-mode dual numbers with K derivative directions.
// ---------------------------------------------------------------------------------------------
constexpr int KD = 4;

struct Dual {
  double v;
  double d[KD];
  Dual() : v(0.0) { for (int k = 0; k < KD; ++k) d[k] = 0.0; }
  Dual(double x) : v(x) { for (int k = 0; k < KD; ++k) d[k] = 0.0; }
};

inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int k = 0; k < KD; ++k) r.d[k] = -a.d[k]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int k = 0; k < KD; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
inline Dual operator+(const Dual& a, double b) { Dual r = a; r.v += b; return r; }
inline Dual operator+(double a, const Dual& b) { Dual r = b; r.v += a; return r; }
inline Dual operator-(const Dual& a, double b) { Dual r = a; r.v -= b; return r; }
inline Dual operator-(double a, const Dual& b) { Dual r = -b; r.v += a; return r; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] * b; return r; }
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { Dual r(a.v / b); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] / b; return r; }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, const Dual& b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, const Dual& b) { a = a * b; return a; }
inline Dual sqrt(const Dual& a) {
  double s = std::sqrt(a.v);
  Dual r(s);
  for (int k = 0; k < KD; ++k) r.d[k] = (s > 0.0) ? a.d[k] / (2.0 * s) : 0.0;
  return r;
}
inline Dual acos(const Dual& a) {
  Dual r(std::acos(a.v));
  double den = std::sqrt(std::max(0.0, 1.0 - a.v * a.v));
  for (int k = 0; k < KD; ++k) r.d[k] = (den > 0.0) ? -a.d[k] / den : 0.0;
  return r;
}
inline Dual cos(const Dual& a) { Dual r(std::cos(a.v)); double s = -std::sin(a.v); for (int k = 0; k < KD; ++k) r.d[k] = s * a.d[k]; return r; }
inline Dual sin(const Dual& a) { Dual r(std::sin(a.v)); double c = std::cos(a.v); for (int k = 0; k < KD; ++k) r.d[k] = c * a.d[k]; return r; }

inline Dual atan2(const Dual& y, const Dual& x) {
  Dual r(std::atan2(y.v, x.v));
  double den = x.v * x.v + y.v * y.v;
  for (int k = 0; k < KD; ++k) r.d[k] = (den > 0.0) ? (x.v * y.d[k] - y.v * x.d[k]) / den : 0.0;
  return r;
}

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::sqrt;
using std::acos;
using std::cos;
using std::sin;
using std::atan2;

// ---------------------------------------------------------------------------------------------
// Lattice (Sec. II.A): D3Q19 velocities are the columns of the matrix M, the rest vector last;
// weights from eq. (d3q19_weight_function); c_s^2 = 1/3.
// ---------------------------------------------------------------------------------------------
constexpr int Q = 19;
const int CX[Q] = {1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0, 0};
const int CY[Q] = {0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0};
const int CZ[Q] = {0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1, 0};
double W[Q];
double CLEN[Q];   // |c_i|
int OPP[Q];

// D3Q7 lattice of the species (not in the paper): +-x, +-y, +-z, rest; c_s^2 = 1/4.
constexpr int Q7 = 7;
const int C7X[Q7] = {1, -1, 0, 0, 0, 0, 0};
const int C7Y[Q7] = {0, 0, 1, -1, 0, 0, 0};
const int C7Z[Q7] = {0, 0, 0, 0, 1, -1, 0};
const double W7[Q7] = {1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 4};
const int OPP7[Q7] = {1, 0, 3, 2, 5, 4, 6};

// Eighth-order isotropic stencil for the solid normal, eq. (normal_vector_solid) with the
// weights of eq. (eigth_order_weight_function): all integer vectors with |e|^2 in
// {1,2,3,4,5,6,8} (92 of them).
std::vector<int> E8X, E8Y, E8Z;
std::vector<double> E8W;

double omega8(int e2) {
  switch (e2) {
    case 1: return 4.0 / 45.0;
    case 2: return 1.0 / 21.0;
    case 3: return 2.0 / 105.0;
    case 4: return 5.0 / 504.0;
    case 5: return 1.0 / 315.0;
    case 6: return 1.0 / 630.0;
    case 8: return 1.0 / 5040.0;
    default: return 0.0;
  }
}

struct TablesInit {
  TablesInit() {
    for (int i = 0; i < Q; ++i) {
      int c2 = CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i];
      W[i] = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
      CLEN[i] = std::sqrt(double(c2));
      for (int j = 0; j < Q; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) OPP[i] = j;
    }
    for (int z = -2; z <= 2; ++z)
      for (int y = -2; y <= 2; ++y)
        for (int x = -2; x <= 2; ++x) {
          double w = omega8(x * x + y * y + z * z);
          if (w > 0.0) { E8X.push_back(x); E8Y.push_back(y); E8Z.push_back(z); E8W.push_back(w); }
        }
  }
} tables_init;

// Equilibrium of eq. (equilibrium_distribution), second-order truncated.
template <class T>
inline T feq(int i, const T& rho, const T& ux, const T& uy, const T& uz) {
  T cu = ux * double(CX[i]) + uy * double(CY[i]) + uz * double(CZ[i]);
  T uu = ux * ux + uy * uy + uz * uz;
  return W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

// Appendix A, eq. (back_transformation_vector): the 19 entries of T^{-1} k* when only the five
// shear central moments k5..k9 are non-zero. Transcribed row by row in lattice order.
template <class T>
void cm_back_transform(const T& ux, const T& uy, const T& uz, const T k[5], T d[Q]) {
  const T& k5 = k[0]; const T& k6 = k[1]; const T& k7 = k[2]; const T& k8 = k[3]; const T& k9 = k[4];
  T x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
  d[0] = (1.0 / 3.0) * (x2 + ux - y2 - z2 + 1.0) * k5 + (1.0 / 6.0) * (x2 + ux - y2 - z2 + 1.0) * k6
         - (2.0 * ux + 1.0) * uy * k7 - (2.0 * ux + 1.0) * uz * k8;
  d[1] = (1.0 / 3.0) * (x2 - ux - y2 - z2 + 1.0) * k5 + (1.0 / 6.0) * (x2 - ux - y2 - z2 + 1.0) * k6
         - (2.0 * ux - 1.0) * uy * k7 - (2.0 * ux - 1.0) * uz * k8;
  d[2] = (1.0 / 6.0) * (x2 - y2 + z2 - uy - 1.0) * k5 + (1.0 / 6.0) * (-x2 + y2 - z2 + uy + 1.0) * k6
         - (2.0 * uy + 1.0) * ux * k7 - (2.0 * uy + 1.0) * uz * k9;
  d[3] = (1.0 / 6.0) * (x2 - y2 + z2 + uy - 1.0) * k5 + (1.0 / 6.0) * (-x2 + y2 - z2 - uy + 1.0) * k6
         - (2.0 * uy - 1.0) * ux * k7 - (2.0 * uy - 1.0) * uz * k9;
  d[4] = (1.0 / 6.0) * (x2 + y2 - z2 - uz - 1.0) * k5 + (1.0 / 3.0) * (x2 + y2 - z2 - uz - 1.0) * k6
         - (2.0 * uz + 1.0) * ux * k8 - (2.0 * uz + 1.0) * uy * k9;
  d[5] = (1.0 / 6.0) * (x2 + y2 - z2 + uz - 1.0) * k5 + (1.0 / 3.0) * (x2 + y2 - z2 + uz - 1.0) * k6
         - (2.0 * uz - 1.0) * ux * k8 - (2.0 * uz - 1.0) * uy * k9;
  d[6] = (1.0 / 12.0) * (-x2 - ux + 2.0 * y2 + 2.0 * uy) * k5 + (1.0 / 12.0) * (x2 + ux + y2 + uy) * k6
         + (1.0 / 12.0) * (12.0 * uy * ux + 6.0 * ux + 6.0 * uy + 3.0) * k7;
  d[7] = (1.0 / 12.0) * (-x2 - ux + 2.0 * y2 - 2.0 * uy) * k5 + (1.0 / 12.0) * (x2 + ux + y2 - uy) * k6
         + (1.0 / 12.0) * (12.0 * uy * ux - 6.0 * ux + 6.0 * uy - 3.0) * k7;
  d[8] = (1.0 / 12.0) * (-x2 - ux + 2.0 * z2 + 2.0 * uz) * k5 + (1.0 / 12.0) * (-2.0 * x2 - 2.0 * ux + z2 + uz) * k6
         + (1.0 / 12.0) * (12.0 * uz * ux + 6.0 * ux + 6.0 * uz + 3.0) * k8;
  d[9] = (1.0 / 12.0) * (-x2 - ux + 2.0 * z2 - 2.0 * uz) * k5 + (1.0 / 12.0) * (-2.0 * x2 - 2.0 * ux + z2 - uz) * k6
         + (1.0 / 12.0) * (12.0 * uz * ux - 6.0 * ux + 6.0 * uz - 3.0) * k8;
  d[10] = (1.0 / 12.0) * (-x2 + ux + 2.0 * y2 + 2.0 * uy) * k5 + (1.0 / 12.0) * (x2 - ux + y2 + uy) * k6
          + (1.0 / 12.0) * (12.0 * uy * ux + 6.0 * ux - 6.0 * uy - 3.0) * k7;
  d[11] = (1.0 / 12.0) * (-x2 + ux + 2.0 * y2 - 2.0 * uy) * k5 + (1.0 / 12.0) * (x2 - ux + y2 - uy) * k6
          + (1.0 / 12.0) * (12.0 * uy * ux - 6.0 * ux - 6.0 * uy + 3.0) * k7;
  d[12] = (1.0 / 12.0) * (-x2 + ux + 2.0 * z2 + 2.0 * uz) * k5 + (1.0 / 12.0) * (-2.0 * x2 + 2.0 * ux + z2 + uz) * k6
          + (1.0 / 12.0) * (12.0 * uz * ux + 6.0 * ux - 6.0 * uz - 3.0) * k8;
  d[13] = (1.0 / 12.0) * (-x2 + ux + 2.0 * z2 - 2.0 * uz) * k5 + (1.0 / 12.0) * (-2.0 * x2 + 2.0 * ux + z2 - uz) * k6
          + (1.0 / 12.0) * (12.0 * uz * ux - 6.0 * ux - 6.0 * uz + 3.0) * k8;
  d[14] = (1.0 / 12.0) * (-y2 - uy - z2 - uz) * k5 + (1.0 / 12.0) * (-2.0 * y2 - 2.0 * uy + z2 + uz) * k6
          + (1.0 / 12.0) * (12.0 * uz * uy + 6.0 * uy + 6.0 * uz + 3.0) * k9;
  d[15] = (1.0 / 12.0) * (-y2 - uy - z2 + uz) * k5 + (1.0 / 12.0) * (-2.0 * y2 - 2.0 * uy + z2 - uz) * k6
          + (1.0 / 12.0) * (12.0 * uz * uy - 6.0 * uy + 6.0 * uz - 3.0) * k9;
  d[16] = (1.0 / 12.0) * (-y2 + uy - z2 - uz) * k5 + (1.0 / 12.0) * (-2.0 * y2 + 2.0 * uy + z2 + uz) * k6
          + (1.0 / 12.0) * (12.0 * uz * uy + 6.0 * uy - 6.0 * uz - 3.0) * k9;
  d[17] = (1.0 / 12.0) * (-y2 + uy - z2 + uz) * k5 + (1.0 / 12.0) * (-2.0 * y2 + 2.0 * uy + z2 - uz) * k6
          + (1.0 / 12.0) * (12.0 * uz * uy - 6.0 * uy - 6.0 * uz + 3.0) * k9;
  d[18] = (1.0 / 3.0) * (-2.0 * x2 + y2 + z2) * k5 + (1.0 / 3.0) * (-x2 - y2 + 2.0 * z2) * k6
          + 4.0 * ux * uy * k7 + 4.0 * ux * uz * k8 + 4.0 * uy * uz * k9;
}

// Akai wetting, eq. (realigned_normal_vectors): both candidates n+ and n-, then the one with the
// smaller Euclidean distance to n (ties keep n+). theta' = arccos(n_s . n). Writing
// t = (n - cos(theta') n_s) / sin(theta') (unit vector in the plane of n and n_s, perpendicular to
// n_s), the candidates are n+- = cos(+-theta) n_s + sin(+-theta) t: n rotated in that plane to the
// angle +-theta. They are undefined for n parallel to n_s, and the rotation plane is set by the
// component of n perpendicular to n_s. n is kept whenever sin(theta') < kAkaiCone = 1e-2 (n within
// 0.57 degrees of +-n_s, an interface parallel to the wall): there the perpendicular component is
// too small to define a plane, and rotating on it would feed rounding noise into the colour field
// (the realigned normal drives recolouring along itself, so any gain above one near the axis grows
// the noise from step to step). The bound also caps the 1/sin(theta') amplification at 100.
// The tests can narrow or widen the cone (orc_set_akai_cone) to show that the equilibrium angle
// does not depend on it.
double kAkaiCone = 1e-2;

template <class T>
void wetting_realign(const T n[3], const double ns[3], const T& theta, T out[3], T np[3], T nm[3]) {
  T cthp = n[0] * ns[0] + n[1] * ns[1] + n[2] * ns[2];
  T cr[3] = {n[1] * ns[2] - n[2] * ns[1], n[2] * ns[0] - n[0] * ns[2], n[0] * ns[1] - n[1] * ns[0]};
  T sthp = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  for (int a = 0; a < 3; ++a) { out[a] = n[a]; np[a] = n[a]; nm[a] = n[a]; }
  if (!(val(sthp) > 0.0)) return;  // exactly parallel: no plane, n is its own limit
  T cp = cos(theta), sp = sin(theta);                // cos(+theta), sin(+theta)
  T cm = cos(-1.0 * theta), sm = sin(-1.0 * theta);  // cos(-theta), sin(-theta)
  for (int a = 0; a < 3; ++a) {
    np[a] = (cp - sp * cthp / sthp) * ns[a] + (sp / sthp) * n[a];
    nm[a] = (cm - sm * cthp / sthp) * ns[a] + (sm / sthp) * n[a];
  }
  double dp = 0.0, dm = 0.0;
  for (int a = 0; a < 3; ++a) {
    double ep = val(np[a]) - val(n[a]), em = val(nm[a]) - val(n[a]);
    dp += ep * ep; dm += em * em;
  }
  const bool minus = dm < dp;
  if (val(sthp) < kAkaiCone) return;  // inside the cone around +-n_s: n is kept
  for (int a = 0; a < 3; ++a) out[a] = minus ? nm[a] : np[a];
}

struct Params {
  int32_t nx, ny, nz;
  int32_t species;   // 0: the paper's model (reaction with C = 1); 1: D3Q7 species on
  int32_t x_open;    // species inlet at x = 0 and outlet at x = nx-1
  int32_t pad_;
  double tau, tau_c, sigma, beta;
  double accel[2][3];
  double c_in, grad_eps;
};

template <class T>
struct Sim {
  Params p;
  T xi;
  int nx, ny, nz;
  long N;
  std::vector<uint8_t> solid, wet, nn, react, ext, ns_ok;
  std::vector<double> ns;     // 3 per node (wetting nodes)
  std::vector<T> theta;       // contact angle per node, radians, through the red colour
  std::vector<T> fr, fp, g;   // post-collision state S_t: [node*19+i], [node*19+i], [node*7+i]
  // Level-t quantities obtained by pulling S_t.
  std::vector<T> Pr, Pp, Pg;
  std::vector<T> rho_r, rho_p, ux, uy, uz, rhoN, C;
  std::vector<T> G, nstar;    // realigned colour gradient and unit normal, 3 per node
  long steps_done = 0;

  long idx(int x, int y, int z) const { return x + long(nx) * (y + long(ny) * z); }
  long nb(int x, int y, int z, int dx, int dy, int dz) const {
    int X = ((x + dx) % nx + nx) % nx, Y = ((y + dy) % ny + ny) % ny, Z = ((z + dz) % nz + nz) % nz;
    return idx(X, Y, Z);
  }
};

template <class T>
Sim<T>* create(const Params& p, T xi, const uint8_t* solid, const T* theta, const uint8_t* reactive,
               const double* rho_r0, const double* rho_p0, const double* c0) {
  Sim<T>* s = new Sim<T>();
  s->p = p; s->xi = xi;
  s->nx = p.nx; s->ny = p.ny; s->nz = p.nz;
  s->N = long(p.nx) * p.ny * p.nz;
  long N = s->N;
  s->solid.assign(solid, solid + N);
  s->theta.resize(N);
  for (long n = 0; n < N; ++n) s->theta[n] = theta[n];
  s->wet.assign(N, 0); s->nn.assign(N, 0); s->react.assign(N, 0); s->ext.assign(N, 0);
  s->ns.assign(3 * N, 0.0); s->ns_ok.assign(N, 0);
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x) {
        long n = s->idx(x, y, z);
        if (s->solid[n]) {
          // A solid node whose colour is read by the gradient stencil: it has a fluid neighbour.
          for (int i = 0; i < Q - 1; ++i)
            if (!s->solid[s->nb(x, y, z, CX[i], CY[i], CZ[i])]) s->ext[n] = 1;
          continue;
        }
        // Eq. (nearest_solid_neighbors): solid face neighbours of a fluid node.
        int cnt = 0;
        for (int i = 0; i < Q; ++i)
          if (CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i] == 1 && s->solid[s->nb(x, y, z, CX[i], CY[i], CZ[i])]) ++cnt;
        s->nn[n] = uint8_t(cnt);
        // Wetting applies where at least one lattice vector points into a solid node.
        for (int i = 0; i < Q - 1; ++i)
          if (s->solid[s->nb(x, y, z, CX[i], CY[i], CZ[i])]) s->wet[n] = 1;
        // Reactive indicator r(x): given mask, else every fluid node touching a wall face.
        s->react[n] = reactive ? (reactive[n] ? 1 : 0) : (cnt > 0 ? 1 : 0);
        if (s->wet[n]) {
          // Eq. (normal_vector_solid): weighted sum of the solid indicator over the E8 stencil.
          double v[3] = {0, 0, 0};
          for (size_t e = 0; e < E8W.size(); ++e) {
            if (s->solid[s->nb(x, y, z, E8X[e], E8Y[e], E8Z[e])]) {
              v[0] += E8W[e] * E8X[e]; v[1] += E8W[e] * E8Y[e]; v[2] += E8W[e] * E8Z[e];
            }
          }
          double len = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
          // The stencil sum is an integer multiple of 1/5040, so any non-zero sum is >= 1/5040.
          if (len > 1e-9) {
            s->ns_ok[n] = 1;
            for (int a = 0; a < 3; ++a) s->ns[3 * n + a] = v[a] / len;
          }
        }
      }
  // Initial state: S_0 = f^eq(rho^k_0, 0) per colour and g = w C_0.
  s->fr.assign(N * Q, T(0.0)); s->fp.assign(N * Q, T(0.0)); s->g.assign(N * Q7, T(0.0));
  for (long n = 0; n < N; ++n) {
    if (s->solid[n]) continue;
    for (int i = 0; i < Q; ++i) {
      s->fr[n * Q + i] = W[i] * rho_r0[n];
      s->fp[n * Q + i] = W[i] * rho_p0[n];
    }
    double c = c0 ? c0[n] : 1.0;
    for (int i = 0; i < Q7; ++i) s->g[n * Q7 + i] = W7[i] * c;
  }
  s->Pr.assign(N * Q, T(0.0)); s->Pp.assign(N * Q, T(0.0)); s->Pg.assign(N * Q7, T(0.0));
  s->rho_r.assign(N, T(0.0)); s->rho_p.assign(N, T(0.0));
  s->ux.assign(N, T(0.0)); s->uy.assign(N, T(0.0)); s->uz.assign(N, T(0.0));
  s->rhoN.assign(N, T(0.0)); s->C.assign(N, T(0.0));
  s->G.assign(3 * N, T(0.0)); s->nstar.assign(3 * N, T(0.0));
  return s;
}

// Step 1: pull streaming of eq. (lattice_boltzmann_equation) with halfway bounce-back of
// eq. (bounce_back) and periodic outer faces, then the moments of eqs. (moments_components),
// (moments_mixture) and the colour function of eq. (color_function).
template <class T>
void pull_and_moments(Sim<T>& s) {
  const Params& p = s.p;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < s.nz; ++z)
    for (int y = 0; y < s.ny; ++y)
      for (int x = 0; x < s.nx; ++x) {
        long n = s.idx(x, y, z);
        if (s.solid[n]) continue;
        T rr(0.0), rp(0.0), mx(0.0), my(0.0), mz(0.0);
        for (int i = 0; i < Q; ++i) {
          long src = s.nb(x, y, z, -CX[i], -CY[i], -CZ[i]);
          T a, b;
          if (s.solid[src]) { a = s.fr[n * Q + OPP[i]]; b = s.fp[n * Q + OPP[i]]; }
          else { a = s.fr[src * Q + i]; b = s.fp[src * Q + i]; }
          s.Pr[n * Q + i] = a; s.Pp[n * Q + i] = b;
          rr += a; rp += b;
          T m = a + b;
          mx += m * double(CX[i]); my += m * double(CY[i]); mz += m * double(CZ[i]);
        }
        T rm = rr + rp;
        s.rho_r[n] = rr; s.rho_p[n] = rp;
        s.ux[n] = mx / rm; s.uy[n] = my / rm; s.uz[n] = mz / rm;
        s.rhoN[n] = (rr - rp) / rm;
        if (p.species) {
          bool inlet = p.x_open && x == 0;
          bool outlet = p.x_open && x == s.nx - 1;
          T c(0.0);
          for (int i = 0; i < Q7; ++i) {
            T v;
            if (i == Q7 - 1) v = s.g[n * Q7 + i];
            else if (outlet && C7X[i] == -1) v = s.g[n * Q7 + i];  // zero-gradient outflow
            else {
              long src = s.nb(x, y, z, -C7X[i], -C7Y[i], -C7Z[i]);
              v = s.solid[src] ? s.g[n * Q7 + OPP7[i]] : s.g[src * Q7 + i];
            }
            s.Pg[n * Q7 + i] = v;
            c += v;
          }
          s.C[n] = inlet ? T(p.c_in) : c;
        } else {
          s.C[n] = T(1.0);
        }
      }
}

// Step 2: colour function inside solid nodes by the lattice-weighted average of
// eq. (color_lattice_weighted_average). Only solid nodes with a fluid neighbour are ever read.
template <class T>
void colour_into_solids(Sim<T>& s) {
#pragma omp parallel for schedule(static)
  for (int z = 0; z < s.nz; ++z)
    for (int y = 0; y < s.ny; ++y)
      for (int x = 0; x < s.nx; ++x) {
        long n = s.idx(x, y, z);
        if (!s.ext[n]) continue;
        T num(0.0);
        double den = 0.0;
        for (int i = 0; i < Q; ++i) {
          long m = s.nb(x, y, z, CX[i], CY[i], CZ[i]);
          if (s.solid[m]) continue;
          num += W[i] * s.rhoN[m];
          den += W[i];
        }
        s.rhoN[n] = num / den;
      }
}

// Step 3: colour gradient by the isotropic finite difference of eq. (finite_difference_scheme),
// unit normal (plus sign, see the header), and at wetting nodes the realignment of
// eq. (realigned_normal_vectors). The realigned gradient keeps the magnitude of the raw one.
template <class T>
void gradient_normal_wetting(Sim<T>& s) {
  const double eps = s.p.grad_eps;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < s.nz; ++z)
    for (int y = 0; y < s.ny; ++y)
      for (int x = 0; x < s.nx; ++x) {
        long n = s.idx(x, y, z);
        if (s.solid[n]) continue;
        T g[3] = {T(0.0), T(0.0), T(0.0)};
        for (int i = 0; i < Q; ++i) {
          long m = s.nb(x, y, z, CX[i], CY[i], CZ[i]);
          T phi = s.rhoN[m];
          g[0] += 3.0 * W[i] * double(CX[i]) * phi;
          g[1] += 3.0 * W[i] * double(CY[i]) * phi;
          g[2] += 3.0 * W[i] * double(CZ[i]) * phi;
        }
        T len = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        T nv[3] = {T(0.0), T(0.0), T(0.0)};
        if (val(len) > eps)
          for (int a = 0; a < 3; ++a) nv[a] = g[a] / len;
        if (s.wet[n] && s.ns_ok[n] && val(len) > eps) {
          T out[3], np[3], nm[3];
          wetting_realign(nv, &s.ns[3 * n], s.theta[n], out, np, nm);
          for (int a = 0; a < 3; ++a) { nv[a] = out[a]; g[a] = len * out[a]; }
        }
        for (int a = 0; a < 3; ++a) { s.G[3 * n + a] = g[a]; s.nstar[3 * n + a] = nv[a]; }
      }
}

// Per-node result of steps 4-8.
template <class T>
struct NodeOut {
  T fr[Q], fp[Q], g[Q7];
  T uphys[3];
  T conversion;
};

// Steps 4-8 at one fluid node: curvature of eq. (interface_curvature), force of
// eq. (continuum_surface_force) and velocity shift of eq. (delta_u), perturbation of
// eq. (operator_perturbation), central-moment collision of eq. (collision_operator) scaled per
// colour as in eq. (single_phase_collision), recolouring of eq. (operator_recoloring), the wall
// reaction and the species update.
template <class T>
void collide_node(const Sim<T>& s, int x, int y, int z, NodeOut<T>& o) {
  const Params& p = s.p;
  long n = s.idx(x, y, z);
  const T rr = s.rho_r[n], rp = s.rho_p[n];
  const T rm = rr + rp;
  const T u[3] = {s.ux[n], s.uy[n], s.uz[n]};
  const T* nc = &s.nstar[3 * n];
  const T* G = &s.G[3 * n];

  // Curvature H = -[(I - n n) . grad] . n with J_ab = d n_a / d x_b from the isotropic stencil.
  // A solid neighbour contributes the centre normal (zero-gradient copy).
  T H(0.0);
  bool has_n = val(nc[0]) != 0.0 || val(nc[1]) != 0.0 || val(nc[2]) != 0.0;
  if (has_n) {
    T J[3][3];
    for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) J[a][b] = T(0.0);
    for (int i = 0; i < Q; ++i) {
      long m = s.nb(x, y, z, CX[i], CY[i], CZ[i]);
      const T* nm = s.solid[m] ? nc : &s.nstar[3 * m];
      const double cb[3] = {double(CX[i]), double(CY[i]), double(CZ[i])};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) J[a][b] += 3.0 * W[i] * cb[b] * nm[a];
    }
    T div = J[0][0] + J[1][1] + J[2][2];
    T nJn(0.0);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) nJn += nc[a] * nc[b] * J[a][b];
    H = -(div - nJn);
  }

  // Velocity shift per colour: F^k / rho^k = (1/2) sigma H grad(rho^N) / rho^m + a^k.
  T du[2][3];
  for (int k = 0; k < 2; ++k)
    for (int a = 0; a < 3; ++a) du[k][a] = 0.5 * p.sigma * H * G[a] / rm + p.accel[k][a];

  const T* fr = &s.Pr[n * Q];
  const T* fp = &s.Pp[n * Q];
  T fm[Q];
  for (int i = 0; i < Q; ++i) fm[i] = fr[i] + fp[i];

  // Central moments k5..k9 of the colour-blind populations about the bare velocity, relaxed
  // with 1 - 1/tau (eq. post_collision_moments), then T^{-1} k*.
  T k[5] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
  for (int i = 0; i < Q; ++i) {
    T cx = double(CX[i]) - u[0], cy = double(CY[i]) - u[1], cz = double(CZ[i]) - u[2];
    k[0] += fm[i] * (cx * cx - cy * cy);
    k[1] += fm[i] * (cy * cy - cz * cz);
    k[2] += fm[i] * cx * cy;
    k[3] += fm[i] * cx * cz;
    k[4] += fm[i] * cy * cz;
  }
  const double relax = 1.0 - 1.0 / p.tau;
  for (int j = 0; j < 5; ++j) k[j] = relax * k[j];
  T d[Q];
  cm_back_transform(u[0], u[1], u[2], k, d);

  // Omega^CM = f^eq(rho^m, u) - f^m + T^{-1} k*.
  T ocm[Q];
  for (int i = 0; i < Q; ++i) ocm[i] = feq(i, rm, u[0], u[1], u[2]) - fm[i] + d[i];

  // Perturbation (exact difference method) and colour share of the collision, per colour.
  T post_r[Q], post_p[Q], fmstar[Q];
  for (int i = 0; i < Q; ++i) {
    T o1r = feq(i, rr, u[0] + du[0][0], u[1] + du[0][1], u[2] + du[0][2]) - feq(i, rr, u[0], u[1], u[2]);
    T o1p = feq(i, rp, u[0] + du[1][0], u[1] + du[1][1], u[2] + du[1][2]) - feq(i, rp, u[0], u[1], u[2]);
    post_r[i] = fr[i] + o1r + (rr / rm) * ocm[i];
    post_p[i] = fp[i] + o1p + (rp / rm) * ocm[i];
    fmstar[i] = post_r[i] + post_p[i];
  }

  // Recolouring (Latva-Kokko form on the colour-blind post-collision populations).
  T bcoef = p.beta * rr * rp / rm;
  for (int i = 0; i < Q; ++i) {
    T B(0.0);
    if (i != Q - 1) {
      T cn = double(CX[i]) * nc[0] + double(CY[i]) * nc[1] + double(CZ[i]) * nc[2];
      B = bcoef * W[i] * cn / CLEN[i];
    }
    o.fr[i] = (rr / rm) * fmstar[i] + B;
    o.fp[i] = (rp / rm) * fmstar[i] - B;
  }

  // Wall reaction, eqs. (reactive_boundary_condition_reactant/product): explicit first-order
  // kinetics at r(x) NN(x) > 0 with the level-t densities, capped at full conversion, applied as
  // a proportional transfer of red populations into product populations.
  T conc = s.C[n];
  T delta(0.0);
  int rnn = s.react[n] ? int(s.nn[n]) : 0;
  if (rnn > 0 && val(rr) > 0.0) {
    if (p.species) {
      if (val(conc) > 0.0) {
        T rate = s.xi * double(rnn) * rr * conc;
        T cap = (val(rr) < val(conc)) ? rr : conc;
        delta = (val(rate) < val(cap)) ? rate : cap;
      }
    } else {
      T frac = s.xi * double(rnn);
      if (val(frac) > 1.0) frac = T(1.0);
      delta = frac * rr;
    }
  }
  if (val(delta) != 0.0) {
    T phi = delta / rr;
    for (int i = 0; i < Q; ++i) {
      T moved = phi * o.fr[i];
      o.fp[i] += moved;
      o.fr[i] -= moved;
    }
  }
  o.conversion = delta;

  // Physical (reported) velocity: bare velocity plus half the total force over rho^m.
  for (int a = 0; a < 3; ++a) o.uphys[a] = u[a] + 0.5 * (rr * du[0][a] + rp * du[1][a]) / rm;

  // Species: BGK towards w_i C (1 + 4 c_i.u), sink equal to the converted amount.
  if (p.species) {
    bool inlet = p.x_open && x == 0;
    T gin[Q7];
    for (int i = 0; i < Q7; ++i) {
      T cu = double(C7X[i]) * o.uphys[0] + double(C7Y[i]) * o.uphys[1] + double(C7Z[i]) * o.uphys[2];
      T geq = W7[i] * conc * (1.0 + 4.0 * cu);
      gin[i] = inlet ? geq : s.Pg[n * Q7 + i];
      o.g[i] = gin[i] - (gin[i] - geq) / p.tau_c;
    }
    if (val(delta) != 0.0) {
      T keep = 1.0 - delta / conc;
      for (int i = 0; i < Q7; ++i) o.g[i] = o.g[i] * keep;
    }
  }
}

template <class T>
struct StepSums { T mass_r, mass_p, conversion, species; double nonfinite; };

// One full time step: S_t -> S_{t+1}. The sums are those of level t (eqs. reactant_mass,
// product_mass, production_rate).
template <class T>
void step(Sim<T>& s, StepSums<T>* sums) {
  pull_and_moments(s);
  colour_into_solids(s);
  gradient_normal_wetting(s);
  std::vector<T> nfr(s.N * Q, T(0.0)), nfp(s.N * Q, T(0.0)), ng(s.N * Q7, T(0.0));
  std::vector<T> zr(s.nz, T(0.0)), zp(s.nz, T(0.0)), zc(s.nz, T(0.0)), zs(s.nz, T(0.0));
  std::vector<double> zn(s.nz, 0.0);
#pragma omp parallel for schedule(static)
  for (int z = 0; z < s.nz; ++z) {
    NodeOut<T> o;
    for (int y = 0; y < s.ny; ++y)
      for (int x = 0; x < s.nx; ++x) {
        long n = s.idx(x, y, z);
        if (s.solid[n]) continue;
        collide_node(s, x, y, z, o);
        bool bad = !std::isfinite(val(s.rho_r[n])) || !std::isfinite(val(s.rho_p[n]));
        for (int i = 0; i < Q; ++i) {
          nfr[n * Q + i] = o.fr[i]; nfp[n * Q + i] = o.fp[i];
          if (!std::isfinite(val(o.fr[i])) || !std::isfinite(val(o.fp[i]))) bad = true;
        }
        if (s.p.species)
          for (int i = 0; i < Q7; ++i) {
            ng[n * Q7 + i] = o.g[i];
            if (!std::isfinite(val(o.g[i]))) bad = true;
          }
        zr[z] += s.rho_r[n]; zp[z] += s.rho_p[n]; zc[z] += o.conversion; zs[z] += s.C[n];
        if (bad) zn[z] += 1.0;
      }
  }
  s.fr.swap(nfr); s.fp.swap(nfp);
  if (s.p.species) s.g.swap(ng);
  s.steps_done++;
  if (sums) {
    T a(0.0), b(0.0), c(0.0), d(0.0);
    double e = 0.0;
    for (int z = 0; z < s.nz; ++z) { a += zr[z]; b += zp[z]; c += zc[z]; d += zs[z]; e += zn[z]; }
    sums->mass_r = a; sums->mass_p = b; sums->conversion = c; sums->species = d; sums->nonfinite = e;
  }
}

}  // namespace

// =============================================================================================
// C interface (ctypes). All arrays are host memory, node index x + nx*(y + ny*z).
// =============================================================================================
extern "C" {

typedef Params orc_params;

void orc_lattice(int* c /*19x3*/, double* w /*19*/, int* opp /*19*/) {
  for (int i = 0; i < Q; ++i) { c[3 * i] = CX[i]; c[3 * i + 1] = CY[i]; c[3 * i + 2] = CZ[i]; w[i] = W[i]; opp[i] = OPP[i]; }
}

int orc_e8(int* e /*92x3*/, double* w /*92*/) {
  for (size_t k = 0; k < E8W.size(); ++k) { e[3 * k] = E8X[k]; e[3 * k + 1] = E8Y[k]; e[3 * k + 2] = E8Z[k]; w[k] = E8W[k]; }
  return int(E8W.size());
}

void orc_feq(double rho, const double* u, double* out) {
  for (int i = 0; i < Q; ++i) out[i] = feq(i, rho, u[0], u[1], u[2]);
}

void orc_cm_back(const double* u, const double* k5_9, double* out) {
  cm_back_transform(u[0], u[1], u[2], k5_9, out);
}

// Half-width of the cone around +-n_s in which n is kept (sin(theta') below it); returns the previous
// value. Test knob: the library's cone is fixed at 1e-2.
double orc_set_akai_cone(double s) {
  const double old = kAkaiCone;
  kAkaiCone = s;
  return old;
}

void orc_wetting(const double* n, const double* ns, double theta, double* nstar, double* np, double* nm) {
  wetting_realign(n, ns, theta, nstar, np, nm);
}

void* orc_create(const orc_params* p, double xi, const uint8_t* solid, const double* theta, const uint8_t* reactive,
                 const double* rho_r0, const double* rho_p0, const double* c0) {
  return create<double>(*p, xi, solid, theta, reactive, rho_r0, rho_p0, c0);
}

void orc_destroy(void* h) { delete static_cast<Sim<double>*>(h); }

void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int orc_get_threads(void) { return omp_get_max_threads(); }

// Runs nsteps; per-step sums (mass_r, mass_p, conversion, species, nonfinite) of level t.
int orc_step(void* h, int nsteps, double* sums) {
  Sim<double>& s = *static_cast<Sim<double>*>(h);
  int bad = 0;
  for (int t = 0; t < nsteps; ++t) {
    StepSums<double> r;
    step(s, &r);
    if (sums) { sums[5 * t] = r.mass_r; sums[5 * t + 1] = r.mass_p; sums[5 * t + 2] = r.conversion; sums[5 * t + 3] = r.species; sums[5 * t + 4] = r.nonfinite; }
    if (r.nonfinite > 0) bad = 1;
  }
  return bad ? -4 : 0;
}

// Level-t fields of the current state (steps 1-4 without storing): rho^r, rho^p, rho^N, the
// reported velocity (3 per node, [a*N + node]) and the species concentration.
void orc_moments(void* h, double* rho_r, double* rho_p, double* rho_n, double* u, double* c) {
  Sim<double>& s = *static_cast<Sim<double>*>(h);
  pull_and_moments(s);
  colour_into_solids(s);
  gradient_normal_wetting(s);
  long N = s.N;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < s.nz; ++z) {
    NodeOut<double> o;
    for (int y = 0; y < s.ny; ++y)
      for (int x = 0; x < s.nx; ++x) {
        long n = s.idx(x, y, z);
        if (s.solid[n]) {
          rho_r[n] = rho_p[n] = rho_n[n] = c[n] = 0.0;
          u[n] = u[N + n] = u[2 * N + n] = 0.0;
          continue;
        }
        collide_node(s, x, y, z, o);
        rho_r[n] = s.rho_r[n]; rho_p[n] = s.rho_p[n]; rho_n[n] = s.rhoN[n]; c[n] = s.C[n];
        u[n] = o.uphys[0]; u[N + n] = o.uphys[1]; u[2 * N + n] = o.uphys[2];
      }
  }
}

// Realigned normal n* and gradient of level t (after orc_moments), 3 per node [a*N + node].
void orc_normals(void* h, double* nstar, double* grad) {
  Sim<double>& s = *static_cast<Sim<double>*>(h);
  for (long n = 0; n < s.N; ++n)
    for (int a = 0; a < 3; ++a) { nstar[a * s.N + n] = s.nstar[3 * n + a]; grad[a * s.N + n] = s.G[3 * n + a]; }
}

// Post-collision state S_t, layout [i*N + node]: fr (19N), fp (19N), g (7N).
void orc_get_state(void* h, double* fr, double* fp, double* g) {
  Sim<double>& s = *static_cast<Sim<double>*>(h);
  for (long n = 0; n < s.N; ++n) {
    for (int i = 0; i < Q; ++i) { fr[i * s.N + n] = s.fr[n * Q + i]; fp[i * s.N + n] = s.fp[n * Q + i]; }
    if (g) for (int i = 0; i < Q7; ++i) g[i * s.N + n] = s.g[n * Q7 + i];
  }
}

void orc_set_state(void* h, const double* fr, const double* fp, const double* g) {
  Sim<double>& s = *static_cast<Sim<double>*>(h);
  for (long n = 0; n < s.N; ++n) {
    for (int i = 0; i < Q; ++i) { s.fr[n * Q + i] = fr[i * s.N + n]; s.fp[n * Q + i] = fp[i * s.N + n]; }
    if (g) for (int i = 0; i < Q7; ++i) s.g[n * Q7 + i] = g[i * s.N + n];
  }
}

// Static geometry: wetting flag, NN, reactive flag, solid-normal validity and n_s (3N, [a*N+n]).
void orc_geometry(void* h, uint8_t* wet, uint8_t* nn, uint8_t* react, uint8_t* ns_ok, double* ns) {
  Sim<double>& s = *static_cast<Sim<double>*>(h);
  for (long n = 0; n < s.N; ++n) {
    wet[n] = s.wet[n]; nn[n] = s.nn[n]; react[n] = s.react[n]; ns_ok[n] = s.ns_ok[n];
    for (int a = 0; a < 3; ++a) ns[a * s.N + n] = s.ns[3 * n + a];
  }
}

int orc_max_dirs(void) { return KD; }

// Gas production L = m^p(T) - m^p(0) = sum over the nsteps of the conversion, and its
// directional derivatives along ndir (<= orc_max_dirs()) directions (dtheta_k, dxi_k), by
// forward-mode dual numbers through the whole step.
int orc_grad(const orc_params* p, double xi, const uint8_t* solid, const double* theta, const uint8_t* reactive,
             const double* rho_r0, const double* rho_p0, const double* c0, int nsteps, int ndir,
             const double* dtheta /*ndir*N*/, const double* dxi /*ndir*/, double* L, double* dL /*ndir*/) {
  if (ndir < 0 || ndir > KD) return -1;
  long N = long(p->nx) * p->ny * p->nz;
  std::vector<Dual> th(N);
  for (long n = 0; n < N; ++n) {
    th[n] = Dual(theta[n]);
    for (int k = 0; k < ndir; ++k) th[n].d[k] = dtheta ? dtheta[k * N + n] : 0.0;
  }
  Dual x(xi);
  for (int k = 0; k < ndir; ++k) x.d[k] = dxi ? dxi[k] : 0.0;
  Sim<Dual>* s = create<Dual>(*p, x, solid, th.data(), reactive, rho_r0, rho_p0, c0);
  Dual total(0.0);
  int bad = 0;
  for (int t = 0; t < nsteps; ++t) {
    StepSums<Dual> r;
    step(*s, &r);
    total += r.conversion;
    if (r.nonfinite > 0) bad = 1;
  }
  *L = total.v;
  for (int k = 0; k < ndir; ++k) dL[k] = total.d[k];
  delete s;
  return bad ? -4 : 0;
}

}  // extern "C"

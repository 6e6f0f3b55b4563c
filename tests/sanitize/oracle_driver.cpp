// The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: its whole C interface on small
// seeded lattices (porous with species and open x faces, one node wide in x, two wide with open
// faces, all solid, all fluid), including the state round trip and the dual-number gradient. The
// oracle's source is compiled into this program, so the sanitizers instrument it. Prints "ok" and
// exits 0 when every result is finite and the state round trip is exact.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "lbm_oracle.cpp"

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);      \
      return 1;                                                     \
    }                                                               \
  } while (0)

static double uniform(uint64_t& s) {
  s = s * 6364136223846793005ull + 1442695040888963407ull;
  return double(s >> 11) * (1.0 / 9007199254740992.0);
}

static bool finite_all(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

static int run(int nx, int ny, int nz, int species, int x_open, double solid_frac, uint64_t seed) {
  orc_params p{};
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.species = species;
  p.x_open = x_open;
  p.tau = 0.8;
  p.tau_c = 0.9;
  p.sigma = 0.02;
  p.beta = 0.7;
  p.accel[0][0] = 1e-5;
  p.accel[1][0] = 1e-5;
  p.c_in = 1.0;
  p.grad_eps = 1e-6;
  const long N = long(nx) * ny * nz;
  std::vector<uint8_t> solid(N);
  std::vector<double> theta(N), rr(N), rp(N);
  for (long n = 0; n < N; ++n) {
    solid[n] = uniform(seed) < solid_frac ? 1 : 0;
    theta[n] = 0.3 + 2.5 * uniform(seed);
    rr[n] = uniform(seed);
    rp[n] = 1.0 - rr[n];
  }
  void* h = orc_create(&p, 0.01, solid.data(), theta.data(), nullptr, rr.data(), rp.data(), nullptr);
  CHECK(h != nullptr);
  const int T = 12;
  std::vector<double> sums(5 * T);
  CHECK(orc_step(h, T, sums.data()) == 0);
  CHECK(finite_all(sums));
  std::vector<double> r(N), q(N), rn(N), u(3 * N), c(N), ns(3 * N), gr(3 * N), sn(3 * N);
  orc_moments(h, r.data(), q.data(), rn.data(), u.data(), c.data());
  orc_normals(h, ns.data(), gr.data());
  CHECK(finite_all(r) && finite_all(q) && finite_all(rn) && finite_all(u) && finite_all(c));
  CHECK(finite_all(ns) && finite_all(gr));
  std::vector<uint8_t> wet(N), nn(N), react(N), ok(N);
  orc_geometry(h, wet.data(), nn.data(), react.data(), ok.data(), sn.data());
  std::vector<double> fr(19 * N), fp(19 * N), g(7 * N);
  orc_get_state(h, fr.data(), fp.data(), g.data());
  orc_set_state(h, fr.data(), fp.data(), g.data());
  std::vector<double> fr2(19 * N), fp2(19 * N), g2(7 * N);
  orc_get_state(h, fr2.data(), fp2.data(), g2.data());
  CHECK(fr == fr2 && fp == fp2 && g == g2);
  CHECK(orc_step(h, 3, nullptr) == 0);
  orc_destroy(h);
  // forward-mode gradient along two directions
  const int D = 2;
  CHECK(orc_max_dirs() >= D);
  std::vector<double> dth(D * N), dxi(D), dL(D);
  for (long i = 0; i < D * N; ++i) dth[i] = uniform(seed) - 0.5;
  dxi[0] = 0.0;
  dxi[1] = 1.0;
  double L = 0;
  CHECK(orc_grad(&p, 0.01, solid.data(), theta.data(), nullptr, rr.data(), rp.data(), nullptr, 5, D, dth.data(),
                 dxi.data(), &L, dL.data()) == 0);
  CHECK(std::isfinite(L) && std::isfinite(dL[0]) && std::isfinite(dL[1]));
  CHECK(orc_grad(&p, 0.01, solid.data(), theta.data(), nullptr, rr.data(), rp.data(), nullptr, 1, orc_max_dirs() + 1,
                 dth.data(), dxi.data(), &L, dL.data()) == -1);
  return 0;
}

int main() {
  orc_set_threads(2);
  if (run(7, 6, 5, 1, 1, 0.3, 1)) return 1;   // porous, species, open x faces
  if (run(1, 5, 4, 0, 0, 0.2, 2)) return 1;   // one node wide in x
  if (run(2, 3, 3, 1, 1, 0.1, 3)) return 1;   // two wide, open x faces
  if (run(4, 4, 4, 1, 0, 1.0, 4)) return 1;   // all solid
  if (run(5, 4, 3, 1, 0, 0.0, 5)) return 1;   // all fluid
  std::printf("ok\n");
  return 0;
}

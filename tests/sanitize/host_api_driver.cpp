// Host-side C ABI under AddressSanitizer and UndefinedBehaviorSanitizer (built with the library's
// host code instrumented, device code untouched; runs without a GPU). Every call here returns before
// touching the device: size and layout queries over all storages and species options, the largest
// lattice, rejected parameters and init inputs, and the per-thread error message of context-free
// calls. Prints "ok" and exits 0 when every expectation holds.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "lbm.h"

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);      \
      return 1;                                                     \
    }                                                               \
  } while (0)

static lbm_params make(int nx, int ny, int nz, int prec, int species, int x_open, int fluid_nodes) {
  lbm_params p;
  std::memset(&p, 0, sizeof(p));
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.precision = prec;
  p.species = species;
  p.x_open = x_open;
  p.tau = 0.8;
  p.tau_species = 0.9;
  p.sigma = 0.01;
  p.beta = 0.7;
  p.xi = 1e-3;
  p.c_inlet = 1.0;
  p.grad_eps = 1e-6;
  p.fp16_scale_log2 = 12;
  p.fluid_nodes = fluid_nodes;
  return p;
}

static int sizes(const lbm_params& p) {
  size_t ws = 0, sb = 0, ab = 0, scr = 0, fb = 0, f = 0, a = 0, g = 0, ps = 0;
  CHECK(lbm_workspace_bytes(&p, &ws) == LBM_OK && ws > 0);
  CHECK(lbm_state_bytes(&p, &sb) == LBM_OK && sb > 0 && ws >= 2 * sb);
  CHECK(lbm_state_layout(&p, &f, &a, &g, &ps) == LBM_OK && a > f && g >= a && sb >= g);
  CHECK(lbm_adjoint_bytes(&p, &ab, &scr) == LBM_OK && ab > 0);
  CHECK(lbm_fields_bytes(&p, &fb) == LBM_OK && fb > 0);
  return 0;
}

static int rejected(const lbm_params& p, const char* needle) {
  size_t b = 0;
  CHECK(lbm_workspace_bytes(&p, &b) == LBM_ERR_ARG);
  const char* e = lbm_last_error(nullptr);
  CHECK(e != nullptr && std::strlen(e) > 0);
  if (needle) CHECK(std::strstr(e, needle) != nullptr);
  return 0;
}

static int init_rejected(const lbm_params& p, const std::vector<uint8_t>& solid, const std::vector<double>& theta,
                         const std::vector<double>& rr, const std::vector<double>& rp, void* ws, size_t bytes) {
  lbm_ctx* ctx = reinterpret_cast<lbm_ctx*>(0x1);  // must stay untouched on failure
  const lbm_status st = lbm_init(&p, solid.data(), theta.empty() ? nullptr : theta.data(), 1.0, nullptr,
                                 rr.data(), rp.data(), nullptr, ws, bytes, nullptr, &ctx);
  CHECK(st == LBM_ERR_ARG);
  CHECK(ctx == reinterpret_cast<lbm_ctx*>(0x1));
  CHECK(std::strlen(lbm_last_error(nullptr)) > 0);
  return 0;
}

int main() {
  CHECK(lbm_version() != nullptr && std::strstr(lbm_version(), "gfx950") != nullptr);
  CHECK(lbm_adjoint_static_scratch_bytes() > 0);
  // size and layout queries
  for (int prec = 0; prec < 4; ++prec)
    for (int species = 0; species < 2; ++species)
      for (int x_open = 0; x_open <= species; ++x_open)
        for (int nf : {0, 64 * 48 * 40 / 2 + 37, 1})
          if (sizes(make(64, 48, 40, prec, species, x_open, nf))) return 1;
  for (int prec = 0; prec < 3; ++prec)
    for (int nf : {0, 1290 * 1290 * 1290 / 2})
      if (sizes(make(1290, 1290, 1290, prec, 1, 0, nf))) return 1;
  // rejected parameters
  if (rejected(make(1291, 1290, 1290, 1, 0, 0, 0), "2^31")) return 1;
  if (rejected(make(1, 8, 8, 1, 1, 1, 0), "x_open")) return 1;
  {
    lbm_params p = make(8, 8, 8, 2, 0, 0, 0);
    lbm_params q = p; q.tau = 0.5; if (rejected(q, nullptr)) return 1;
    q = p; q.tau = std::nan(""); if (rejected(q, nullptr)) return 1;
    q = p; q.sigma = -1; if (rejected(q, nullptr)) return 1;
    q = p; q.beta = -0.1; if (rejected(q, nullptr)) return 1;
    q = p; q.xi = -1e-3; if (rejected(q, nullptr)) return 1;
    q = p; q.grad_eps = 0; if (rejected(q, nullptr)) return 1;
    q = p; q.nx = 0; if (rejected(q, nullptr)) return 1;
    q = p; q.precision = 7; if (rejected(q, nullptr)) return 1;
    q = p; q.fluid_nodes = -1; if (rejected(q, nullptr)) return 1;
    q = p; q.fluid_nodes = 8 * 8 * 8 + 1; if (rejected(q, nullptr)) return 1;
    q = p; q.fp16_scale_log2 = 40; if (rejected(q, nullptr)) return 1;
  }
  // init inputs rejected on the host, before any device call
  {
    const int N = 4 * 4 * 4;
    lbm_params p = make(4, 4, 4, 1, 0, 0, 0);
    size_t need = 0;
    CHECK(lbm_workspace_bytes(&p, &need) == LBM_OK);
    std::vector<uint8_t> solid(N, 0);
    std::vector<double> rr(N, 1.0), rp(N, 0.0), theta;
    void* ws = reinterpret_cast<void*>(uintptr_t(256));
    if (init_rejected(p, solid, theta, rr, rp, ws, need - 1)) return 1;                            // too small
    if (init_rejected(p, solid, theta, rr, rp, reinterpret_cast<void*>(uintptr_t(257)), need)) return 1;  // misaligned
    std::vector<double> bad = rr;
    bad[5] = -1.0;
    if (init_rejected(p, solid, theta, bad, rp, ws, need)) return 1;  // negative density
    bad = rr;
    bad[7] = std::nan("");
    if (init_rejected(p, solid, theta, bad, rp, ws, need)) return 1;  // non-finite density
    theta.assign(N, 1.0);
    theta[3] = 4.0;
    if (init_rejected(p, solid, theta, rr, rp, ws, need)) return 1;  // angle outside [0, pi]
    theta.clear();
    lbm_params q = make(4, 4, 4, 1, 0, 0, 10);  // fluid count differs from the mask's 64
    size_t need_q = 0;
    CHECK(lbm_workspace_bytes(&q, &need_q) == LBM_OK);
    if (init_rejected(q, solid, theta, rr, rp, ws, need_q)) return 1;
  }
  // the context-free error message is per thread
  std::string ea, eb;
  std::thread ta([&] {
    lbm_params p = make(1, 8, 8, 1, 1, 1, 0);
    size_t b;
    lbm_workspace_bytes(&p, &b);
    ea = lbm_last_error(nullptr);
  });
  std::thread tb([&] {
    lbm_params p = make(1291, 1290, 1290, 1, 0, 0, 0);
    size_t b;
    lbm_workspace_bytes(&p, &b);
    eb = lbm_last_error(nullptr);
  });
  ta.join();
  tb.join();
  CHECK(ea.find("x_open") != std::string::npos && eb.find("2^31") != std::string::npos);
  std::printf("ok\n");
  return 0;
}

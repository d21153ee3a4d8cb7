// Host-side driver of liblbf for the sanitizer test (tests/test_sanitizers.py):
// built with AddressSanitizer and UndefinedBehaviorSanitizer on the host code
// together with an equally instrumented build of the library, it runs every
// host path that needs no device (sizes, parameter validation, refusals,
// NULL handles, per-thread error text) and, without a device, the failing
// allocation of a valid parameter set.  Exit status 0 when every expectation
// holds; the sanitizers abort on the first finding.
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>
#include "lbf.h"
#include "lbf3.h"
#include "lbf_pre.h"

static int fails = 0;
#define EXPECT(c) do { if (!(c)) { std::printf("FAILED %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } } while (0)

static lbf_params base() {
  lbf_params p;
  std::memset(&p, 0, sizeof p);
  p.nx = 24; p.ny = 16; p.periodic_x = 1; p.periodic_y = 0;
  p.thermal_bc[0] = 1;
  p.latch_fs = 1;
  p.rho_l = 1; p.rho_g = 0.1; p.rho_s = 0.9; p.mu_l = 0.1; p.mu_g = 0.01; p.mu_s = 0.1;
  p.lam_l = 0.1; p.lam_g = 0.01; p.lam_s = 0.1; p.cp_l = p.cp_g = p.cp_s = 1;
  p.latent = 1; p.T_m = 0; p.sigma = 1e-3; p.eps = 4; p.mobility = 0.1; p.rho_ref = 0.1;
  p.pcm_floor = 0.01;
  return p;
}

int main() {
  // sizes
  EXPECT(lbf_workspace_bytes(0, 5, 0, 0) == 0);
  EXPECT(lbf_workspace_bytes(24, 16, 0, 0) > 0);
  EXPECT(lbf_workspace_bytes(24, 16, 0, 4) > 0);
  EXPECT(lbf_workspace_bytes(24, 16, 7, 0) == 0);
  EXPECT(lbf_workspace_bytes(24, 16, 0, 3) == 0);
  EXPECT(lbf_ch_workspace_bytes(10, 10, 1) == 2 * 512);
  EXPECT(lbf_ch_noalloc_max_nodes() == (size_t)1 << 22);
  // invalid parameter sets are refused before any device call
  struct Mut { const char* what; void (*f)(lbf_params&); };
  std::vector<Mut> muts = {
    {"nx", [](lbf_params& p) { p.nx = 0; }},
    {"rho_g", [](lbf_params& p) { p.rho_g = -1; }},
    {"mu_l", [](lbf_params& p) { p.mu_l = 0; }},
    {"eps", [](lbf_params& p) { p.eps = 0; }},
    {"pcm_floor", [](lbf_params& p) { p.pcm_floor = 1.0; }},
    {"rho_ref", [](lbf_params& p) { p.rho_ref = 1.0; }},
    {"plane_pad", [](lbf_params& p) { p.plane_pad = 65; }},
    {"mrt rate", [](lbf_params& p) { p.mrt = 1; p.s_b = 2.5; }},
    {"phi_src_mdot", [](lbf_params& p) { p.phi_src_mdot = 3; }},
    {"row_block", [](lbf_params& p) { p.row_block = 6; }},
    {"thermal_bc", [](lbf_params& p) { p.thermal_bc[2] = 5; }},
    {"grav", [](lbf_params& p) { p.grav[0] = 1.0 / 0.0; }},
  };
  for (auto& m : muts) {
    lbf_params p = base();
    m.f(p);
    lbf_sim* s = nullptr;
    const int rc = lbf_create(&p, nullptr, nullptr, 0, &s);
    if (!(rc == LBF_EINVAL && s == nullptr)) {
      std::printf("mutation %s: rc %d (%s)\n", m.what, rc, lbf_last_error());
      ++fails;
    }
  }
  // a valid set: without a device the allocation (or the device query) fails cleanly
  {
    lbf_params p = base();
    lbf_sim* s = nullptr;
    const int rc = lbf_create(&p, nullptr, nullptr, 0, &s);
    EXPECT(rc != LBF_OK || s != nullptr);
    if (s) lbf_destroy(s);
    EXPECT(std::strlen(lbf_last_error()) < 512);
  }
  // NULL handles everywhere
  EXPECT(lbf_step(nullptr, 1) == LBF_EINVAL);
  EXPECT(lbf_reduce(nullptr, nullptr) == LBF_EINVAL);
  EXPECT(lbf_batch_create(nullptr, 0, nullptr) == LBF_EINVAL);
  lbf_destroy(nullptr);
  // smoothing: refusals on the host
  {
    lbf_ch_params c;
    std::memset(&c, 0, sizeof c);
    c.nx = 8; c.ny = 8; c.nz = 1; c.A = 1; c.kappa = 2; c.mobility = 1; c.dt = 0.05;
    uint8_t img[64] = {0};
    float out[64];
    EXPECT(lbf_ch_smooth(&c, img, 0, out, 0, 1, nullptr, nullptr, 0) == LBF_EINVAL);
    c.dt = 0.02; c.nz = (1 << 22) / 64 + 1;
    EXPECT(lbf_ch_smooth_noalloc(&c, img, out, 1, nullptr) == LBF_EINVAL);
    EXPECT(lbf_ch_smooth_noalloc(nullptr, img, out, 1, nullptr) == LBF_EINVAL);
  }
  // 3D refusals
  EXPECT(lbf3_workspace_bytes(0, 1, 1, 0, 0) == 0);
  EXPECT(lbf3_workspace_bytes(8, 8, 8, 0, 16) > 0);
  EXPECT(lbf3_workspace_bytes(8, 8, 8, 0, 5) == 0);
  // error text is per thread
  std::thread t([] { lbf_step(nullptr, -1); });
  t.join();
  std::printf("driver done, %d failures\n", fails);
  return fails ? 1 : 0;
}

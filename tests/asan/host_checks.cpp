// Host-side checks of libcapred under AddressSanitizer (host code only; no
// GPU is touched).  Built and run by tests/test_host_asan.py against a copy of
// the library whose host code is compiled with -fsanitize=address.  Exercises
// the argument validation of every entry point family, the error strings, the
// tile cut of the persistent launch, the workspace-size query and the plan's
// error-path cleanup; exits non-zero on a wrong status, and ASan aborts on any
// out-of-bounds access, use after free or double free on the way.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "capred.h"

static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, cap_last_error());
    ++failures;
  }
}

static void expect_status(cap_status got, cap_status want, const char* what) {
  expect(got == want, what);
  if (got != CAP_OK) expect(std::strlen(cap_last_error()) > 0, "error string set");
}

int main() {
  expect(cap_abi_version() == CAP_ABI_VERSION, "abi version");

  // ---- tile cut: every human's units covered by P, P/2 and P/4 tiles
  std::mt19937 rng(7);
  for (int it = 0; it < 300; ++it) {
    const int n = 1 + (int)(rng() % 40);
    const int Ps[3] = {1, 2, 4};
    const int P = Ps[rng() % 3];
    const int C = 1 + (int)(rng() % 300);
    const int R = C * (1 + (int)(rng() % 4));
    std::vector<int32_t> units(n);
    for (auto& u : units) u = (int32_t)(rng() % 3000);
    std::vector<int32_t> counts((size_t)3 * n, -1);
    expect_status(cap_plan_tile_split(units.data(), n, P, R, C, counts.data()), CAP_OK,
                  "tile split");
    const int sz[3] = {P, P / 2, P / 4};
    for (int i = 0; i < n; ++i) {
      long cover = 0;
      for (int k = 0; k < 3; ++k) cover += (long)counts[3 * i + k] * sz[k];
      expect(cover == units[i], "tile split covers the units");
    }
  }
  expect_status(cap_plan_tile_split(nullptr, 3, 4, 8, 8, nullptr), CAP_E_INVALID,
                "tile split without arrays");

  // ---- workspace query
  expect(cap_loglik_backward_workspace(1024, 8, 9, 0) > 0, "workspace size");
  expect(cap_loglik_backward_workspace(0, 8, 9, 0) == 0, "workspace of an empty batch");

  // ---- model validation (belief update), predict and normalise arguments
  float beta[2] = {1.f, 0.f};
  float goals[4] = {0, 0, 1, 1};
  cap_model m{};
  m.K = 8; m.speed = 1.0; m.dt = 0.1; m.B = 2; m.beta = beta; m.G = 2; m.goals = goals;
  void* fake = reinterpret_cast<void*>(256);
  expect_status(cap_belief_update(&m, (const float*)fake, 1, (double*)fake, nullptr, nullptr),
                CAP_E_INVALID, "beta of 0 rejected");
  beta[1] = 2.f;
  m.K = 1;
  expect_status(cap_belief_update(&m, (const float*)fake, 1, (double*)fake, nullptr, nullptr),
                CAP_E_INVALID, "K < 2 rejected");
  m.K = 8;
  cap_grid g{0.0, 0.0, 0.0, 16, 16};
  const double z0[2] = {0.5, 0.5};
  expect_status(cap_predict_occupancy(&m, &g, z0, (const double*)fake, 16, 4, 0, 0, 0,
                                      (uint32_t*)fake, nullptr, nullptr, nullptr, nullptr),
                CAP_E_INVALID, "zero cell size rejected");
  expect_status(cap_normalize(nullptr, 16, 4, (float*)fake, nullptr), CAP_E_INVALID,
                "normalise without counts");

  // ---- log-likelihood, MPPI, probes
  expect_status(cap_loglik(8, 1.0, 0.1, nullptr, nullptr, 4, 4, nullptr, 2, nullptr, 2, 0,
                           nullptr, nullptr),
                CAP_E_INVALID, "log-likelihood without buffers");
  const double z[4] = {0, 0, 1, 0};
  expect_status(cap_mppi_step(z, z, 0, 0.1, 8, (double*)fake, (const double*)fake, nullptr, 0,
                              nullptr, nullptr, (double*)fake, nullptr),
                CAP_E_INVALID, "MPPI without cost");
  expect_status(cap_probe(9, 1, 1, (float*)fake, nullptr), CAP_E_INVALID, "unknown probe");
  expect_status(cap_probe_global_atomic(1, 1, nullptr, 10, nullptr), CAP_E_INVALID,
                "atomic probe without buffer");

  // ---- plan: invalid configurations, then a valid one that fails at the
  // first device call (no GPU) and must clean up what it built
  cap_plan_config cfg{};
  cfg.n_slots = 0; cfg.K = 16; cfg.speed = 1.2; cfg.dt = 0.02; cfg.max_obs = 1;
  cap_plan* plan = reinterpret_cast<cap_plan*>(fake);
  expect_status(cap_plan_create(&cfg, &plan), CAP_E_INVALID, "zero slots rejected");
  expect(plan == nullptr, "no plan returned on error");
  cfg.n_slots = 4; cfg.block_threads = 384;
  expect_status(cap_plan_create(&cfg, &plan), CAP_E_INVALID, "block size rejected");
  cfg.block_threads = 256; cfg.particles_per_thread = 4;
  const cap_status st = cap_plan_create(&cfg, &plan);
  if (st == CAP_OK) {
    cap_plan_destroy(plan);   // a device is present after all
  } else {
    expect(st == CAP_E_HIP, "plan creation without a device fails with CAP_E_HIP");
    expect(plan == nullptr, "no plan returned on a device error");
  }
  cap_plan_destroy(nullptr);
  const int32_t one_slot[1] = {0};
  const float one_xy[2] = {0.f, 0.f};
  expect_status(cap_plan_stage_obs_many(nullptr, 1, one_slot, one_xy), CAP_E_INVALID,
                "staging without a plan");

  if (failures) std::fprintf(stderr, "%d host check(s) failed\n", failures);
  else std::printf("host checks passed\n");
  return failures ? 1 : 0;
}

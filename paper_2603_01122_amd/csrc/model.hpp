// model.hpp -- host-side validation and descriptor construction shared by the
// single-human entry points and the batched plan.
#pragma once

#include <cstdio>

#include "rollout.hpp"

namespace capred {

// Continuous-model constants of the belief update and the log-likelihood.
struct BeliefModel {
  int32_t K, B, G;
  float sx[CAP_MAX_K], sy[CAP_MAX_K], s2[CAP_MAX_K];  // fl32 steps (m), fl32(|s|^2)
  float cth[CAP_MAX_K], sth[CAP_MAX_K];              // fl32(cos, sin theta_k)
  float beta[CAP_MAX_B];
  float gx[CAP_MAX_G], gy[CAP_MAX_G];
};

inline cap_status check_model_shape(int K, double speed, double dt) {
  if (K < 2 || K > CAP_MAX_K) return fail(CAP_E_INVALID, "K must be in [2, 32]");
  if (!(speed > 0.0) || !std::isfinite(speed)) return fail(CAP_E_INVALID, "speed must be > 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CAP_E_INVALID, "dt must be > 0");
  return CAP_OK;
}

inline cap_status check_model(const cap_model* m) {
  if (!m) return fail(CAP_E_INVALID, "model is NULL");
  cap_status s = check_model_shape(m->K, m->speed, m->dt);
  if (s != CAP_OK) return s;
  if (m->B < 1 || m->B > CAP_MAX_B) return fail(CAP_E_INVALID, "B must be in [1, 16]");
  if (m->G < 1 || m->G > CAP_MAX_G) return fail(CAP_E_INVALID, "G must be in [1, 64]");
  if (m->G * m->B > CAP_MAX_J) return fail(CAP_E_INVALID, "G * B must be <= 512");
  if (!m->beta || !m->goals) return fail(CAP_E_INVALID, "model beta/goals pointer is NULL");
  for (int b = 0; b < m->B; ++b)
    if (!(m->beta[b] > 0.f) || !std::isfinite(m->beta[b]))
      return fail(CAP_E_INVALID, "every beta must be finite and > 0");
  for (int g = 0; g < 2 * m->G; ++g)
    if (!std::isfinite(m->goals[g])) return fail(CAP_E_INVALID, "goals must be finite");
  return CAP_OK;
}

inline cap_status check_grid(const cap_grid* g) {
  if (!g) return fail(CAP_E_INVALID, "grid is NULL");
  if (!(g->cell > 0.0) || !std::isfinite(g->cell) || !std::isfinite(g->x0) ||
      !std::isfinite(g->y0))
    return fail(CAP_E_INVALID, "grid origin/cell must be finite, cell > 0");
  if (g->nx < 1 || g->ny < 1 || g->nx > 16384 || g->ny > 16384)
    return fail(CAP_E_INVALID, "grid nx, ny must be in [1, 16384]");
  return CAP_OK;
}

inline BeliefModel make_belief_model(int K, double speed, double dt, int B, const float* beta,
                                     int G, const float* goals) {
  BeliefModel bm;
  std::memset(&bm, 0, sizeof(bm));
  bm.K = K;
  bm.B = B;
  bm.G = G;
  for (int k = 0; k < K; ++k) {
    continuous_step(k, K, speed, dt, &bm.sx[k], &bm.sy[k]);
    const double sx = bm.sx[k], sy = bm.sy[k];
    bm.s2[k] = (float)(sx * sx + sy * sy);
    const double th = heading_angle(k, K);
    bm.cth[k] = (float)std::cos(th);
    bm.sth[k] = (float)std::sin(th);
  }
  for (int b = 0; b < B && beta; ++b) bm.beta[b] = beta[b];
  for (int g = 0; g < G && goals; ++g) {
    bm.gx[g] = goals[2 * g];
    bm.gy[g] = goals[2 * g + 1];
  }
  return bm;
}

// Rollout descriptor of one human.  The start position arrives in metres
// (host) or is filled in later on the device (batched plans); goals and the
// step table are rounded to the lattice here, in FP64.
inline cap_status make_rollout_desc(int K, double speed, double dt, int B, const float* beta,
                                    int G, const float* goals, const cap_grid& grid, int N, int H,
                                    RolloutDesc* out) {
  if (N < 1 || N > (1 << 30)) return fail(CAP_E_INVALID, "N must be in [1, 2^30]");
  if (H < 1 || H > 4096) return fail(CAP_E_INVALID, "H must be in [1, 4096]");
  RolloutDesc& d = *out;
  std::memset(&d, 0, sizeof(d));
  d.N = N;
  d.H = H;
  d.K = K;
  d.B = B;
  d.G = G;
  d.nx = grid.nx;
  d.ny = grid.ny;
  const double q = lattice_pitch(grid.cell);
  int32_t rx = 0, ry = 0;
  for (int k = 0; k < K; ++k) {
    lattice_step(k, K, speed, dt, grid.cell, &d.Sx[k], &d.Sy[k]);
    const double fx = d.Sx[k], fy = d.Sy[k];
    d.T.fx[k] = (float)fx;
    d.T.fy[k] = (float)fy;
    d.T.s2[k] = (float)(fx * fx + fy * fy);
    rx = std::max(rx, std::abs(d.Sx[k]));
    ry = std::max(ry, std::abs(d.Sy[k]));
  }
  if (std::max(rx, ry) < 2)
    return fail(CAP_E_INVALID, "step v*dt is shorter than 2 lattice units (cell/2^15)");
  d.Rx = rx;
  d.Ry = ry;
  d.sym = (K % 2 == 0) ? 1 : 0;
  for (int k = 0; k < K / 2 && d.sym; ++k)
    if (d.Sx[k + K / 2] != -d.Sx[k] || d.Sy[k + K / 2] != -d.Sy[k]) d.sym = 0;
  // reach check: start +- H steps must stay within int32 (checked again per start)
  const double reach = (double)H * (double)std::max(rx, ry);
  if (reach + (double)grid.nx * kLatticeScale > 2.0e9 || reach + (double)grid.ny * kLatticeScale > 2.0e9)
    return fail(CAP_E_INVALID, "grid size + H steps exceed the int32 lattice");
  double max_beta = 0.0;
  for (int b = 0; b < B; ++b) {
    d.ibeta[b] = (float)(1.0 / (-(double)beta[b] * q * (double)kLog2e));
    max_beta = std::max(max_beta, (double)beta[b]);
  }
  d.shift = max_beta * speed * dt > kNoShiftLimit ? 1 : 0;
  for (int g = 0; g < G; ++g) {
    const double gx = lattice_coord(goals[2 * g], grid.x0, grid.cell);
    const double gy = lattice_coord(goals[2 * g + 1], grid.y0, grid.cell);
    if (std::fabs(gx) > 2.0e9 || std::fabs(gy) > 2.0e9)
      return fail(CAP_E_INVALID, "a goal lies outside the int32 lattice of the grid");
    d.GX[g] = (int32_t)gx;
    d.GY[g] = (int32_t)gy;
  }
  return CAP_OK;
}

inline cap_status set_start(RolloutDesc* d, double zx, double zy, const cap_grid& grid) {
  if (!std::isfinite(zx) || !std::isfinite(zy)) return fail(CAP_E_INVALID, "start is not finite");
  const double X = lattice_coord(zx, grid.x0, grid.cell);
  const double Y = lattice_coord(zy, grid.y0, grid.cell);
  const double reach = (double)d->H * (double)std::max(d->Rx, d->Ry);
  if (std::fabs(X) + reach > 2.1e9 || std::fabs(Y) + reach > 2.1e9)
    return fail(CAP_E_INVALID, "start + H steps leave the int32 lattice of the grid");
  d->X0 = (int32_t)X;
  d->Y0 = (int32_t)Y;
  return CAP_OK;
}

}  // namespace capred

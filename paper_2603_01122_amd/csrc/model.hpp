// model.hpp -- host-side validation and descriptor construction shared by the
// single-human entry points and the batched plan.
#pragma once

#include <cstdio>

#include "rollout.hpp"

namespace capred {

// Control set: S speeds x K headings, control u = s K + k; `mask` (bit s,
// never 0 after validation) selects the speeds the prediction may use.
struct Controls {
  int K = 0, S = 1;
  double v[CAP_MAX_S] = {};
  uint32_t mask = 1u;
  int U() const { return K * S; }
};

// Continuous-model constants of the belief update and the log-likelihood.
struct BeliefModel {
  int32_t K, S, U, B, G;
  float sx[CAP_MAX_U], sy[CAP_MAX_U], s2[CAP_MAX_U];  // fl32 steps (m), fl32(|s|^2)
  float cth[CAP_MAX_K], sth[CAP_MAX_K];              // fl32(cos, sin theta_k)
  float vdt[CAP_MAX_S];                              // fl32(v_s dt)
  float beta[CAP_MAX_B];
  float gx[CAP_MAX_G], gy[CAP_MAX_G];
};

inline cap_status check_model_shape(int K, double speed, double dt) {
  if (K < 2 || K > CAP_MAX_K) return fail(CAP_E_INVALID, "K must be in [2, 32]");
  if (!(speed > 0.0) || !std::isfinite(speed)) return fail(CAP_E_INVALID, "speed must be > 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CAP_E_INVALID, "dt must be > 0");
  return CAP_OK;
}

// Control set of (K, speed) or (n_speeds, speeds) with a prediction mask.
inline cap_status make_controls(int K, double speed, double dt, int n_speeds,
                                const double* speeds, uint32_t mask, Controls* c) {
  if (n_speeds < 0 || n_speeds > CAP_MAX_S) return fail(CAP_E_INVALID, "n_speeds must be in [0, 8]");
  if (n_speeds == 0) {
    cap_status st = check_model_shape(K, speed, dt);
    if (st != CAP_OK) return st;
    c->K = K;
    c->S = 1;
    c->v[0] = speed;
    c->mask = 1u;
    return CAP_OK;
  }
  if (!speeds) return fail(CAP_E_INVALID, "speeds is NULL");
  for (int s = 0; s < n_speeds; ++s) {
    cap_status st = check_model_shape(K, speeds[s], dt);
    if (st != CAP_OK) return st;
  }
  if (K * n_speeds > CAP_MAX_U) return fail(CAP_E_INVALID, "n_speeds * K must be <= 128");
  const uint32_t full = (1u << n_speeds) - 1u;
  if (mask == 0u) mask = full;
  if ((mask & full) == 0u || (mask & ~full) != 0u)
    return fail(CAP_E_INVALID, "speed_mask must select at least one of the n_speeds speeds");
  c->K = K;
  c->S = n_speeds;
  for (int s = 0; s < n_speeds; ++s) c->v[s] = speeds[s];
  c->mask = mask;
  return CAP_OK;
}

inline cap_status check_model(const cap_model* m, Controls* c) {
  if (!m) return fail(CAP_E_INVALID, "model is NULL");
  cap_status s = make_controls(m->K, m->speed, m->dt, m->n_speeds, m->speeds, m->speed_mask, c);
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

inline BeliefModel make_belief_model(const Controls& c, double dt, int B, const float* beta,
                                     int G, const float* goals) {
  BeliefModel bm;
  std::memset(&bm, 0, sizeof(bm));
  const int K = c.K;
  bm.K = K;
  bm.S = c.S;
  bm.U = c.U();
  bm.B = B;
  bm.G = G;
  for (int s = 0; s < c.S; ++s) {
    bm.vdt[s] = (float)(c.v[s] * dt);
    for (int k = 0; k < K; ++k) {
      const int u = s * K + k;
      continuous_step(k, K, c.v[s], dt, &bm.sx[u], &bm.sy[u]);
      const double sx = bm.sx[u], sy = bm.sy[u];
      bm.s2[u] = (float)(sx * sx + sy * sy);
    }
  }
  for (int k = 0; k < K; ++k) {
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
inline cap_status make_rollout_desc(const Controls& c, double dt, int B, const float* beta,
                                    int G, const float* goals, const cap_grid& grid, int N, int H,
                                    RolloutDesc* out) {
  if (N < 1 || N > (1 << 30)) return fail(CAP_E_INVALID, "N must be in [1, 2^30]");
  if (H < 1 || H > 4096) return fail(CAP_E_INVALID, "H must be in [1, 4096]");
  RolloutDesc& d = *out;
  std::memset(&d, 0, sizeof(d));
  const int K = c.K, U = c.U();
  d.N = N;
  d.H = H;
  d.K = K;
  d.S = c.S;
  d.B = B;
  d.G = G;
  d.nx = grid.nx;
  d.ny = grid.ny;
  d.smask = c.mask;
  d.s_last = 0;
  for (int s = 0; s < c.S; ++s)
    if ((c.mask >> s) & 1u) d.s_last = s;
  const double q = lattice_pitch(grid.cell);
  int32_t rx = 0, ry = 0;
  double vmax = 0.0;
  for (int s = 0; s < c.S; ++s) {
    vmax = std::max(vmax, c.v[s]);
    for (int k = 0; k < K; ++k) {
      int32_t sx = 0, sy = 0;
      lattice_step(k, K, c.v[s], dt, grid.cell, &sx, &sy);
      if (std::abs(sx) >= (1 << 24) || std::abs(sy) >= (1 << 24))
        return fail(CAP_E_INVALID, "a step spans 256 cells or more");
      const int u = s * K + k;
      const double fx = sx, fy = sy;
      d.T.fx[u] = (float)fx;
      d.T.fy[u] = (float)fy;
      d.T.s2[u] = (float)(fx * fx + fy * fy);
      rx = std::max(rx, std::abs(sx));
      ry = std::max(ry, std::abs(sy));
    }
  }
  for (int s = 0; s < c.S; ++s) {
    int32_t mx = 0;
    for (int k = 0; k < K; ++k)
      mx = std::max(mx, (int32_t)std::max(std::fabs(d.T.fx[s * K + k]), std::fabs(d.T.fy[s * K + k])));
    if (mx < 2) return fail(CAP_E_INVALID, "step v*dt is shorter than 2 lattice units (cell/2^15)");
  }
  d.Rx = rx;
  d.Ry = ry;
  d.sym = (K % 2 == 0) ? 1 : 0;
  for (int s = 0; s < c.S && d.sym; ++s)
    for (int k = 0; k < K / 2 && d.sym; ++k) {
      const int a = s * K + k, b = a + K / 2;
      if (d.T.fx[b] != -d.T.fx[a] || d.T.fy[b] != -d.T.fy[a]) d.sym = 0;
    }
  (void)U;
  // reach check: start +- H steps must stay within int32 (checked again per start)
  const double reach = (double)H * (double)std::max(rx, ry);
  if (reach + (double)grid.nx * kLatticeScale > 2.0e9 || reach + (double)grid.ny * kLatticeScale > 2.0e9)
    return fail(CAP_E_INVALID, "grid size + H steps exceed the int32 lattice");
  double max_beta = 0.0;
  for (int b = 0; b < B; ++b) {
    d.ibeta[b] = (float)(1.0 / (-(double)beta[b] * q * (double)kLog2e));
    max_beta = std::max(max_beta, (double)beta[b]);
  }
  d.shift = max_beta * vmax * dt > kNoShiftLimit ? 1 : 0;
  for (int g = 0; g < G; ++g) {
    const double gx = lattice_coord(goals[2 * g], grid.x0, grid.cell);
    const double gy = lattice_coord(goals[2 * g + 1], grid.y0, grid.cell);
    if (std::fabs(gx) > 2.0e9 || std::fabs(gy) > 2.0e9)
      return fail(CAP_E_INVALID, "a goal lies outside the int32 lattice of the grid");
    d.GX[g] = (int32_t)gx;
    d.GY[g] = (int32_t)gy;
  }
  if (c.S > 1 && (!d.sym || (K != 4 && K != 8 && K != 16 && K != 32)))
    return fail(CAP_E_UNSUPPORTED,
                "several speeds need K in {4, 8, 16, 32} and a point-symmetric step table");
  return CAP_OK;
}

// Allowed speeds of an existing descriptor (the rest of the table unchanged).
inline cap_status set_speed_mask(RolloutDesc* d, uint32_t mask) {
  const uint32_t full = (1u << d->S) - 1u;
  if (mask == 0u) mask = full;
  if ((mask & full) == 0u || (mask & ~full) != 0u)
    return fail(CAP_E_INVALID, "speed_mask must select at least one speed");
  d->smask = mask;
  for (int s = 0; s < d->S; ++s)
    if ((mask >> s) & 1u) d->s_last = s;
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

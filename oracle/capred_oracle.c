/*
 * capred_oracle.c -- plain FP64 CPU oracle for confidence-aware particle
 * prediction (Lu, Bui, Lyu, Chen, "Fast Confidence-Aware Human Prediction via
 * Hardware-accelerated Bayesian Inference for Safe Robot Navigation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no source, header, table
 * generator or helper with the HIP path.
 *
 * Everything is written for obviousness, not speed: FP64 throughout, libm
 * exp/hypot, sequential sums in index order, OpenMP only over independent
 * particles / tracks with private histograms (integer sums, so the result
 * does not depend on the thread count).
 *
 * Conventions (readings of the paper that it leaves open; each one is listed
 * in the design notes):
 *   - headings theta_k = 2*pi*k/K counter-clockwise from +x; one prediction
 *     step moves by v*dt*(cos theta_k, sin theta_k) (discretised 2-D
 *     kinematic model, Sec. III-A running example).  The control set is
 *     speeds {v_0..v_{S-1}} x headings, control u = s*K + k (S = 1: one fixed
 *     speed).  A speed mask (bit s) removes the controls of the other speeds
 *     from the prediction policy (Q = -inf, Sec. IV-B stationary humans).
 *   - Q(x,u;g) = -|x + v*dt*u - g|  (the running example's Q printed in the
 *     paper does not depend on the heading, so the next-state distance is used).
 *   - policy pi(k|x;beta,g) = exp(beta*Q_k) / sum_j exp(beta*Q_j)
 *     (Boltzmann policy, Eq. human_softmax_policy).
 *   - prediction state lives on an integer lattice of pitch q = cell/2^16
 *     relative to the grid origin; the step table is S_k = rint(v*dt*(cos,sin)/q);
 *     start and goals are rounded to the lattice with rint (half-even).
 *   - random numbers: Philox4x32-10 with key (seed lo, seed hi);
 *       pair draw     counter (i, 0,           h, 2*cycle)     word 0
 *       heading draw  counter (i, (t-1)/4,     h, 2*cycle+1)   word (t-1)%4
 *       track sim.    counter (n, (t-1)/4, stream, 0xFFFFFFFF) word (t-1)%4
 *     uniform u = (2*(w>>9)+1) * 2^-24, exactly representable in FP32 and FP64.
 *   - inverse CDF: k = min{k : u*C_{K-1} < C_k}, else K-1.
 *   - pair index j = g*B + b over the belief laid out [G][B]; pair = min{j :
 *     u < P_j} with P the sequential FP64 prefix sum, else the last j with
 *     b_j > 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_MAXK 256
#define ORC_SIM_TAG 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the
 * published round definition: two 32x32->64 products per round, a fixed
 * permutation of the four words, and a Weyl key schedule. */
static void orc_philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  const uint32_t o0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k[0];
  const uint32_t o1 = (uint32_t)p1;
  const uint32_t o2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k[1];
  const uint32_t o3 = (uint32_t)p0;
  c[0] = o0; c[1] = o1; c[2] = o2; c[3] = o3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
    orc_philox_round(c, k);
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Bulk form used by the tests: n counters (c0 = base0 + i, c1, c2, c3). */
void orc_philox_bulk(int64_t n, uint32_t base0, uint32_t c1, uint32_t c2, uint32_t c3,
                     uint64_t seed, uint32_t* out /* [n][4] */) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t i = 0; i < n; ++i) {
    uint32_t ctr[4] = {base0 + (uint32_t)i, c1, c2, c3};
    orc_philox4x32_10(ctr, key, out + 4 * i);
  }
}

double orc_uniform24(uint32_t w) {
  return ((double)(w >> 9) * 2.0 + 1.0) * (1.0 / 16777216.0);
}

static double orc_draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                       int word) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return orc_uniform24(out[word]);
}

/* ------------------------------------------------------------------------ */
/* Lattice (integer positions of pitch q = cell / 65536 from the grid origin). */
static double orc_pitch(double cell) { return cell / 65536.0; }

static int64_t orc_to_lattice(double z, double origin, double cell) {
  return (int64_t)rint((z - origin) / orc_pitch(cell));
}

/* floor(v / 65536) for signed v. */
static int64_t orc_cell_of(int64_t v) {
  if (v >= 0) return v / 65536;
  return -((-v + 65535) / 65536);
}

#define ORC_MAXS 8

/* Control set: S speeds x K headings, u = s*K + k. */
static int orc_check_controls(int K, int S, const double* speeds) {
  if (K < 2 || S < 1 || S > ORC_MAXS || K * S > ORC_MAXK || !speeds) return -1;
  for (int s = 0; s < S; ++s)
    if (!(speeds[s] > 0)) return -1;
  return 0;
}

int orc_lattice_steps(int K, int S, const double* speeds, double dt, double cell, int32_t* Sx,
                      int32_t* Sy) {
  if (orc_check_controls(K, S, speeds) || !(dt > 0) || !(cell > 0)) return -1;
  const double q = orc_pitch(cell);
  for (int s = 0; s < S; ++s) {
    const double L = speeds[s] * dt;
    for (int k = 0; k < K; ++k) {
      const double th = 2.0 * ORC_PI * (double)k / (double)K;
      Sx[s * K + k] = (int32_t)rint(L * cos(th) / q);
      Sy[s * K + k] = (int32_t)rint(L * sin(th) / q);
    }
  }
  return 0;
}

/* allowed[u] = 1 for the controls whose speed bit is set in mask (mask 0: all). */
static int orc_allowed(int K, int S, uint32_t mask, unsigned char* allowed) {
  const uint32_t full = S >= 32 ? 0xFFFFFFFFu : ((1u << S) - 1u);
  if (mask == 0) mask = full;
  if ((mask & full) == 0) return -1;
  for (int s = 0; s < S; ++s)
    for (int k = 0; k < K; ++k) allowed[s * K + k] = (unsigned char)((mask >> s) & 1u);
  return 0;
}

/* Continuous step vectors used by the belief update and the log-likelihood:
 * the FP32 roundings of v_s*dt*(cos theta_k, sin theta_k), u = s*K + k. */
static void orc_cont_steps(int K, int S, const double* speeds, double dt, double* sx,
                           double* sy) {
  for (int s = 0; s < S; ++s) {
    const double L = speeds[s] * dt;
    for (int k = 0; k < K; ++k) {
      const double th = 2.0 * ORC_PI * (double)k / (double)K;
      sx[s * K + k] = (double)(float)(L * cos(th));
      sy[s * K + k] = (double)(float)(L * sin(th));
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Policy on the lattice: cumulative unnormalised weights C_u over the U
 * controls for a particle at (X,Y), goal (GX,GY) and rationality beta.  d_u is
 * the distance to the goal after control u; w_u = exp(-beta (d_u - min d))
 * over the allowed controls, 0 for the others (allowed NULL: all). */
static void orc_lattice_cdf(int U, const int32_t* Sx, const int32_t* Sy,
                            const unsigned char* allowed, double q, int64_t X, int64_t Y,
                            int64_t GX, int64_t GY, double beta, double* C) {
  double d[ORC_MAXK];
  double dmin = INFINITY;
  for (int u = 0; u < U; ++u) {
    const double ax = (double)(X + Sx[u] - GX) * q;
    const double ay = (double)(Y + Sy[u] - GY) * q;
    d[u] = hypot(ax, ay);
    if ((!allowed || allowed[u]) && d[u] < dmin) dmin = d[u];
  }
  double acc = 0.0;
  for (int u = 0; u < U; ++u) {
    if (!allowed || allowed[u]) acc += exp(-beta * (d[u] - dmin));
    C[u] = acc;
  }
}

static int orc_pick(int K, const double* C, double u) {
  const double thr = u * C[K - 1];
  for (int k = 0; k < K; ++k)
    if (thr < C[k]) return k;
  return K - 1;
}

/* Pair CDF over j = g*B + b, sequential FP64 prefix sum of the belief. */
static int orc_pair_cdf(int J, const double* belief, double* P, int* last_pos) {
  double acc = 0.0;
  int last = -1;
  for (int j = 0; j < J; ++j) {
    if (!(belief[j] >= 0.0)) return -1;
    acc += belief[j];
    P[j] = acc;
    if (belief[j] > 0.0) last = j;
  }
  *last_pos = last;
  return last < 0 ? -1 : 0;
}

static int orc_pick_pair(int J, const double* P, int last, double u) {
  for (int j = 0; j < J; ++j)
    if (u < P[j]) return j;
  return last;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 (hardware-accelerated human prediction) step by step, for particle
 * indices idx[0..n_idx) (or 0..N-1 when idx is NULL):
 *   draw (beta,g) once from the belief (bootstrapped belief, Sec. III-B);
 *   for t = 1..H: draw a control u = s*K + k from the Boltzmann policy at the
 *   particle's own state, move one step, emplace the new position on grid t.
 * counts [H][ny][nx] and offgrid [H] are accumulated (caller zeroes them).
 * trace_k [n][H] receives chosen controls u, trace_pair [n] the pair index,
 * trace_cell [n][H] the flattened cell (-1 when off the grid). */
int orc_predict(int K, int S, const double* speeds, uint32_t speed_mask, double dt,
                int B, const float* beta, int G, const float* goals,
                double x0, double y0, double cell, int nx, int ny,
                double zx, double zy, const double* belief,
                int64_t N, int H, uint64_t seed, uint32_t human, uint32_t cycle,
                const int64_t* idx, int64_t n_idx,
                uint32_t* counts, uint32_t* offgrid,
                uint8_t* trace_k, int32_t* trace_pair, int32_t* trace_cell,
                int nthreads) {
  if (B < 1 || G < 1 || N < 1 || H < 1 || nx < 1 || ny < 1) return -1;
  int32_t Sx[ORC_MAXK], Sy[ORC_MAXK];
  unsigned char allowed[ORC_MAXK];
  if (orc_lattice_steps(K, S, speeds, dt, cell, Sx, Sy)) return -1;
  if (orc_allowed(K, S, speed_mask, allowed)) return -1;
  const int U = K * S;
  const double q = orc_pitch(cell);
  const int J = G * B;
  double* P = (double*)malloc(sizeof(double) * J);
  int64_t* GX = (int64_t*)malloc(sizeof(int64_t) * G);
  int64_t* GY = (int64_t*)malloc(sizeof(int64_t) * G);
  int last = -1;
  if (!P || !GX || !GY || orc_pair_cdf(J, belief, P, &last)) {
    free(P); free(GX); free(GY);
    return -1;
  }
  for (int g = 0; g < G; ++g) {
    GX[g] = orc_to_lattice((double)goals[2 * g], x0, cell);
    GY[g] = orc_to_lattice((double)goals[2 * g + 1], y0, cell);
  }
  const int64_t X0 = orc_to_lattice(zx, x0, cell);
  const int64_t Y0 = orc_to_lattice(zy, y0, cell);
  const int64_t n_run = idx ? n_idx : N;
  const int64_t cells = (int64_t)nx * ny;
  const uint32_t c3_pair = 2u * cycle, c3_head = 2u * cycle + 1u;
  int err = 0;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
  {
    uint32_t* hist = NULL;
    uint32_t* off = NULL;
    if (counts) hist = (uint32_t*)calloc((size_t)(cells * H), sizeof(uint32_t));
    if (offgrid) off = (uint32_t*)calloc((size_t)H, sizeof(uint32_t));
    double C[ORC_MAXK];
#pragma omp for schedule(static)
    for (int64_t r = 0; r < n_run; ++r) {
      const int64_t i = idx ? idx[r] : r;
      if (i < 0 || i >= N) { err = 1; continue; }
      const double up = orc_draw(seed, (uint32_t)i, 0u, human, c3_pair, 0);
      const int j = orc_pick_pair(J, P, last, up);
      const int g = j / B, b = j % B;
      if (trace_pair) trace_pair[r] = j;
      const double bt = (double)beta[b];
      int64_t X = X0, Y = Y0;
      for (int t = 1; t <= H; ++t) {
        orc_lattice_cdf(U, Sx, Sy, allowed, q, X, Y, GX[g], GY[g], bt, C);
        const double u = orc_draw(seed, (uint32_t)i, (uint32_t)((t - 1) / 4), human, c3_head,
                                  (t - 1) % 4);
        const int k = orc_pick(U, C, u);
        X += Sx[k];
        Y += Sy[k];
        if (trace_k) trace_k[r * H + (t - 1)] = (uint8_t)k;
        const int64_t cx = orc_cell_of(X), cy = orc_cell_of(Y);
        const int in = (cx >= 0 && cx < nx && cy >= 0 && cy < ny);
        if (trace_cell) trace_cell[r * H + (t - 1)] = in ? (int32_t)(cy * nx + cx) : -1;
        if (in) {
          if (hist) hist[(int64_t)(t - 1) * cells + cy * nx + cx] += 1u;
        } else if (off) {
          off[t - 1] += 1u;
        }
      }
    }
#pragma omp critical
    {
      if (hist) for (int64_t c = 0; c < cells * H; ++c) counts[c] += hist[c];
      if (off) for (int t = 0; t < H; ++t) offgrid[t] += off[t];
    }
    free(hist);
    free(off);
  }
  free(P); free(GX); free(GY);
  return err ? -1 : 0;
}

/* Replays particles with the oracle and compares with another implementation's
 * choices (pair index and heading trace).  Per particle:
 *   status 0 = identical, 1 = first difference explained by a CDF tie within
 *   `window` at that draw, 2 = unexplained difference;
 *   first[r] = first differing step (0 = pair draw, t>=1 = heading step, -1 none). */
int orc_tie_check(int K, int S, const double* speeds, uint32_t speed_mask, double dt,
                  int B, const float* beta, int G, const float* goals,
                  double x0, double y0, double cell,
                  double zx, double zy, const double* belief,
                  int64_t N, int H, uint64_t seed, uint32_t human, uint32_t cycle,
                  const int64_t* idx, int64_t n_idx,
                  const int32_t* other_pair, const uint8_t* other_k, double window,
                  double pair_window, int32_t* status, int32_t* first, int nthreads) {
  int32_t Sx[ORC_MAXK], Sy[ORC_MAXK];
  unsigned char allowed[ORC_MAXK];
  if (orc_lattice_steps(K, S, speeds, dt, cell, Sx, Sy)) return -1;
  if (orc_allowed(K, S, speed_mask, allowed)) return -1;
  const int U = K * S;
  const double q = orc_pitch(cell);
  const int J = G * B;
  double* P = (double*)malloc(sizeof(double) * J);
  int64_t* GX = (int64_t*)malloc(sizeof(int64_t) * G);
  int64_t* GY = (int64_t*)malloc(sizeof(int64_t) * G);
  int last = -1;
  if (!P || !GX || !GY || orc_pair_cdf(J, belief, P, &last)) {
    free(P); free(GX); free(GY);
    return -1;
  }
  for (int g = 0; g < G; ++g) {
    GX[g] = orc_to_lattice((double)goals[2 * g], x0, cell);
    GY[g] = orc_to_lattice((double)goals[2 * g + 1], y0, cell);
  }
  const int64_t X0 = orc_to_lattice(zx, x0, cell);
  const int64_t Y0 = orc_to_lattice(zy, y0, cell);
  const int64_t n_run = idx ? n_idx : N;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int64_t r = 0; r < n_run; ++r) {
    const int64_t i = idx ? idx[r] : r;
    double C[ORC_MAXK];
    status[r] = 0;
    first[r] = -1;
    const double up = orc_draw(seed, (uint32_t)i, 0u, human, 2u * cycle, 0);
    const int j = orc_pick_pair(J, P, last, up);
    const int jo = other_pair[r];
    if (jo != j) {
      first[r] = 0;
      int ok = 0;
      if (jo >= 0 && jo < J) {
        /* other chose a later pair: all of P[j..jo-1] must sit within window of u */
        if (jo > j) ok = (P[jo - 1] - up) <= pair_window;
        else ok = (up - P[jo]) <= pair_window;
      }
      status[r] = ok ? 1 : 2;
      continue;
    }
    const int g = j / B, b = j % B;
    const double bt = (double)beta[b];
    int64_t X = X0, Y = Y0;
    for (int t = 1; t <= H; ++t) {
      orc_lattice_cdf(U, Sx, Sy, allowed, q, X, Y, GX[g], GY[g], bt, C);
      const double u = orc_draw(seed, (uint32_t)i, (uint32_t)((t - 1) / 4), human,
                                2u * cycle + 1u, (t - 1) % 4);
      const int k = orc_pick(U, C, u);
      const int ko = other_k[r * H + (t - 1)];
      if (ko != k) {
        first[r] = t;
        int ok = 0;
        if (ko >= 0 && ko < U && allowed[ko]) {
          const double tot = C[U - 1];
          if (ko > k) ok = (C[ko - 1] / tot - u) <= window;
          else ok = (u - C[ko] / tot) <= window;
        }
        status[r] = ok ? 1 : 2;
        break;
      }
      X += Sx[k];
      Y += Sy[k];
    }
  }
  free(P); free(GX); free(GY);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Control recovery (flatness of the kinematic model: the control follows from
 * two consecutive positions): the control nearest to the displacement dz.
 * Every speed shares the heading k* = argmax_k <dz, (cos,sin)theta_k> (lowest
 * k on ties); the speed is the one whose step v_s dt is nearest to the
 * projection p = <dz, (cos,sin)theta_k*> (lowest s on ties).  u* = s* K + k*;
 * -1 when |dz| < 1e-9 m (no information, the step is skipped).
 * margin[t] (nullable) = best minus second-best heading projection. */
int orc_recover_controls(int K, int S, const double* speeds, double dt, const float* obs,
                         int n_obs, int32_t* ustar, double* margin) {
  if (orc_check_controls(K, S, speeds) || !(dt > 0) || n_obs < 0) return -1;
  for (int t = 0; t < n_obs; ++t) {
    const double dx = (double)obs[2 * (t + 1)] - (double)obs[2 * t];
    const double dy = (double)obs[2 * (t + 1) + 1] - (double)obs[2 * t + 1];
    if (hypot(dx, dy) < 1e-9) {
      ustar[t] = -1;
      if (margin) margin[t] = INFINITY;
      continue;
    }
    int best = 0;
    double bv = -INFINITY, second = -INFINITY;
    for (int k = 0; k < K; ++k) {
      const double th = 2.0 * ORC_PI * (double)k / (double)K;
      const double v = dx * cos(th) + dy * sin(th);
      if (v > bv) { second = bv; bv = v; best = k; }
      else if (v > second) second = v;
    }
    int sb = 0;
    double err = INFINITY;
    for (int s = 0; s < S; ++s) {
      const double e = fabs(speeds[s] * dt - bv);
      if (e < err) { err = e; sb = s; }
    }
    ustar[t] = sb * K + best;
    if (margin) margin[t] = bv - second;
  }
  return 0;
}

/* log pi(u*|z;beta,g) over the U controls of the continuous model (FP64,
 * max-shifted log-sum-exp). */
static double orc_log_policy(int K, const double* sx, const double* sy, double zx, double zy,
                             double gx, double gy, double beta, int kstar) {
  double d[ORC_MAXK];
  double dmin = INFINITY;
  for (int k = 0; k < K; ++k) {
    d[k] = hypot(zx + sx[k] - gx, zy + sy[k] - gy);
    if (d[k] < dmin) dmin = d[k];
  }
  double s = 0.0;
  for (int k = 0; k < K; ++k) s += exp(-beta * (d[k] - dmin));
  return -beta * (d[kstar] - dmin) - log(s);
}

/* Bayesian (beta,g) update (Eq. beta_update, in the log form the paper gives):
 * log b(beta,g) += sum_t log pi(u_t|z_t;beta,g), then subtract the log-sum-exp
 * over all pairs.  (beta,g) is static between observations, so applying the
 * update once per transition equals applying the summed log-likelihood once;
 * `sequential` != 0 renormalises after every transition instead.
 * log_belief [G][B] in/out, belief [G][B] out (nullable), ell [n_obs][G][B]
 * per-transition log-likelihoods out (nullable). */
int orc_belief_update(int K, int S, const double* speeds, double dt, int B, const float* beta,
                      int G, const float* goals, const float* obs, int n_obs,
                      double* log_belief, double* belief, double* ell, int sequential) {
  if (orc_check_controls(K, S, speeds) || !(dt > 0) || B < 1 || G < 1 || n_obs < 0) return -1;
  double sx[ORC_MAXK], sy[ORC_MAXK];
  orc_cont_steps(K, S, speeds, dt, sx, sy);
  const int U = K * S;
  int32_t* ks = (int32_t*)malloc(sizeof(int32_t) * (n_obs > 0 ? n_obs : 1));
  if (!ks) return -1;
  orc_recover_controls(K, S, speeds, dt, obs, n_obs, ks, NULL);
  const int J = G * B;
  double* acc = (double*)calloc((size_t)J, sizeof(double));
  for (int t = 0; t < n_obs; ++t) {
    for (int g = 0; g < G; ++g)
      for (int b = 0; b < B; ++b) {
        double l = 0.0;
        if (ks[t] >= 0)
          l = orc_log_policy(U, sx, sy, (double)obs[2 * t], (double)obs[2 * t + 1],
                             (double)goals[2 * g], (double)goals[2 * g + 1], (double)beta[b],
                             ks[t]);
        if (ell) ell[((int64_t)t * G + g) * B + b] = l;
        if (sequential) log_belief[g * B + b] += l;
        else acc[g * B + b] += l;
      }
    if (sequential) {
      double m = -INFINITY;
      for (int j = 0; j < J; ++j) if (log_belief[j] > m) m = log_belief[j];
      double s = 0.0;
      for (int j = 0; j < J; ++j) s += exp(log_belief[j] - m);
      const double lse = m + log(s);
      for (int j = 0; j < J; ++j) log_belief[j] -= lse;
    }
  }
  if (!sequential) {
    for (int j = 0; j < J; ++j) log_belief[j] += acc[j];
  }
  double m = -INFINITY;
  for (int j = 0; j < J; ++j) if (log_belief[j] > m) m = log_belief[j];
  double s = 0.0;
  for (int j = 0; j < J; ++j) s += exp(log_belief[j] - m);
  const double lse = m + log(s);
  for (int j = 0; j < J; ++j) {
    log_belief[j] -= lse;
    if (belief) belief[j] = exp(log_belief[j]);
  }
  free(acc);
  free(ks);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Trajectory log-likelihood over tracks (product form of Eq. beta_update
 * without normalisation): LL[n][b][g] = sum_{t < len_n} log pi(k*_t|z_t; beta_{n,b}, g),
 * beta = exp(log_beta); log_beta is [B] (shared) or [N][B] (per track).
 * tracks [N][Tmax+1][2] FP32 metres, goals [G][2] FP64 metres. */
int orc_loglik(int K, double speed, double dt, const float* tracks, const int32_t* lengths,
               int N, int Tmax, const double* goals, int G, const double* log_beta, int B,
               int per_track_beta, double* LL, int nthreads) {
  if (K < 2 || K > ORC_MAXK || N < 0 || Tmax < 0 || G < 1 || B < 1) return -1;
  double sx[ORC_MAXK], sy[ORC_MAXK];
  orc_cont_steps(K, 1, &speed, dt, sx, sy);
  if (nthreads < 1) nthreads = 1;
  int err = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int n = 0; n < N; ++n) {
    const float* z = tracks + (int64_t)n * (Tmax + 1) * 2;
    const int len = lengths[n];
    if (len < 0 || len > Tmax) { err = 1; continue; }
    int32_t* ks = (int32_t*)malloc(sizeof(int32_t) * (len > 0 ? len : 1));
    orc_recover_controls(K, 1, &speed, dt, z, len, ks, NULL);
    for (int b = 0; b < B; ++b) {
      const double bt = exp(per_track_beta ? log_beta[(int64_t)n * B + b] : log_beta[b]);
      for (int g = 0; g < G; ++g) {
        double acc = 0.0;
        for (int t = 0; t < len; ++t) {
          if (ks[t] < 0) continue;
          acc += orc_log_policy(K, sx, sy, (double)z[2 * t], (double)z[2 * t + 1],
                                goals[2 * g], goals[2 * g + 1], bt, ks[t]);
        }
        LL[((int64_t)n * B + b) * G + g] = acc;
      }
    }
    free(ks);
  }
  return err ? -1 : 0;
}

/* Analytic gradient of sum_{n,b,g} dLL[n,b,g] * LL[n,b,g] with respect to the
 * goals and log beta.  With d_k = |z + s_k - g|, p = softmax(-beta d) and
 * yhat_k = (z + s_k - g)/d_k (0 when d_k = 0):
 *   d ell / d g        = beta (yhat_{k*} - sum_k p_k yhat_k)
 *   d ell / d log beta = -beta (d_{k*} - sum_k p_k d_k). */
int orc_loglik_grad(int K, double speed, double dt, const float* tracks, const int32_t* lengths,
                    int N, int Tmax, const double* goals, int G, const double* log_beta, int B,
                    int per_track_beta, const double* dLL, double* dgoals, double* dlog_beta) {
  if (K < 2 || K > ORC_MAXK || N < 0 || Tmax < 0 || G < 1 || B < 1) return -1;
  double sx[ORC_MAXK], sy[ORC_MAXK];
  orc_cont_steps(K, 1, &speed, dt, sx, sy);
  memset(dgoals, 0, sizeof(double) * 2 * G);
  memset(dlog_beta, 0, sizeof(double) * (per_track_beta ? (int64_t)N * B : B));
  double d[ORC_MAXK], yx[ORC_MAXK], yy[ORC_MAXK], p[ORC_MAXK];
  for (int n = 0; n < N; ++n) {
    const float* z = tracks + (int64_t)n * (Tmax + 1) * 2;
    const int len = lengths[n];
    if (len < 0 || len > Tmax) return -1;
    int32_t* ks = (int32_t*)malloc(sizeof(int32_t) * (len > 0 ? len : 1));
    orc_recover_controls(K, 1, &speed, dt, z, len, ks, NULL);
    for (int t = 0; t < len; ++t) {
      if (ks[t] < 0) continue;
      const double zx = (double)z[2 * t], zy = (double)z[2 * t + 1];
      for (int g = 0; g < G; ++g) {
        double dmin = INFINITY;
        for (int k = 0; k < K; ++k) {
          const double ax = zx + sx[k] - goals[2 * g];
          const double ay = zy + sy[k] - goals[2 * g + 1];
          d[k] = hypot(ax, ay);
          yx[k] = d[k] > 0.0 ? ax / d[k] : 0.0;
          yy[k] = d[k] > 0.0 ? ay / d[k] : 0.0;
          if (d[k] < dmin) dmin = d[k];
        }
        for (int b = 0; b < B; ++b) {
          const double lb = per_track_beta ? log_beta[(int64_t)n * B + b] : log_beta[b];
          const double bt = exp(lb);
          double s = 0.0;
          for (int k = 0; k < K; ++k) { p[k] = exp(-bt * (d[k] - dmin)); s += p[k]; }
          double ex = 0.0, ey = 0.0, ed = 0.0;
          for (int k = 0; k < K; ++k) {
            p[k] /= s;
            ex += p[k] * yx[k];
            ey += p[k] * yy[k];
            ed += p[k] * d[k];
          }
          const double w = dLL[((int64_t)n * B + b) * G + g];
          dgoals[2 * g] += w * bt * (yx[ks[t]] - ex);
          dgoals[2 * g + 1] += w * bt * (yy[ks[t]] - ey);
          const double gl = -bt * (d[ks[t]] - ed);
          if (per_track_beta) dlog_beta[(int64_t)n * B + b] += w * gl;
          else dlog_beta[b] += w * gl;
        }
      }
    }
    free(ks);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Synthetic humans: n tracks of T lattice steps, each driven by the same
 * Boltzmann policy with its own fixed (beta, goal).  Positions are reported on
 * the lattice (lat, [n][T+1][2]) and as FP32 metres (pos, origin + X*q). */
int orc_simulate_tracks(int K, int S, const double* speeds, double dt, double x0, double y0,
                        double cell, int n, int T, const double* start, const float* beta,
                        const float* goal, uint64_t seed, uint32_t stream, int64_t* lat,
                        float* pos) {
  if (n < 0 || T < 0) return -1;
  int32_t Sx[ORC_MAXK], Sy[ORC_MAXK];
  if (orc_lattice_steps(K, S, speeds, dt, cell, Sx, Sy)) return -1;
  const int U = K * S;
  const double q = orc_pitch(cell);
  double C[ORC_MAXK];
  for (int r = 0; r < n; ++r) {
    int64_t X = orc_to_lattice(start[2 * r], x0, cell);
    int64_t Y = orc_to_lattice(start[2 * r + 1], y0, cell);
    const int64_t GX = orc_to_lattice((double)goal[2 * r], x0, cell);
    const int64_t GY = orc_to_lattice((double)goal[2 * r + 1], y0, cell);
    for (int t = 0; t <= T; ++t) {
      if (t > 0) {
        orc_lattice_cdf(U, Sx, Sy, NULL, q, X, Y, GX, GY, (double)beta[r], C);
        const double u = orc_draw(seed, (uint32_t)r, (uint32_t)((t - 1) / 4), stream,
                                  ORC_SIM_TAG, (t - 1) % 4);
        const int k = orc_pick(U, C, u);
        X += Sx[k];
        Y += Sy[k];
      }
      const int64_t o = ((int64_t)r * (T + 1) + t) * 2;
      if (lat) { lat[o] = X; lat[o + 1] = Y; }
      if (pos) {
        pos[o] = (float)(x0 + (double)X * q);
        pos[o + 1] = (float)(y0 + (double)Y * q);
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Gaussian-smoothed occupancy (Sec. III-B: a Gaussian convolution of the
 * particle batch before emplacement).  Reading: convolving the particle set
 * with a Gaussian and emplacing equals convolving the point histogram with a
 * discrete Gaussian kernel, so
 *   p~_t(x, y) = (1/N) sum_{|dx|<=r, |dy|<=r} w(dx, dy) count_t(x - dx, y - dy),
 *   w(dx, dy) = exp(-(dx^2 + dy^2) / (2 sigma^2)) / Z,  Z = sum of the numerators
 * over the square (2r+1)^2 window, with counts outside the grid taken as zero
 * (mass that the kernel spreads past the border is dropped, like particles
 * that leave the grid).  sigma and r are in cells.  Written as the direct 2-D
 * sum in FP64.  cells[0..n_cells) selects flattened (t, y, x) outputs, written
 * to out[i]; cells == NULL computes all H*ny*nx outputs in order. */
int orc_smooth(const uint32_t* counts, int H, int ny, int nx, int64_t N, double sigma,
               int radius, const int64_t* cells, int64_t n_cells, double* out, int nthreads) {
  if (H < 0 || ny < 1 || nx < 1 || N < 1 || radius < 0 || radius > 64) return -1;
  if (radius > 0 && !(sigma > 0)) return -1;
  const int W = 2 * radius + 1;
  double* w = (double*)malloc(sizeof(double) * W * W);
  if (!w) return -2;
  double Z = 0.0;
  for (int dy = -radius; dy <= radius; ++dy)
    for (int dx = -radius; dx <= radius; ++dx) {
      const double v = radius == 0 ? 1.0 : exp(-(double)(dx * dx + dy * dy) / (2.0 * sigma * sigma));
      w[(dy + radius) * W + (dx + radius)] = v;
      Z += v;
    }
  const int64_t plane = (int64_t)ny * nx;
  const int64_t n = cells ? n_cells : (int64_t)H * plane;
  int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) reduction(|:bad)
#endif
  for (int64_t i = 0; i < n; ++i) {
    const int64_t c = cells ? cells[i] : i;
    if (c < 0 || c >= (int64_t)H * plane) { bad |= 1; continue; }
    const int64_t t = c / plane;
    const int y = (int)((c % plane) / nx), x = (int)(c % nx);
    double acc = 0.0;
    for (int dy = -radius; dy <= radius; ++dy) {
      const int sy = y - dy;
      if (sy < 0 || sy >= ny) continue;
      for (int dx = -radius; dx <= radius; ++dx) {
        const int sx = x - dx;
        if (sx < 0 || sx >= nx) continue;
        acc += w[(dy + radius) * W + (dx + radius)] / Z *
               (double)counts[t * plane + (int64_t)sy * nx + sx];
      }
    }
    out[i] = acc / (double)N;
  }
  free(w);
  return bad ? -1 : 0;
}

/* Point-wise maximum over humans of per-step grids (Sec. IV-B: the union of
 * several humans' predictions on one grid).  grids[h] points to a float32
 * [n] array; out[i] = max_h grids[h][i] in FP64 of the FP32 values. */
int orc_union_max(const float* const* grids, int n_humans, int64_t n, float* out) {
  if (n_humans < 1 || n < 0) return -1;
  for (int64_t i = 0; i < n; ++i) {
    float m = grids[0][i];
    for (int h = 1; h < n_humans; ++h)
      if (grids[h][i] > m) m = grids[h][i];
    out[i] = m;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* MPPI consumer of the predictions (Sec. III-C, local planner), FP64.
 * Robot: 4-D Dubins car z = (x, y, v, theta) with controls u = (a, omega)
 * (Eq. robot_model), forward Euler over dt:
 *   x += v cos(theta) dt,  y += v sin(theta) dt,  v += a dt,  theta += omega dt.
 * Sample i applies u'_t = U_t + delta_{t,i} for t = 1..T (delta laid out
 * [T][N][2]) from z_0 and accumulates
 *   S_i = sum_{t<T} [ (z_t-g)' Q (z_t-g) + u'_t' diag(R) u'_t
 *                     + w_coll * 1{p_t(z_t) >= p_coll} + c_time ]
 *       + (z_T-g)' Qf (z_T-g),
 * with p_t the occupancy probability of the cell holding (x_t, y_t) in grid
 * t of occ [H][ny][nx] (0 off the grid, or when t > H).  Then
 *   U*_t = U_t + sum_i w_i delta_{t,i} / sum_i w_i,  w_i = exp(-(S_i - min S)/tau)
 * (the weighted average of the paper's update, shifted by min S, which
 * cancels).  near[i] (nullable) counts the steps of sample i that read the
 * grid at a position within 1e-9 m of a cell edge, where another
 * implementation's rounding may pick the neighbouring cell.  Readings: the
 * control cost is the quadratic u' diag(R) u (the cost is called quadratic;
 * the printed R^T u is read as that), the collision probability of the robot at
 * step t is the predicted occupancy of its cell in grid t, and the robot step
 * equals the prediction step. */
int orc_mppi(const double* z0, const double* goal, int T, double dt, int N, const double* U,
             const double* delta, const float* occ, int H, double x0, double y0, double cell,
             int nx, int ny, const double* Q, const double* Qf, const double* R, double w_coll,
             double p_coll, double c_time, double tau, double* S, double* U_out,
             int32_t* near) {
  if (T < 1 || N < 1 || !(dt > 0) || !(tau > 0) || !(cell > 0) || nx < 1 || ny < 1 || H < 0)
    return -1;
  for (int i = 0; i < N; ++i) {
    double x = z0[0], y = z0[1], v = z0[2], th = z0[3];
    double s = 0.0;
    int nn = 0;
    for (int t = 1; t <= T; ++t) {
      const double a = U[2 * (t - 1)] + delta[((int64_t)(t - 1) * N + i) * 2];
      const double w = U[2 * (t - 1) + 1] + delta[((int64_t)(t - 1) * N + i) * 2 + 1];
      const double nxp = x + v * cos(th) * dt, nyp = y + v * sin(th) * dt;
      v = v + a * dt;
      th = th + w * dt;
      x = nxp;
      y = nyp;
      const double e[4] = {x - goal[0], y - goal[1], v - goal[2], th - goal[3]};
      if (t < T) {
        for (int k = 0; k < 4; ++k) s += Q[k] * e[k] * e[k];
        s += R[0] * a * a + R[1] * w * w;
        const double fx = (x - x0) / cell, fy = (y - y0) / cell;
        const double cx = floor(fx), cy = floor(fy);
        if (occ && t <= H &&
            (fabs(fx - rint(fx)) * cell < 1e-9 || fabs(fy - rint(fy)) * cell < 1e-9))
          ++nn;
        if (occ && t <= H && cx >= 0 && cx < nx && cy >= 0 && cy < ny) {
          const float p = occ[((int64_t)(t - 1) * ny + (int64_t)cy) * nx + (int64_t)cx];
          if ((double)p >= p_coll) s += w_coll;
        }
        s += c_time;
      } else {
        for (int k = 0; k < 4; ++k) s += Qf[k] * e[k] * e[k];
      }
    }
    S[i] = s;
    if (near) near[i] = nn;
  }
  double smin = INFINITY;
  for (int i = 0; i < N; ++i) if (S[i] < smin) smin = S[i];
  double den = 0.0;
  double* wts = (double*)malloc(sizeof(double) * N);
  if (!wts) return -2;
  for (int i = 0; i < N; ++i) {
    wts[i] = exp(-(S[i] - smin) / tau);
    den += wts[i];
  }
  for (int t = 0; t < T; ++t)
    for (int k = 0; k < 2; ++k) {
      double num = 0.0;
      for (int i = 0; i < N; ++i) num += wts[i] * delta[((int64_t)t * N + i) * 2 + k];
      U_out[2 * t + k] = U[2 * t + k] + num / den;
    }
  free(wts);
  return 0;
}

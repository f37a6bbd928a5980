/*
 * capred.h -- C ABI of the MI355X (gfx950) confidence-aware particle
 * prediction library (libcapred.so).
 *
 * Method: Lu, Bui, Lyu, Chen, "Fast Confidence-Aware Human Prediction via
 * Hardware-accelerated Bayesian Inference for Safe Robot Navigation".
 *   - belief over (rationality beta, goal g) updated from observed steps by
 *     Bayes' rule, Eq. (beta_update), in the log form of Sec. III-B;
 *   - Boltzmann heading policy pi(u|z;beta,g) ~ exp(beta Q(z,u;g)),
 *     Eq. (human_softmax_policy), with Q = -|z + v dt u - g|;
 *   - Alg. 1: particles draw (beta,g) once from the belief, roll H steps of
 *     the discretised kinematic model (Eq. human_dynamics) with Boltzmann
 *     headings, and are emplaced per step on occupancy grids.
 *
 * Conventions shared by every call:
 *   controls      headings theta_k = 2 pi k / K, counter-clockwise from +x, at one
 *                 speed v, or S speeds x K headings with control u = s K + k
 *                 (step v_s dt (cos, sin) theta_k); U = S K.
 *   pair index    j = g * B + b; beliefs are FP64 arrays laid out [G][B].
 *   lattice       prediction state is int32 on a lattice of pitch q = cell/2^16
 *                 from the grid origin; steps S_k = rint(v dt (cos,sin)theta_k / q);
 *                 start and goals are rounded with rint((z - origin)/q).
 *   cells         cell = floor(X / 2^16); grid t (1..H) holds positions after t steps.
 *   random draws  Philox4x32-10, key (seed lo, seed hi), uniform
 *                 u = (2 (w >> 9) + 1) 2^-24:
 *                   pair      counter (i, 0,       human, 2 cycle)     word 0
 *                   control t counter (i, (t-1)/4, human, 2 cycle + 1) word (t-1)%4
 *                   simulated track n, step t: counter (n, (t-1)/4, stream, 0xFFFFFFFF)
 *   inverse CDF   control u = min{u : x C_{U-1} < C_u} (else U-1); pair j = min{j :
 *                 u < P_j} over the sequential FP64 prefix sums P (else the last
 *                 j with positive belief).
 *
 * Memory: every pointer named *_dev is device memory owned by the caller; host
 * pointers are read during the call only.  No call allocates device memory
 * except cap_plan_create (descriptors, owned by the plan).  Every call is
 * asynchronous on the caller's stream (a hipStream_t passed as void*; NULL is
 * the null stream) and never synchronises it.  Calls return a cap_status and
 * never throw; cap_last_error() gives a thread-local message for the last
 * failure.
 */
#ifndef CAPRED_H
#define CAPRED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CAP_ABI_VERSION 2
#define CAP_MAX_K 32   /* headings per model                       */
#define CAP_MAX_B 16   /* rationality values per model             */
#define CAP_MAX_G 64   /* goals per model                          */
#define CAP_MAX_J 512  /* (beta, g) pairs, G * B                    */
#define CAP_MAX_S 8    /* speeds of a multi-speed control set        */
#define CAP_MAX_U 128  /* controls S * K                             */

typedef enum cap_status {
  CAP_OK = 0,
  CAP_E_INVALID = -1,     /* an argument is out of range or a required pointer is NULL */
  CAP_E_HIP = -2,         /* a HIP runtime call failed (message in cap_last_error)    */
  CAP_E_WORKSPACE = -3,   /* the workspace is NULL or smaller than required             */
  CAP_E_UNSUPPORTED = -4, /* no gfx950 device or a feature not built in                 */
  CAP_E_CAPACITY = -5     /* a plan has no room (slots, particles, grid cells)           */
} cap_status;

/* Human model (Sec. III-A).  Host memory. */
typedef struct cap_model {
  int32_t K;            /* headings, 2..CAP_MAX_K                                   */
  double speed;         /* walking speed v in m/s, > 0 (used when n_speeds == 0)    */
  double dt;            /* prediction / observation step in s, > 0                  */
  int32_t B;            /* rationality values, 1..CAP_MAX_B                         */
  const float* beta;    /* host [B], every value > 0                                */
  int32_t G;            /* goals, 1..CAP_MAX_G, with G * B <= CAP_MAX_J             */
  const float* goals;   /* host [G][2], metres, world frame                         */
  /* Multi-speed control set (the |U| = 96 experiments of Sec. IV, e.g. 6 speeds x
   * 16 headings): n_speeds = 0 keeps the one speed above; 1..CAP_MAX_S uses
   * speeds[s] (m/s, > 0) x K headings, S K <= CAP_MAX_U, and `speed` is ignored. */
  int32_t n_speeds;
  const double* speeds;  /* host [n_speeds]                                          */
  /* Prediction-only mask of allowed speeds (bit s; 0 = all): the controls of the
   * other speeds get Q = -inf, as for a human detected standing still
   * (Sec. IV-B).  The belief update always uses every control. */
  uint32_t speed_mask;
} cap_model;

/* Occupancy grid: nx * ny cells of side `cell` metres, lower-left corner at
 * (x0, y0).  1 <= nx, ny <= 16384. */
typedef struct cap_grid {
  double x0, y0, cell;
  int32_t nx, ny;
} cap_grid;

/* Library / device queries. */
int32_t cap_abi_version(void);
const char* cap_last_error(void);
/* Number of compute units of the current device (0 on failure). */
int32_t cap_device_cu_count(void);

/* ------------------------------------------------------------------------
 * Belief update, Eq. (beta_update) in log space (Sec. III-B):
 *   for each observed transition (z_t, z_{t+1}) the control is recovered as the
 *   nearest one: heading k* = argmax_k <z_{t+1} - z_t, (cos, sin) theta_k> (lowest k
 *   on ties), speed s* = argmin_s |v_s dt - p| with p that projection (lowest s
 *   on ties), u* = s* K + k*; a transition shorter than 1e-9 m is skipped; and
 *   log b(beta,g) += sum_t log pi(u*_t | z_t; beta, g) over all U controls,
 *   followed by one log-sum-exp renormalisation over all (beta, g) in FP64.
 * The policy terms are FP32 (continuous steps fl32(v_s dt (cos,sin) theta_k)),
 * accumulated in FP64.
 *   obs_dev         [n_obs + 1][2] FP32 metres, n_obs >= 0
 *   log_belief_dev  [G][B] FP64, in: prior (log), out: posterior (log);
 *                   entries may be -inf (pairs ruled out).
 *   belief_dev      [G][B] FP64 out: exp(log posterior); may be NULL.
 * Errors: CAP_E_INVALID for a bad model, n_obs < 0, NULL obs (n_obs > 0) or NULL
 * log_belief. */
cap_status cap_belief_update(const cap_model* model, const float* obs_dev, int32_t n_obs,
                             double* log_belief_dev, double* belief_dev, void* stream);

/* Uniform prior b^1 = 1 / (|B| |G|) (Sec. III-B) written to log_belief_dev [G][B]. */
cap_status cap_belief_reset(int32_t G, int32_t B, double* log_belief_dev, void* stream);

/* ------------------------------------------------------------------------
 * Alg. 1 for one human: N particles start at z0 (host, metres), each draws
 * (beta, g) from belief_dev once (bootstrapped belief, Sec. III-B) and takes H
 * Boltzmann control steps over the allowed controls (model->speed_mask); grid t
 * receives the particles after t steps.
 *   belief_dev   [G][B] FP64, non-negative, summing to 1 (not renormalised).
 *   counts_dev   [H][ny][nx] uint32 out; zeroed by the call.
 *   offgrid_dev  [H] uint32 out (particles outside the grid), zeroed; may be NULL.
 *   trace_k_dev  [N][H] uint8 out, chosen control u per step; may be NULL.
 *   trace_pair_dev [N] int32 out, pair index j per particle; may be NULL.
 *   1 <= N <= 2^30, 1 <= H <= 4096, cycle < 2^31 - 1.
 * Errors: CAP_E_INVALID for a bad model/grid/size, a start or goal whose
 * lattice coordinates (plus H steps) leave the int32 range, or a step shorter
 * than 2 lattice units. */
cap_status cap_predict_occupancy(const cap_model* model, const cap_grid* grid,
                                 const double z0[2], const double* belief_dev, int32_t N,
                                 int32_t H, uint64_t seed, uint32_t human_id, uint32_t cycle,
                                 uint32_t* counts_dev, uint32_t* offgrid_dev,
                                 uint8_t* trace_k_dev, int32_t* trace_pair_dev, void* stream);

/* Occupancy probabilities p = (float)count / (float)N (IEEE FP32 division),
 * the output p(z_{t'+t} | z_{1:t'}) of Alg. 1.
 *   counts_dev [n_cells] uint32, probs_dev [n_cells] FP32; N >= 1. */
cap_status cap_normalize(const uint32_t* counts_dev, int64_t n_cells, int32_t N,
                         float* probs_dev, void* stream);

/* Gaussian-smoothed occupancy probabilities: the Gaussian convolution of the
 * particle batch before emplacement (Sec. III-B), taken as the convolution of
 * each step's point histogram with the discrete kernel w(dx) w(dy),
 *   w(d) = exp(-d^2 / (2 sigma^2)) / sum_{|e| <= radius} exp(-e^2 / (2 sigma^2)),
 * over the square window |dx|, |dy| <= radius (cells), counts outside the grid
 * being zero, divided by N:
 *   probs[t][y][x] = sum_{dx,dy} w(dx) w(dy) counts[t][y-dy][x-dx] / N.
 *   counts_dev [H][ny][nx] uint32 (device), probs_dev [H][ny][nx] FP32
 *   (device, must not alias counts); radius in [0, 16] (0 gives count / N);
 *   sigma > 0 in cells when radius > 0.  FP32 arithmetic: relative error at
 *   most (4 radius + 6) 2^-24 per output.  Asynchronous on `stream`.
 * Errors: CAP_E_INVALID for a bad size, radius, sigma or pointer. */
cap_status cap_smooth_occupancy(const uint32_t* counts_dev, int32_t H, int32_t ny, int32_t nx,
                                int32_t N, double sigma, int32_t radius, float* probs_dev,
                                void* stream);

/* Union of several humans' predictions on one grid by the point-wise maximum
 * (Sec. IV-B): out[i] = max_h grids[h][i], i < n_cells.
 *   grids: HOST array of n_humans (1..CAP_MAX_SLOTS) DEVICE pointers, each to
 *   at least n_cells FP32 probabilities (no NaN) laid out alike, e.g. [H][ny][nx]
 *   of humans sharing one grid frame; out_dev [n_cells] FP32 (device), may
 *   alias grids[0].  The pointer array is read before the call returns.
 * Errors: CAP_E_INVALID for a bad count or a NULL pointer. */
cap_status cap_union_max(const float* const* grids, int32_t n_humans, int64_t n_cells,
                         float* out_dev, void* stream);

/* Raw Philox4x32-10 blocks of the library's generator, for counters
 * (c0 + i, c1, c2, c3), i < n, key (seed lo, seed hi): out_dev [n][4] uint32.
 * Exposed so that the random-number contract above can be checked directly. */
cap_status cap_philox_blocks(int64_t n, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                             uint64_t seed, uint32_t* out_dev, void* stream);

/* ------------------------------------------------------------------------
 * Synthetic humans: n tracks of T lattice steps, each following the Boltzmann
 * policy with its own fixed (beta, goal) (the model of Sec. III-A, used as a
 * simulator) over the control set of (K, speed) or (n_speeds, speeds) as in
 * cap_model (every control allowed).  The lattice frame (x0, y0, cell) fixes q.
 *   start_dev [n][2] FP64 metres, beta_dev [n] FP32, goal_dev [n][2] FP32 metres.
 *   lat_dev   [n][T+1][2] int32 lattice positions out (may be NULL).
 *   pos_dev   [n][T+1][2] FP32 metres out: fl32(origin + X q) (may be NULL). */
cap_status cap_simulate_tracks(int32_t K, double speed, int32_t n_speeds, const double* speeds,
                               double dt, double x0, double y0,
                               double cell, int32_t n, int32_t T, const double* start_dev,
                               const float* beta_dev, const float* goal_dev, uint64_t seed,
                               uint32_t stream_id, int32_t* lat_dev, float* pos_dev,
                               void* stream);

/* ------------------------------------------------------------------------
 * Trajectory log-likelihood over tracks (product form of Eq. beta_update,
 * unnormalised):  LL[n][b][g] = sum_{t < len_n} log pi(k*_t | z_t; exp(log_beta), g)
 *   tracks_dev   [N][Tmax+1][2] FP32 metres; lengths_dev [N] int32 in [0, Tmax].
 *   goals_dev    [G][2] FP32 metres (continuous, differentiable).
 *   log_beta_dev [B] FP32, or [N][B] when per_track_beta != 0.
 *   LL_dev       [N][B][G] FP64 out.
 * FP32 policy terms, FP64 sums over t.  No workspace.
 * CAP_E_INVALID (nothing launched) for a bad K, speed or dt, N < 0, Tmax < 0,
 * G outside [1, CAP_MAX_G], B outside [1, CAP_MAX_B], N * G above 2^25, or a
 * NULL pointer with N > 0; N = 0 writes nothing. */
cap_status cap_loglik(int32_t K, double speed, double dt, const float* tracks_dev,
                      const int32_t* lengths_dev, int32_t N, int32_t Tmax,
                      const float* goals_dev, int32_t G, const float* log_beta_dev, int32_t B,
                      int32_t per_track_beta, double* LL_dev, void* stream);

/* Adjoint of cap_loglik: given dLL_dev [N][B][G] FP64,
 *   dgoals_dev   [G][2] FP64 = sum_{n,b,t} dLL * beta (yhat_{k*} - E_p[yhat]),
 *   dlog_beta_dev [B] (or [N][B]) FP64 = sum_{n,g,t} dLL * (-beta)(d_{k*} - E_p[d]),
 * with d_k = |z_t + s_k - g|, yhat_k = (z_t + s_k - g)/d_k, p = pi(.|z_t).
 * Reductions are FP64 and deterministic (fixed-order two-stage sums through
 * the workspace; no floating-point atomics).
 *   ws_dev / ws_bytes: workspace of at least cap_loglik_backward_workspace(...) bytes. */
cap_status cap_loglik_backward(int32_t K, double speed, double dt, const float* tracks_dev,
                               const int32_t* lengths_dev, int32_t N, int32_t Tmax,
                               const float* goals_dev, int32_t G, const float* log_beta_dev,
                               int32_t B, int32_t per_track_beta, const double* dLL_dev,
                               double* dgoals_dev, double* dlog_beta_dev, void* ws_dev,
                               size_t ws_bytes, void* stream);
size_t cap_loglik_backward_workspace(int32_t N, int32_t G, int32_t B, int32_t per_track_beta);

/* cap_loglik_backward without a workspace, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, layout, results (bit for bit) and
 * errors as cap_loglik_backward minus ws_dev / ws_bytes; the partial sums go
 * to a library-owned static device array of CAP_LOGLIK_SCRATCH_BYTES, one per
 * device, held until the process ends (its address is looked up once per
 * device, with that device current, on the first call there).
 *   Limit: cap_loglik_backward_workspace(N, G, B, per_track_beta) must not
 *   exceed CAP_LOGLIK_SCRATCH_BYTES (e.g. N * G <= 47662 at B = 9), else
 *   CAP_E_CAPACITY before any launch.  Calls no allocator.
 *   Calls that overlap on one device (different streams, or host threads
 *   without ordering) share the array and race: order them on one stream. */
#define CAP_LOGLIK_SCRATCH_BYTES ((size_t)4 << 20)
cap_status cap_loglik_backward_noalloc(int32_t K, double speed, double dt,
                                       const float* tracks_dev, const int32_t* lengths_dev,
                                       int32_t N, int32_t Tmax, const float* goals_dev,
                                       int32_t G, const float* log_beta_dev, int32_t B,
                                       int32_t per_track_beta, const double* dLL_dev,
                                       double* dgoals_dev, double* dlog_beta_dev, void* stream);

/* ------------------------------------------------------------------------
 * Batched many-human prediction: one persistent launch per cycle for all
 * humans (replacing the sequential per-human loop of Sec. IV-B), captured in
 * hipGraphs together with the belief update, the grid clear and the
 * normalisation.  A plan has `n_slots` slots sharing one model family (K,
 * speed, dt); each slot holds one human with its own N, H, goals, beta grid,
 * grid geometry and output buffers.  Slots are filled and emptied between
 * cycles (continuous batching) without re-capture: the graphs read compact
 * per-cycle descriptors that cap_plan_run copies to the device.
 *
 * Cycles may overlap on the device: cycle c uses ring entry e = c % ring of
 * every per-cycle buffer (descriptors, posterior, grids), and cap_plan_run
 * waits on the host only when the entry it needs is still in flight.  Belief
 * updates of consecutive cycles are ordered by an event even when the caller
 * alternates streams.
 *
 * Results are keyed by the human id and cycle, never by the slot, so a human
 * gets the same grids alone or in any mix. */
typedef struct cap_plan cap_plan;

typedef struct cap_plan_config {
  int32_t n_slots;              /* 1..CAP_MAX_SLOTS                             */
  int32_t K;                    /* headings (shared)                            */
  double speed, dt;             /* shared                                       */
  int32_t max_obs;              /* new observed positions per slot per cycle, 1..8 */
  int32_t ring;                 /* per-cycle buffer ring depth, 1..4            */
  int32_t block_threads;        /* 0 = default; else 256, 512 or 1024           */
  int32_t particles_per_thread; /* 0 = default; else 1, 2 or 4                  */
  int32_t lds_bytes;            /* 0 = default; LDS histogram window per block  */
  int32_t grid_blocks;          /* 0 = default: fill every CU at each rollout
                                   variant's occupancy; else persistent blocks */
  int32_t max_smooth_radius;    /* 0 = no smoothing stage; 1..16 = largest radius a
                                   slot may ask for (sizes the stage's LDS tile) */
  int32_t n_speeds;             /* shared control set as in cap_model: 0 = one speed */
  double speeds[CAP_MAX_S];     /* m/s, first n_speeds entries                   */
} cap_plan_config;

#define CAP_MAX_SLOTS 256

typedef struct cap_slot_desc {
  uint32_t human_id;            /* stable id keying the random streams          */
  int32_t N, H;                 /* particles (<= 2^30), horizon                 */
  int32_t B;                    /* beta values                                  */
  const float* beta;            /* host [B]                                     */
  int32_t G;                    /* goals                                        */
  const float* goals;           /* host [G][2] metres                           */
  cap_grid grid;                /* per-human grid                               */
  float last_xy[2];             /* last observed position before the first staged one */
  uint32_t* counts_dev;         /* [ring][H][ny][nx] uint32, caller-owned       */
  uint32_t* offgrid_dev;        /* [ring][H] uint32 or NULL                     */
  float* probs_dev;             /* [ring][H][ny][nx] FP32 or NULL (skip normalisation) */
  double* log_belief_dev;       /* [G][B] FP64 belief state, caller-owned, in/out */
  double* belief_dev;           /* [ring][G][B] FP64 posterior out (read by the rollout) */
  int32_t reset_belief;         /* 1: write the uniform prior before the first update */
  int32_t smooth_radius;        /* 0: probs = count / N; 1..max_smooth_radius: probs
                                   are the Gaussian-smoothed occupancy of
                                   cap_smooth_occupancy (requires probs_dev)       */
  double smooth_sigma;          /* kernel width in cells, > 0 when smooth_radius > 0 */
  uint32_t speed_mask;          /* allowed speeds of the prediction (bit s; 0 = all) */
} cap_slot_desc;

cap_status cap_plan_create(const cap_plan_config* cfg, cap_plan** out);
void cap_plan_destroy(cap_plan* plan);
/* Admit a human into an empty slot (validated like cap_predict_occupancy). */
cap_status cap_plan_set_slot(cap_plan* plan, int32_t slot, const cap_slot_desc* desc);
/* Retire the human in `slot`; its buffers are not touched by later cycles. */
cap_status cap_plan_clear_slot(cap_plan* plan, int32_t slot);
/* From the next cycle on, predict `slot` with the allowed speeds `mask` (bit s;
 * 0 = all): a human detected standing still gets only the slow controls
 * (Q = -inf for the others, Sec. IV-B).  Errors: no allowed speed. */
cap_status cap_plan_set_speed_mask(cap_plan* plan, int32_t slot, uint32_t mask);
/* Re-uniformise the belief of `slot` before the next cycle's update, as after
 * the human leaves a goal (Sec. IV-B). */
cap_status cap_plan_reset_belief(cap_plan* plan, int32_t slot);
/* Stage the new observed positions of `slot` for the next cycle:
 * xy [n_new][2] FP32 metres (host), 0 <= n_new <= max_obs.  The first one
 * continues from the slot's last observed position. */
cap_status cap_plan_stage_obs(cap_plan* plan, int32_t slot, const float* xy, int32_t n_new);
/* The same for many slots in one call (a serving loop stages every human's
 * new position each cycle): entry i stages one position xy[i] ([n][2] FP32
 * metres, host) for slots[i] (host [n]); a slot listed twice stages two
 * positions in list order.  Every entry is validated before any is staged, so
 * a rejected call (inactive slot, too many staged positions, a position whose
 * horizon leaves the lattice) stages nothing. */
cap_status cap_plan_stage_obs_many(cap_plan* plan, int32_t n, const int32_t* slots,
                                   const float* xy);
/* Run one cycle on `stream`: copy the compact descriptors (with staged
 * observations) to ring entry cycle % ring and launch the captured graphs:
 * belief update -> grid clear -> persistent batched rollout -> normalisation
 * (-> Gaussian smoothing of the slots that ask for it, when the plan was
 * created with max_smooth_radius > 0).
 * Every active slot is predicted from its newest observed position.  The
 * staging area is reusable when this returns.  cycle < 2^31 - 1. */
cap_status cap_plan_run(cap_plan* plan, uint64_t seed, uint32_t cycle, void* stream);
/* Re-launch the rollout of the most recent cycle alone (grid clear, then the
 * persistent rollout kernel), recording ev_start / ev_end (hipEvent_t, may be
 * NULL) on `stream` immediately around the rollout launch.  The outputs are
 * recomputed identically (same keys).  Used to time the rollout kernel. */
cap_status cap_plan_replay_rollout(cap_plan* plan, void* stream, void* ev_start, void* ev_end);
/* Block the host until the last run has completed on the device. */
cap_status cap_plan_sync(cap_plan* plan);
/* Totals over the active slots: particles, particle-steps, and tiles of
 * particles_per_thread * block_threads particles (the per-human launches'
 * tiles; the persistent launch cuts the same particles into tiles of that
 * size, half of it and a quarter of it, sized per cycle to the resident
 * blocks). */
cap_status cap_plan_stats(const cap_plan* plan, int64_t* particles, int64_t* particle_steps,
                          int32_t* tiles);
/* Union stage (Sec. IV-B: the planner reads one occupancy map of all humans):
 * from the next cycle on, every cycle also writes the point-wise maximum of
 * the probabilities (count / N, or the smoothed ones) of each active slot
 * whose grid equals `frame` (same origin, cell, nx, ny) and that has probs_dev,
 * into union_dev[cycle % ring][t][ny][nx] for t < H (a slot contributes its
 * steps t < min(H, its horizon); cells that no such slot reaches are 0).  It is
 * computed inside the cycle's graph: cleared with the grids, then raised by
 * the normalisation / smoothing stages with integer atomic max on the FP32
 * bits (exact, independent of order).  cap_plan_run_plain does the same in its
 * per-human launches.  union_dev: caller-owned [ring][H][ny][nx] FP32;
 * NULL switches the stage off.  Errors: bad frame, H outside [1, 4096]. */
cap_status cap_plan_set_union(cap_plan* plan, const cap_grid* frame, int32_t H, float* union_dev);
/* Effective tuning of the plan (after defaults are resolved). */
cap_status cap_plan_tuning(const cap_plan* plan, cap_plan_config* out);
/* The cut of a cycle's particles into the persistent launch's tiles (host
 * only, no device work; the plan applies it every cycle): units[i] =
 * ceil(N_i / block_threads) for the n active humans (HOST array, each >= 0),
 * particles_per_thread P in {1, 2, 4}, resident_blocks R >= 1 on cus C >= 1
 * compute units.  Writes counts[i][k] (HOST array [n][3]): the number of tiles
 * of human i holding P >> k units (k = 0, 1, 2; only sizes >= 1 occur), with
 * sum_k counts[i][k] (P >> k) = units[i].  Whole rounds of big tiles (one per
 * block) come first; the remainder is spread over the CUs one tile per CU at
 * a time, largest first.  CAP_E_INVALID on bad sizes or NULL pointers. */
cap_status cap_plan_tile_split(const int32_t* units, int32_t n, int32_t particles_per_thread,
                               int32_t resident_blocks, int32_t cus, int32_t* counts);

/* Plain per-human reference of one serving cycle (the paper's sequential
 * multi-human procedure, Sec. IV-B): for each active slot in turn, belief
 * update -> clear -> single-human rollout -> normalisation, one launch each,
 * on `stream`.  Same kernels' arithmetic and random keys as cap_plan_run, so
 * the outputs are identical; used to measure the batched form against it. */
cap_status cap_plan_run_plain(cap_plan* plan, uint64_t seed, uint32_t cycle, void* stream);

/* ------------------------------------------------------------------------
 * MPPI consumer of the predictions (Sec. III-C, local planner; weights of the
 * running example).  Robot: 4-D Dubins car z = (x, y, v, theta), controls
 * u = (a, omega) (Eq. robot_model), forward Euler over dt.  Sample i applies
 * u'_t = U_t + delta_{t,i}, t = 1..T, from z0 and costs
 *   S_i = sum_{t<T} [ (z_t-g)' diag(Q) (z_t-g) + u'_t' diag(R) u'_t
 *                     + w_coll [p_t(z_t) >= p_coll] + c_time ]
 *         + (z_T-g)' diag(Qf) (z_T-g),
 * p_t(z) = occupancy probability of the cell holding (x, y) in prediction grid
 * t (occ [H][ny][nx], the robot step equal to the prediction step; 0 off the
 * grid or for t > H).  Then U_t += sum_i w_i delta_{t,i} / sum_i w_i with
 * w_i = exp(-(S_i - min S) / tau).  FP64 throughout (the collision term is a
 * step function of the cell).
 *   z0, goal: host [4]; U_dev [T][2] FP64 in/out; delta_dev [T][N][2] FP64,
 *   16-byte aligned (perturbations drawn by the caller); occ_dev FP32 or NULL
 *   (no collision term); S_dev [N] FP64 out.  1 <= T <= 65535, 1 <= N <= 2^24.
 * Errors: CAP_E_INVALID for bad sizes, tau <= 0, NULL or misaligned buffers. */
typedef struct cap_mppi_cost {
  double Q[4];     /* running state weights (paper: 3, 3, 10, 0)    */
  double Qf[4];    /* terminal state weights (paper: Q / 5)          */
  double R[2];     /* control weights (paper: 2, 1)                  */
  double w_coll;   /* collision penalty (paper: 1000)                */
  double p_coll;   /* collision probability threshold (paper: 0.1)  */
  double c_time;   /* per-step time cost (the planning interval)     */
  double tau;      /* temperature, > 0                               */
} cap_mppi_cost;

cap_status cap_mppi_step(const double z0[4], const double goal[4], int32_t T, double dt,
                         int32_t N, double* U_dev, const double* delta_dev, const float* occ_dev,
                         int32_t H, const cap_grid* grid, const cap_mppi_cost* cost,
                         double* S_dev, void* stream);

/* ------------------------------------------------------------------------
 * Measurement probes for the roofline of the rollout (not part of the method):
 * cap_probe runs `blocks` x 256 threads, each issuing 8 independent chains of
 * `iters` operations of one kind: 0 FP32 FMA, 1 exp2, 2 sqrt, 3 reciprocal,
 * 4 32x32->64-bit multiply (the Philox round product), 5 LDS atomic add,
 * 6 one exp2 with one multiply and three FMA (mixed issue).
 * Time it with events on `stream`; sink_dev is a [blocks] FP32 buffer that is
 * written only to keep the chains alive.  cap_copy is a plain device copy of
 * `bytes` (16-byte aligned), used to calibrate hardware byte counters.
 * cap_probe_global_atomic runs `blocks` x 256 threads, each issuing 8 chains
 * of `iters` relaxed device-scope adds of 1 (no return value, as the
 * histogram flush issues them) to pseudo-random words of counts_dev, a
 * caller-owned device buffer of 2^log2_words uint32 (log2_words in [6, 30]);
 * after the launch the words sum to blocks * 2048 * iters more than before.
 * Errors: CAP_E_INVALID for a null buffer or out-of-range arguments. */
cap_status cap_probe(int32_t kind, int64_t iters, int32_t blocks, float* sink_dev, void* stream);
cap_status cap_probe_global_atomic(int64_t iters, int32_t blocks, uint32_t* counts_dev,
                                   int32_t log2_words, void* stream);
cap_status cap_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CAPRED_H */

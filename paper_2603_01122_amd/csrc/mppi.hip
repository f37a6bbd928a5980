// mppi.hip -- MPPI consumer of the predicted occupancy grids (Sec. III-C,
// local planner): N sampled control sequences for the 4-D Dubins robot of
// Eq. (robot_model), their trajectory costs against the device-resident
// prediction grids, and the exponentially weighted update of the reference
// controls.
//
// Layout on gfx950: one lane per sample for the rollout (perturbations laid
// out [T][N][2] so that a wavefront reads 64 consecutive (a, omega) pairs per
// step; the reference control of step t is uniform and comes through scalar
// loads).  The robot state and the cost run in FP64: the collision term is a
// step function of the grid cell, and FP64 positions keep the cell decisions
// of this kernel and of an FP64 reference identical except within ~1e-12 m of
// a cell edge.  The update runs one block per step t; every block recomputes
// min S and the weight sum with the same fixed-order reduction, so the result
// does not depend on the launch.
#include <algorithm>

#include "common.hpp"

namespace capred {

constexpr int kMppiThreads = 256;

struct MppiArgs {
  double z0[4], goal[4];
  double Q[4], Qf[4], R[2];
  double w_coll, p_coll, c_time, tau, dt;
  double x0, y0, cell;
  int32_t T, N, H, nx, ny;
  const double* U;      // [T][2]
  const double* delta;  // [T][N][2]
  const float* occ;     // [H][ny][nx] or null
  double* S;            // [N]
};

__global__ void __launch_bounds__(kMppiThreads) mppi_rollout_kernel(const MppiArgs a) {
  // every product and sum rounded on its own, like a plain FP64 reference
#pragma clang fp contract(off)
  const int i = blockIdx.x * kMppiThreads + threadIdx.x;
  if (i >= a.N) return;
  double x = a.z0[0], y = a.z0[1], v = a.z0[2], th = a.z0[3];
  double s = 0.0;
  const double2* dl = reinterpret_cast<const double2*>(a.delta);
  const size_t plane = (size_t)a.nx * a.ny;
  for (int t = 1; t <= a.T; ++t) {
    const double2 d = dl[(size_t)(t - 1) * a.N + i];
    const double ua = a.U[2 * (t - 1)] + d.x;
    const double uw = a.U[2 * (t - 1) + 1] + d.y;
    const double nxp = x + v * cos(th) * a.dt, nyp = y + v * sin(th) * a.dt;
    v = v + ua * a.dt;
    th = th + uw * a.dt;
    x = nxp;
    y = nyp;
    const double e0 = x - a.goal[0], e1 = y - a.goal[1], e2 = v - a.goal[2], e3 = th - a.goal[3];
    if (t < a.T) {
      s += a.Q[0] * e0 * e0;
      s += a.Q[1] * e1 * e1;
      s += a.Q[2] * e2 * e2;
      s += a.Q[3] * e3 * e3;
      s += a.R[0] * ua * ua + a.R[1] * uw * uw;
      if (a.occ && t <= a.H) {
        const double cx = floor((x - a.x0) / a.cell), cy = floor((y - a.y0) / a.cell);
        if (cx >= 0.0 && cx < (double)a.nx && cy >= 0.0 && cy < (double)a.ny) {
          const float p = a.occ[(size_t)(t - 1) * plane + (size_t)cy * a.nx + (size_t)cx];
          if ((double)p >= a.p_coll) s += a.w_coll;
        }
      }
      s += a.c_time;
    } else {
      s += a.Qf[0] * e0 * e0;
      s += a.Qf[1] * e1 * e1;
      s += a.Qf[2] * e2 * e2;
      s += a.Qf[3] * e3 * e3;
    }
  }
  a.S[i] = s;
}

// Block-wide reduction in a fixed order (per-thread partials, then a tree in LDS).
template <bool MIN>
__device__ __forceinline__ double block_fold(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = kMppiThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      red[threadIdx.x] = MIN ? fmin(red[threadIdx.x], red[threadIdx.x + o])
                             : red[threadIdx.x] + red[threadIdx.x + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Block t: U[t] += sum_i w_i delta[t][i] / sum_i w_i, w_i = exp(-(S_i - min S) / tau).
__global__ void __launch_bounds__(kMppiThreads)
    mppi_update_kernel(const double* __restrict__ S, const double* __restrict__ delta, int N,
                       double tau, double* __restrict__ U) {
  __shared__ double red[kMppiThreads];
  const int t = blockIdx.x;
  double m = INFINITY;
  for (int i = threadIdx.x; i < N; i += kMppiThreads) m = fmin(m, S[i]);
  const double smin = block_fold<true>(m, red);
  double den = 0.0, n0 = 0.0, n1 = 0.0;
  const double2* dl = reinterpret_cast<const double2*>(delta) + (size_t)t * N;
  for (int i = threadIdx.x; i < N; i += kMppiThreads) {
    const double w = exp(-(S[i] - smin) / tau);
    const double2 d = dl[i];
    den += w;
    n0 += w * d.x;
    n1 += w * d.y;
  }
  den = block_fold<false>(den, red);
  n0 = block_fold<false>(n0, red);
  n1 = block_fold<false>(n1, red);
  if (threadIdx.x == 0) {
    U[2 * t] += n0 / den;
    U[2 * t + 1] += n1 / den;
  }
}

}  // namespace capred

using namespace capred;

extern "C" cap_status cap_mppi_step(const double z0[4], const double goal[4], int32_t T,
                                    double dt, int32_t N, double* U_dev,
                                    const double* delta_dev, const float* occ_dev, int32_t H,
                                    const cap_grid* grid, const cap_mppi_cost* cost,
                                    double* S_dev, void* stream) {
  if (!z0 || !goal || !cost) return fail(CAP_E_INVALID, "z0, goal or cost is NULL");
  if (T < 1 || T > 65535 || N < 1 || N > (1 << 24))
    return fail(CAP_E_INVALID, "T must be in [1, 65535] and N in [1, 2^24]");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CAP_E_INVALID, "dt must be > 0");
  if (!(cost->tau > 0.0) || !std::isfinite(cost->tau)) return fail(CAP_E_INVALID, "tau must be > 0");
  if (!U_dev || !delta_dev || !S_dev) return fail(CAP_E_INVALID, "U, delta or S is NULL");
  if (occ_dev) {
    if (!grid || !(grid->cell > 0.0) || grid->nx < 1 || grid->ny < 1 || H < 0 ||
        !std::isfinite(grid->x0) || !std::isfinite(grid->y0))
      return fail(CAP_E_INVALID, "occupancy needs a valid grid and H >= 0");
  }
  if ((reinterpret_cast<uintptr_t>(delta_dev) & 15u) != 0)
    return fail(CAP_E_INVALID, "delta must be 16-byte aligned");
  MppiArgs a{};
  for (int k = 0; k < 4; ++k) {
    a.z0[k] = z0[k];
    a.goal[k] = goal[k];
    a.Q[k] = cost->Q[k];
    a.Qf[k] = cost->Qf[k];
  }
  a.R[0] = cost->R[0];
  a.R[1] = cost->R[1];
  a.w_coll = cost->w_coll;
  a.p_coll = cost->p_coll;
  a.c_time = cost->c_time;
  a.tau = cost->tau;
  a.dt = dt;
  a.T = T;
  a.N = N;
  a.U = U_dev;
  a.delta = delta_dev;
  a.S = S_dev;
  if (occ_dev) {
    a.occ = occ_dev;
    a.H = H;
    a.x0 = grid->x0;
    a.y0 = grid->y0;
    a.cell = grid->cell;
    a.nx = grid->nx;
    a.ny = grid->ny;
  } else {
    a.cell = 1.0;
    a.nx = a.ny = 1;
  }
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(mppi_rollout_kernel, dim3((unsigned)((N + kMppiThreads - 1) / kMppiThreads)),
                     dim3(kMppiThreads), 0, s, a);
  hipLaunchKernelGGL(mppi_update_kernel, dim3((unsigned)T), dim3(kMppiThreads), 0, s,
                     (const double*)S_dev, delta_dev, (int)N, cost->tau, U_dev);
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

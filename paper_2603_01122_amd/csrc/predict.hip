// predict.hip -- single-human Alg. 1 (cap_predict_occupancy), grid clearing,
// normalisation (cap_normalize) and the track simulator (cap_simulate_tracks).
#include <algorithm>

#include "model.hpp"

namespace capred {

// LDS budget of the histogram windows of the single-human kernel (two
// buffers: the step being binned and the step being flushed).
constexpr int kPlainThreads = 256;
constexpr int kPlainLdsBytes = 40 * 1024;

__global__ void __launch_bounds__(256) zero_u32_kernel(uint32_t* __restrict__ p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t head = (reinterpret_cast<uintptr_t>(p) & 15u) ? 0 : n / 4;
  uint4* p4 = reinterpret_cast<uint4*>(p);
  for (size_t v = i; v < head; v += stride) p4[v] = make_uint4(0u, 0u, 0u, 0u);
  for (size_t v = head * 4 + i; v < n; v += stride) p[v] = 0u;
}

__global__ void __launch_bounds__(256) normalize_kernel(const uint32_t* __restrict__ c,
                                                        float* __restrict__ p, size_t n,
                                                        float inv_n_unused, float N) {
  (void)inv_n_unused;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool aligned = ((reinterpret_cast<uintptr_t>(c) | reinterpret_cast<uintptr_t>(p)) & 15u) == 0;
  const size_t head = aligned ? n / 4 : 0;
  const uint4* c4 = reinterpret_cast<const uint4*>(c);
  float4* p4 = reinterpret_cast<float4*>(p);
  for (size_t v = i; v < head; v += stride) {
    const uint4 x = c4[v];
    p4[v] = make_float4((float)x.x / N, (float)x.y / N, (float)x.z / N, (float)x.w / N);
  }
  for (size_t v = head * 4 + i; v < n; v += stride) p[v] = (float)c[v] / N;
}

template <int KT, int P, bool SHIFT, bool MS>
__global__ void __launch_bounds__(kPlainThreads)
    rollout_plain_kernel(const RolloutDesc d, uint32_t seed_lo, uint32_t seed_hi, int cap) {
  __shared__ TileShared sh;
  __shared__ float4 ctl[MS ? CAP_MAX_U : 1];
  extern __shared__ uint32_t win[];
  for (int i = threadIdx.x; i < 2 * cap; i += blockDim.x) win[i] = 0u;
  // the first barrier inside rollout_tile orders this clear before any binning
  const int64_t first = (int64_t)blockIdx.x * P * blockDim.x;
  rollout_tile<KT, P, SHIFT, MS>(d, first, seed_lo, seed_hi, sh, win, cap, ctl);
}

// Track simulator: one thread per track, the same control draw as the rollout
// with the track's own (beta, goal) and the simulation counter domain.
template <int KT, bool MS>
__global__ void __launch_bounds__(256)
    simulate_kernel(const RolloutDesc d, int32_t n, int32_t T, const double* __restrict__ start,
                    const float* __restrict__ beta, const float* __restrict__ goal, double x0,
                    double y0, double cell, uint32_t stream_id, uint32_t seed_lo,
                    uint32_t seed_hi, int32_t* __restrict__ lat, float* __restrict__ pos) {
#pragma clang fp contract(off)
  __shared__ float4 ctl[MS ? CAP_MAX_U : 1];
  if constexpr (MS) {
    for (int u = threadIdx.x; u < d.K * d.S; u += blockDim.x)
      ctl[u] = make_float4(d.T.fx[u], d.T.fy[u], d.T.s2[u], 0.f);
    __syncthreads();
  }
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double q = cell / kLatticeScale;
  int32_t X = (int32_t)rint((start[2 * r] - x0) / q);
  int32_t Y = (int32_t)rint((start[2 * r + 1] - y0) / q);
  const int32_t GX = (int32_t)rint(((double)goal[2 * r] - x0) / q);
  const int32_t GY = (int32_t)rint(((double)goal[2 * r + 1] - y0) / q);
  const float ib = (float)(1.0 / (-(double)beta[r] * q * (double)kLog2e));
  const bool shift = (double)beta[r] * (double)max(d.Rx, d.Ry) * q > kNoShiftLimit;
  uint4 w = make_uint4(0u, 0u, 0u, 0u);
  for (int t = 0; t <= T; ++t) {
    if (t > 0) {
      const int s = (t - 1) & 3;
      if (s == 0) w = philox10((uint32_t)r, (uint32_t)((t - 1) >> 2), stream_id, 0xFFFFFFFFu,
                               seed_lo, seed_hi);
      const float u = uniform24f(pick_word(w, s));
      int k;
      if constexpr (MS)
        k = shift ? draw_control<KT, true>((float)(X - GX), (float)(Y - GY), ib, u, d.T, d.S,
                                           d.smask, d.s_last, ctl)
                  : draw_control<KT, false>((float)(X - GX), (float)(Y - GY), ib, u, d.T, d.S,
                                            d.smask, d.s_last, ctl);
      else
        k = shift ? draw_heading<KT, true>((float)(X - GX), (float)(Y - GY), ib, u, d.T, d.K)
                  : draw_heading<KT, false>((float)(X - GX), (float)(Y - GY), ib, u, d.T, d.K);
      X += (int32_t)d.T.fx[k];
      Y += (int32_t)d.T.fy[k];
    }
    const size_t o = ((size_t)r * (T + 1) + t) * 2;
    if (lat) {
      lat[o] = X;
      lat[o + 1] = Y;
    }
    if (pos) {
      pos[o] = (float)(x0 + (double)X * q);
      pos[o + 1] = (float)(y0 + (double)Y * q);
    }
  }
}

__global__ void __launch_bounds__(256)
    philox_blocks_kernel(int64_t n, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t slo, uint32_t shi, uint4* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = philox10(c0 + (uint32_t)i, c1, c2, c3, slo, shi);
}

cap_status launch_zero(uint32_t* p, size_t n, hipStream_t s) {
  if (n == 0) return CAP_OK;
  const size_t blocks = std::min<size_t>((n / 4 + 255) / 256 + 1, 4096);
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

template <int KT, int P, bool MS>
static cap_status launch_plain_t(const RolloutDesc& d, uint32_t slo, uint32_t shi, int cap,
                                 hipStream_t s) {
  const int64_t per_block = (int64_t)P * kPlainThreads;
  const int64_t blocks = (d.N + per_block - 1) / per_block;
  const size_t lds = window_lds_bytes(cap, P * kPlainThreads);
  if (d.shift)
    hipLaunchKernelGGL((rollout_plain_kernel<KT, P, true, MS>), dim3((unsigned)blocks),
                       dim3(kPlainThreads), lds, s, d, slo, shi, cap);
  else
    hipLaunchKernelGGL((rollout_plain_kernel<KT, P, false, MS>), dim3((unsigned)blocks),
                       dim3(kPlainThreads), lds, s, d, slo, shi, cap);
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

static cap_status launch_plain(const RolloutDesc& d, uint32_t slo, uint32_t shi, hipStream_t s) {
  const int cap = kPlainLdsBytes / (2 * (int)sizeof(uint32_t));
  // specialised kernels assume a point-symmetric step table; several speeds
  // need one (checked when the descriptor is built)
  if (d.S > 1) {
    switch (d.K) {
      case 4: return launch_plain_t<4, 1, true>(d, slo, shi, cap, s);
      case 8: return launch_plain_t<8, 1, true>(d, slo, shi, cap, s);
      case 16: return launch_plain_t<16, 1, true>(d, slo, shi, cap, s);
      default: return launch_plain_t<32, 1, true>(d, slo, shi, cap, s);
    }
  }
  switch (d.sym ? d.K : 0) {
    case 4: return launch_plain_t<4, 1, false>(d, slo, shi, cap, s);
    case 8: return launch_plain_t<8, 1, false>(d, slo, shi, cap, s);
    case 16: return launch_plain_t<16, 1, false>(d, slo, shi, cap, s);
    case 32: return launch_plain_t<32, 1, false>(d, slo, shi, cap, s);
    default: return launch_plain_t<0, 1, false>(d, slo, shi, cap, s);
  }
}

}  // namespace capred

using namespace capred;

extern "C" cap_status cap_predict_occupancy(const cap_model* model, const cap_grid* grid,
                                            const double z0[2], const double* belief_dev,
                                            int32_t N, int32_t H, uint64_t seed,
                                            uint32_t human_id, uint32_t cycle,
                                            uint32_t* counts_dev, uint32_t* offgrid_dev,
                                            uint8_t* trace_k_dev, int32_t* trace_pair_dev,
                                            void* stream) {
  Controls c;
  cap_status st = check_model(model, &c);
  if (st != CAP_OK) return st;
  if ((st = check_grid(grid)) != CAP_OK) return st;
  if (!z0 || !belief_dev || !counts_dev) return fail(CAP_E_INVALID, "z0, belief or counts is NULL");
  if (cycle >= 0x7FFFFFFFu) return fail(CAP_E_INVALID, "cycle must be < 2^31 - 1");
  RolloutDesc d;
  st = make_rollout_desc(c, model->dt, model->B, model->beta, model->G, model->goals, *grid, N,
                         H, &d);
  if (st != CAP_OK) return st;
  if ((st = set_start(&d, z0[0], z0[1], *grid)) != CAP_OK) return st;
  d.human = human_id;
  d.cycle = cycle;
  d.belief = belief_dev;
  d.counts = counts_dev;
  d.offgrid = offgrid_dev;
  d.trace_k = trace_k_dev;
  d.trace_pair = trace_pair_dev;
  hipStream_t s = as_stream(stream);
  if ((st = launch_zero(counts_dev, (size_t)H * grid->nx * grid->ny, s)) != CAP_OK) return st;
  if (offgrid_dev && (st = launch_zero(offgrid_dev, (size_t)H, s)) != CAP_OK) return st;
  return launch_plain(d, (uint32_t)seed, (uint32_t)(seed >> 32), s);
}

extern "C" cap_status cap_normalize(const uint32_t* counts_dev, int64_t n_cells, int32_t N,
                                    float* probs_dev, void* stream) {
  if (n_cells < 0 || N < 1) return fail(CAP_E_INVALID, "n_cells must be >= 0 and N >= 1");
  if (n_cells == 0) return CAP_OK;
  if (!counts_dev || !probs_dev) return fail(CAP_E_INVALID, "counts or probs is NULL");
  const size_t n = (size_t)n_cells;
  const size_t blocks = std::min<size_t>((n / 4 + 255) / 256 + 1, 8192);
  hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream),
                     counts_dev, probs_dev, n, 0.f, (float)N);
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

extern "C" cap_status cap_simulate_tracks(int32_t K, double speed, int32_t n_speeds,
                                          const double* speeds, double dt, double x0,
                                          double y0, double cell, int32_t n, int32_t T,
                                          const double* start_dev, const float* beta_dev,
                                          const float* goal_dev, uint64_t seed,
                                          uint32_t stream_id, int32_t* lat_dev, float* pos_dev,
                                          void* stream) {
  Controls c;
  cap_status st = make_controls(K, speed, dt, n_speeds, speeds, 0u, &c);
  if (st != CAP_OK) return st;
  if (n < 0 || T < 0 || T > (1 << 24)) return fail(CAP_E_INVALID, "n >= 0 and 0 <= T <= 2^24 required");
  if (!(cell > 0.0) || !std::isfinite(x0) || !std::isfinite(y0))
    return fail(CAP_E_INVALID, "frame origin must be finite and cell > 0");
  if (n == 0) return CAP_OK;
  if (!start_dev || !beta_dev || !goal_dev) return fail(CAP_E_INVALID, "start/beta/goal is NULL");
  const float one = 1.0f;
  const float zero2[2] = {0.f, 0.f};
  cap_grid g{x0, y0, cell, 1, 1};
  RolloutDesc d;
  st = make_rollout_desc(c, dt, 1, &one, 1, zero2, g, 1, 1, &d);
  if (st != CAP_OK) return st;
  d.shift = 0;
  const uint32_t slo = (uint32_t)seed, shi = (uint32_t)(seed >> 32);
  const dim3 grid_dim((unsigned)((n + 255) / 256)), blk(256);
  hipStream_t s = as_stream(stream);
#define CAP_SIM(KT, MS)                                                                          \
  hipLaunchKernelGGL((simulate_kernel<KT, MS>), grid_dim, blk, 0, s, d, n, T, start_dev, beta_dev, \
                     goal_dev, x0, y0, cell, stream_id, slo, shi, lat_dev, pos_dev)
  switch (d.S > 1 ? -K : (d.sym ? K : 0)) {
    case -4: CAP_SIM(4, true); break;
    case -8: CAP_SIM(8, true); break;
    case -16: CAP_SIM(16, true); break;
    case -32: CAP_SIM(32, true); break;
    case 4: CAP_SIM(4, false); break;
    case 8: CAP_SIM(8, false); break;
    case 16: CAP_SIM(16, false); break;
    case 32: CAP_SIM(32, false); break;
    default: CAP_SIM(0, false); break;
  }
#undef CAP_SIM
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

extern "C" cap_status cap_philox_blocks(int64_t n, uint32_t c0, uint32_t c1, uint32_t c2,
                                        uint32_t c3, uint64_t seed, uint32_t* out_dev,
                                        void* stream) {
  if (n < 0 || n > ((int64_t)1 << 32)) return fail(CAP_E_INVALID, "n must be in [0, 2^32]");
  if (n == 0) return CAP_OK;
  if (!out_dev) return fail(CAP_E_INVALID, "out is NULL");
  if (reinterpret_cast<uintptr_t>(out_dev) & 15u) return fail(CAP_E_INVALID, "out must be 16-byte aligned");
  hipLaunchKernelGGL(philox_blocks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     as_stream(stream), n, c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32),
                     reinterpret_cast<uint4*>(out_dev));
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

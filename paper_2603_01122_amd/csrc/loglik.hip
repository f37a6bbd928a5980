// loglik.hip -- batched trajectory log-likelihood (product form of
// Eq. beta_update over each track) and its adjoint with respect to the goal
// positions and log beta.  A wavefront takes 64 / L goals of one track, and
// each goal's L lanes stride over the observed steps (L = 64: one goal per
// wave).  FP32 policy terms are accumulated per lane in FP64 and reduced
// across each goal's lanes by a fixed butterfly, so for a given L results are
// bitwise reproducible.  The adjoint writes per-(track, goal) partials to the
// workspace and a second kernel sums them in a fixed order (no atomics).
#include <algorithm>
#include <mutex>

#include "belief.hpp"

namespace capred {

constexpr int kLLThreads = 256;  // 4 wavefronts

// Sum over the 2^lg lanes of this lane's goal (a butterfly inside the group).
__device__ __forceinline__ double group_sum(double v, int lg) {
  for (int o = (1 << lg) >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// This lane's (track, goal, first step) for 2^lg lanes per goal; `on` is false
// for the lanes of a wave's last goal slots beyond G (they add nothing but
// take part in the group sums).
struct LLItem {
  int n, g, sub;
  bool on;
};

__device__ __forceinline__ bool ll_item(int G, int N, int lg, LLItem* it) {
  const int lane = threadIdx.x & 63;
  const int gpw = 64 >> lg;                    // goals per wave
  const int groups = (G + gpw - 1) / gpw;      // waves per track
  const int wave = blockIdx.x * (kLLThreads / 64) + (threadIdx.x >> 6);
  if (wave >= N * groups) return false;        // whole wavefront exits together
  it->n = wave / groups;
  const int g = (wave - it->n * groups) * gpw + (lane >> lg);
  it->on = g < G;
  it->g = it->on ? g : 0;
  it->sub = lane & ((1 << lg) - 1);
  return true;
}

struct LLArgs {
  BeliefModel m;           // K, continuous steps and heading unit vectors
  const float* tracks;     // [N][Tmax+1][2]
  const int32_t* lengths;  // [N]
  int32_t N, Tmax, G, B, per_track;
  const float* goals;      // [G][2]
  const float* log_beta;   // [B] or [N][B]
};

__device__ __forceinline__ void load_beta(const LLArgs& a, int n, float* beta) {
  const float* lb = a.per_track ? a.log_beta + (size_t)n * a.B : a.log_beta;
  for (int b = 0; b < a.B; ++b) beta[b] = expf(lb[b]);
}

template <int KT>
__global__ void __launch_bounds__(kLLThreads)
    loglik_kernel(const LLArgs a, int lg, double* __restrict__ LL) {
  LLItem it;
  if (!ll_item(a.G, a.N, lg, &it)) return;
  const int n = it.n, g = it.g;
  const int len = it.on ? a.lengths[n] : 0;
  const float* z = a.tracks + (size_t)n * (a.Tmax + 1) * 2;
  const float gx = a.goals[2 * g], gy = a.goals[2 * g + 1];
  float beta[CAP_MAX_B], terms[CAP_MAX_B];
  load_beta(a, n, beta);
  double acc[CAP_MAX_B];
  for (int b = 0; b < a.B; ++b) acc[b] = 0.0;
  for (int t = it.sub; t < len; t += 1 << lg) {
    const float zx = z[2 * t], zy = z[2 * t + 1];
    const int ks = recover_control(a.m, z[2 * t + 2] - zx, z[2 * t + 3] - zy);
    if constexpr (KT > 0)
      policy_terms_fixed<KT>(a.m, zx, zy, ks, gx, gy, beta, a.B, terms);
    else
      policy_terms<CAP_MAX_K>(a.m, zx, zy, ks, gx, gy, beta, a.B, terms);
    for (int b = 0; b < a.B; ++b) acc[b] += (double)terms[b];
  }
  for (int b = 0; b < a.B; ++b) {
    const double s = group_sum(acc[b], lg);
    if (it.on && it.sub == 0) LL[((size_t)n * a.B + b) * a.G + g] = s;
  }
}

// Per-step adjoint terms for one (z, goal) and every beta:
//   d ell/d g        = -beta (E_p[yhat] - yhat_{k*}),
//   d ell/d log beta = -beta (Delta_{k*} - E_p[Delta]),
// with yhat_k = (a + s_k)/d_k and, to avoid cancellation between unit vectors,
//   yhat_k - yhat_* = a (Delta_* - Delta_k)/(d_k d_*) + s_k/d_k - s_*/d_*.
// KT > 0: the model has KT headings (loops over headings fully unrolled, so
// the per-heading arrays stay in registers); KT == 0: any K.
template <int KT>
__global__ void __launch_bounds__(kLLThreads)
    loglik_backward_kernel(const LLArgs a, int lg, const double* __restrict__ dLL,
                           double* __restrict__ ws_g, double* __restrict__ ws_b) {
  constexpr int KM = KT > 0 ? KT : CAP_MAX_K;
  LLItem it;
  if (!ll_item(a.G, a.N, lg, &it)) return;
  const int n = it.n, g = it.g;
  const int len = it.on ? a.lengths[n] : 0;
  const int K = KT > 0 ? KT : a.m.K, B = a.B;
  const float* z = a.tracks + (size_t)n * (a.Tmax + 1) * 2;
  const float gx = a.goals[2 * g], gy = a.goals[2 * g + 1];
  float beta[CAP_MAX_B], w[CAP_MAX_B];
  load_beta(a, n, beta);
  for (int b = 0; b < B; ++b) w[b] = (float)dLL[((size_t)n * B + b) * a.G + g];
  double agx = 0.0, agy = 0.0, ab[CAP_MAX_B];
  for (int b = 0; b < B; ++b) ab[b] = 0.0;
  float dl[KM], dk[KM];
  for (int t = it.sub; t < len; t += 1 << lg) {
    const float zx = z[2 * t], zy = z[2 * t + 1];
    const int ks = recover_control(a.m, z[2 * t + 2] - zx, z[2 * t + 3] - zy);
    if (ks < 0) continue;
    const float ax = zx - gx, bx = ax - zx;
    const float ax_lo = (zx - (ax - bx)) + (-gx - bx);
    const float ay = zy - gy, by = ay - zy;
    const float ay_lo = (zy - (ay - by)) + (-gy - by);
    const float D2 = fmaf(ax, ax, ay * ay);
    const float D = fast_sqrt(D2);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      if (KT == 0 && k >= K) break;
      const float corr = fmaf(2.f * ax_lo, a.m.sx[k], fmaf(2.f * ay_lo, a.m.sy[k], a.m.s2[k]));
      const float nk = fmaf(ax + ax, a.m.sx[k], fmaf(ay + ay, a.m.sy[k], corr));
      // hardware square root and reciprocal, as in the forward's fixed-K path
      dk[k] = fast_sqrt(fmaxf(D2 + nk, 0.f));
      dl[k] = nk * fast_rcp(dk[k] + D);
    }
    if constexpr (KT > 0) {
      const float ds = dk[ks], dls = dl[ks], sxs = a.m.sx[ks], sys = a.m.sy[ks];
      // the unit vectors take hardware reciprocals (within 1 ulp) in place of
      // IEEE divisions, one per heading instead of three (11 % of the kernel's
      // time at K = 32); the gradient's error bar is 1e-5 of its norm
      const float rds = ds > 0.f ? __builtin_amdgcn_rcpf(ds) : 0.f;
      const float sxs_ds = sxs * rds, sys_ds = sys * rds;
      // yhat_k - yhat_* once per heading (independent of beta; yhat := 0 where
      // the distance is 0), and max_k (-beta dl_k) = -beta min_k dl_k exactly
      // (the rounded product is monotone in dl_k)
      float ux[KM], uy[KM];
      float dmin = INFINITY;
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        const float rk = __builtin_amdgcn_rcpf(dk[k]);
        if (dk[k] > 0.f && ds > 0.f) {
          const float v = (dls - dl[k]) * (rk * rds);
          ux[k] = fmaf(ax, v, fmaf(a.m.sx[k], rk, -sxs_ds));
          uy[k] = fmaf(ay, v, fmaf(a.m.sy[k], rk, -sys_ds));
        } else if (dk[k] > 0.f) {
          ux[k] = (ax + a.m.sx[k]) * rk;
          uy[k] = (ay + a.m.sy[k]) * rk;
        } else if (ds > 0.f) {
          ux[k] = -(ax + sxs) * rds;
          uy[k] = -(ay + sys) * rds;
        } else {
          ux[k] = 0.f;
          uy[k] = 0.f;
        }
        dmin = fminf(dmin, dl[k]);
      }
      for (int b = 0; b < B; ++b) {
        const float nbt = -beta[b];
        // base-2 exponents with the shift folded into one FMA (p is a ratio,
        // so the shift's rounding cancels)
        const float nb2 = nbt * kLog2e, mx2 = nb2 * dmin;
        float s = 0.f, ex = 0.f, ey = 0.f, ed = 0.f;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const float p = fast_exp2(fmaf(nb2, dl[k], -mx2));
          s += p;
          ex = fmaf(p, ux[k], ex);
          ey = fmaf(p, uy[k], ey);
          ed = fmaf(p, dl[k] - dls, ed);
        }
        const float inv = 1.f / s;
        // E[yhat] - yhat_* = ex/s ; E[Delta] - Delta_* = ed/s
        agx += (double)(w[b] * (nbt * (ex * inv)));
        agy += (double)(w[b] * (nbt * (ey * inv)));
        ab[b] += (double)(w[b] * (beta[b] * (ed * inv)));
      }
    } else {
      // any K: per (beta, heading), without per-heading arrays beyond dl and dk
      const float ds = dk[ks];
      for (int b = 0; b < B; ++b) {
        const float nbt = -beta[b];
        float mx = -INFINITY;
        for (int k = 0; k < K; ++k) mx = fmaxf(mx, nbt * dl[k]);
        float s = 0.f, ex = 0.f, ey = 0.f, ed = 0.f;
        for (int k = 0; k < K; ++k) {
          const float p = exp_nonpos(nbt * dl[k] - mx);
          s += p;
          // yhat_k - yhat_*  (yhat := 0 where the distance is 0)
          float ux, uy;
          if (dk[k] > 0.f && ds > 0.f) {
            const float v = (dl[ks] - dl[k]) / (dk[k] * ds);
            ux = fmaf(ax, v, a.m.sx[k] / dk[k] - a.m.sx[ks] / ds);
            uy = fmaf(ay, v, a.m.sy[k] / dk[k] - a.m.sy[ks] / ds);
          } else if (dk[k] > 0.f) {
            ux = (ax + a.m.sx[k]) / dk[k];
            uy = (ay + a.m.sy[k]) / dk[k];
          } else if (ds > 0.f) {
            ux = -(ax + a.m.sx[ks]) / ds;
            uy = -(ay + a.m.sy[ks]) / ds;
          } else {
            ux = 0.f;
            uy = 0.f;
          }
          ex = fmaf(p, ux, ex);
          ey = fmaf(p, uy, ey);
          ed = fmaf(p, dl[k] - dl[ks], ed);
        }
        const float inv = 1.f / s;
        // E[yhat] - yhat_* = ex/s ; E[Delta] - Delta_* = ed/s
        agx += (double)(w[b] * (nbt * (ex * inv)));
        agy += (double)(w[b] * (nbt * (ey * inv)));
        ab[b] += (double)(w[b] * (beta[b] * (ed * inv)));
      }
    }
  }
  const double sgx = group_sum(agx, lg), sgy = group_sum(agy, lg);
  if (it.on && it.sub == 0) {
    ws_g[((size_t)n * a.G + g) * 2] = sgx;
    ws_g[((size_t)n * a.G + g) * 2 + 1] = sgy;
  }
  for (int b = 0; b < B; ++b) {
    const double s = group_sum(ab[b], lg);
    if (it.on && it.sub == 0) ws_b[((size_t)n * a.G + g) * B + b] = s;
  }
}

// Fixed-order second stage.  Long sums -- the goals over tracks, a shared log
// beta over (track, goal) -- take one block per output: thread t adds terms
// t, t + 256, ... in ascending order, then a fixed tree combines the 256
// partials.  Per-track log beta (a sum over the goals only) takes one thread
// per output.  Every order is fixed, so results are bitwise reproducible.
constexpr int kSumThreads = 256;

__global__ void __launch_bounds__(kSumThreads)
    loglik_sum_kernel(int N, int G, int B, const double* __restrict__ ws_g,
                      const double* __restrict__ ws_b, double* __restrict__ dgoals,
                      double* __restrict__ dlog_beta) {
  __shared__ double red[kSumThreads];
  const int o = blockIdx.x;
  double s = 0.0;
  if (o < 2 * G) {
    const int g = o >> 1, c = o & 1;
    for (int n = threadIdx.x; n < N; n += kSumThreads) s += ws_g[((size_t)n * G + g) * 2 + c];
  } else {
    const int jb = o - 2 * G;
    const int total = N * G;  // term i = n G + g
    for (int i = threadIdx.x; i < total; i += kSumThreads) s += ws_b[(size_t)i * B + jb];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kSumThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (o < 2 * G) dgoals[o] = red[0];
    else dlog_beta[o - 2 * G] = red[0];
  }
}

__global__ void loglik_track_beta_kernel(int N, int G, int B, const double* __restrict__ ws_b,
                                         double* __restrict__ dlog_beta) {
  const int jb = blockIdx.x * blockDim.x + threadIdx.x;
  if (jb >= N * B) return;
  const int n = jb / B, b = jb - n * B;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += ws_b[((size_t)n * G + g) * B + b];
  dlog_beta[jb] = s;
}

// log2 of the lanes per (track, goal) for a launch.  Fewer lanes per goal
// leave fewer idle in a track's last pass over its steps (200 steps: 78 % of
// the lanes busy at 64 lanes per goal, 89 % at 32, 96 % at 16) but make fewer
// waves.  Each width is scored by its busy fraction (from Tmax, and the goal
// slots the last wave of a track leaves empty) times the fraction of
// `target_waves` resident wave slots its waves fill; ties keep the wider form.
static int ll_lanes_log2(int N, int G, int Tmax, double target_waves) {
  int best = 6;
  double best_score = -1.0;
  for (int lg = 6; lg >= 3; --lg) {
    const int L = 1 << lg, gpw = 64 >> lg;
    const long groups = (G + gpw - 1) / gpw;
    const double waves = (double)N * (double)groups;
    const double passes = Tmax > 0 ? (double)((Tmax + L - 1) / L) : 1.0;
    const double busy = (Tmax > 0 ? Tmax / (L * passes) : 1.0) * ((double)G / ((double)groups * gpw));
    const double score = busy * std::min(1.0, waves / target_waves);
    if (score > best_score + 1e-9) {
      best = lg;
      best_score = score;
    }
  }
  return best;
}

// Resident wave slots of the device's 1024 SIMDs (256 CUs x 4) at each
// kernel's occupancy: the forward holds four waves per SIMD at every K; the
// adjoint two at K = 32 (247 VGPRs), three at K = 16 and in the any-K build
// (kt = 0), four at K <= 8.
constexpr double kSimds = 1024.0;
static double ll_forward_waves() { return 4.0 * kSimds; }
static double ll_backward_waves(int kt) {
  return (kt == 32 ? 2.0 : kt == 16 || kt == 0 ? 3.0 : 4.0) * kSimds;
}

static cap_status make_ll_args(int32_t K, double speed, double dt, const float* tracks,
                               const int32_t* lengths, int32_t N, int32_t Tmax,
                               const float* goals, int32_t G, const float* log_beta, int32_t B,
                               int32_t per_track, LLArgs* a) {
  Controls c;
  cap_status st = make_controls(K, speed, dt, 0, nullptr, 0u, &c);
  if (st != CAP_OK) return st;
  if (N < 0 || Tmax < 0) return fail(CAP_E_INVALID, "N and Tmax must be >= 0");
  if (G < 1 || G > CAP_MAX_G || B < 1 || B > CAP_MAX_B)
    return fail(CAP_E_INVALID, "G in [1, 64] and B in [1, 16] required");
  // one wave (64 threads) per (track, goal) at most: thread indices stay in int
  if ((int64_t)N * G > ((int64_t)1 << 25)) return fail(CAP_E_INVALID, "N * G above 2^25");
  if (N > 0 && (!tracks || !lengths || !goals || !log_beta))
    return fail(CAP_E_INVALID, "tracks/lengths/goals/log_beta is NULL");
  a->m = make_belief_model(c, dt, 0, nullptr, 0, nullptr);
  a->tracks = tracks;
  a->lengths = lengths;
  a->N = N;
  a->Tmax = Tmax;
  a->G = G;
  a->B = B;
  a->per_track = per_track ? 1 : 0;
  a->goals = goals;
  a->log_beta = log_beta;
  return CAP_OK;
}

}  // namespace capred

using namespace capred;

extern "C" cap_status cap_loglik(int32_t K, double speed, double dt, const float* tracks_dev,
                                 const int32_t* lengths_dev, int32_t N, int32_t Tmax,
                                 const float* goals_dev, int32_t G, const float* log_beta_dev,
                                 int32_t B, int32_t per_track_beta, double* LL_dev, void* stream) {
  LLArgs a;
  cap_status st = make_ll_args(K, speed, dt, tracks_dev, lengths_dev, N, Tmax, goals_dev, G,
                               log_beta_dev, B, per_track_beta, &a);
  if (st != CAP_OK) return st;
  if (N == 0) return CAP_OK;
  if (!LL_dev) return fail(CAP_E_INVALID, "LL is NULL");
  const int lg = ll_lanes_log2(N, G, Tmax, ll_forward_waves());
  const int gpw = 64 >> lg, per_block = kLLThreads / 64;
  const long waves = (long)N * ((G + gpw - 1) / gpw);
  const dim3 grid((unsigned)((waves + per_block - 1) / per_block)), block(kLLThreads);
  hipStream_t s = as_stream(stream);
  switch (a.m.U) {
    case 4: hipLaunchKernelGGL(loglik_kernel<4>, grid, block, 0, s, a, lg, LL_dev); break;
    case 8: hipLaunchKernelGGL(loglik_kernel<8>, grid, block, 0, s, a, lg, LL_dev); break;
    case 16: hipLaunchKernelGGL(loglik_kernel<16>, grid, block, 0, s, a, lg, LL_dev); break;
    case 32: hipLaunchKernelGGL(loglik_kernel<32>, grid, block, 0, s, a, lg, LL_dev); break;
    default: hipLaunchKernelGGL(loglik_kernel<0>, grid, block, 0, s, a, lg, LL_dev); break;
  }
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

extern "C" size_t cap_loglik_backward_workspace(int32_t N, int32_t G, int32_t B,
                                                int32_t per_track_beta) {
  (void)per_track_beta;
  if (N < 0 || G < 0 || B < 0) return 0;
  return (size_t)N * G * (2 + B) * sizeof(double);
}

namespace capred {

// The adjoint's launches with the partial sums in ws (cap_loglik_backward_workspace bytes).
static cap_status loglik_backward_launch(const LLArgs& a, int32_t per_track_beta,
                                         const double* dLL_dev, double* dgoals_dev,
                                         double* dlog_beta_dev, void* ws_dev, hipStream_t s) {
  const int32_t N = a.N, G = a.G, B = a.B;
  double* ws_g = static_cast<double*>(ws_dev);
  double* ws_b = ws_g + (size_t)N * G * 2;
  if (N > 0) {
    const int kt = a.m.K == 4 || a.m.K == 8 || a.m.K == 16 || a.m.K == 32 ? a.m.K : 0;
    const int lg = ll_lanes_log2(N, G, a.Tmax, ll_backward_waves(kt));
    const int gpw = 64 >> lg, per_block = kLLThreads / 64;
    const long waves = (long)N * ((G + gpw - 1) / gpw);
    const dim3 grid((unsigned)((waves + per_block - 1) / per_block)), block(kLLThreads);
    switch (kt) {
      case 4: hipLaunchKernelGGL(loglik_backward_kernel<4>, grid, block, 0, s, a, lg, dLL_dev, ws_g, ws_b); break;
      case 8: hipLaunchKernelGGL(loglik_backward_kernel<8>, grid, block, 0, s, a, lg, dLL_dev, ws_g, ws_b); break;
      case 16: hipLaunchKernelGGL(loglik_backward_kernel<16>, grid, block, 0, s, a, lg, dLL_dev, ws_g, ws_b); break;
      case 32: hipLaunchKernelGGL(loglik_backward_kernel<32>, grid, block, 0, s, a, lg, dLL_dev, ws_g, ws_b); break;
      default: hipLaunchKernelGGL(loglik_backward_kernel<0>, grid, block, 0, s, a, lg, dLL_dev, ws_g, ws_b); break;
    }
    CAP_HIP(hipGetLastError());
  }
  // with N = 0 the sums are empty: the kernels write zeros
  const int long_sums = 2 * G + (per_track_beta ? 0 : B);
  hipLaunchKernelGGL(loglik_sum_kernel, dim3(long_sums), dim3(kSumThreads), 0, s, N, G, B, ws_g,
                     ws_b, dgoals_dev, dlog_beta_dev);
  if (per_track_beta && N > 0)
    hipLaunchKernelGGL(loglik_track_beta_kernel, dim3((N * B + 255) / 256), dim3(256), 0, s, N, G,
                       B, ws_b, dlog_beta_dev);
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

// Device-resident partial sums of the allocation-free adjoint.  Each device
// holds its own copy (until the process ends); host code reaches it only
// through the per-device address from hipGetSymbolAddress, never through the
// array's name, which on the host is a stand-in and not a device address.
__device__ __align__(256) double loglik_scratch[CAP_LOGLIK_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// loglik_scratch's address on the current device (looked up once per device).
static cap_status scratch_of_current_device(void** out) {
  int dev = 0;
  CAP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CAP_E_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    CAP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(loglik_scratch)));
    if (!p) return fail(CAP_E_HIP, "hipGetSymbolAddress returned no address for the scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CAP_OK;
}

}  // namespace capred

extern "C" cap_status cap_loglik_backward(int32_t K, double speed, double dt,
                                          const float* tracks_dev, const int32_t* lengths_dev,
                                          int32_t N, int32_t Tmax, const float* goals_dev,
                                          int32_t G, const float* log_beta_dev, int32_t B,
                                          int32_t per_track_beta, const double* dLL_dev,
                                          double* dgoals_dev, double* dlog_beta_dev, void* ws_dev,
                                          size_t ws_bytes, void* stream) {
  LLArgs a;
  cap_status st = make_ll_args(K, speed, dt, tracks_dev, lengths_dev, N, Tmax, goals_dev, G,
                               log_beta_dev, B, per_track_beta, &a);
  if (st != CAP_OK) return st;
  if (!dgoals_dev || !dlog_beta_dev) return fail(CAP_E_INVALID, "dgoals/dlog_beta is NULL");
  if (N > 0 && !dLL_dev) return fail(CAP_E_INVALID, "dLL is NULL");
  const size_t need = cap_loglik_backward_workspace(N, G, B, per_track_beta);
  if (need > 0 && (!ws_dev || ws_bytes < need))
    return fail(CAP_E_WORKSPACE, "workspace smaller than cap_loglik_backward_workspace()");
  return loglik_backward_launch(a, per_track_beta, dLL_dev, dgoals_dev, dlog_beta_dev, ws_dev,
                                as_stream(stream));
}

extern "C" cap_status cap_loglik_backward_noalloc(int32_t K, double speed, double dt,
                                                  const float* tracks_dev,
                                                  const int32_t* lengths_dev, int32_t N,
                                                  int32_t Tmax, const float* goals_dev, int32_t G,
                                                  const float* log_beta_dev, int32_t B,
                                                  int32_t per_track_beta, const double* dLL_dev,
                                                  double* dgoals_dev, double* dlog_beta_dev,
                                                  void* stream) {
  LLArgs a;
  cap_status st = make_ll_args(K, speed, dt, tracks_dev, lengths_dev, N, Tmax, goals_dev, G,
                               log_beta_dev, B, per_track_beta, &a);
  if (st != CAP_OK) return st;
  if (!dgoals_dev || !dlog_beta_dev) return fail(CAP_E_INVALID, "dgoals/dlog_beta is NULL");
  if (N > 0 && !dLL_dev) return fail(CAP_E_INVALID, "dLL is NULL");
  if (cap_loglik_backward_workspace(N, G, B, per_track_beta) > CAP_LOGLIK_SCRATCH_BYTES)
    return fail(CAP_E_CAPACITY,
                "N * G * (2 + B) * 8 bytes exceed CAP_LOGLIK_SCRATCH_BYTES; use cap_loglik_backward "
                "with a caller workspace");
  void* scratch = nullptr;
  st = scratch_of_current_device(&scratch);
  if (st != CAP_OK) return st;
  // every partial-sum slot the launches read is written first (one per (track,
  // goal) item), so the previous call's contents need no clearing
  return loglik_backward_launch(a, per_track_beta, dLL_dev, dgoals_dev, dlog_beta_dev, scratch,
                                as_stream(stream));
}

// belief.hpp -- device side of the (beta, g) belief update, Eq. (beta_update)
// in the log form of Sec. III-B, for one human per thread block.
#pragma once

#include "dfloat.hpp"
#include "model.hpp"

namespace capred {

constexpr int kBeliefThreads = 256;
constexpr int kDeltaSlots = 1024;  // Delta of one transition for a chunk of goals x all controls
                                   // (8 KiB: the update fits beside the rollout blocks of a busy CU)

struct BeliefShared {
  double dl[kDeltaSlots];
  double red[kBeliefThreads / 64];
};

// Control recovered from one observed transition (the nearest control):
// heading k* = argmax_k <dz, (cos, sin)theta_k> with the lowest k on ties, then
// the speed whose step v_s dt is nearest to that projection (lowest s on
// ties); returns u* = s* K + k*, or -1 when the displacement is below 1e-9 m.
__device__ __forceinline__ int recover_control(const BeliefModel& m, float dx, float dy) {
  if (fmaf(dx, dx, dy * dy) < 1e-18f) return -1;
  int ks = 0;
  float best = -INFINITY;
  for (int k = 0; k < m.K; ++k) {
    const float v = fmaf(dx, m.cth[k], dy * m.sth[k]);
    if (v > best) {
      best = v;
      ks = k;
    }
  }
  int ss = 0;
  float err = INFINITY;
  for (int s = 0; s < m.S; ++s) {
    const float e = fabsf(m.vdt[s] - best);
    if (e < err) {
      err = e;
      ss = s;
    }
  }
  return ss * m.K + ks;
}

// log pi(u* | z; beta_b, g) for every b over the U controls in plain FP32 (the
// trajectory log-likelihood's terms: its bar is relative to |LL|, a sum of
// hundreds of terms, so FP32 logits meet it; the posterior update uses the
// compensated policy_delta and policy_term_from below).
// Delta_u = |a + s_u| - |a| with a = z - g carried as an unevaluated sum
// (hi + lo, exact subtraction), from the cancellation-free quotient
// (2 a.s_u + |s_u|^2) / (|a + s_u| + |a|); then l_u = -beta Delta_u and
// log pi = l_{u*} - max l - log sum exp(l - max l).  NMAX bounds U.
// exp(x) for the policy's shifted logits (x <= 0) through the hardware base-2
// exponential: one multiply by log2(e) and V_EXP_F32.  Relative error below
// 2e-7 + |x| 6e-8, against 1e-5 for the posterior and log-likelihood bars.
__device__ __forceinline__ float exp_nonpos(float x) { return fast_exp2(x * kLog2e); }

// Hardware base-2 logarithm (within 1 ulp for the normal arguments it gets
// here: sums of K weights whose largest is 1).
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
constexpr float kLn2 = 0.6931471805599453f;

template <int NMAX>
__device__ __forceinline__ void policy_terms(const BeliefModel& m, float zx, float zy, int ks,
                                             float gx, float gy, const float* beta, int B,
                                             float* out) {
  if (ks < 0) {
    for (int b = 0; b < B; ++b) out[b] = 0.f;
    return;
  }
  const int U = m.U;
  const float ax = zx - gx, bx = ax - zx;
  const float ax_lo = (zx - (ax - bx)) + (-gx - bx);
  const float ay = zy - gy, by = ay - zy;
  const float ay_lo = (zy - (ay - by)) + (-gy - by);
  const float D2 = fmaf(ax, ax, ay * ay);
  const float D = sqrtf(D2);
  const float ax2 = ax + ax, ay2 = ay + ay;
  float dl[NMAX];
  float dmin = INFINITY;
  for (int k = 0; k < U; ++k) {
    const float corr = fmaf(2.f * ax_lo, m.sx[k], fmaf(2.f * ay_lo, m.sy[k], m.s2[k]));
    const float n = fmaf(ax2, m.sx[k], fmaf(ay2, m.sy[k], corr));
    const float d = sqrtf(fmaxf(D2 + n, 0.f));
    dl[k] = n / (d + D);
    dmin = fminf(dmin, dl[k]);
  }
  for (int b = 0; b < B; ++b) {
    const float nbt = -beta[b];
    // max_k (nbt dl_k) for nbt <= 0: the rounded product is monotone in dl_k
    const float mx = nbt * dmin;
    float s = 0.f;
    for (int k = 0; k < U; ++k) s += exp_nonpos(nbt * dl[k] - mx);
    out[b] = (nbt * dl[ks] - mx) - logf(s);
  }
}

// policy_terms for a model of exactly KT controls (KT > 0), for the batched
// log-likelihood: the loops over the controls are unrolled (the KT distance
// chains are independent, which the runtime-length loops above hide from the
// scheduler), the chosen control's Delta is picked by a select in the loop
// instead of a dynamic index, and the distances take the hardware square root
// and reciprocal (within 1 ulp) in place of the IEEE ones: the log-likelihood's
// error bar is 1e-5 of its magnitude, not the posterior's absolute 1e-5.
template <int KT>
__device__ __forceinline__ void policy_terms_fixed(const BeliefModel& m, float zx, float zy,
                                                   int ks, float gx, float gy,
                                                   const float* beta, int B, float* out) {
  if (ks < 0) {
    for (int b = 0; b < B; ++b) out[b] = 0.f;
    return;
  }
  const float ax = zx - gx, bx = ax - zx;
  const float ax_lo = (zx - (ax - bx)) + (-gx - bx);
  const float ay = zy - gy, by = ay - zy;
  const float ay_lo = (zy - (ay - by)) + (-gy - by);
  const float D2 = fmaf(ax, ax, ay * ay);
  const float D = fast_sqrt(D2);
  const float ax2 = ax + ax, ay2 = ay + ay;
  float dl[KT];
  float dmin = INFINITY, dks = 0.f;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const float corr = fmaf(2.f * ax_lo, m.sx[k], fmaf(2.f * ay_lo, m.sy[k], m.s2[k]));
    const float n = fmaf(ax2, m.sx[k], fmaf(ay2, m.sy[k], corr));
    const float d = fast_sqrt(fmaxf(D2 + n, 0.f));
    dl[k] = n * fast_rcp(d + D);
    dmin = fminf(dmin, dl[k]);
    dks = k == ks ? dl[k] : dks;
  }
  // logits in base 2: a_k = -beta log2(e) Delta_k - c with the shift c = -beta
  // log2(e) min_k Delta_k (rounded), so pi_k = 2^a_k / sum_j 2^a_j for any c
  // and the term is (a_k* - log2 sum_j 2^a_j) ln 2; each exponent is one FMA
  for (int b = 0; b < B; ++b) {
    const float nb2 = -beta[b] * kLog2e;
    const float mx2 = nb2 * dmin;
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < KT; ++k) s += fast_exp2(fmaf(nb2, dl[k], -mx2));
    out[b] = (fmaf(nb2, dks, -mx2) - fast_log2(s)) * kLn2;
  }
}

// Delta_u = |a + s_u| - |a| for a = z - g, the distance change of control u
// that the policy's logits -beta Delta_u are built from (the shift-invariant
// form of beta Q).  The posterior multiplies up to thousands of these terms
// into a log that must stay within 1e-5 of the exact one, and a logit's
// rounding error scales with beta |s| (about 15 at beta = 100 and a 0.15 m
// step): plain FP32 Delta errs by a few 1e-6 per transition.  So Delta is
// evaluated in compensated FP32 (hi + lo pairs, about 46 bits): a = z - g
// exactly, |a|^2, n_u = 2 a.s_u + |s_u|^2 and the cancellation-free quotient
// n_u / (|a + s_u| + |a|), rounded once to FP64, where the rest of the term
// (the product with beta and the log-sum-exp over the controls) runs.
struct GoalOffset {
  dfl ax, ay, D2, D;
};

__device__ __forceinline__ GoalOffset goal_offset(float zx, float zy, float gx, float gy) {
  GoalOffset o;
  o.ax = two_sum(zx, -gx);
  o.ay = two_sum(zy, -gy);
  o.D2 = df_add(df_mul(o.ax, o.ax), df_mul(o.ay, o.ay));
  o.D = df_sqrt(o.D2);
  return o;
}

__device__ __forceinline__ double policy_delta(const GoalOffset& o, float sx, float sy) {
  const dfl s2 = df_add(two_prod(sx, sx), two_prod(sy, sy));
  const dfl dot = df_add(df_mul_f(o.ax, sx), df_mul_f(o.ay, sy));
  const dfl n = df_add(dfl{2.f * dot.hi, 2.f * dot.lo}, s2);
  const dfl d = df_sqrt(df_add(o.D2, n));
  return df_to_double(df_div(n, df_add(d, o.D)));
}

// log pi(u* | z; beta, g) from the U values -Delta_u: l_u = -beta Delta_u and
// log pi = (l_{u*} - max l) - log sum exp(l - max l), FP64, one pass with a
// running maximum.
__device__ __forceinline__ double policy_term_from(const double* dl, int U, int ks, double beta) {
  double mx = -INFINITY, s = 0.0, lks = 0.0;
  for (int u = 0; u < U; ++u) {
    const double l = -beta * dl[u];
    if (u == ks) lks = l;
    if (l > mx) {
      s = s * exp(mx - l) + 1.0;
      mx = l;
    } else {
      s += exp(l - mx);
    }
  }
  return (lks - mx) - log(s);
}

__device__ __forceinline__ double block_reduce(double v, bool is_max, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double x = __shfl_xor(v, o, 64);
    v = is_max ? fmax(v, x) : v + x;
  }
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < nw; ++w) r = is_max ? fmax(r, red[w]) : r + red[w];
  return r;
}

// One human's update: log_belief[j] += sum_t ell_t(j), renormalised by one
// FP64 log-sum-exp.  Per transition and chunk of goals, the threads first
// evaluate every (goal, control) Delta once into LDS, then every (goal, beta)
// term from them; thread tid owns pairs j = tid + r blockDim.x and adds their
// terms in transition order, so all sums run in a fixed order (bitwise
// reproducible).
__device__ void belief_update_block(const BeliefModel& m, const float* __restrict__ obs,
                                    int n_obs, double* __restrict__ log_belief,
                                    double* __restrict__ belief_out, BeliefShared& sh) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int G = m.G, B = m.B, U = m.U, J = G * B;
  const int gchunk = max(1, kDeltaSlots / U);
  constexpr int kPerThread = CAP_MAX_J / kBeliefThreads;
  double acc[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) acc[r] = 0.0;
  for (int t = 0; t < n_obs; ++t) {
    const float zx = obs[2 * t], zy = obs[2 * t + 1];
    const int ks = recover_control(m, obs[2 * t + 2] - zx, obs[2 * t + 3] - zy);
    if (ks < 0) continue;  // no displacement: no information (uniform across the block)
    for (int g0 = 0; g0 < G; g0 += gchunk) {
      const int gn = min(gchunk, G - g0);
      for (int item = tid; item < gn * U; item += nthr) {
        const int gl = item / U, u = item - gl * U;
        const GoalOffset o = goal_offset(zx, zy, m.gx[g0 + gl], m.gy[g0 + gl]);
        sh.dl[item] = policy_delta(o, m.sx[u], m.sy[u]);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kPerThread; ++r) {
        const int j = tid + r * nthr, g = j / B;
        if (j < J && g >= g0 && g < g0 + gn)
          acc[r] += policy_term_from(sh.dl + (g - g0) * U, U, ks, (double)m.beta[j - g * B]);
      }
      __syncthreads();
    }
  }
  double v[kPerThread];
  double mx = -INFINITY;
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int j = tid + r * nthr;
    v[r] = j < J ? log_belief[j] + acc[r] : -INFINITY;
    mx = fmax(mx, v[r]);
  }
  mx = block_reduce(mx, true, sh.red);
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int j = tid + r * nthr;
    if (j < J) s += exp(v[r] - mx);
  }
  s = block_reduce(s, false, sh.red);
  const double lse = mx + log(s);
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int j = tid + r * nthr;
    if (j < J) {
      const double lb = v[r] - lse;
      log_belief[j] = lb;
      if (belief_out) belief_out[j] = exp(lb);
    }
  }
}

}  // namespace capred

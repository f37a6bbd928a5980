// common.hpp -- internal definitions shared by the libcapred translation units:
// error reporting, host-side model tables, and the device building blocks of
// the rollout (counter-based Philox, Boltzmann heading choice).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/capred.h"

namespace capred {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
cap_status fail(cap_status code, const std::string& msg);
cap_status hip_fail(hipError_t e, const char* what);

#define CAP_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr double kPi = 3.14159265358979323846;
constexpr int kLatticeShift = 16;          // q = cell / 2^16
constexpr double kLatticeScale = 65536.0;
constexpr float kLog2e = 1.4426950408889634f;

// Largest beta * step length (metres) for which exp2 of the unshifted logits
// cannot overflow in FP32 (sum of up to 32 terms of 2^(80 log2 e)).
constexpr double kNoShiftLimit = 80.0;

// ---------------------------------------------------------------- host lattice
// Lattice pitch and rounding of metres to lattice units (round half to even).
// Written without FP contraction so that every host computes identical bits.
inline double lattice_pitch(double cell) { return cell / kLatticeScale; }

inline double lattice_coord(double z, double origin, double cell) {
#pragma clang fp contract(off)
  return std::nearbyint((z - origin) / lattice_pitch(cell));
}

inline double heading_angle(int k, int K) {
#pragma clang fp contract(off)
  return 2.0 * kPi * (double)k / (double)K;
}

// Lattice step of heading k: rint(v dt cos(theta_k) / q), rint(v dt sin(theta_k) / q).
inline void lattice_step(int k, int K, double speed, double dt, double cell, int32_t* sx,
                         int32_t* sy) {
#pragma clang fp contract(off)
  const double L = speed * dt;
  const double q = lattice_pitch(cell);
  const double th = heading_angle(k, K);
  *sx = (int32_t)std::nearbyint(L * std::cos(th) / q);
  *sy = (int32_t)std::nearbyint(L * std::sin(th) / q);
}

// Continuous step of heading k in metres, rounded to FP32.
inline void continuous_step(int k, int K, double speed, double dt, float* sx, float* sy) {
#pragma clang fp contract(off)
  const double L = speed * dt;
  const double th = heading_angle(k, K);
  *sx = (float)(L * std::cos(th));
  *sy = (float)(L * std::sin(th));
}

// ---------------------------------------------------------------- device
// Three-input exclusive or in one gfx950 V_BITOP3_B32 (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon et al., SC'11): per round two 32x32->64-bit products of
// counter words 0 and 2, recombined with words 1 and 3 and the round key; the
// key advances by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one v_mad_u64_u32 per product gives both halves
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// u = (2 (w >> 9) + 1) 2^-24: 24 significant bits, exact in FP32 and FP64.
// In FP32 as two instructions: one funnel shift places w >> 9 in the mantissa
// of 1.0 (x = 1 + (w >> 9) 2^-23), then x - (1 - 2^-24), exact by Sterbenz's
// lemma (x and 1 - 2^-24 are within a factor of two).
__device__ __forceinline__ float uniform24f(uint32_t w) {
  const uint32_t x = __builtin_amdgcn_alignbit(0x7Fu, w, 9u);  // 0x3F800000 | (w >> 9)
  return __uint_as_float(x) - 0x1.fffffep-1f;
}
__device__ __forceinline__ double uniform24d(uint32_t w) {
  return (double)((w >> 9) * 2u + 1u) * 5.9604644775390625e-8;
}

// Global-memory (address space 1) view of a generic pointer.  Pointers that a
// kernel loads from descriptor tables in device memory are generic to the
// compiler, which then emits FLAT accesses; a FLAT access also counts on the
// LDS wait counter, so every later LDS wait (each barrier, each LDS atomic
// whose result is used) would wait for its round trip to memory.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ global_ptr<T> as_global(T* p) {
  return (global_ptr<T>)p;
}

// Relaxed device-scope integer add through the global path (no return value).
__device__ __forceinline__ void global_add(uint32_t* p, uint32_t v) {
  __hip_atomic_fetch_add(as_global(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Per-model control constants for the lattice rollout, in lattice units:
// step (fx, fy) of control u = s K + k (integers, exact in FP32) and its
// squared length s2 (FP32).
struct HeadingTable {
  float fx[CAP_MAX_U];
  float fy[CAP_MAX_U];
  float s2[CAP_MAX_U];
};

// Inverse CDF over K non-decreasing prefix sums: #{k < K-1 : C_k <= thr},
// which equals min{k : thr < C_k} (capped at K-1).  For K a power of two the
// count is found by a branchless binary search whose register selections are
// explicit conditional moves (per-lane dynamic indexing of registers would
// spill to scratch); otherwise by counting.
template <int KT>
__device__ __forceinline__ int cdf_index(const float* C, float thr, int Krt) {
  constexpr bool kPow2 = KT >= 4 && (KT & (KT - 1)) == 0;
  if constexpr (kPow2) {
    // Level l probes C[c * (KT >> l) + (KT >> (l + 1)) - 1] where the bits
    // b_0..b_{l-1} decided so far spell c (b_0 most significant); the probe is
    // picked by a tree of 2^l - 1 conditional moves on those bits.
    constexpr int L = KT == 4 ? 2 : KT == 8 ? 3 : KT == 16 ? 4 : KT == 32 ? 5 : 6;
    bool b[L];
    int pos = 0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
      float v[KT / 2];
#pragma unroll
      for (int c = 0; c < (1 << l); ++c) v[c] = C[c * (KT >> l) + (KT >> (l + 1)) - 1];
#pragma unroll
      for (int st = l - 1; st >= 0; --st)
#pragma unroll
        for (int j = 0; j < (1 << st); ++j) v[j] = b[st] ? v[2 * j + 1] : v[2 * j];
      b[l] = v[0] <= thr;
      pos += b[l] ? (KT >> (l + 1)) : 0;
    }
    return pos;
  } else {
    constexpr int KM = KT > 0 ? KT : CAP_MAX_K;
    const int K = KT > 0 ? KT : Krt;
    int kk = 0;
#pragma unroll
    for (int k = 0; k < KM - 1; ++k) {
      if (KT == 0 && k >= K - 1) break;
      kk += (C[k] <= thr) ? 1 : 0;
    }
    return kk;
  }
}

// Boltzmann heading draw at lattice offset a = x - g (lattice units).  The
// logit of heading k is beta (|a| - |a + s_k|) (shift-invariant form of
// beta Q_k); it is computed from the cancellation-free difference
//   Delta_k = |a + s_k| - |a| = n_k / (|a + s_k| + |a|),  n_k = 2 a.s_k + |s_k|^2,
// whose absolute error stays a few ulp of the step length however far the
// goal is.  With nb = -beta q log2(e) and ib = 1/nb (both per particle), the
// base-2 exponent nb Delta_k is n_k / (|a + s_k| ib + |a| ib): one FMA, one
// reciprocal and one multiply.  |a + s_k|^2 = |a|^2 + n_k is taken through
// |.| (a free source modifier) against rounding below zero at the goal.
// Weights w_k = exp2(exponent) (optionally shifted by the largest exponent),
// prefix sums C_k, heading = cdf_index(C, u C_{K-1}).
//
// For KT > 0 the step table is point-symmetric (s_{k+KT/2} = -s_k, checked on
// the host), so one dot product 2 a.s_k serves both opposite headings:
// n_{k} = |s_k|^2 + 2 a.s_k and n_{k+KT/2} = |s_k|^2 - 2 a.s_k.  KT == 0 is the
// general table with a run-time K.
//
// SHIFT (a compile-time variant, used when beta * step is large enough for
// exp2 to overflow) subtracts the largest exponent before exponentiating.
//
// draw_headings: M particles' draws in one pass (KT > 0): the operations of each particle
// are the same and in the same order for every M, so its heading is the same
// bit for bit; with M = 2 the two particles' heading terms stand side by side,
// which gives the scheduler two independent sqrt -> rcp -> exp2 chains.
template <int KT, bool SHIFT, int M>
__device__ __forceinline__ void draw_headings(const float* ax, const float* ay, const float* ib,
                                              const float* u, const HeadingTable& T, int* k_out) {
  static_assert(KT > 0 && KT % 2 == 0, "needs a compile-time, point-symmetric table");
  constexpr int KH = KT / 2;
  float D2[M], Dib[M], ax2[M], ay2[M], acc[M];
  float C[M][KT];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    D2[m] = fmaf(ax[m], ax[m], ay[m] * ay[m]);
    Dib[m] = fast_sqrt(D2[m]) * ib[m];
    ax2[m] = ax[m] + ax[m];
    ay2[m] = ay[m] + ay[m];
  }
  // exponents of both halves, then the prefix sum in heading order
#pragma unroll
  for (int k = 0; k < KH; ++k) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const float dot = fmaf(ax2[m], T.fx[k], ay2[m] * T.fy[k]);
      const float np = T.s2[k] + dot, nm = T.s2[k] - dot;
      const float dp = fast_sqrt(fabsf(D2[m] + np)), dm = fast_sqrt(fabsf(D2[m] + nm));
      C[m][k] = np * fast_rcp(fmaf(dp, ib[m], Dib[m]));
      C[m][k + KH] = nm * fast_rcp(fmaf(dm, ib[m], Dib[m]));
    }
  }
  if constexpr (SHIFT) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
      float mx = C[m][0];
#pragma unroll
      for (int k = 1; k < KT; ++k) mx = fmaxf(mx, C[m][k]);
#pragma unroll
      for (int k = 0; k < KT; ++k) C[m][k] -= mx;
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    acc[m] = fast_exp2(C[m][0]);
    C[m][0] = acc[m];
  }
#pragma unroll
  for (int k = 1; k < KT; ++k)
#pragma unroll
    for (int m = 0; m < M; ++m) {
      acc[m] += fast_exp2(C[m][k]);
      C[m][k] = acc[m];
    }
#pragma unroll
  for (int m = 0; m < M; ++m) k_out[m] = cdf_index<KT>(C[m], u[m] * acc[m], KT);
}

template <int KT, bool SHIFT>
__device__ __forceinline__ int draw_heading(float ax, float ay, float ib, float u,
                                            const HeadingTable& T, int Krt) {
  if constexpr (KT > 0) {
    int k;
    draw_headings<KT, SHIFT, 1>(&ax, &ay, &ib, &u, T, &k);
    return k;
  } else {
    const float D2 = fmaf(ax, ax, ay * ay);
    const float D = fast_sqrt(D2);
    const float Dib = D * ib;
    const float ax2 = ax + ax, ay2 = ay + ay;
    float C[CAP_MAX_K];
    float acc = 0.f;
    float m = -INFINITY;
#pragma unroll
    for (int k = 0; k < CAP_MAX_K; ++k) {
      if (k >= Krt) break;
      const float n = fmaf(ax2, T.fx[k], fmaf(ay2, T.fy[k], T.s2[k]));
      const float d = fast_sqrt(fabsf(D2 + n));
      C[k] = n * fast_rcp(fmaf(d, ib, Dib));
      if constexpr (SHIFT) m = fmaxf(m, C[k]);
    }
#pragma unroll
    for (int k = 0; k < CAP_MAX_K; ++k) {
      if (k >= Krt) break;
      acc += fast_exp2(SHIFT ? C[k] - m : C[k]);
      C[k] = acc;
    }
    return cdf_index<KT>(C, u * acc, Krt);
  }
}

// Multi-speed draw: the inverse CDF over all U = S KT controls (u = s KT + k,
// prefix sums in u order) in two passes.  Pass 1 accumulates the weights of
// every allowed speed block in u order and keeps the running sum at the end of
// each block; the speed block s* = min{s : x < sum_s} (x = u C_{U-1}, capped at
// the last allowed speed) follows from those S sums.  Pass 2 recomputes block
// s* from the same constants (LDS copy `ctl`, per-lane index) starting from the
// sum before it, so its prefix sums are bit-identical to the flat sequence,
// and the heading is cdf_index over them.  Blocks of masked speeds add nothing
// (weight 0, Q = -inf).  Requires a point-symmetric table per speed.
template <int KT, bool SHIFT>
__device__ __forceinline__ int draw_control(float ax, float ay, float ib, float u,
                                            const HeadingTable& T, int S, uint32_t smask,
                                            int s_last, const float4* ctl) {
  static_assert(KT >= 4 && (KT & (KT - 1)) == 0, "multi-speed draw needs a power-of-two K");
  constexpr int KH = KT / 2;
  const float D2 = fmaf(ax, ax, ay * ay);
  const float D = fast_sqrt(D2);
  const float Dib = D * ib;
  const float ax2 = ax + ax, ay2 = ay + ay;
  float m = 0.f;
  if constexpr (SHIFT) {
    m = -INFINITY;
#pragma unroll
    for (int s = 0; s < CAP_MAX_S; ++s) {
      if (s >= S) break;
      if (!((smask >> s) & 1u)) continue;
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int c = s * KT + k;
        const float dot = fmaf(ax2, T.fx[c], ay2 * T.fy[c]);
        const float np = T.s2[c] + dot, nm = T.s2[c] - dot;
        const float dp = fast_sqrt(fabsf(D2 + np)), dm = fast_sqrt(fabsf(D2 + nm));
        m = fmaxf(m, fmaxf(np * fast_rcp(fmaf(dp, ib, Dib)), nm * fast_rcp(fmaf(dm, ib, Dib))));
      }
    }
  }
  float bs[CAP_MAX_S];
  float acc = 0.f;
#pragma unroll
  for (int s = 0; s < CAP_MAX_S; ++s) {
    if (s < S && ((smask >> s) & 1u)) {
      float e[KT];
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int c = s * KT + k;
        const float dot = fmaf(ax2, T.fx[c], ay2 * T.fy[c]);
        const float np = T.s2[c] + dot, nm = T.s2[c] - dot;
        const float dp = fast_sqrt(fabsf(D2 + np)), dm = fast_sqrt(fabsf(D2 + nm));
        e[k] = np * fast_rcp(fmaf(dp, ib, Dib));
        e[k + KH] = nm * fast_rcp(fmaf(dm, ib, Dib));
      }
#pragma unroll
      for (int k = 0; k < KT; ++k) acc += fast_exp2(SHIFT ? e[k] - m : e[k]);
    }
    bs[s] = acc;
  }
  const float thr = u * acc;
  int ss = 0;
#pragma unroll
  for (int s = 0; s < CAP_MAX_S - 1; ++s) ss += (s < s_last && bs[s] <= thr) ? 1 : 0;
  float base = 0.f;
#pragma unroll
  for (int s = 0; s < CAP_MAX_S - 1; ++s) base = (s == ss - 1) ? bs[s] : base;
  float C[KT];
  const float4* cb = ctl + ss * KT;
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const float4 c = cb[k];
    const float dot = fmaf(ax2, c.x, ay2 * c.y);
    const float np = c.z + dot, nm = c.z - dot;
    const float dp = fast_sqrt(fabsf(D2 + np)), dm = fast_sqrt(fabsf(D2 + nm));
    C[k] = np * fast_rcp(fmaf(dp, ib, Dib));
    C[k + KH] = nm * fast_rcp(fmaf(dm, ib, Dib));
  }
  float a2 = base;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    a2 += fast_exp2(SHIFT ? C[k] - m : C[k]);
    C[k] = a2;
  }
  return ss * KT + cdf_index<KT>(C, thr, KT);
}

}  // namespace capred

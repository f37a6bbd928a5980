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
// Philox4x32-10 (Salmon et al., SC'11): per round two 32x32->64-bit products of
// counter words 0 and 2, recombined with words 1 and 3 and the round key; the
// key advances by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// u = (2 (w >> 9) + 1) 2^-24: 24 significant bits, exact in FP32 and FP64.
__device__ __forceinline__ float uniform24f(uint32_t w) {
  return (float)((w >> 9) * 2u + 1u) * 5.9604644775390625e-8f;
}
__device__ __forceinline__ double uniform24d(uint32_t w) {
  return (double)((w >> 9) * 2u + 1u) * 5.9604644775390625e-8;
}

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Per-model heading constants for the lattice rollout, in lattice units:
// step (fx, fy) and its squared length s2 (all FP32).
struct HeadingTable {
  float fx[CAP_MAX_K];
  float fy[CAP_MAX_K];
  float s2[CAP_MAX_K];
};

// Boltzmann heading draw at lattice offset a = x - g (lattice units) with
// nb = -beta q log2(e).  The logit of heading k is beta (d_0 - d_k) up to a
// constant; it is computed from the cancellation-free difference
//   Delta_k = |a + s_k| - |a| = (2 a.s_k + |s_k|^2) / (|a + s_k| + |a|),
// so its absolute error stays a few ulp of the step length however far the
// goal is.  Weights w_k = exp2(nb Delta_k) (optionally shifted by the largest
// exponent), prefix sums C_k, and k = #{k < K-1 : C_k <= u C_{K-1}}, which is
// min{k : u C_{K-1} < C_k} because C is non-decreasing.
template <int KT>
__device__ __forceinline__ int draw_heading(float ax, float ay, float nb, float u, bool shift,
                                            const HeadingTable& T, int Krt) {
  constexpr int KM = KT > 0 ? KT : CAP_MAX_K;
  const int K = KT > 0 ? KT : Krt;
  const float D2 = fmaf(ax, ax, ay * ay);
  const float D = fast_sqrt(D2);
  const float ax2 = ax + ax, ay2 = ay + ay;
  float C[KM];
  float acc = 0.f;
  if (!shift) {
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      if (KT == 0 && k >= K) break;
      const float n = fmaf(ax2, T.fx[k], fmaf(ay2, T.fy[k], T.s2[k]));
      const float d = fast_sqrt(fmaxf(D2 + n, 0.f));
      const float l = n * fast_rcp(d + D);
      acc += fast_exp2(nb * l);
      C[k] = acc;
    }
  } else {
    float m = -INFINITY;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      if (KT == 0 && k >= K) break;
      const float n = fmaf(ax2, T.fx[k], fmaf(ay2, T.fy[k], T.s2[k]));
      const float d = fast_sqrt(fmaxf(D2 + n, 0.f));
      C[k] = nb * (n * fast_rcp(d + D));
      m = fmaxf(m, C[k]);
    }
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      if (KT == 0 && k >= K) break;
      acc += fast_exp2(C[k] - m);
      C[k] = acc;
    }
  }
  const float thr = u * acc;
  int kk = 0;
#pragma unroll
  for (int k = 0; k < KM - 1; ++k) {
    if (KT == 0 && k >= K - 1) break;
    kk += (C[k] <= thr) ? 1 : 0;
  }
  return kk;
}

}  // namespace capred

// dfloat.hpp -- compensated FP32 arithmetic: a value is the unevaluated sum
// hi + lo of two floats with |lo| <= ulp(hi) / 2 (about 48 significant bits).
// Built from the error-free transformations of Knuth (two-sum), Dekker
// (fast two-sum) and the FMA product residual; division and square root take
// one FP32 estimate and correct it with the exact residual.  Relative error
// of each operation is a few 2^-48, against 2^-24 for plain FP32.
#pragma once

#include <hip/hip_runtime.h>

namespace capred {

struct dfl {
  float hi, lo;
};

// a + b exactly, any magnitudes.
__device__ __forceinline__ dfl two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return dfl{s, (a - (s - bb)) + (b - bb)};
}

// a + b exactly when |a| >= |b| (or a == 0).
__device__ __forceinline__ dfl fast_two_sum(float a, float b) {
  const float s = a + b;
  return dfl{s, b - (s - a)};
}

// a * b exactly: the rounded product and its FMA residual.
__device__ __forceinline__ dfl two_prod(float a, float b) {
  const float p = a * b;
  return dfl{p, fmaf(a, b, -p)};
}

__device__ __forceinline__ dfl df_add(dfl x, dfl y) {
  dfl s = two_sum(x.hi, y.hi);
  const dfl t = two_sum(x.lo, y.lo);
  s = fast_two_sum(s.hi, s.lo + t.hi);
  return fast_two_sum(s.hi, s.lo + t.lo);
}

__device__ __forceinline__ dfl df_neg(dfl x) { return dfl{-x.hi, -x.lo}; }

__device__ __forceinline__ dfl df_mul_f(dfl x, float b) {
  const dfl p = two_prod(x.hi, b);
  return fast_two_sum(p.hi, fmaf(x.lo, b, p.lo));
}

__device__ __forceinline__ dfl df_mul(dfl x, dfl y) {
  const dfl p = two_prod(x.hi, y.hi);
  return fast_two_sum(p.hi, fmaf(x.hi, y.lo, fmaf(x.lo, y.hi, p.lo)));
}

// x / y for y != 0: the hardware reciprocal estimate of 1/y.hi (within 1 ulp)
// gives q1 = x.hi / y.hi to 2^-22; two corrections with the residuals
// x - q y evaluated in hi + lo arithmetic shrink the error to about 2^-46.
__device__ __forceinline__ dfl df_div(dfl x, dfl y) {
  const float ry = __builtin_amdgcn_rcpf(y.hi);
  const float q1 = x.hi * ry;
  const dfl r = df_add(x, df_neg(df_mul_f(y, q1)));
  const float q2 = r.hi * ry;
  const dfl r2 = df_add(r, df_neg(df_mul_f(y, q2)));
  const float q3 = r2.hi * ry;
  const dfl q = fast_two_sum(q1, q2);
  return df_add(q, dfl{q3, 0.f});
}

// sqrt(x) for x >= 0 (negative inputs, from rounding at zero, give 0): the
// hardware root s (within 1 ulp) corrected by (x - s^2) / (2 s) with x - s^2
// evaluated exactly (one Newton step: error about 2^-45 relative).
__device__ __forceinline__ dfl df_sqrt(dfl x) {
  if (!(x.hi > 0.f)) return dfl{0.f, 0.f};
  const float s = __builtin_amdgcn_sqrtf(x.hi);
  const dfl r = df_add(x, df_neg(two_prod(s, s)));
  return fast_two_sum(s, r.hi * (0.5f * __builtin_amdgcn_rcpf(s)));
}

// The value rounded once to double (relative error at most 2^-53).
__device__ __forceinline__ double df_to_double(dfl x) { return (double)x.hi + (double)x.lo; }

}  // namespace capred

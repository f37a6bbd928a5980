// smooth.hpp -- the Gaussian smoothing stage shared by the single-grid entry
// point and the batched plan: host-side kernel weights and the device routine
// that smooths one (band of rows x 256 columns) tile of one step's grid.
#pragma once

#include <vector>

#include "common.hpp"

namespace capred {

constexpr int kSmoothThreads = 256;   // output columns per tile (one per thread)
constexpr int kBandRows = 32;         // output rows per tile
constexpr int kMaxSmoothRadius = 16;  // LDS tile (kBandRows + 2r) x 256 floats <= 64 KiB

struct SmoothWeights {
  float w[2 * kMaxSmoothRadius + 1];
};

inline cap_status check_smoothing(double sigma, int radius, int max_radius) {
  if (radius < 0 || radius > max_radius)
    return fail(CAP_E_INVALID, "smoothing radius must be in [0, " + std::to_string(max_radius) + "]");
  if (radius > 0 && !(sigma > 0.0 && std::isfinite(sigma)))
    return fail(CAP_E_INVALID, "smoothing sigma must be finite and > 0");
  return CAP_OK;
}

// w[d + r] = fl32(exp(-d^2 / (2 sigma^2)) / sum_{|e| <= r} exp(-e^2 / (2 sigma^2))), FP64 then
// rounded once; r = 0 gives the single weight 1.
inline void smooth_weights(double sigma, int r, SmoothWeights* W) {
  std::vector<double> e(2 * r + 1);
  double Z = 0.0;
  for (int d = -r; d <= r; ++d) {
    e[d + r] = r == 0 ? 1.0 : std::exp(-(double)(d * d) / (2.0 * sigma * sigma));
    Z += e[d + r];
  }
  for (int i = 0; i < 2 * kMaxSmoothRadius + 1; ++i) W->w[i] = i <= 2 * r ? (float)(e[i] / Z) : 0.f;
}

inline size_t smooth_lds_bytes(int r) {
  return (size_t)(kBandRows + 2 * r) * kSmoothThreads * sizeof(float);
}

// Smooths output rows [y0, y0 + kBandRows) x columns [x0, x0 + 256) of one
// step: c and o point at that step's [ny][nx] counts and probabilities.
// Pass 1 blurs rows y0 - r .. y0 + kBandRows + r - 1 along x from the uint32
// grid into the LDS tile (the 2r+1 shifted loads of a row share cache lines);
// pass 2 blurs the tile along y and writes row-coalesced.  Every thread of the
// block must call it (it contains a barrier); the caller separates two calls
// that reuse `tile` with another barrier.  un (nullable): that step's plane of
// a union grid of the same frame, raised to each nonzero output by an integer
// atomic max on the FP32 bits (exact for values >= 0).
__device__ __forceinline__ void smooth_block(const uint32_t* __restrict__ c,
                                             float* __restrict__ o, int ny, int nx, int r,
                                             float Nf, const float* __restrict__ w, int y0,
                                             int x0, float* tile, float* un = nullptr) {
  const int x = x0 + (int)threadIdx.x;
  const int rows = kBandRows + 2 * r;
  for (int i = 0; i < rows; ++i) {
    const int y = y0 - r + i;
    float h = 0.f;
    if (y >= 0 && y < ny && x < nx) {
      const uint32_t* __restrict__ row = c + (size_t)y * nx;
      for (int d = -r; d <= r; ++d) {
        const int sx = x - d;
        if (sx >= 0 && sx < nx) h = fmaf(w[d + r], (float)row[sx], h);
      }
    }
    tile[i * kSmoothThreads + threadIdx.x] = h;
  }
  __syncthreads();
  if (x < nx) {
    const int yend = min(kBandRows, ny - y0);
    for (int j = 0; j < yend; ++j) {
      float acc = 0.f;
      for (int d = -r; d <= r; ++d)
        acc = fmaf(w[d + r], tile[(j + r - d) * kSmoothThreads + threadIdx.x], acc);
      const float v = acc / Nf;
      o[(size_t)(y0 + j) * nx + x] = v;
      if (un && v > 0.f)
        __hip_atomic_fetch_max(reinterpret_cast<uint32_t*>(un) + (size_t)(y0 + j) * nx + x,
                               __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace capred

// smooth.hip -- Gaussian-smoothed occupancy (cap_smooth_occupancy) and the
// point-wise maximum union of several humans' grids (cap_union_max).
//
// Smoothing (Sec. III-B, the Gaussian convolution applied before emplacement):
// the histogram of step t is convolved with the separable discrete Gaussian
// w(dx) w(dy), w(d) = exp(-d^2 / (2 sigma^2)) / sum_{|e|<=r} exp(-e^2 / (2 sigma^2)),
// counts outside the grid being zero, and divided by N.  The separable form is
// the same kernel as the 2-D one over the square window (the 2-D Gaussian
// factorises and so does its normaliser).
//
// Layout on gfx950: one 256-thread block per (step, band of kBandRows output
// rows, 256 output columns).  Pass 1 blurs the band's rows plus r halo rows
// above and below along x straight from the uint32 grid (the 2r+1 shifted
// loads of one row hit the same cache lines, so HBM sees each count about
// (1 + 2r / kBandRows) times) into an LDS tile; pass 2 blurs the tile along y
// and writes FP32 probabilities row-coalesced.  The kernel is HBM-bound:
// 4 B read and 4 B written per cell.
#include <algorithm>
#include <vector>

#include "smooth.hpp"

namespace capred {

__global__ void __launch_bounds__(kSmoothThreads)
smooth_kernel(const uint32_t* __restrict__ counts, float* __restrict__ out, int ny, int nx,
              int r, float Nf, SmoothWeights W) {
  extern __shared__ float tile[];  // [kBandRows + 2r][kSmoothThreads]
  const size_t plane = (size_t)ny * nx;
  smooth_block(counts + (size_t)blockIdx.z * plane, out + (size_t)blockIdx.z * plane, ny, nx, r,
               Nf, W.w, (int)blockIdx.y * kBandRows, (int)blockIdx.x * kSmoothThreads, tile);
}

struct UnionPtrs {
  const float* g[CAP_MAX_SLOTS];
};

__global__ void __launch_bounds__(256) union_max_kernel(UnionPtrs P, int n_humans, size_t n,
                                                        float* out, bool vec) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t head = vec ? n / 4 : 0;
  for (size_t v = i0; v < head; v += stride) {
    float4 m = reinterpret_cast<const float4*>(P.g[0])[v];
    for (int h = 1; h < n_humans; ++h) {
      const float4 a = reinterpret_cast<const float4*>(P.g[h])[v];
      m.x = fmaxf(m.x, a.x);
      m.y = fmaxf(m.y, a.y);
      m.z = fmaxf(m.z, a.z);
      m.w = fmaxf(m.w, a.w);
    }
    reinterpret_cast<float4*>(out)[v] = m;
  }
  for (size_t v = head * 4 + i0; v < n; v += stride) {
    float m = P.g[0][v];
    for (int h = 1; h < n_humans; ++h) m = fmaxf(m, P.g[h][v]);
    out[v] = m;
  }
}

}  // namespace capred

using namespace capred;

extern "C" cap_status cap_smooth_occupancy(const uint32_t* counts_dev, int32_t H, int32_t ny,
                                           int32_t nx, int32_t N, double sigma, int32_t radius,
                                           float* probs_dev, void* stream) {
  if (H < 0 || ny < 1 || nx < 1 || N < 1)
    return fail(CAP_E_INVALID, "H >= 0, ny >= 1, nx >= 1 and N >= 1 required");
  cap_status st = check_smoothing(sigma, radius, kMaxSmoothRadius);
  if (st != CAP_OK) return st;
  if (ny > (1 << 20) || nx > (1 << 20)) return fail(CAP_E_INVALID, "grid side above 2^20");
  if (H == 0) return CAP_OK;
  if (H > 65535) return fail(CAP_E_INVALID, "H above 65535");
  if (!counts_dev || !probs_dev) return fail(CAP_E_INVALID, "counts or probs is NULL");
  if ((const void*)counts_dev == (const void*)probs_dev)
    return fail(CAP_E_INVALID, "probs must not alias counts");
  SmoothWeights W;
  smooth_weights(sigma, radius, &W);
  const dim3 grid((unsigned)((nx + kSmoothThreads - 1) / kSmoothThreads),
                  (unsigned)((ny + kBandRows - 1) / kBandRows), (unsigned)H);
  const size_t lds = smooth_lds_bytes(radius);
  hipLaunchKernelGGL(smooth_kernel, grid, dim3(kSmoothThreads), lds, as_stream(stream),
                     counts_dev, probs_dev, (int)ny, (int)nx, (int)radius, (float)N, W);
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

extern "C" cap_status cap_union_max(const float* const* grids, int32_t n_humans,
                                    int64_t n_cells, float* out_dev, void* stream) {
  if (n_humans < 1 || n_humans > CAP_MAX_SLOTS)
    return fail(CAP_E_INVALID, "n_humans must be in [1, 256]");
  if (n_cells < 0) return fail(CAP_E_INVALID, "n_cells must be >= 0");
  if (!grids || !out_dev) return fail(CAP_E_INVALID, "grids or out is NULL");
  UnionPtrs P{};
  uintptr_t align = reinterpret_cast<uintptr_t>(out_dev);
  for (int h = 0; h < n_humans; ++h) {
    if (!grids[h]) return fail(CAP_E_INVALID, "a grid pointer is NULL");
    P.g[h] = grids[h];
    align |= reinterpret_cast<uintptr_t>(grids[h]);
  }
  if (n_cells == 0) return CAP_OK;
  const size_t n = (size_t)n_cells;
  const size_t blocks = std::min<size_t>((n / 4 + 255) / 256 + 1, 8192);
  hipLaunchKernelGGL(union_max_kernel, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream),
                     P, (int)n_humans, n, out_dev, (align & 15u) == 0);
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

// probe.hip -- throughput probes for the roofline of the rollout: FP32 FMA,
// the three transcendentals of a heading evaluation (exp2, sqrt, rcp), the
// 32x32->64 multiply of Philox, LDS atomics, device-scope global atomics (the
// histogram flush), and a plain copy kernel whose known traffic calibrates
// the HBM byte counters.
#include <algorithm>

#include "common.hpp"

namespace capred {

constexpr int kProbeChains = 8;

template <int KIND>
__global__ void __launch_bounds__(256) probe_kernel(int64_t iters, float seed,
                                                    float* __restrict__ sink) {
  float x[kProbeChains], y[kProbeChains];
  uint32_t u[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) {
    x[c] = seed + 0.001f * (float)(threadIdx.x + 7 * c);
    y[c] = x[c] * 0.5f;
    u[c] = threadIdx.x * 2654435761u + c;
  }
  __shared__ uint32_t lds[4096];
  if (KIND == 5) {
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) lds[i] = 0u;
    __syncthreads();
  }
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) {
      if (KIND == 0) x[c] = fmaf(x[c], 0.999f, 1e-4f);
      if (KIND == 1) x[c] = fast_exp2(x[c] * -0.5f);
      if (KIND == 2) x[c] = fast_sqrt(x[c] + 0.25f);
      if (KIND == 3) x[c] = fast_rcp(x[c] + 1.5f);
      if (KIND == 4) {
        const uint64_t p = (uint64_t)u[c] * 0xD2511F53u;
        u[c] = (uint32_t)(p >> 32) ^ (uint32_t)p;
      }
      if (KIND == 6) {
        x[c] = fast_exp2(x[c] * -0.5f);
        y[c] = fmaf(y[c], 0.999f, 1e-4f);
        y[c] = fmaf(y[c], 0.999f, 1e-4f);
        y[c] = fmaf(y[c], 0.999f, 1e-4f);
      }
      if (KIND == 5) atomicAdd(&lds[(u[c] + (uint32_t)i * 97u + c * 509u) & 4095u], 1u);
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) acc += x[c] + y[c] + (float)u[c];
  if (KIND == 5) {
    __syncthreads();
    acc += (float)lds[threadIdx.x];
  }
  if (acc == 123.456f) sink[blockIdx.x] = acc;  // keeps the chains alive
}

// Relaxed device-scope adds without return, as the histogram flush issues
// them: every lane of every chain draws a fresh address from its own linear
// congruential sequence and adds 1 to that word of a 2^log2_words buffer (the
// top bits of the state; lanes of a wave land on different lines).
__global__ void __launch_bounds__(256) probe_global_atomic_kernel(int64_t iters,
                                                                  uint32_t* __restrict__ counts,
                                                                  uint32_t shift) {
  uint32_t u[kProbeChains];
  const uint32_t lane = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) u[c] = lane * 2654435761u + (uint32_t)c * 0x9E3779B9u;
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) {
      u[c] = u[c] * 1664525u + 1013904223u;
      global_add(counts + (u[c] >> shift), 1u);
    }
  }
}

__global__ void __launch_bounds__(256) copy_kernel(const uint4* __restrict__ a,
                                                   uint4* __restrict__ b, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) b[i] = a[i];
}

}  // namespace capred

using namespace capred;

extern "C" cap_status cap_probe(int32_t kind, int64_t iters, int32_t blocks, float* sink_dev,
                                void* stream) {
  if (kind < 0 || kind > 6 || iters < 1 || blocks < 1 || !sink_dev)
    return fail(CAP_E_INVALID, "probe: kind in [0,6], iters >= 1, blocks >= 1, sink required");
  hipStream_t s = as_stream(stream);
  const dim3 g((unsigned)blocks), b(256);
  switch (kind) {
    case 0: hipLaunchKernelGGL(probe_kernel<0>, g, b, 0, s, iters, 0.5f, sink_dev); break;
    case 1: hipLaunchKernelGGL(probe_kernel<1>, g, b, 0, s, iters, 0.5f, sink_dev); break;
    case 2: hipLaunchKernelGGL(probe_kernel<2>, g, b, 0, s, iters, 0.5f, sink_dev); break;
    case 3: hipLaunchKernelGGL(probe_kernel<3>, g, b, 0, s, iters, 0.5f, sink_dev); break;
    case 4: hipLaunchKernelGGL(probe_kernel<4>, g, b, 0, s, iters, 0.5f, sink_dev); break;
    case 5: hipLaunchKernelGGL(probe_kernel<5>, g, b, 0, s, iters, 0.5f, sink_dev); break;
    default: hipLaunchKernelGGL(probe_kernel<6>, g, b, 0, s, iters, 0.5f, sink_dev); break;
  }
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

extern "C" cap_status cap_probe_global_atomic(int64_t iters, int32_t blocks, uint32_t* counts_dev,
                                               int32_t log2_words, void* stream) {
  if (iters < 1 || blocks < 1 || !counts_dev || log2_words < 6 || log2_words > 30)
    return fail(CAP_E_INVALID,
                "probe_global_atomic: iters >= 1, blocks >= 1, log2_words in [6,30], buffer required");
  hipLaunchKernelGGL(probe_global_atomic_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     as_stream(stream), iters, counts_dev, (uint32_t)(32 - log2_words));
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

extern "C" cap_status cap_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream) {
  if (!src_dev || !dst_dev || (bytes & 15u) ||
      ((reinterpret_cast<uintptr_t>(src_dev) | reinterpret_cast<uintptr_t>(dst_dev)) & 15u))
    return fail(CAP_E_INVALID, "copy: 16-byte aligned pointers and size required");
  const size_t n16 = bytes / 16;
  if (n16 == 0) return CAP_OK;
  const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 8192);
  hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, as_stream(stream),
                     static_cast<const uint4*>(src_dev), static_cast<uint4*>(dst_dev), n16);
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

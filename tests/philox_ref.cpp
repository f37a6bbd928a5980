// Thin C shim over PyTorch's header-only Philox4x32-10 engine, used as an
// independent library reference for the oracle's and the GPU's Philox.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>

extern "C" void ref_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                           uint32_t* out) {
  const uint64_t offset = static_cast<uint64_t>(c0) | (static_cast<uint64_t>(c1) << 32);
  const uint64_t subseq = static_cast<uint64_t>(c2) | (static_cast<uint64_t>(c3) << 32);
  at::philox_engine e(seed, subseq, offset);
  for (int i = 0; i < 4; ++i) out[i] = e();
}

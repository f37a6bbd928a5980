// belief.hip -- cap_belief_update and cap_belief_reset (single human).
#include "belief.hpp"

namespace capred {

__global__ void __launch_bounds__(kBeliefThreads)
    belief_update_kernel(const BeliefModel m, const float* __restrict__ obs, int n_obs,
                         double* __restrict__ log_belief, double* __restrict__ belief_out) {
  __shared__ BeliefShared sh;
  belief_update_block(m, obs, n_obs, log_belief, belief_out, sh);
}

__global__ void belief_reset_kernel(int J, double* __restrict__ log_belief) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < J) log_belief[j] = -log((double)J);
}

}  // namespace capred

using namespace capred;

extern "C" cap_status cap_belief_update(const cap_model* model, const float* obs_dev,
                                        int32_t n_obs, double* log_belief_dev,
                                        double* belief_dev, void* stream) {
  Controls c;
  cap_status st = check_model(model, &c);
  if (st != CAP_OK) return st;
  if (n_obs < 0) return fail(CAP_E_INVALID, "n_obs must be >= 0");
  if (!log_belief_dev) return fail(CAP_E_INVALID, "log_belief is NULL");
  if (n_obs > 0 && !obs_dev) return fail(CAP_E_INVALID, "obs is NULL");
  const BeliefModel m = make_belief_model(c, model->dt, model->B, model->beta, model->G,
                                          model->goals);
  hipLaunchKernelGGL(belief_update_kernel, dim3(1), dim3(kBeliefThreads), 0, as_stream(stream),
                     m, obs_dev, n_obs, log_belief_dev, belief_dev);
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

extern "C" cap_status cap_belief_reset(int32_t G, int32_t B, double* log_belief_dev,
                                       void* stream) {
  if (G < 1 || B < 1 || G > CAP_MAX_G || B > CAP_MAX_B || G * B > CAP_MAX_J)
    return fail(CAP_E_INVALID, "G, B out of range");
  if (!log_belief_dev) return fail(CAP_E_INVALID, "log_belief is NULL");
  hipLaunchKernelGGL(belief_reset_kernel, dim3(1), dim3(CAP_MAX_J), 0, as_stream(stream), G * B,
                     log_belief_dev);
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

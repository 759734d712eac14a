// optim.hip -- the optimisation protocol of Sec. 3.3 on top of the parameter
// gradient: Adam (Sec. 3.3.1), the learning-rate schedule (Sec. 3.3.2) and
// the dynamic loss weights (Sec. 3.3.3).
#include <cmath>

#include "model.hpp"

namespace nepmi {

// One Adam step on FP32 parameters, first and second moments:
//   m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2,
//   p <- p - (lr / c1) m / (sqrt(v) / sqrt(c2) + eps),  c1 = 1 - b1^t, c2 = 1 - b2^t.
// omb1 = 1 - b1 and omb2 = 1 - b2 come from the host in double precision
// (1 - 0.999f in float would be off by 1e-5 relative).
__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float b1, float omb1, float b2, float omb2, float step_size,
                       float inv_sqrt_c2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = fmaf(b1, m[i], omb1 * gi);
  const float vi = fmaf(b2, v[i], omb2 * gi * gi);
  m[i] = mi;
  v[i] = vi;
  p[i] -= step_size * mi / (sqrtf(vi) * inv_sqrt_c2 + eps);
}

}  // namespace nepmi

using namespace nepmi;

extern "C" {

int nepmi_adam_step(int64_t n, float* dev_params, const float* dev_grad, float* dev_m, float* dev_v, int64_t t,
                    double lr, double beta1, double beta2, double eps, void* stream) {
  if (n < 0 || (n > 0 && (!dev_params || !dev_grad || !dev_m || !dev_v)) || t < 1 || !(lr >= 0) ||
      !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0)) {
    set_error("invalid Adam arguments");
    return NEPMI_INVALID_ARG;
  }
  if (n == 0) return NEPMI_OK;
  const double c1 = 1.0 - std::pow(beta1, (double)t), c2 = 1.0 - std::pow(beta2, (double)t);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n, dev_params,
                     dev_grad, dev_m, dev_v, (float)beta1, (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2),
                     (float)(lr / c1), (float)(1.0 / std::sqrt(c2)), (float)eps);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

int nepmi_lr_schedule(int64_t step, int64_t warmup_steps, int64_t total_steps, double lr_start, double lr_end,
                      double start_factor, double* lr_out) {
  if (!lr_out || step < 0 || warmup_steps < 0 || total_steps < warmup_steps || !(lr_start > 0) || !(lr_end >= 0) ||
      !(start_factor > 0 && start_factor <= 1)) {
    set_error("invalid schedule arguments");
    return NEPMI_INVALID_ARG;
  }
  double lr;
  if (step < warmup_steps) {
    // linear warmup: factor start_factor -> 1 over warmup_steps
    lr = lr_start * (start_factor + (1.0 - start_factor) * (double)step / (double)warmup_steps);
  } else {
    // cosine annealing lr_start -> lr_end over the remaining steps
    const int64_t T = total_steps - warmup_steps;
    const double s = T > 0 ? (double)(step - warmup_steps < T ? step - warmup_steps : T) / (double)T : 1.0;
    lr = lr_end + 0.5 * (lr_start - lr_end) * (1.0 + std::cos(3.14159265358979323846 * s));
  }
  *lr_out = lr;
  return NEPMI_OK;
}

int nepmi_loss_weights(double lr, double lr_start, const double* w_start, const double* w_end, int32_t normalised,
                       double* w_out) {
  if (!w_start || !w_end || !w_out || !(lr >= 0) || (normalised && !(lr_start > 0))) {
    set_error("invalid loss-weight arguments");
    return NEPMI_INVALID_ARG;
  }
  const double x = normalised ? lr / lr_start : lr;
  for (int c = 0; c < 3; ++c) w_out[c] = w_start[c] * x + w_end[c] * (1.0 - x);
  return NEPMI_OK;
}

}  // extern "C"

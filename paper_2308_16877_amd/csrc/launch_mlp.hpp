// Launchers of the MLP surrogate kernels (mlp_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpac {

// MLP surrogate (parameters: one FP32 array, see mlp_kernels.hip).
struct MlpArgs {
  int64_t n;
  const float *in[5];
  float *out[2];
  const float *params;
  float in_center[5], in_scale[5], out_mean[2], out_scale[2];
  float out_shift[2];  // > 0: outputs are exp(v) - shift (the network models log(y + shift))
  float box_lo[5], box_hi[5];
  int32_t *queue;
  int32_t *queue_count;
};
struct MlpGradArgs {
  int64_t n;
  const float *x[5];
  const float *t[2];
  const float *params;
  float in_center[5], in_scale[5], out_mean[2], out_scale[2];
  float out_shift[2];  // > 0: targets are taken as log(t + shift)
  float inv_count;  // 1 / number of items the loss averages over
  float *grad_partials;
  float *loss_partials;
};
struct AdamArgs {
  const float *grad_partials;
  int64_t blocks;
  float *params, *m, *v;
  float lr, beta1, beta2, eps, bc1, bc2;
};
int mlp_num_params();
hipError_t launch_mlp_infer(const MlpArgs &a, hipStream_t stream);
hipError_t launch_mlp_grad(const MlpGradArgs &a, hipStream_t stream);
hipError_t launch_mlp_adam(const AdamArgs &a, hipStream_t stream);

}  // namespace hpac

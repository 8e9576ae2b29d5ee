// Launchers of the Greeks backward kernels (greeks_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpac {

// Greeks backward: grad_in[j] = gC * dC/dx_j + gP * dP/dx_j for the five
// inputs, from a saved Jacobian (10 columns) or recomputed from the inputs.
// gC or gP may be null (treated as zero).
struct VjpArgs {
  int64_t n;
  const float *jac[10];  // used by the saved-Jacobian kernel
  const float *in[5];    // used by the recomputing kernels
  const int32_t *src;    // used by the by-reference kernel: source item of each item
  const float *gC, *gP;
  float *gin[5];
};
hipError_t launch_bs_vjp(const VjpArgs &a, hipStream_t stream);
hipError_t launch_bs_adjoint(const VjpArgs &a, hipStream_t stream);
hipError_t launch_bs_vjp_ref(const VjpArgs &a, hipStream_t stream);

}  // namespace hpac

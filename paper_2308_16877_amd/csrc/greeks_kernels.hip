// Backward kernels for the Black-Scholes Greeks (vector-Jacobian products).
//
// The forward region HPAC_REGION_BS_PRICE_GRAD writes the prices and their
// Jacobian; under iACT a reused table entry carries its Jacobian too, so the
// backward pass contracts the saved Jacobian with the upstream gradients and
// reuses the memoized derivatives.  When nothing was memoized the backward
// can instead recompute the derivatives from the inputs (k_bs_adjoint),
// which moves 48 instead of 68 bytes per item.  Both contract with the same
// separately rounded products and sum, so on the same derivatives they agree
// bit for bit.
#include "launch_greeks.hpp"
#include "region_bs.hpp"

namespace hpac {

// gc * a + gp * b with both products and the sum rounded separately.
__device__ __forceinline__ float contract2(float gc, float a, float gp, float b) {
#pragma clang fp contract(off)
  return gc * a + gp * b;
}

__global__ void __launch_bounds__(256) k_bs_vjp(VjpArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    const float gc = a.gC ? a.gC[i] : 0.0f;
    const float gp = a.gP ? a.gP[i] : 0.0f;
#pragma unroll
    for (int j = 0; j < 5; ++j) a.gin[j][i] = contract2(gc, a.jac[j][i], gp, a.jac[5 + j][i]);
  }
}

__global__ void __launch_bounds__(256) k_bs_adjoint(VjpArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    const float gc = a.gC ? a.gC[i] : 0.0f;
    const float gp = a.gP ? a.gP[i] : 0.0f;
    const float x[5] = {a.in[0][i], a.in[1][i], a.in[2][i], a.in[3][i], a.in[4][i]};
    float y[RegionBSPriceGrad::kOut];
    RegionBSPriceGrad::eval(x, y);
#pragma unroll
    for (int j = 0; j < 5; ++j) a.gin[j][i] = contract2(gc, y[2 + j], gp, y[7 + j]);
  }
}

// Backward of the by-reference memo: item i's derivatives are those of its
// source item j = src[i] (itself where the forward computed, the stored
// entry's source where iACT reused one), recomputed from j's inputs with the
// forward's region, so they equal bit for bit the Jacobian the price-and-
// Jacobian region would have stored and reused.  An index outside [0, n)
// (a column not written by such a forward) gives NaN gradients and reads
// nothing.
__global__ void __launch_bounds__(256) k_bs_vjp_ref(VjpArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    const float gc = a.gC ? a.gC[i] : 0.0f;
    const float gp = a.gP ? a.gP[i] : 0.0f;
    const int64_t j = a.src[i];
    if (j < 0 || j >= a.n) {
#pragma unroll
      for (int k = 0; k < 5; ++k) a.gin[k][i] = __builtin_nanf("");
      continue;
    }
    const float x[5] = {a.in[0][j], a.in[1][j], a.in[2][j], a.in[3][j], a.in[4][j]};
    float y[RegionBSPriceGrad::kOut];
    RegionBSPriceGrad::eval(x, y);
#pragma unroll
    for (int k = 0; k < 5; ++k) a.gin[k][i] = contract2(gc, y[2 + k], gp, y[7 + k]);
  }
}

static dim3 grid_items(int64_t n) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1 << 20) blocks = 1 << 20;  // grid-stride beyond this
  return dim3((unsigned)(blocks < 1 ? 1 : blocks));
}

hipError_t launch_bs_vjp(const VjpArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(k_bs_vjp, grid_items(a.n), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_bs_vjp_ref(const VjpArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(k_bs_vjp_ref, grid_items(a.n), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_bs_adjoint(const VjpArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(k_bs_adjoint, grid_items(a.n), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace hpac

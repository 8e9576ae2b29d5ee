// Black-Scholes-Merton region bodies (FP32) for the approximation kernels.
// The paper's Black-Scholes benchmark prices a portfolio of European options
// analytically (section 4, Table 1); the whole price calculation is the
// approximated region.  Textbook formula, no dividends:
//   d1 = (ln(S/K) + (r + v^2/2) T) / (v sqrt T),  d2 = d1 - v sqrt T,
//   C = S N(d1) - K e^{-rT} N(d2),  P = K e^{-rT} N(-d2) - S N(-d1).
// N is evaluated through the tail probability Q(|d|) = 1 - Phi(|d|), so N(d)
// and N(-d) are both accurate in relative terms in the tails.
#pragma once
#include <hip/hip_runtime.h>

#include "io_types.hpp"
#include "tail_q_coeffs.hpp"

namespace hpac {

struct BSCore {
  float sqT, vs, d1, d2, disc, D;
  float Nd1, Nmd1, Nd2, Nmd2;
};

constexpr float kLog2e = 1.44269504088896341f;
constexpr float kLn2 = 0.693147180559945309f;
constexpr float kInvSqrt2Pi = 0.398942280401432678f;
// -log2(e)/2 split into a float and the float of its remainder
constexpr float kHalfL2eHi = -0.721347510814666748f;
constexpr float kHalfL2eLo = -9.62981495e-09f;

// Upper tail Q(z) = 1 - Phi(z) for z >= 0, relative error below 1e-6 where
// Q is an FP32 normal number: Q = phi(z) M(z).  The density's exponent
// -z^2/2 (in base 2) is carried to about twice FP32 precision, because its
// rounding error would otherwise be multiplied by z^2/2 in Q.  The Mills
// ratio M uses the fitted form of tail_q_coeffs.hpp.
__device__ __forceinline__ float tail_q(float z) {
  const float u = z * z;
  const float eu = __builtin_fmaf(z, z, -u);  // z^2 = u + eu exactly
  const float ah = u * kHalfL2eHi;
  const float al = __builtin_fmaf(u, kHalfL2eHi, -ah) + __builtin_fmaf(u, kHalfL2eLo, eu * kHalfL2eHi);
  const float phi = __builtin_amdgcn_exp2f(ah) * __builtin_fmaf(al, kLn2, 1.0f) * kInvSqrt2Pi;
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(kTailP, z, 1.0f));
  float m = kTailC[kTailK - 1];
#pragma unroll
  for (int k = kTailK - 2; k >= 0; --k) m = __builtin_fmaf(m, t, kTailC[k]);
  return phi * (m * t);
}

// N(d) and N(-d) from the tail of |d|: the smaller one is the tail itself,
// the larger one 1 - tail, so both keep their relative accuracy.
__device__ __forceinline__ void bs_normal_pair(float d, float &Nd, float &Nmd) {
  const float q = tail_q(fabsf(d));
  const float c = 1.0f - q;
  Nd = d >= 0.0f ? c : q;
  Nmd = d >= 0.0f ? q : c;
}

// Hardware transcendentals (v_sqrt, v_rcp, v_log, v_exp; about 1 ulp): the
// common rounding of d1 and d2 cancels to first order in both prices, since
// S phi(d1) = K e^{-rT} phi(d2).
__device__ __forceinline__ BSCore bs_core(float S, float K, float T, float r, float v) {
  BSCore c;
  c.sqT = __builtin_amdgcn_sqrtf(T);
  c.vs = v * c.sqT;
  const float lnSK = __builtin_amdgcn_logf(S * __builtin_amdgcn_rcpf(K)) * kLn2;
  c.d1 = __builtin_fmaf(0.5f * v * v + r, T, lnSK) * __builtin_amdgcn_rcpf(c.vs);
  c.d2 = c.d1 - c.vs;
  c.disc = __builtin_amdgcn_exp2f(-r * T * kLog2e);
  c.D = K * c.disc;
  bs_normal_pair(c.d1, c.Nd1, c.Nmd1);
  bs_normal_pair(c.d2, c.Nd2, c.Nmd2);
  return c;
}

// Region: inputs (S, K, T, r, v) -> outputs (call, put).
struct RegionBSPrice {
  static constexpr int kIn = 5;
  static constexpr int kOut = 2;
  using io = IoF32;
  __device__ __forceinline__ static void eval(const float (&x)[kIn], float (&y)[kOut]) {
    const float S = x[0], K = x[1], T = x[2], r = x[3], v = x[4];
    const BSCore c = bs_core(S, K, T, r, v);
    y[0] = S * c.Nd1 - c.D * c.Nd2;
    y[1] = c.D * c.Nmd2 - S * c.Nmd1;
  }
};

// Region: inputs (S, K, T, r, v) -> (call, put, source item).  The prices of
// RegionBSPrice; output kIndexOut is the index of the item whose evaluation
// produced them (its bits stored in the FP32 column), filled in by the
// kernels: the item itself on an accurate path, the stored entry's source
// item when iACT reuses an entry.  A backward pass can then recompute the
// derivatives at the source item's inputs: the reused gradient is reached by
// reference instead of being carried as ten columns.
struct RegionBSPriceRef {
  static constexpr int kIn = 5;
  static constexpr int kOut = 3;
  static constexpr int kIndexOut = 2;
  using io = IoF32;
  __device__ __forceinline__ static void eval(const float (&x)[kIn], float (&y)[kOut]) {
    float p[2];
    RegionBSPrice::eval(x, p);
    y[0] = p[0];
    y[1] = p[1];
    y[2] = 0.0f;
  }
};

// Region: inputs (S, K, T, r, v) -> (call, put, dC/dx[5], dP/dx[5]), x in
// input order.  Closed-form sensitivities; the put row is written with the
// tail probabilities (dP/dS = -N(-d1), dP/dK = e^{-rT} N(-d2), ...), the same
// values as the parity-derived forms without their cancellation.
struct RegionBSPriceGrad {
  static constexpr int kIn = 5;
  static constexpr int kOut = 12;
  using io = IoF32;
  __device__ __forceinline__ static void eval(const float (&x)[kIn], float (&y)[kOut]) {
    const float S = x[0], K = x[1], T = x[2], r = x[3], v = x[4];
    const BSCore c = bs_core(S, K, T, r, v);
    const float phi = kInvSqrt2Pi * __builtin_amdgcn_exp2f(c.d1 * c.d1 * kHalfL2eHi);
    const float Sphi = S * phi;
    const float theta_common = Sphi * v * 0.5f * __builtin_amdgcn_rcpf(c.sqT);
    y[0] = S * c.Nd1 - c.D * c.Nd2;
    y[1] = c.D * c.Nmd2 - S * c.Nmd1;
    y[2] = c.Nd1;                              // dC/dS
    y[3] = -c.disc * c.Nd2;                    // dC/dK
    y[4] = theta_common + r * c.D * c.Nd2;     // dC/dT
    y[5] = T * c.D * c.Nd2;                    // dC/dr
    y[6] = Sphi * c.sqT;                       // dC/dv
    y[7] = -c.Nmd1;                            // dP/dS
    y[8] = c.disc * c.Nmd2;                    // dP/dK
    y[9] = theta_common - r * c.D * c.Nmd2;    // dP/dT
    y[10] = -T * c.D * c.Nmd2;                 // dP/dr
    y[11] = y[6];                              // dP/dv
  }
};

}  // namespace hpac

// Black-Scholes-Merton region bodies (FP32) for the approximation kernels.
// The paper's Black-Scholes benchmark prices a portfolio of European options
// analytically (section 4, Table 1); the whole price calculation is the
// approximated region.  Textbook formula, no dividends:
//   d1 = (ln(S/K) + (r + v^2/2) T) / (v sqrt T),  d2 = d1 - v sqrt T,
//   C = S N(d1) - K e^{-rT} N(d2),  P = K e^{-rT} N(-d2) - S N(-d1).
// N is evaluated through the tail probability Q(|d|) = erfc(|d|/sqrt2)/2,
// so N(d) and N(-d) are both accurate in relative terms in the tails.
#pragma once
#include <hip/hip_runtime.h>

namespace hpac {

struct BSCore {
  float sqT, vs, d1, d2, disc, D;
  float Nd1, Nmd1, Nd2, Nmd2;
};

__device__ __forceinline__ void bs_normal_pair(float d, float &Nd, float &Nmd) {
  const float q = 0.5f * erfcf(fabsf(d) * 0.70710678118654752f);
  const float c = 1.0f - q;
  Nd = d >= 0.0f ? c : q;
  Nmd = d >= 0.0f ? q : c;
}

__device__ __forceinline__ BSCore bs_core(float S, float K, float T, float r, float v) {
  BSCore c;
  c.sqT = sqrtf(T);
  c.vs = v * c.sqT;
  c.d1 = (logf(S / K) + (r + 0.5f * v * v) * T) / c.vs;
  c.d2 = c.d1 - c.vs;
  c.disc = expf(-r * T);
  c.D = K * c.disc;
  bs_normal_pair(c.d1, c.Nd1, c.Nmd1);
  bs_normal_pair(c.d2, c.Nd2, c.Nmd2);
  return c;
}

// Region: inputs (S, K, T, r, v) -> outputs (call, put).
struct RegionBSPrice {
  static constexpr int kIn = 5;
  static constexpr int kOut = 2;
  __device__ __forceinline__ static void eval(const float (&x)[kIn], float (&y)[kOut]) {
    const float S = x[0], K = x[1], T = x[2], r = x[3], v = x[4];
    const BSCore c = bs_core(S, K, T, r, v);
    y[0] = S * c.Nd1 - c.D * c.Nd2;
    y[1] = c.D * c.Nmd2 - S * c.Nmd1;
  }
};

// Region: inputs (S, K, T, r, v) -> (call, put, dC/dx[5], dP/dx[5]), x in
// input order.  Closed-form sensitivities; the put row is written with the
// tail probabilities (dP/dS = -N(-d1), dP/dK = e^{-rT} N(-d2), ...), the same
// values as the parity-derived forms without their cancellation.
struct RegionBSPriceGrad {
  static constexpr int kIn = 5;
  static constexpr int kOut = 12;
  __device__ __forceinline__ static void eval(const float (&x)[kIn], float (&y)[kOut]) {
    const float S = x[0], K = x[1], T = x[2], r = x[3], v = x[4];
    const BSCore c = bs_core(S, K, T, r, v);
    const float phi = 0.39894228040143268f * expf(-0.5f * c.d1 * c.d1);
    const float Sphi = S * phi;
    const float theta_common = Sphi * v / (2.0f * c.sqT);
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

// Reduced-precision variants of the Black-Scholes region and half-precision
// column I/O.
//
// RegionBSPriceF16 evaluates the same formula as RegionBSPrice with every
// operation in FP16 (hardware v_log/v_exp/v_sqrt/v_rcp/v_fma _f16).
// RegionBSPriceBF16 evaluates it with BF16 precision: each operation is done
// in FP32 and its result rounded to the nearest BF16 (8-bit significand).
// Both take and return floats, so they compose with every technique; the
// column element type is a separate choice (IoF32, IoF16, IoBF16), applied
// when a column is loaded or stored.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "io_types.hpp"
#include "region_bs.hpp"
#include "tail_q_coeffs.hpp"

namespace hpac {

// -------------------------------------------------------------- FP16 body

struct RegionBSPriceF16 {
  static constexpr int kIn = 5;
  static constexpr int kOut = 2;
  using io = IoF32;
  using h = _Float16;

  __device__ __forceinline__ static h tail(h z) {
    const h phi = __builtin_exp2f16(z * z * (h)kHalfL2eHi) * (h)kInvSqrt2Pi;
    const h t = __builtin_amdgcn_rcph(__builtin_fmaf16((h)kTailP, z, (h)1.0f));
    h m = (h)kTailC[kTailK - 1];
#pragma unroll
    for (int k = kTailK - 2; k >= 0; --k) m = __builtin_fmaf16(m, t, (h)kTailC[k]);
    return phi * (m * t);
  }

  __device__ __forceinline__ static void eval(const float (&x)[kIn], float (&y)[kOut]) {
    const h S = (h)x[0], K = (h)x[1], T = (h)x[2], r = (h)x[3], v = (h)x[4];
    const h sqT = __builtin_sqrtf16(T);
    const h vs = v * sqT;
    const h lnSK = __builtin_log2f16(S * __builtin_amdgcn_rcph(K)) * (h)kLn2;
    const h d1 = __builtin_fmaf16((h)0.5f * v * v + r, T, lnSK) * __builtin_amdgcn_rcph(vs);
    const h d2 = d1 - vs;
    const h D = K * __builtin_exp2f16(-r * T * (h)kLog2e);
    const h q1 = tail(d1 >= (h)0 ? d1 : -d1), q2 = tail(d2 >= (h)0 ? d2 : -d2);
    const h one = (h)1.0f;
    const h Nd1 = d1 >= (h)0 ? one - q1 : q1, Nmd1 = d1 >= (h)0 ? q1 : one - q1;
    const h Nd2 = d2 >= (h)0 ? one - q2 : q2, Nmd2 = d2 >= (h)0 ? q2 : one - q2;
    y[0] = (float)(S * Nd1 - D * Nd2);
    y[1] = (float)(D * Nmd2 - S * Nmd1);
  }
};

// -------------------------------------------------------------- BF16 body

// FP32 value carried at BF16 precision: every operation's result is rounded
// to the nearest BF16.
struct Bf {
  float v;
  __device__ __forceinline__ static Bf r(float f) { return Bf{(float)(__bf16)f}; }
};
__device__ __forceinline__ Bf operator+(Bf a, Bf b) { return Bf::r(a.v + b.v); }
__device__ __forceinline__ Bf operator-(Bf a, Bf b) { return Bf::r(a.v - b.v); }
__device__ __forceinline__ Bf operator*(Bf a, Bf b) { return Bf::r(a.v * b.v); }
__device__ __forceinline__ Bf operator-(Bf a) { return Bf{-a.v}; }
__device__ __forceinline__ Bf bfma(Bf a, Bf b, Bf c) { return Bf::r(__builtin_fmaf(a.v, b.v, c.v)); }
__device__ __forceinline__ Bf brcp(Bf a) { return Bf::r(__builtin_amdgcn_rcpf(a.v)); }
__device__ __forceinline__ Bf bsqrt(Bf a) { return Bf::r(__builtin_amdgcn_sqrtf(a.v)); }
__device__ __forceinline__ Bf blog2(Bf a) { return Bf::r(__builtin_amdgcn_logf(a.v)); }
__device__ __forceinline__ Bf bexp2(Bf a) { return Bf::r(__builtin_amdgcn_exp2f(a.v)); }

struct RegionBSPriceBF16 {
  static constexpr int kIn = 5;
  static constexpr int kOut = 2;
  using io = IoF32;

  __device__ __forceinline__ static Bf tail(Bf z) {
    const Bf phi = bexp2(z * z * Bf::r(kHalfL2eHi)) * Bf::r(kInvSqrt2Pi);
    const Bf t = brcp(bfma(Bf::r(kTailP), z, Bf{1.0f}));
    Bf m = Bf::r(kTailC[kTailK - 1]);
#pragma unroll
    for (int k = kTailK - 2; k >= 0; --k) m = bfma(m, t, Bf::r(kTailC[k]));
    return phi * (m * t);
  }

  __device__ __forceinline__ static void eval(const float (&x)[kIn], float (&y)[kOut]) {
    const Bf S = Bf::r(x[0]), K = Bf::r(x[1]), T = Bf::r(x[2]), r = Bf::r(x[3]), v = Bf::r(x[4]);
    const Bf sqT = bsqrt(T);
    const Bf vs = v * sqT;
    const Bf lnSK = blog2(S * brcp(K)) * Bf::r(kLn2);
    const Bf d1 = bfma(Bf{0.5f} * v * v + r, T, lnSK) * brcp(vs);
    const Bf d2 = d1 - vs;
    const Bf D = K * bexp2(-r * T * Bf::r(kLog2e));
    const Bf q1 = tail(Bf{fabsf(d1.v)}), q2 = tail(Bf{fabsf(d2.v)});
    const Bf one{1.0f};
    const bool p1 = d1.v >= 0.0f, p2 = d2.v >= 0.0f;
    const Bf Nd1 = p1 ? one - q1 : q1, Nmd1 = p1 ? q1 : one - q1;
    const Bf Nd2 = p2 ? one - q2 : q2, Nmd2 = p2 ? q2 : one - q2;
    y[0] = (S * Nd1 - D * Nd2).v;
    y[1] = (D * Nmd2 - S * Nmd1).v;
  }
};

}  // namespace hpac

// Reduced-precision variants of the Black-Scholes region and half-precision
// column I/O.
//
// RegionBSPriceF16 evaluates the same formula as RegionBSPrice with every
// operation in FP16 (hardware v_log/v_exp/v_sqrt/v_rcp/v_fma _f16), each
// written operation rounded on its own (no contraction), so that the
// single-item and the packed pair forms agree bit for bit.
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
#pragma clang fp contract(off)
    const h phi = __builtin_exp2f16(z * z * (h)kHalfL2eHi) * (h)kInvSqrt2Pi;
    const h t = __builtin_amdgcn_rcph(__builtin_fmaf16((h)kTailP, z, (h)1.0f));
    h m = (h)kTailC[kTailK - 1];
#pragma unroll
    for (int k = kTailK - 2; k >= 0; --k) m = __builtin_fmaf16(m, t, (h)kTailC[k]);
    return phi * (m * t);
  }

  __device__ __forceinline__ static void eval(const float (&x)[kIn], float (&y)[kOut]) {
#pragma clang fp contract(off)
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

  // The same operations on a pair of items in packed FP16 (v_pk_add / mul /
  // fma _f16; the transcendentals have no packed form and go element by
  // element): each element is rounded as in eval, so eval2 gives eval's
  // results bit for bit, at about half the instructions.
  static constexpr bool kPaired = true;
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  template <class F>
  __device__ __forceinline__ static h2 each(h2 v, F f) {
    return h2{(h)f(v.x), (h)f(v.y)};
  }
  __device__ __forceinline__ static h2 fma2(h2 a, h2 b, h2 c) { return __builtin_elementwise_fma(a, b, c); }
  __device__ __forceinline__ static h2 sel(h2 c_ge0, h2 a, h2 b) {  // c >= 0 ? a : b, element-wise
    return h2{c_ge0.x >= (h)0 ? a.x : b.x, c_ge0.y >= (h)0 ? a.y : b.y};
  }
  __device__ __forceinline__ static h2 tail2(h2 z) {
#pragma clang fp contract(off)
    const h2 phi = each(z * z * (h)kHalfL2eHi, [](h t) { return __builtin_exp2f16(t); }) * (h)kInvSqrt2Pi;
    const h2 t = each(fma2((h2)(h)kTailP, z, (h2)(h)1.0f), [](h q) { return __builtin_amdgcn_rcph(q); });
    h2 m = (h2)(h)kTailC[kTailK - 1];
#pragma unroll
    for (int k = kTailK - 2; k >= 0; --k) m = fma2(m, t, (h2)(h)kTailC[k]);
    return phi * (m * t);
  }
  __device__ __forceinline__ static void eval2(const float (&xa)[kIn], const float (&xb)[kIn], float (&ya)[kOut],
                                               float (&yb)[kOut]) {
#pragma clang fp contract(off)
    const h2 S{(h)xa[0], (h)xb[0]}, K{(h)xa[1], (h)xb[1]}, T{(h)xa[2], (h)xb[2]}, r{(h)xa[3], (h)xb[3]},
        v{(h)xa[4], (h)xb[4]};
    const h2 sqT = each(T, [](h q) { return __builtin_sqrtf16(q); });
    const h2 vs = v * sqT;
    const h2 lnSK = each(S * each(K, [](h q) { return __builtin_amdgcn_rcph(q); }),
                         [](h q) { return __builtin_log2f16(q); }) * (h)kLn2;
    const h2 d1 = fma2((h)0.5f * v * v + r, T, lnSK) * each(vs, [](h q) { return __builtin_amdgcn_rcph(q); });
    const h2 d2 = d1 - vs;
    const h2 D = K * each(-r * T * (h)kLog2e, [](h q) { return __builtin_exp2f16(q); });
    const h2 q1 = tail2(sel(d1, d1, -d1)), q2 = tail2(sel(d2, d2, -d2));
    const h2 one = (h2)(h)1.0f;
    const h2 Nd1 = sel(d1, one - q1, q1), Nmd1 = sel(d1, q1, one - q1);
    const h2 Nd2 = sel(d2, one - q2, q2), Nmd2 = sel(d2, q2, one - q2);
    const h2 c = S * Nd1 - D * Nd2, p = D * Nmd2 - S * Nmd1;
    ya[0] = (float)c.x;
    ya[1] = (float)p.x;
    yb[0] = (float)c.y;
    yb[1] = (float)p.y;
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

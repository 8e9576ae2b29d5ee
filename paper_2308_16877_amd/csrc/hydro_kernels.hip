// Lagrangian hydrodynamics on a structured hexahedral mesh (a Sedov point
// blast) with the paper's techniques applied across timesteps to two
// per-element regions: the hourglass-force region (TAF or herded
// perforation) and the EOS region (TAF).  The paper approximates the
// hourglass computation of its hydrodynamics proxy and reports the final
// origin energy as quantity of interest (section 4, Table 1 and 4.1).
//
// Scheme (our own, from published methods; FP32 state, FP64 time step):
//   n^3 elements on [0, side]^3, (n+1)^3 nodes, symmetry planes x=0, y=0,
//   z=0, free outer faces.  Element (i,j,k), corner a + 2b + 4c is node
//   (i+a, j+b, k+c); reference coordinates s = (2a-1, 2b-1, 2c-1).
//   k_hydro_force  per element: volume V and its gradient B = dV/dx in
//                  closed form (exact for a trilinear hexahedron);
//                  corner forces (p + q) B + hourglass forces (viscous
//                  Flanagan-Belytschko form); the element's FP64 time-step
//                  bound, reduced per workgroup.
//   k_hydro_dt     dt = min(growth * previous dt, all bounds); time += dt.
//   k_hydro_node   per node: gather of the adjacent corner forces in corner
//                  order (no atomics), u' = u + dt F / M, zero normal
//                  velocity on the symmetry planes, x += dt (u + u') / 2.
//   k_hydro_eos    per element: compatible energy update m de = -dt
//                  sum F . (u + u')/2 (Caramana et al. 1998), ideal-gas
//                  pressure, von Neumann-Richtmyer viscosity from the
//                  volume rate sum B(x') . (u + u')/2, sound speed.
// One element per lane, so a wave is 64 consecutive elements and a TAF
// "step" is a timestep: windows live in HBM.  At wave level the countdown
// and push count of each wave are one int each, read by the whole wave and
// written by its first lane; at thread level every element has its own.
// An approximate EOS step reads only the countdown; an approximate
// hourglass step adds the last accurate hourglass forces -- the newest slot
// of its window -- instead of computing them.  A perforated hourglass
// iteration adds nothing.
#include "launch_hydro.hpp"
#include "wave.hpp"

#include <mutex>

namespace hpac {

namespace {

constexpr float sgnf(int c, int d) { return ((c >> d) & 1) ? 1.0f : -1.0f; }

// Hourglass base vectors: products of reference coordinates.
constexpr float gamma_base(int a, int k) {
  return a == 0 ? sgnf(k, 1) * sgnf(k, 2)
       : a == 1 ? sgnf(k, 0) * sgnf(k, 2)
       : a == 2 ? sgnf(k, 0) * sgnf(k, 1)
                : sgnf(k, 0) * sgnf(k, 1) * sgnf(k, 2);
}

// Volume and, with kGrad, B = dV/dx of the trilinear hexahedron, in closed
// form.  Writing the map in the Walsh-Hadamard basis of the corner signs,
// x(xi) = a0 + a1 xi + a2 eta + a3 zeta + a4 xi eta + a5 xi zeta + a6 eta zeta
// + a7 xi eta zeta with a_k = 1/8 sum_c h_k(c) x_c, and integrating det J
// over the reference cube, the odd monomials vanish and
//   V = 8 [a1, a2, a3] + 8/3 ([a1, a4, a5] + [a4, a2, a6] + [a5, a6, a3]),
// [x, y, z] = x . (y cross z); a0 and a7 drop out.  Then dV/da_k = g_k (cross
// products of the others) and B_c = 1/8 sum_k g_k h_k(c): two 8-point
// Hadamard transforms and twelve cross products, about a quarter of the
// Gauss-point work, and the same values (the Gauss rule is exact here).
// The transform is taken of x_c - x_0, differences that neighbouring FP32
// coordinates give almost exactly, since the coordinates themselves far
// exceed an element's size.
__device__ __forceinline__ void cross3(const float (&u)[3], const float (&v)[3], float (&w)[3]) {
  w[0] = __builtin_fmaf(u[1], v[2], -u[2] * v[1]);
  w[1] = __builtin_fmaf(u[2], v[0], -u[0] * v[2]);
  w[2] = __builtin_fmaf(u[0], v[1], -u[1] * v[0]);
}
__device__ __forceinline__ float dot3(const float (&u)[3], const float (&v)[3]) {
  return __builtin_fmaf(u[0], v[0], __builtin_fmaf(u[1], v[1], u[2] * v[2]));
}

template <bool kGrad>
__device__ __forceinline__ float hex_volume(const float (&x)[8][3], float (&B)[8][3]) {
  // A[m] = 8 a_m: Hadamard transform of the corner offsets; bit 0 of m is
  // the xi factor, bit 1 eta, bit 2 zeta (a1 = A[1], a2 = A[2], a3 = A[4],
  // a4 = A[3], a5 = A[5], a6 = A[6])
  float A[8][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float d[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) d[c] = c ? x[c][i] - x[0][i] : 0.0f;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (!((c >> j) & 1)) {
          const float lo = d[c], hi = d[c | (1 << j)];
          d[c] = lo + hi;
          d[c | (1 << j)] = hi - lo;
        }
#pragma unroll
    for (int m = 0; m < 8; ++m) A[m][i] = d[m];
  }
  const float(&A1)[3] = A[1], (&A2)[3] = A[2], (&A3)[3] = A[4], (&A4)[3] = A[3], (&A5)[3] = A[5],
               (&A6)[3] = A[6];
  constexpr float kThird = 1.0f / 3.0f;
  float x23[3], x45[3], x26[3], x63[3];
  cross3(A2, A3, x23);
  cross3(A4, A5, x45);
  cross3(A2, A6, x26);
  cross3(A6, A3, x63);
  // G1 = A2 x A3 + (A4 x A5) / 3 = 64 dV/dA1 (times 8 a1 . G1 it gives the leading terms)
  float G1[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) G1[i] = __builtin_fmaf(x45[i], kThird, x23[i]);
  const float V = (dot3(A1, G1) + (dot3(A4, x26) + dot3(A5, x63)) * kThird) * (1.0f / 64.0f);
  if (kGrad) {
    float x31[3], x64[3], x12[3], x56[3], x51[3], x14[3], x42[3], x35[3];
    cross3(A3, A1, x31);
    cross3(A6, A4, x64);
    cross3(A1, A2, x12);
    cross3(A5, A6, x56);
    cross3(A5, A1, x51);
    cross3(A1, A4, x14);
    cross3(A4, A2, x42);
    cross3(A3, A5, x35);
    // E[m] = 64 dV/dA_m at the Hadamard position m, then the inverse transform
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      float E[8];
      E[0] = 0.0f;
      E[7] = 0.0f;
      E[1] = G1[i];
      E[2] = __builtin_fmaf(x64[i], kThird, x31[i]);
      E[4] = __builtin_fmaf(x56[i], kThird, x12[i]);
      E[3] = (x51[i] + x26[i]) * kThird;
      E[5] = (x14[i] + x63[i]) * kThird;
      E[6] = (x42[i] + x35[i]) * kThird;
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int m = 0; m < 8; ++m)
          if (!((m >> j) & 1)) {
            const float u = E[m], v = E[m | (1 << j)];
            E[m] = u - v;
            E[m | (1 << j)] = u + v;
          }
#pragma unroll
      for (int c = 0; c < 8; ++c) B[c][i] = E[c] * (1.0f / 64.0f);
    }
  }
  return V;
}

__device__ __forceinline__ void hourglass(const float (&x)[8][3], const float (&u)[8][3], const float (&B)[8][3],
                                          float V, float rho, float c, float khg, float (&f)[8][3]) {
  const float inv_v = 1.0f / V;
  float h[4][3];
  float gam[4][8];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    float gx[3];
    // both sums vanish on constants (the base vectors and the hourglass
    // vectors sum to zero), so they are taken relative to corner 0
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      float s = 0.0f;
#pragma unroll
      for (int k = 1; k < 8; ++k) s = __builtin_fmaf(gamma_base(a, k), x[k][i] - x[0][i], s);
      gx[i] = s * inv_v;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      gam[a][k] = gamma_base(a, k) - (gx[0] * B[k][0] + gx[1] * B[k][1] + gx[2] * B[k][2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      float s = 0.0f;
#pragma unroll
      for (int k = 1; k < 8; ++k) s = __builtin_fmaf(gam[a][k], u[k][i] - u[0][i], s);
      h[a][i] = s;
    }
  }
  const float cv = cbrtf(V);
  const float coef = -(khg * 0.125f) * rho * c * (cv * cv);
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      float s = 0.0f;
#pragma unroll
      for (int a = 0; a < 4; ++a) s = __builtin_fmaf(gam[a][k], h[a][i], s);
      f[k][i] = coef * s;
    }
}

struct ElemIdx {
  int64_t z;
  int64_t node0;  // node of corner 0
  __device__ ElemIdx(int64_t z_, const DivBy &dn) : z(z_) {
    const int64_t n = dn.d, m = n + 1;
    const uint32_t t = dn.quo((uint32_t)z_), k = dn.quo(t);
    const int64_t i = z_ - (int64_t)t * n, j = (int64_t)t - (int64_t)k * n;
    node0 = i + m * (j + m * k);
  }
  __device__ int64_t node(int c, int n) const {
    const int64_t m = n + 1;
    return node0 + (c & 1) + m * (((c >> 1) & 1) + m * ((c >> 2) & 1));
  }
};

__device__ __forceinline__ void gather3(const float *const *src, const ElemIdx &e, int n, float (&v)[8][3]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int64_t nd = e.node(c, n);
#pragma unroll
    for (int d = 0; d < 3; ++d) v[c][d] = src[d][nd];
  }
}

// Whether the RSD of every output over the h window slots is below theta.
// The value y in slot `fresh`, just pushed by this thread, is read back as
// a pivot.  With the deviations d_q = w_q - y of the other slots (exact in
// FP64 for FP32 data), s' = sum d_q and Q = sum d_q^2, the two-pass
// statistic is
//   D = sum_q (h w_q - s)^2 = h (h Q - s'^2),   s = sum_q w_q = h y + s',
// shifted by a sample so that it does not cancel (h Q >= s'^2 by
// Cauchy-Schwarz, so D >= 0).  Division-free test D < h theta^2 s^2, and D
// == 0 (a constant window) passes whenever theta > 0, as in the
// Black-Scholes TAF.  Outputs go in groups of G, a slot of a whole group per
// memory round trip; the first failing group decides.
template <int NO, int G>
__device__ __forceinline__ bool window_rsd_below(const float *win, int64_t E, int64_t z, int h, int fresh,
                                                 double th2, bool th_pos) {
  static_assert(NO % G == 0, "outputs come in whole groups");
  for (int o0 = 0; o0 < NO; o0 += G) {
    double y[G], s1[G], Q[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      y[g] = (double)win[((int64_t)fresh * NO + o0 + g) * E + z];
      s1[g] = 0.0;
      Q[g] = 0.0;
    }
    for (int q = 0; q < h; ++q) {
      if (q == fresh) continue;
      float wq[G];
#pragma unroll
      for (int g = 0; g < G; ++g) wq[g] = win[((int64_t)q * NO + o0 + g) * E + z];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const double d = (double)wq[g] - y[g];
        s1[g] += d;
        Q[g] = __builtin_fma(d, d, Q[g]);
      }
    }
    bool ok = true;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const double D = (double)h * __builtin_fma((double)h, Q[g], -(s1[g] * s1[g]));
      const double sum = __builtin_fma((double)h, y[g], s1[g]);
      ok = ok && (D == 0.0 ? th_pos : D < (double)h * th2 * (sum * sum));
    }
    if (!ok) return false;
  }
  return true;
}

// Workgroups are dispatched to the 8 XCDs in turn (workgroup b to XCD b mod
// 8).  Renumbered this way, XCD x runs one contiguous stretch of the range,
// so neighbouring planes of the mesh, which share nodes, meet in the same L2.
// A bijection of [0, nb): XCD x takes nb/8 workgroups, one more if x < nb mod 8.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b & 7, j = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ double block_min(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  return red[0];
}

}  // namespace

// ------------------------------------------------------------------ init

__global__ void __launch_bounds__(256) k_hydro_init_elem(HydroArgs a, double e_origin) {
  const int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.E) return;
  const int64_t n = a.n;
  const uint32_t t = a.dn.quo((uint32_t)z), kk = a.dn.quo(t);
  const int64_t i = z - (int64_t)t * n, j = (int64_t)t - (int64_t)kk * n, k = kk;
  float x[8][3], B[8][3];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    x[c][0] = a.h * (float)(i + (c & 1));
    x[c][1] = a.h * (float)(j + ((c >> 1) & 1));
    x[c][2] = a.h * (float)(k + ((c >> 2) & 1));
  }
  const float V = hex_volume<false>(x, B);
  const float rho0 = 1.0f;
  a.vol[z] = V;
  a.mass[z] = rho0 * V;
  const float e = z == 0 ? (float)e_origin : 0.0f;
  const float p = (a.gamma - 1.0f) * rho0 * e;
  a.e[z] = e;
  a.p[z] = p;
  a.q[z] = 0.0f;
  a.c[z] = sqrtf(a.gamma * fmaxf(p, 0.0f) / rho0);
}

__global__ void __launch_bounds__(256) k_hydro_init_node(HydroArgs a) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= a.Nn) return;
  const int n = a.n;
  const int64_t m = n + 1;
  const uint32_t t = a.dm.quo((uint32_t)v), kk = a.dm.quo(t);
  const int64_t i = v - (int64_t)t * m, j = (int64_t)t - (int64_t)kk * m, k = kk;
  a.x[0][v] = a.h * (float)i;
  a.x[1][v] = a.h * (float)j;
  a.x[2][v] = a.h * (float)k;
  float M = 0.0f;
  for (int c = 0; c < 8; ++c) {
    const int64_t ei = i - (c & 1), ej = j - ((c >> 1) & 1), ek = k - ((c >> 2) & 1);
    if (ei < 0 || ej < 0 || ek < 0 || ei >= n || ej >= n || ek >= n) continue;
    M += a.mass[ei + n * (ej + (int64_t)n * ek)] * 0.125f;
  }
  a.mnode[v] = M;
  for (int d = 0; d < 3; ++d) {
    a.u[d][v] = 0.0f;
    a.un[d][v] = 0.0f;
  }
}

// TAF decision-group state, over one entry per element (the largest grouping)
__global__ void __launch_bounds__(256) k_hydro_init_groups(HydroArgs a, double dt0) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) {
    a.clock[0] = 0.0;
    a.clock[1] = dt0;
    *a.status = 0;
  }
  if (g >= a.E) return;
  if (a.rho_eos) a.rho_eos[g] = 0, a.z_eos[g] = 0;
  if (a.rho_hg) a.rho_hg[g] = 0, a.z_hg[g] = 0;
}

// ------------------------------------------------------------------ force

// Corner forces (p + q) B + f of one element, f = NULL for none.
__device__ __forceinline__ void store_forces(float *force, int64_t E, int64_t z, float pq, const float (&B)[8][3],
                                             const float (*f)[3]) {
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) force[(c * 3 + d) * E + z] = f ? __builtin_fmaf(pq, B[c][d], f[c][d]) : pq * B[c][d];
}

template <int HG>
__global__ void __launch_bounds__(256) k_hydro_force(HydroArgs a) {
  __shared__ double red[256];
  const int n = a.n;
  const int64_t E = a.E;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);  // element block: the block-level group
  const int64_t l = blk * blockDim.x + threadIdx.x;
  const int lane = lane_id();
  constexpr bool kTaf = HG == kHgTafWave || HG == kHgTafThread || HG == kHgTafBlock;
  __shared__ int tally[3];  // block level: active elements, votes to approximate, waves that voted
  if (HG == kHgTafBlock) {
    if (threadIdx.x < 3) tally[threadIdx.x] = 0;
    __syncthreads();
  }
  double bound = INFINITY;
  for (int k = 0; k < a.hg_ipt; ++k) {
    const int64_t z = l + (int64_t)k * a.hg_L;
    const bool active = z < E;
    const int64_t w = l >> 6;  // TAF: one element per lane
    bool compute_hg = HG != kHgNone;
    int rho = 0, pushes = 0;
    if (HG == kHgPerfo) {
      const int M = a.perfo_param;
      if (M > 0) {
        switch (a.perfo_kind) {
          case 0: compute_hg = (int)(((int64_t)k + a.step) % M) != M - 1; break;
          case 1: compute_hg = (int)(((int64_t)k + a.step) % M) == 0; break;
          case 2: compute_hg = z >= (int64_t)M * E / 100; break;
          default: compute_hg = z < E - (int64_t)M * E / 100; break;
        }
      }
    }
    if (HG == kHgTafWave && w < a.W) {
      rho = a.rho_hg[w];
      pushes = a.z_hg[w];
      compute_hg = rho <= 0;
    }
    if (HG == kHgTafThread && active) {
      rho = a.rho_hg[z];
      pushes = a.z_hg[z];
      compute_hg = rho <= 0;
    }
    if (HG == kHgTafBlock) {
      rho = a.rho_hg[blk];
      pushes = a.z_hg[blk];
      compute_hg = rho <= 0;
    }
    bool crit = false, voted = false;
    if (active) {
      const ElemIdx ei(z, a.dn);
      float x[8][3], u[8][3], B[8][3];
      gather3(a.x, ei, n, x);
      gather3(a.u, ei, n, u);
      const float V = hex_volume<true>(x, B);
      a.vol[z] = V;
      if (!(V > 0.0f)) atomicOr(a.status, kHydroBadVolume);  // tangled (or NaN) element
      const float pq = a.p[z] + a.q[z];
      // volume rate sum B . u (B sums to zero, so relative to corner 0)
      float vdot = 0.0f;
#pragma unroll
      for (int c = 1; c < 8; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) vdot = __builtin_fmaf(B[c][d], u[c][d] - u[0][d], vdot);
      if (compute_hg) {
        float f[8][3];
        hourglass(x, u, B, V, a.mass[z] / V, a.c[z], a.khg, f);
        store_forces(a.force, E, z, pq, B, f);
        if (kTaf) {  // push the accurate forces
          const int slot = pushes % a.hg_h;
#pragma unroll
          for (int o = 0; o < 24; ++o) a.whg[((int64_t)slot * 24 + o) * E + z] = f[o / 3][o % 3];
        }
      } else if (kTaf) {
        // TAF's approximate path: the newest window slot holds the last
        // accurate forces (a countdown is only set after a push)
        const int slot = (pushes - 1) % a.hg_h;
        float f[8][3];
#pragma unroll
        for (int o = 0; o < 24; ++o) f[o / 3][o % 3] = a.whg[((int64_t)slot * 24 + o) * E + z];
        store_forces(a.force, E, z, pq, B, f);
      } else {
        store_forces(a.force, E, z, pq, B, nullptr);  // perforated: no hourglass force
      }
      // time-step bound in FP64
      const double Vd = (double)V, rd = (double)a.mass[z] / Vd;
      const double ceff2 = a.gamma_d * fmax((double)pq, 0.0) / rd;
      double b = ceff2 > 0.0 ? a.cfl * cbrt(Vd) / sqrt(ceff2) : INFINITY;
      if (vdot != 0.0f) b = fmin(b, a.dvmax * Vd / fabs((double)vdot));
      bound = fmin(bound, b);
      if (kTaf && compute_hg && pushes + 1 >= a.hg_h) {  // the window is full: vote
        voted = true;
        const double th = (double)a.hg_theta;
        crit = window_rsd_below<24, 8>(a.whg, E, z, a.hg_h, pushes % a.hg_h, th * th, th > 0.0);
      }
    }
    if (HG == kHgTafThread && active) {
      if (!compute_hg) {
        a.rho_hg[z] = rho - 1;
      } else {
        a.z_hg[z] = pushes + 1;
        if (crit) a.rho_hg[z] = a.hg_p;
      }
      if (a.dec_hg) a.dec_hg[z] = compute_hg ? 0 : 1;
    }
    if (HG == kHgTafWave && w < a.W) {
      const uint64_t amask = ballot(active);
      const uint64_t vmask = ballot(crit);
      const bool any_vote = ballot(voted) != 0;
      if (lane == 0) {
        if (!compute_hg) {
          a.rho_hg[w] = rho - 1;
        } else {
          a.z_hg[w] = pushes + 1;
          if (any_vote && majority(popc(vmask), popc(amask))) a.rho_hg[w] = a.hg_p;
        }
        if (a.dec_hg) a.dec_hg[w] = compute_hg ? 0 : 1;
      }
    }
    if (HG == kHgTafBlock) {  // every lane of the workgroup reaches the barrier
      const uint64_t amask = ballot(active);
      const uint64_t vmask = ballot(crit);
      const bool any_vote = ballot(voted) != 0;
      if (lane == 0 && compute_hg) {
        atomicAdd(&tally[0], popc(amask));
        atomicAdd(&tally[1], popc(vmask));
        if (any_vote) atomicAdd(&tally[2], 1);
      }
      __syncthreads();
      if (threadIdx.x == 0 && blk * blockDim.x < E) {
        if (!compute_hg) {
          a.rho_hg[blk] = rho - 1;
        } else {
          a.z_hg[blk] = pushes + 1;
          if (tally[2] > 0 && majority(tally[1], tally[0])) a.rho_hg[blk] = a.hg_p;
        }
        if (a.dec_hg) a.dec_hg[blk] = compute_hg ? 0 : 1;
      }
    }
  }
  const double m = block_min(bound, red);
  if (threadIdx.x == 0) a.dt_partials[blockIdx.x] = m;
}

// ------------------------------------------------------------------ dt

__global__ void __launch_bounds__(256) k_hydro_dt(HydroArgs a, int64_t parts) {
  __shared__ double red[256];
  // sixteen independent loads per thread in flight at once: the partials
  // were just written by every XCD, so each round trip is a memory latency
  constexpr int kU = 16;
  double m = INFINITY;
  for (int64_t b0 = threadIdx.x; b0 < parts; b0 += (int64_t)blockDim.x * kU) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t b = b0 + (int64_t)u * blockDim.x;
      v[u] = b < parts ? a.dt_partials[b] : INFINITY;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) m = fmin(m, v[u]);
  }
  m = block_min(m, red);
  if (threadIdx.x == 0) {
    const double dt = fmin(m, a.growth * a.clock[1]);
    if (!(dt > 0.0) || !isfinite(dt)) atomicOr(a.status, kHydroBadDt);
    a.clock[0] += dt;
    a.clock[1] = dt;
  }
}

// ------------------------------------------------------------------ nodes

__global__ void __launch_bounds__(256) k_hydro_node(HydroArgs a) {
  const int64_t v = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (v >= a.Nn) return;
  const int n = a.n;
  const int64_t m = n + 1, E = a.E;
  const uint32_t t = a.dm.quo((uint32_t)v), kk = a.dm.quo(t);
  const int64_t i = v - (int64_t)t * m, j = (int64_t)t - (int64_t)kk * m, k = kk;
  float F[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int64_t ei = i - (c & 1), ej = j - ((c >> 1) & 1), ek = k - ((c >> 2) & 1);
    if (ei < 0 || ej < 0 || ek < 0 || ei >= n || ej >= n || ek >= n) continue;
    const int64_t z = ei + n * (ej + (int64_t)n * ek);
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] += a.force[(c * 3 + d) * E + z];
  }
  const float dt = (float)a.clock[1];
  const float inv_m = 1.0f / a.mnode[v];
  const int64_t idx[3] = {i, j, k};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float u0 = a.u[d][v];
    float u1 = __builtin_fmaf(dt, F[d] * inv_m, u0);
    if (idx[d] == 0) u1 = 0.0f;
    a.un[d][v] = u1;
    a.x[d][v] = __builtin_fmaf(dt, 0.5f * (u0 + u1), a.x[d][v]);
  }
}

// ------------------------------------------------------------------ EOS

template <int EOS>
__global__ void __launch_bounds__(256) k_hydro_eos(HydroArgs a) {
  constexpr bool kTaf = EOS != kEosExact;
  const int n = a.n;
  const int64_t E = a.E;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);  // element block: the block-level group
  const int64_t z = blk * blockDim.x + threadIdx.x;
  const int64_t w = z >> 6;
  // whole waves past the last element leave, except at block level, where
  // every lane of the workgroup must reach its barriers
  if (EOS != kEosTafBlock && w >= a.W) return;
  const int lane = lane_id();
  const bool active = z < E;
  int pushes = 0;
  __shared__ int tally[3];  // block level: active elements, votes to approximate, waves that voted
  if (EOS == kEosTafBlock) {
    const int rho = a.rho_eos[blk];
    if (rho > 0) {  // the same for the whole workgroup
      if (threadIdx.x == 0) {
        a.rho_eos[blk] = rho - 1;
        if (a.dec_eos) a.dec_eos[blk] = 1;
      }
      return;
    }
    pushes = a.z_eos[blk];
    if (threadIdx.x < 3) tally[threadIdx.x] = 0;
    __syncthreads();
  }
  if (EOS == kEosTafWave) {
    const int rho = a.rho_eos[w];
    if (rho > 0) {
      if (lane == 0) {
        a.rho_eos[w] = rho - 1;
        if (a.dec_eos) a.dec_eos[w] = 1;
      }
      return;
    }
    pushes = a.z_eos[w];
  }
  if (EOS == kEosTafThread) {
    if (!active) return;
    const int rho = a.rho_eos[z];
    if (rho > 0) {
      a.rho_eos[z] = rho - 1;
      if (a.dec_eos) a.dec_eos[z] = 1;
      return;
    }
    pushes = a.z_eos[z];
  }
  bool crit = false, voted = false;
  if (active) {
    const ElemIdx ei(z, a.dn);
    float x[8][3], u0[8][3], u1[8][3], B[8][3];
    gather3(a.x, ei, n, x);
    gather3(a.u, ei, n, u0);
    gather3(a.un, ei, n, u1);
    float W = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) W = __builtin_fmaf(a.force[(c * 3 + d) * E + z], 0.5f * (u0[c][d] + u1[c][d]), W);
    const float V1 = hex_volume<true>(x, B);
    if (!(V1 > 0.0f)) atomicOr(a.status, kHydroBadVolume);
    // volume rate sum B . u (B sums to zero, so relative to corner 0)
    float vdot = 0.0f;
#pragma unroll
    for (int c = 1; c < 8; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        vdot = __builtin_fmaf(B[c][d], 0.5f * (u0[c][d] + u1[c][d]) - 0.5f * (u0[0][d] + u1[0][d]), vdot);
    const float dt = (float)a.clock[1];
    const float m = a.mass[z];
    const float e1 = a.e[z] - dt * W / m;
    const float rho1 = m / V1;
    const float cv = cbrtf(V1);
    const float du = vdot / (cv * cv);
    const float q1 = du < 0.0f ? rho1 * (a.cq * du * du + a.cl * a.c[z] * fabsf(du)) : 0.0f;
    const float p1 = (a.gamma - 1.0f) * rho1 * e1;
    const float c1 = sqrtf(a.gamma * fmaxf(p1, 0.0f) / rho1);
    a.e[z] = e1;
    a.p[z] = p1;
    a.q[z] = q1;
    a.c[z] = c1;
    if (kTaf) {
      const int slot = pushes % a.eos_h;
      const float y[4] = {e1, p1, q1, c1};
#pragma unroll
      for (int o = 0; o < 4; ++o) a.weos[((int64_t)slot * 4 + o) * E + z] = y[o];
      if (pushes + 1 >= a.eos_h) {
        voted = true;
        const double th = (double)a.eos_theta;
        crit = window_rsd_below<4, 4>(a.weos, E, z, a.eos_h, slot, th * th, th > 0.0);
      }
    }
  }
  if (EOS == kEosTafThread) {
    a.z_eos[z] = pushes + 1;
    if (crit) a.rho_eos[z] = a.eos_p;
    if (a.dec_eos) a.dec_eos[z] = 0;
  }
  if (EOS == kEosTafWave) {
    const uint64_t amask = ballot(active);
    const uint64_t vmask = ballot(crit);
    const bool any_vote = ballot(voted) != 0;
    if (lane == 0) {
      a.z_eos[w] = pushes + 1;
      if (any_vote && majority(popc(vmask), popc(amask))) a.rho_eos[w] = a.eos_p;
      if (a.dec_eos) a.dec_eos[w] = 0;
    }
  }
  if (EOS == kEosTafBlock) {
    const uint64_t amask = ballot(active);
    const uint64_t vmask = ballot(crit);
    const bool any_vote = ballot(voted) != 0;
    if (lane == 0) {
      atomicAdd(&tally[0], popc(amask));
      atomicAdd(&tally[1], popc(vmask));
      if (any_vote) atomicAdd(&tally[2], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a.z_eos[blk] = pushes + 1;
      if (tally[2] > 0 && majority(tally[1], tally[0])) a.rho_eos[blk] = a.eos_p;
      if (a.dec_eos) a.dec_eos[blk] = 0;
    }
  }
}

// --------------------------------------------------------------- launchers

int64_t hydro_lanes(int64_t E, int ipt) { return 64 * (((E + ipt - 1) / ipt + 63) / 64); }

int64_t hydro_partials(int64_t E) { return (hydro_lanes(E, 1) + 255) / 256; }

// Partial time-step minima of the allocation-free step: one double per
// workgroup of the force kernel, held in a file-scope device array rather
// than a caller buffer.  Every GPU the library runs on holds its own copy,
// at its own address, until the process ends.  In host code `scratch` names
// a host-side stand-in, never passed to a kernel: its device address is
// looked up once per device, with that device current, and kept.
static __device__ __align__(256) double scratch[kHydroScratchPartials];

hipError_t hydro_scratch(hipStream_t stream, double **ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  int cur = 0, dev = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  dev = cur;
  if (stream && (e = hipStreamGetDevice(stream, &dev)) != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = (double *)p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_hydro_init(const HydroArgs &a, double e_origin, double dt0, hipStream_t s) {
  hipLaunchKernelGGL(k_hydro_init_elem, dim3((unsigned)((a.E + 255) / 256)), dim3(256), 0, s, a, e_origin);
  hipLaunchKernelGGL(k_hydro_init_node, dim3((unsigned)((a.Nn + 255) / 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_hydro_init_groups, dim3((unsigned)((a.E + 255) / 256)), dim3(256), 0, s, a, dt0);
  return hipGetLastError();
}

hipError_t launch_hydro_step(const HydroArgs &a, int hg_mode, int eos_mode, hipStream_t s) {
  const unsigned fblocks = (unsigned)((a.hg_L + 255) / 256);
  if (hg_mode == kHgPerfo && a.hg_ipt == 1 && a.perfo_param > 0 && (a.perfo_kind == 0 || a.perfo_kind == 1)) {
    // one item per lane: the herded rule keeps or drops the whole step
    const int r = (int)((int64_t)a.step % a.perfo_param);
    const bool keep = a.perfo_kind == 0 ? r != a.perfo_param - 1 : r == 0;
    hg_mode = keep ? kHgExact : kHgNone;
  }
  switch (hg_mode) {
    case kHgExact: hipLaunchKernelGGL(k_hydro_force<kHgExact>, dim3(fblocks), dim3(256), 0, s, a); break;
    case kHgTafWave: hipLaunchKernelGGL(k_hydro_force<kHgTafWave>, dim3(fblocks), dim3(256), 0, s, a); break;
    case kHgTafThread: hipLaunchKernelGGL(k_hydro_force<kHgTafThread>, dim3(fblocks), dim3(256), 0, s, a); break;
    case kHgTafBlock: hipLaunchKernelGGL(k_hydro_force<kHgTafBlock>, dim3(fblocks), dim3(256), 0, s, a); break;
    case kHgNone: hipLaunchKernelGGL(k_hydro_force<kHgNone>, dim3(fblocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(k_hydro_force<kHgPerfo>, dim3(fblocks), dim3(256), 0, s, a); break;
  }
  hipLaunchKernelGGL(k_hydro_dt, dim3(1), dim3(256), 0, s, a, (int64_t)fblocks);
  hipLaunchKernelGGL(k_hydro_node, dim3((unsigned)((a.Nn + 255) / 256)), dim3(256), 0, s, a);
  const unsigned eblocks = (unsigned)((hydro_lanes(a.E, 1) + 255) / 256);
  switch (eos_mode) {
    case kEosExact: hipLaunchKernelGGL(k_hydro_eos<kEosExact>, dim3(eblocks), dim3(256), 0, s, a); break;
    case kEosTafWave: hipLaunchKernelGGL(k_hydro_eos<kEosTafWave>, dim3(eblocks), dim3(256), 0, s, a); break;
    case kEosTafThread: hipLaunchKernelGGL(k_hydro_eos<kEosTafThread>, dim3(eblocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(k_hydro_eos<kEosTafBlock>, dim3(eblocks), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace hpac

// Binomial Options region (Cox-Ross-Rubinstein tree, American or European
// call and put) with the paper's techniques.  The paper's Binomial Options
// benchmark has a whole group of threads price one option, so its decisions
// are taken per option by that group (section 4.1); here that group is one
// wavefront:
//
//   * one wave prices one option: lane j holds tree nodes jC .. jC+C-1 in
//     registers (C = ceil((N+1)/64), rounded up to an instantiated size); a time
//     step updates every node from itself and its upper neighbour, which for
//     a lane's last node is the next lane's first node (one cross-lane
//     permute per step and value array), so no barrier and no LDS array is
//     needed;
//   * a wave is the decision unit ("logical lane") of the techniques: unit u
//     of L = 64 ceil(ceil(n/IPT)/64) units processes options u + kL,
//     k < IPT, and decides alone for each (the thread level of section
//     3.1.2, the unit being the wave);
//   * iACT: the unit's table (tSize <= 64 entries of 5 inputs and 2 outputs)
//     is spread over the lanes, lane e holding entry e; distances are taken
//     in parallel with the oracle's FP32 rounding sequence, the minimum and
//     the lowest arg-min slot by a wave reduction and a ballot; a unit that
//     computed writes its entry round-robin;
//   * TAF: the unit's window of its last h accurate outputs, FP64 RSD test,
//     pSize approximate options after a passing test;
//   * perforation: herded over the unit's option loop (small, large, ini,
//     fini); a skipped option is neither read nor written.
//
// Node prices S u^(2i-n) are carried by one multiplication per step and
// recomputed from exp2 every 32 steps, which bounds their FP32 drift.
#include "launch_binomial.hpp"
#include <type_traits>
#include "wave.hpp"

namespace hpac {

namespace {

template <int N>
__device__ __forceinline__ float bo_dist2(const float (&x)[N], const float (&e)[N]) {
#pragma clang fp contract(off)
  float t = x[0] - e[0];
  float acc = t * t;
#pragma unroll
  for (int j = 1; j < N; ++j) {
    const float u = x[j] - e[j];
    acc = __builtin_fmaf(u, u, acc);
  }
  return acc;
}

// value of lane (lane + 1); the last lane reads its own (unused)
__device__ __forceinline__ float from_next_lane(float v) {
  const int src = lane_id() < 63 ? lane_id() + 1 : 63;
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

struct BoOut {
  float call, put;
};

// CRR tree of one option over the 64 lanes of the calling wave; every lane
// returns the prices.
template <int C>
__device__ __forceinline__ BoOut bo_tree(float S, float K, float T, float r, float v, int N, bool american) {
  const int lane = lane_id();
  // tree parameters in FP64 (uniform), used in FP32
  const double dt = (double)T / N;
  const double u = exp((double)v * sqrt(dt)), d = 1.0 / u, a = exp((double)r * dt);
  const double p = (a - d) / (u - d);
  const float uf = (float)u, pu = (float)(p / a), pd = (float)((1.0 - p) / a);
  const float log2u = (float)(log2(u));
  float X[C], Vc[C], Vp[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int i = lane * C + c;
    // nodes past the last leaf are padding: zero, never read by a live node
    X[c] = i <= N ? S * __builtin_amdgcn_exp2f((float)(2 * i - N) * log2u) : 0.0f;
    Vc[c] = i <= N ? fmaxf(X[c] - K, 0.0f) : 0.0f;
    Vp[c] = i <= N ? fmaxf(K - X[c], 0.0f) : 0.0f;
  }
  // the step loop, with the exercise test compiled in or out (a runtime
  // flag would cost two lane selects per node and step)
  auto steps = [&](auto american_tag) {
    constexpr bool kAmerican = decltype(american_tag)::value;
    for (int n = N - 1; n >= 0; --n) {
      const float nc = from_next_lane(Vc[0]), np = from_next_lane(Vp[0]);
      if (kAmerican) {
        if ((n & 31) == 0) {
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const int i = lane * C + c;
            X[c] = i <= n ? S * __builtin_amdgcn_exp2f((float)(2 * i - n) * log2u) : 0.0f;
          }
        } else {
#pragma unroll
          for (int c = 0; c < C; ++c) X[c] *= uf;
        }
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const float up_c = c + 1 < C ? Vc[c + 1] : nc;
        const float up_p = c + 1 < C ? Vp[c + 1] : np;
        float vc = __builtin_fmaf(pu, up_c, pd * Vc[c]);
        float vp = __builtin_fmaf(pu, up_p, pd * Vp[c]);
        if (kAmerican) {
          vc = fmaxf(vc, X[c] - K);
          vp = fmaxf(vp, K - X[c]);
        }
        Vc[c] = vc;
        Vp[c] = vp;
      }
    }
  };
  if (american)
    steps(std::true_type{});
  else
    steps(std::false_type{});
  // node 0 is lane 0's first node
  BoOut o;
  o.call = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Vc[0])));
  o.put = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Vp[0])));
  return o;
}

// Division-free FP64 RSD test over the h window slots (slot h-1 newest):
// var < theta^2 mu^2  <=>  D < h theta^2 s^2, D == 0 passes iff theta > 0.
template <int H>
__device__ __forceinline__ bool bo_rsd_below(const float (&w)[H][2], double th2, bool th_pos) {
  bool ok = true;
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < H; ++q) s += (double)w[q][o];
    double D = 0.0;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      const double dd = (double)H * (double)w[q][o] - s;
      D = __builtin_fma(dd, dd, D);
    }
    ok = ok && (D == 0.0 ? th_pos : D < (double)H * th2 * (s * s));
  }
  return ok;
}

// per-block counters: lane 0 of each wave adds into LDS, thread 0 publishes
struct BoStats {
  unsigned long long *g, *s;
  __device__ void begin() {
    if (!g) return;
    if (threadIdx.x < 4) s[threadIdx.x] = 0;
    __syncthreads();
  }
  __device__ void end(unsigned long long visited, unsigned long long approx) {
    if (!g) return;
    if (lane_id() == 0) {
      atomicAdd(&s[0], visited);
      atomicAdd(&s[1], approx);
      atomicAdd(&s[2], approx);
      atomicAdd(&s[3], visited);
    }
    __syncthreads();
    if (threadIdx.x < 4 && s[threadIdx.x]) atomicAdd(&g[threadIdx.x], s[threadIdx.x]);
  }
};

__device__ __forceinline__ uint32_t bo_trace_word(bool approx, bool voted, bool crit) {
  return 0x80000000u | (crit ? 1u : 0u) | ((approx ? 1u : 0u) << 8) | ((approx ? 1u : 0u) << 24) |
         ((voted ? 1u : 0u) << 25);
}

}  // namespace

// TECH: 0 exact, 1 iACT, 2 TAF, 3 perforation, 4 dense small/large
// perforation.  H: TAF history (1..8).
//
// Dense perforation (no trace or counters): the region keeps no state, so
// the options a herded small/large pattern keeps -- whole steps k, i.e. the
// option ranges [kL, (k+1)L) -- can be priced by any wavefronts: one option
// per wavefront over the kept ranges only, so every SIMD gets the same share
// of trees whatever the options per unit.  The outputs are those of TECH 3.
template <int C, int TECH, int H>
__global__ void __launch_bounds__(256) k_binomial(BoArgs a) {
  __shared__ unsigned long long sums[4];
  const int lane = lane_id();
  const int64_t unit = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (TECH == 4) {
    // wavefront -> r-th kept step; kept steps repeat with period M: small
    // keeps every position of a period but `special`, large only `special`
    const int64_t r = unit / a.L;
    const int64_t P = r / a.kept_per_period;
    const int rem = (int)(r - P * a.kept_per_period);
    const int pos = a.kind == 1 ? a.special : (rem < a.special ? rem : rem + 1);
    const int64_t i = (P * a.param + pos) * a.L + (unit - r * a.L);
    if (i < a.n) {
      float x[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) x[j] = a.in[j][i];
      const BoOut y = bo_tree<C>(x[0], x[1], x[2], x[3], x[4], a.steps, a.american);
      if (lane == 0) {
        a.out[0][i] = y.call;
        a.out[1][i] = y.put;
      }
    }
    return;
  }
  BoStats stats{a.counters, sums};
  stats.begin();
  unsigned long long visited = 0, approxd = 0;
  // iACT: lane e holds entry e
  float ex[5] = {0, 0, 0, 0, 0}, ey[2] = {0, 0};
  int cnt = 0, ins = 0;
  const float thr2 = a.threshold * a.threshold;
  // TAF
  float win[H][2];
#pragma unroll
  for (int q = 0; q < H; ++q) win[q][0] = win[q][1] = 0.0f;
  int fill = 0, rho = 0;
  const double th = (double)a.threshold;

  for (int k = 0; k < a.ipt && unit < a.L; ++k) {
    const int64_t i = unit + (int64_t)k * a.L;
    if (i >= a.n) break;
    visited += 1;
    if (TECH == 3) {
      bool skip = false;
      const int M = a.param;
      if (M > 0) {
        switch (a.kind) {
          case 0: skip = (int)(((int64_t)k + a.offset) % M) == M - 1; break;
          case 1: skip = (int)(((int64_t)k + a.offset) % M) != 0; break;
          case 2: skip = i < (int64_t)M * a.n / 100; break;
          default: skip = i >= a.n - (int64_t)M * a.n / 100; break;
        }
      }
      if (skip) {
        approxd += 1;
        if (a.trace && lane == 0) a.trace[unit * a.ipt + k] = bo_trace_word(true, false, false);
        continue;
      }
    }
    if (TECH == 2 && rho > 0) {
      rho -= 1;
      approxd += 1;
      if (lane == 0) {
        a.out[0][i] = win[H - 1][0];
        a.out[1][i] = win[H - 1][1];
        if (a.trace) a.trace[unit * a.ipt + k] = bo_trace_word(true, false, false);
      }
      continue;
    }
    float x[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) x[j] = a.in[j][i];
    if (TECH == 1 && cnt > 0) {
      const float d2 = lane < cnt ? bo_dist2<5>(x, ex) : INFINITY;
      const float md2 = -wave_max(-d2);
      if (md2 < thr2) {
        const int arg = lowest_lane(ballot(lane < cnt && d2 == md2));
        const float yc = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ey[0]), arg));
        const float yp = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ey[1]), arg));
        approxd += 1;
        if (lane == 0) {
          a.out[0][i] = yc;
          a.out[1][i] = yp;
          if (a.trace) a.trace[unit * a.ipt + k] = bo_trace_word(true, true, true);
        }
        continue;
      }
    }
    const BoOut y = bo_tree<C>(x[0], x[1], x[2], x[3], x[4], a.steps, a.american);
    if (lane == 0) {
      a.out[0][i] = y.call;
      a.out[1][i] = y.put;
    }
    bool voted = false, crit = false;
    if (TECH == 1) {
      const int slot = ins % a.tsize;
      if (lane == slot) {
#pragma unroll
        for (int j = 0; j < 5; ++j) ex[j] = x[j];
        ey[0] = y.call;
        ey[1] = y.put;
      }
      cnt = cnt < a.tsize ? cnt + 1 : a.tsize;
      ins += 1;
      voted = true;
    }
    if (TECH == 2) {
#pragma unroll
      for (int q = 0; q + 1 < H; ++q) {
        win[q][0] = win[q + 1][0];
        win[q][1] = win[q + 1][1];
      }
      win[H - 1][0] = y.call;
      win[H - 1][1] = y.put;
      fill = fill < H ? fill + 1 : H;
      if (fill == H) {
        voted = true;
        crit = bo_rsd_below<H>(win, th * th, th > 0.0);
        if (crit) rho = a.psize;
      }
    }
    if (a.trace && lane == 0) a.trace[unit * a.ipt + k] = bo_trace_word(false, voted, crit);
  }
  stats.end(visited, approxd);
}

// --------------------------------------------------------------- launchers

int64_t bo_units(int64_t n, int ipt) { return 64 * (((n + ipt - 1) / ipt + 63) / 64); }

// nodes per lane: the instantiated sizes, so that at most one lane's worth of
// slots is padding for every N up to 1023
int bo_nodes_per_lane(int steps) {
  const int need = (steps + 1 + 63) / 64;
  for (int c : {2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 14, 16})
    if (need <= c) return c;
  return 0;
}

template <int C, int TECH>
static void bo_go_h(const BoArgs &a, int block, hipStream_t s) {
  if (TECH == 3 && !a.trace && !a.counters && a.param > 0) {
    if (a.kind == 0 || a.kind == 1) {
      // small / large: the kept steps below the last one that holds options
      const int M = a.param;
      const int off = (int)(a.offset % M);
      BoArgs b = a;
      b.special = a.kind == 0 ? ((M - 1 - off) % M + M) % M : ((M - off) % M + M) % M;
      b.kept_per_period = a.kind == 0 ? M - 1 : 1;
      if (b.kept_per_period == 0) return;  // small with M = 1 drops every step
      const int64_t steps = (a.n + a.L - 1) / a.L;
      int64_t kept = (steps / M) * b.kept_per_period;
      for (int64_t st = (steps / M) * M; st < steps; ++st) {
        const int pos = (int)(st % M);
        kept += a.kind == 0 ? pos != b.special : pos == b.special;
      }
      if (kept == 0) return;
      if (kept * a.L * 64 > 0xFFFFFFFFll) {  // beyond a 32-bit grid: one unit per lane group, as traced
        hipLaunchKernelGGL((k_binomial<C, TECH, 1>), dim3((unsigned)(a.L * 64 / block)), dim3(block), 0, s, a);
        return;
      }
      hipLaunchKernelGGL((k_binomial<C, 4, 1>), dim3((unsigned)(kept * a.L * 64 / block)), dim3(block), 0, s, b);
      return;
    }
    // ini / fini: the kept options are one contiguous range, one per unit
    const int64_t cut = ((int64_t)a.param * a.n) / 100;
    const int64_t lo = a.kind == 2 ? cut : 0;
    BoArgs b = a;
    b.n = a.n - cut;
    if (b.n == 0) return;
    b.ipt = 1;
    b.L = bo_units(b.n, 1);
    if (b.L * 64 > 0xFFFFFFFFll) {  // beyond a 32-bit grid: the caller's units, as traced
      hipLaunchKernelGGL((k_binomial<C, TECH, 1>), dim3((unsigned)(a.L * 64 / block)), dim3(block), 0, s, a);
      return;
    }
    for (int j = 0; j < 5; ++j) b.in[j] = a.in[j] + lo;
    for (int o = 0; o < 2; ++o) b.out[o] = a.out[o] + lo;
    hipLaunchKernelGGL((k_binomial<C, 0, 1>), dim3((unsigned)(b.L * 64 / block)), dim3(block), 0, s, b);
    return;
  }
  const dim3 grid((unsigned)(a.L * 64 / block));
  if (TECH != 2) {
    hipLaunchKernelGGL((k_binomial<C, TECH, 1>), grid, dim3(block), 0, s, a);
    return;
  }
  switch (a.hsize) {
    case 1: hipLaunchKernelGGL((k_binomial<C, 2, 1>), grid, dim3(block), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_binomial<C, 2, 2>), grid, dim3(block), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_binomial<C, 2, 3>), grid, dim3(block), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_binomial<C, 2, 4>), grid, dim3(block), 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_binomial<C, 2, 5>), grid, dim3(block), 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_binomial<C, 2, 6>), grid, dim3(block), 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_binomial<C, 2, 7>), grid, dim3(block), 0, s, a); break;
    default: hipLaunchKernelGGL((k_binomial<C, 2, 8>), grid, dim3(block), 0, s, a); break;
  }
}

template <int C>
static void bo_go_c(const BoArgs &a, int tech, int block, hipStream_t s) {
  switch (tech) {
    case 0: bo_go_h<C, 0>(a, block, s); break;
    case 1: bo_go_h<C, 1>(a, block, s); break;
    case 2: bo_go_h<C, 2>(a, block, s); break;
    default: bo_go_h<C, 3>(a, block, s); break;
  }
}

hipError_t launch_binomial(const BoArgs &a, int tech, int block, hipStream_t s) {
  switch (bo_nodes_per_lane(a.steps)) {
    case 2: bo_go_c<2>(a, tech, block, s); break;
    case 3: bo_go_c<3>(a, tech, block, s); break;
    case 4: bo_go_c<4>(a, tech, block, s); break;
    case 5: bo_go_c<5>(a, tech, block, s); break;
    case 6: bo_go_c<6>(a, tech, block, s); break;
    case 7: bo_go_c<7>(a, tech, block, s); break;
    case 8: bo_go_c<8>(a, tech, block, s); break;
    case 9: bo_go_c<9>(a, tech, block, s); break;
    case 10: bo_go_c<10>(a, tech, block, s); break;
    case 12: bo_go_c<12>(a, tech, block, s); break;
    case 14: bo_go_c<14>(a, tech, block, s); break;
    case 16: bo_go_c<16>(a, tech, block, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace hpac

// Fused region + approximation kernels for gfx950.
//
// One lane per logical thread of the grid-stride loop: lane l visits items
// i = l + k L for k = 0 .. ipt-1 (sections 3.1.3 and 3.3).  Every kernel
// loads its inputs and stores its outputs as structure-of-arrays columns, so
// each wave reads and writes 64 consecutive floats per column per step.
//
//  k_exact   the region on every item.
//  k_iact    input memoization (sections 2.3, 3.1.4, 3.3): tables in LDS,
//            shared by 64/g lanes of a wave; nearest-entry search, vote,
//            single-writer round-robin insert.
//  k_taf     output memoization (sections 2.3, 3.1.3, 3.3): each lane's
//            window of recent accurate outputs lives in VGPRs; the RSD test
//            runs in FP64 after each accurate step; a passing group skips
//            both the region and its input loads for pSize steps.
//  k_perfo   herded perforation (section 3.1.5): whole steps are dropped by
//            every lane, so a dropped step issues no memory traffic at all.
//
// Decision levels (section 3.1.2): THREAD lanes decide alone (divergent);
// WAVE uses ballot + popcount; BLOCK adds the per-wave counts in LDS and
// reads the total after a barrier (section 3.3).
#include "launch.hpp"
#include "region_bs.hpp"
#include "wave.hpp"

#include <math.h>

namespace hpac {

enum { kThread = 0, kWaveLvl = 1, kBlock = 2 };
enum { kSmall = 0, kLarge = 1, kIni = 2, kFini = 3 };

// ------------------------------------------------------------------ helpers

template <class R>
__device__ __forceinline__ void load_inputs(const KArgs &a, int64_t i, float (&x)[R::kIn]) {
#pragma unroll
  for (int j = 0; j < R::kIn; ++j) x[j] = a.in[j][i];
}

template <class R>
__device__ __forceinline__ void store_outputs(const KArgs &a, int64_t i, const float (&y)[R::kOut]) {
#pragma unroll
  for (int o = 0; o < R::kOut; ++o) a.out[o][i] = y[o];
}

__device__ __forceinline__ uint32_t trace_word(int votes, int napprox, int writer, bool approx, bool voted) {
  uint32_t t = 0x80000000u | (uint32_t)(votes & 0x7F) | ((uint32_t)(napprox & 0x7F) << 8);
  if (writer >= 0) t |= ((uint32_t)writer << 16) | (1u << 22);
  if (approx) t |= 1u << 24;
  if (voted) t |= 1u << 25;
  return t;
}

// Per-wave tallies, wave-uniform, flushed once per wave at kernel end.
struct WaveStats {
  uint64_t lane_steps = 0, approx_lanes = 0, approx_wsteps = 0, wsteps = 0;
  __device__ __forceinline__ void add(int active, int napprox, bool wave_approx) {
    lane_steps += active;
    approx_lanes += napprox;
    approx_wsteps += wave_approx ? 1 : 0;
    wsteps += 1;
  }
  __device__ __forceinline__ void flush(unsigned long long *c) const {
    if (c && lane_id() == 0 && wsteps) {
      atomicAdd(&c[0], (unsigned long long)lane_steps);
      atomicAdd(&c[1], (unsigned long long)approx_lanes);
      atomicAdd(&c[2], (unsigned long long)approx_wsteps);
      atomicAdd(&c[3], (unsigned long long)wsteps);
    }
  }
};

// Block-level majority (section 3.3): lane 0 of each wave adds its wave's
// counts into LDS; the total is read after a barrier.  Three rotating tally
// slots let one barrier per step suffice: slot (k+1)%3 is cleared at step k,
// after every wave has finished reading it at step k-2 and before anyone
// adds into it at step k+1.
struct BlockTally {
  int *t;  // [3][2] in LDS
  __device__ __forceinline__ void init() {
    if (threadIdx.x < 6) t[threadIdx.x] = 0;
    __syncthreads();
  }
  __device__ __forceinline__ bool decide(int k, int wave_votes, int wave_active, bool *any_active) {
    int *cur = t + 2 * (k % 3);
    if (threadIdx.x == 0) {
      int *nxt = t + 2 * ((k + 1) % 3);
      nxt[0] = 0;
      nxt[1] = 0;
    }
    if (lane_id() == 0 && (wave_votes | wave_active)) {
      atomicAdd(&cur[0], wave_votes);
      atomicAdd(&cur[1], wave_active);
    }
    __syncthreads();
    const int votes = cur[0], act = cur[1];
    *any_active = act > 0;
    return majority(votes, act);
  }
};

// --------------------------------------------------------------- exact path

template <class R, bool kStats>
__global__ void __launch_bounds__(256) k_exact(KArgs a) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wbase = l - lane_id();
  if (wbase >= a.L) return;
  WaveStats st;
  for (int k = 0; k < a.ipt; ++k) {
    const int64_t i = l + (int64_t)k * a.L;
    if (wbase + (int64_t)k * a.L >= a.n) break;
    const bool active = i < a.n;
    if (active) {
      float x[R::kIn], y[R::kOut];
      load_inputs<R>(a, i, x);
      R::eval(x, y);
      store_outputs<R>(a, i, y);
    }
    if (kStats) {
      const int nact = popc(ballot(active));
      st.add(nact, 0, false);
      if (a.trace && lane_id() == 0) a.trace[(wbase >> 6) * a.ipt + k] = trace_word(0, 0, -1, false, false);
    }
  }
  if (kStats) st.flush(a.counters);
}

// ---------------------------------------------------------------- perforation

template <class R>
__global__ void __launch_bounds__(256) k_perfo(KArgs a, int kind, int param, int offset) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wbase = l - lane_id();
  if (wbase >= a.L) return;
  const int64_t cut = (kind == kIni || kind == kFini) ? ((int64_t)param * a.n) / 100 : 0;
  WaveStats st;
  for (int k = 0; k < a.ipt; ++k) {
    const int64_t i = l + (int64_t)k * a.L;
    if (wbase + (int64_t)k * a.L >= a.n) break;
    const bool active = i < a.n;
    const int64_t kk = (int64_t)k + offset;
    bool skip = false;  // herded: identical for every lane at step k
    if (kind == kSmall) skip = param > 0 && (kk % param) == param - 1;
    if (kind == kLarge) skip = param > 0 && (kk % param) != 0;
    if (kind == kIni) skip = i < cut;
    if (kind == kFini) skip = i >= a.n - cut;
    if (active && !skip) {
      float x[R::kIn], y[R::kOut];
      load_inputs<R>(a, i, x);
      R::eval(x, y);
      store_outputs<R>(a, i, y);
    }
    if (a.trace || a.counters) {
      const int nact = popc(ballot(active));
      const int nskip = popc(ballot(active && skip));
      st.add(nact, nskip, nskip > 0);
      if (a.trace && lane_id() == 0)
        a.trace[(wbase >> 6) * a.ipt + k] = trace_word(0, nskip, -1, nskip > 0, false);
    }
  }
  st.flush(a.counters);
}

// ------------------------------------------------------------------- iACT

template <class R>
constexpr int entry_floats() { return (R::kIn + R::kOut + 3) & ~3; }

// Squared Euclidean distance in FP32 with a fixed rounding sequence:
// t0*t0, then fma(tj, tj, acc).  No other contraction is allowed here.
template <int N>
__device__ __forceinline__ float dist2(const float (&x)[N], const float *e) {
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

template <class R, int LEVEL>
__global__ void __launch_bounds__(256) k_iact(KArgs a, int tsize, float theta, int tpw) {
  extern __shared__ float lds[];
  __shared__ int tally_mem[6];
  constexpr int E = entry_floats<R>();
  const int lane = lane_id();
  const int wib = threadIdx.x >> 6;
  const int lpt = kWave / tpw;  // lanes per table
  const int tab_in_wave = lane / lpt;
  float *tab = lds + ((size_t)wib * tpw + tab_in_wave) * tsize * E;
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wbase = l - lane;
  const int64_t bbase = (int64_t)blockIdx.x * blockDim.x;
  if (LEVEL != kBlock && wbase >= a.L) return;
  BlockTally tally{tally_mem};
  if (LEVEL == kBlock) tally.init();
  const float thr2 = theta * theta;
  const int seg0 = tab_in_wave * lpt;
  const uint64_t segmask = lpt == kWave ? ~0ull : (((1ull << lpt) - 1) << seg0);
  int cnt = 0, ins = 0;  // valid entries and insertions of this lane's table
  WaveStats st;

  for (int k = 0; k < a.ipt; ++k) {
    const int64_t step0 = (int64_t)k * a.L;
    if (LEVEL != kBlock && wbase + step0 >= a.n) break;
    if (LEVEL == kBlock && bbase + step0 >= a.n) break;
    const int64_t i = l + step0;
    const bool active = l < a.L && i < a.n;
    // read phase: nearest valid entry of this lane's table
    float x[R::kIn];
    float md2 = INFINITY;
    int arg = -1;
    if (active) {
      load_inputs<R>(a, i, x);
      for (int e = 0; e < cnt; ++e) {
        const float d2 = dist2<R::kIn>(x, tab + e * E);
        if (d2 < md2) {
          md2 = d2;
          arg = e;
        }
      }
    }
    const bool hit = active && arg >= 0 && md2 < thr2;
    const uint64_t amask = ballot(active);
    const uint64_t vmask = ballot(hit);
    bool group_approx;
    bool wave_live = amask != 0;
    if (LEVEL == kThread) {
      group_approx = hit;
    } else if (LEVEL == kWaveLvl) {
      group_approx = majority(popc(vmask), popc(amask));
    } else {
      bool any;
      group_approx = tally.decide(k, popc(vmask), popc(amask), &any);
    }
    const bool lane_approx = active && group_approx && arg >= 0;
    const bool computes = active && !lane_approx;
    float y[R::kOut];
    if (lane_approx) {
#pragma unroll
      for (int o = 0; o < R::kOut; ++o) y[o] = tab[arg * E + R::kIn + o];
    }
    if (computes) R::eval(x, y);
    if (active) store_outputs<R>(a, i, y);
    // write phase: one writer per table among the lanes that computed
    const uint64_t cmask = ballot(computes);
    int writer0 = -1;
    if (cmask) {
      const float key = computes ? md2 : -1.0f;
      const float m = segment_max(key, lpt);
      const uint64_t cand = ballot(computes && key == m);
      const uint64_t mine = cand & segmask;
      if (mine) {
        if (lane == lowest_lane(mine)) {
          float *slot = tab + (ins % tsize) * E;
#pragma unroll
          for (int j = 0; j < R::kIn; ++j) slot[j] = x[j];
#pragma unroll
          for (int o = 0; o < R::kOut; ++o) slot[R::kIn + o] = y[o];
        }
        cnt = cnt < tsize ? cnt + 1 : tsize;
        ins += 1;
      }
      const uint64_t cand0 = cand & (lpt == kWave ? ~0ull : ((1ull << lpt) - 1));
      writer0 = cand0 ? lowest_lane(cand0) : -1;
      wave_lds_fence();
    }
    if (wave_live && (a.trace || a.counters)) {
      const int nact = popc(amask);
      const int napx = popc(ballot(lane_approx));
      const bool wave_approx = LEVEL == kThread ? napx > 0 : group_approx;
      st.add(nact, napx, wave_approx);
      if (a.trace && lane == 0)
        a.trace[(wbase >> 6) * a.ipt + k] = trace_word(popc(vmask), napx, writer0, wave_approx, true);
    }
  }
  st.flush(a.counters);
}

// -------------------------------------------------------------------- TAF

// RSD criterion of one lane, FP64, all outputs must pass.
template <int H, int NO>
__device__ __forceinline__ bool rsd_below(const float (&w)[H][NO], double th, double th2) {
  bool ok = true;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < H; ++q) s += (double)w[q][o];
    const double mu = s / H;
    double var = 0.0;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      const double d = (double)w[q][o] - mu;
      var += d * d;
    }
    var /= H;
    const bool v = var == 0.0 ? th > 0.0 : var < th2 * (mu * mu);
    ok = ok && v;
  }
  return ok;
}

template <class R, int LEVEL, int H>
__global__ void __launch_bounds__(256) k_taf(KArgs a, int psize, float theta) {
  __shared__ int tally_mem[6];
  const int lane = lane_id();
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wbase = l - lane;
  const int64_t bbase = (int64_t)blockIdx.x * blockDim.x;
  if (LEVEL != kBlock && wbase >= a.L) return;
  BlockTally tally{tally_mem};
  if (LEVEL == kBlock) tally.init();
  const double th = (double)theta;
  const double th2 = th * th;
  float win[H][R::kOut];  // win[H-1] is the newest accurate output
#pragma unroll
  for (int q = 0; q < H; ++q)
#pragma unroll
    for (int o = 0; o < R::kOut; ++o) win[q][o] = 0.0f;
  int fill = 0;
  int rho = 0;  // remaining approximate steps (uniform per group)
  WaveStats st;

  for (int k = 0; k < a.ipt; ++k) {
    const int64_t step0 = (int64_t)k * a.L;
    if (LEVEL != kBlock && wbase + step0 >= a.n) break;
    if (LEVEL == kBlock && bbase + step0 >= a.n) break;
    const int64_t i = l + step0;
    const bool active = l < a.L && i < a.n;
    const bool stable = rho > 0;
    const bool lane_approx = active && stable;
    const bool computes = active && !stable;
    bool crit = false, voted = false;
    if (lane_approx) {
#pragma unroll
      for (int o = 0; o < R::kOut; ++o) a.out[o][i] = win[H - 1][o];
    }
    if (computes) {
      float x[R::kIn], y[R::kOut];
      load_inputs<R>(a, i, x);
      R::eval(x, y);
      store_outputs<R>(a, i, y);
#pragma unroll
      for (int q = 0; q + 1 < H; ++q)
#pragma unroll
        for (int o = 0; o < R::kOut; ++o) win[q][o] = win[q + 1][o];
#pragma unroll
      for (int o = 0; o < R::kOut; ++o) win[H - 1][o] = y[o];
      fill = fill < H ? fill + 1 : H;
      if (fill == H) {
        voted = true;
        crit = rsd_below<H, R::kOut>(win, th, th2);
      }
    }
    const uint64_t amask = ballot(active);
    const uint64_t vmask = ballot(crit);
    const bool any_vote = ballot(voted) != 0;
    bool wave_approx;
    if (LEVEL == kThread) {
      if (stable) rho -= 1;
      else if (crit) rho = psize;
      wave_approx = ballot(lane_approx) != 0;
    } else if (LEVEL == kWaveLvl) {
      wave_approx = stable && amask != 0;
      if (stable) rho -= 1;
      else if (any_vote && majority(popc(vmask), popc(amask))) rho = psize;
    } else {
      // every wave of the block takes part in the tally at every step; the
      // result only matters after an accurate step whose windows were full
      // (before that no lane's criterion holds, so the majority fails)
      bool any;
      const bool pass = tally.decide(k, popc(vmask), popc(amask), &any);
      wave_approx = stable && amask != 0;
      if (stable) rho -= 1;
      else if (pass) rho = psize;
    }
    if (amask && (a.trace || a.counters)) {
      const int nact = popc(amask);
      const int napx = popc(ballot(lane_approx));
      st.add(nact, napx, wave_approx);
      if (a.trace && lane == 0)
        a.trace[(wbase >> 6) * a.ipt + k] = trace_word(any_vote ? popc(vmask) : 0, napx, -1, wave_approx, any_vote);
    }
  }
  st.flush(a.counters);
}

// ------------------------------------------------------------------ probe

__global__ void __launch_bounds__(256) k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

// --------------------------------------------------------------- launchers

static inline dim3 grid_for(const KArgs &a, int block) { return dim3((unsigned)((a.L + block - 1) / block)); }

int64_t iact_lds_bytes(int region, int block, int table_size, int tables_per_wave) {
  const int E = region == 1 ? entry_floats<RegionBSPriceGrad>() : entry_floats<RegionBSPrice>();
  return (int64_t)(block / kWave) * tables_per_wave * table_size * E * (int64_t)sizeof(float);
}

template <class R>
static hipError_t exact_r(const LaunchCfg &c, const KArgs &a) {
  if (a.trace || a.counters)
    hipLaunchKernelGGL((k_exact<R, true>), grid_for(a, c.block), dim3(c.block), 0, c.stream, a);
  else
    hipLaunchKernelGGL((k_exact<R, false>), grid_for(a, c.block), dim3(c.block), 0, c.stream, a);
  return hipGetLastError();
}

hipError_t launch_exact(const LaunchCfg &c, const KArgs &a) {
  return c.region == 1 ? exact_r<RegionBSPriceGrad>(c, a) : exact_r<RegionBSPrice>(c, a);
}

template <class R>
static hipError_t perfo_r(const LaunchCfg &c, const KArgs &a, int kind, int param, int offset) {
  hipLaunchKernelGGL((k_perfo<R>), grid_for(a, c.block), dim3(c.block), 0, c.stream, a, kind, param, offset);
  return hipGetLastError();
}

hipError_t launch_perfo(const LaunchCfg &c, const KArgs &a, int kind, int param, int offset) {
  return c.region == 1 ? perfo_r<RegionBSPriceGrad>(c, a, kind, param, offset)
                       : perfo_r<RegionBSPrice>(c, a, kind, param, offset);
}

template <class R>
static hipError_t iact_r(const LaunchCfg &c, const KArgs &a, int level, int t, float thr, int tpw) {
  const size_t lds = (size_t)iact_lds_bytes(c.region, c.block, t, tpw);
  const dim3 g = grid_for(a, c.block), b(c.block);
  switch (level) {
    case kThread: hipLaunchKernelGGL((k_iact<R, kThread>), g, b, lds, c.stream, a, t, thr, tpw); break;
    case kWaveLvl: hipLaunchKernelGGL((k_iact<R, kWaveLvl>), g, b, lds, c.stream, a, t, thr, tpw); break;
    default: hipLaunchKernelGGL((k_iact<R, kBlock>), g, b, lds, c.stream, a, t, thr, tpw); break;
  }
  return hipGetLastError();
}

hipError_t launch_iact(const LaunchCfg &c, const KArgs &a, int level, int table_size, float threshold,
                       int tables_per_wave) {
  return c.region == 1 ? iact_r<RegionBSPriceGrad>(c, a, level, table_size, threshold, tables_per_wave)
                       : iact_r<RegionBSPrice>(c, a, level, table_size, threshold, tables_per_wave);
}

template <class R, int LEVEL, int H>
static void taf_go(const LaunchCfg &c, const KArgs &a, int p, float thr) {
  hipLaunchKernelGGL((k_taf<R, LEVEL, H>), grid_for(a, c.block), dim3(c.block), 0, c.stream, a, p, thr);
}

template <class R, int LEVEL>
static void taf_h(const LaunchCfg &c, const KArgs &a, int h, int p, float thr) {
  switch (h) {
    case 1: taf_go<R, LEVEL, 1>(c, a, p, thr); break;
    case 2: taf_go<R, LEVEL, 2>(c, a, p, thr); break;
    case 3: taf_go<R, LEVEL, 3>(c, a, p, thr); break;
    case 4: taf_go<R, LEVEL, 4>(c, a, p, thr); break;
    case 5: taf_go<R, LEVEL, 5>(c, a, p, thr); break;
    case 6: taf_go<R, LEVEL, 6>(c, a, p, thr); break;
    case 7: taf_go<R, LEVEL, 7>(c, a, p, thr); break;
    default: taf_go<R, LEVEL, 8>(c, a, p, thr); break;
  }
}

template <class R>
static hipError_t taf_r(const LaunchCfg &c, const KArgs &a, int level, int h, int p, float thr) {
  switch (level) {
    case kThread: taf_h<R, kThread>(c, a, h, p, thr); break;
    case kWaveLvl: taf_h<R, kWaveLvl>(c, a, h, p, thr); break;
    default: taf_h<R, kBlock>(c, a, h, p, thr); break;
  }
  return hipGetLastError();
}

hipError_t launch_taf(const LaunchCfg &c, const KArgs &a, int level, int history_size, int prediction_size,
                      float threshold) {
  return c.region == 1 ? taf_r<RegionBSPriceGrad>(c, a, level, history_size, prediction_size, threshold)
                       : taf_r<RegionBSPrice>(c, a, level, history_size, prediction_size, threshold);
}

hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t stream) {
  const int64_t n4 = bytes / 16;
  int64_t blocks = (n4 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, stream, (const float4 *)src, (float4 *)dst, n4);
  return hipGetLastError();
}

}  // namespace hpac

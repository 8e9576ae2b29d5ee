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
#include "region_half.hpp"
#include "wave.hpp"

#include <math.h>

#include <type_traits>

namespace hpac {

enum { kThread = 0, kWaveLvl = 1, kBlock = 2 };
enum { kSmall = 0, kLarge = 1, kIni = 2, kFini = 3 };

// ------------------------------------------------------------------ helpers

// Regions with an output that names the item whose evaluation produced the
// outputs (RegionBSPriceRef): the accurate path writes the item's own index
// there, as int32 bits; a reused iACT entry carries its source's.
template <class R, class = void>
struct HasIndexOut : std::false_type {};
template <class R>
struct HasIndexOut<R, std::void_t<decltype(R::kIndexOut)>> : std::true_type {};

template <class R>
__device__ __forceinline__ void eval_at(const float (&x)[R::kIn], int64_t i, float (&y)[R::kOut]) {
  R::eval(x, y);
  if constexpr (HasIndexOut<R>::value) y[R::kIndexOut] = __int_as_float((int)i);
}

template <class R>
__device__ __forceinline__ void load_inputs(const KArgs &a, int64_t i, float (&x)[R::kIn]) {
#pragma unroll
  for (int j = 0; j < R::kIn; ++j) x[j] = R::io::load(a.in[j], i);
}

template <class R>
__device__ __forceinline__ void store_outputs(const KArgs &a, int64_t i, const float (&y)[R::kOut]) {
#pragma unroll
  for (int o = 0; o < R::kOut; ++o) R::io::store(a.out[o], i, y[o]);
}

__device__ __forceinline__ uint32_t trace_word(int votes, int napprox, int writer, bool approx, bool voted) {
  uint32_t t = 0x80000000u | (uint32_t)(votes & 0x7F) | ((uint32_t)(napprox & 0x7F) << 8);
  if (writer >= 0) t |= ((uint32_t)writer << 16) | (1u << 22);
  if (approx) t |= 1u << 24;
  if (voted) t |= 1u << 25;
  return t;
}

// Per-wave tallies (wave-uniform).  At kernel end each wave adds them into
// the block's LDS sums and one thread adds those into the caller's counters,
// so a launch issues at most 4 global atomics per workgroup.
struct WaveStats {
  uint64_t lane_steps = 0, approx_lanes = 0, approx_wsteps = 0, wsteps = 0;
  __device__ __forceinline__ void add(int active, int napprox, bool wave_approx) {
    lane_steps += active;
    approx_lanes += napprox;
    approx_wsteps += wave_approx ? 1 : 0;
    wsteps += 1;
  }
};

// Every thread of the block calls begin() and end() (no early returns in the
// kernels), and both are no-ops unless counters were requested.
struct StatsSink {
  unsigned long long *g;  // caller's counters or nullptr
  unsigned long long *s;  // 4 sums in LDS
  __device__ __forceinline__ void begin() {
    if (!g) return;
    if (threadIdx.x < 4) s[threadIdx.x] = 0;
    __syncthreads();
  }
  __device__ __forceinline__ void end(const WaveStats &st) {
    if (!g) return;
    if (lane_id() == 0 && st.wsteps) {
      atomicAdd(&s[0], (unsigned long long)st.lane_steps);
      atomicAdd(&s[1], (unsigned long long)st.approx_lanes);
      atomicAdd(&s[2], (unsigned long long)st.approx_wsteps);
      atomicAdd(&s[3], (unsigned long long)st.wsteps);
    }
    __syncthreads();
    if (threadIdx.x < 4 && s[threadIdx.x]) atomicAdd(&g[threadIdx.x], s[threadIdx.x]);
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
  __device__ __forceinline__ bool decide(int k, int wave_votes, int wave_active) {
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
    return majority(cur[0], cur[1]);
  }
};

// Geometry of one lane in the grid-stride loop.
struct LaneGeom {
  int64_t l;      // logical lane
  int64_t wbase;  // first lane of the wave
  int64_t bbase;  // first lane of the block
  __device__ __forceinline__ LaneGeom() : LaneGeom((int64_t)blockIdx.x) {}
  // the lanes of workgroup `block` of the full grid
  __device__ __forceinline__ explicit LaneGeom(int64_t block) {
    bbase = block * blockDim.x;
    l = bbase + threadIdx.x;
    wbase = l - lane_id();
  }
  // the wave (or block) has an active lane at step k
  __device__ __forceinline__ bool wave_has(const KArgs &a, int k) const {
    return wbase < a.L && wbase + (int64_t)k * a.L < a.n;
  }
  __device__ __forceinline__ bool block_has(const KArgs &a, int k) const { return bbase + (int64_t)k * a.L < a.n; }
  __device__ __forceinline__ bool active(const KArgs &a, int k) const {
    return l < a.L && l + (int64_t)k * a.L < a.n;
  }
  __device__ __forceinline__ int64_t item(const KArgs &a, int k) const { return l + (int64_t)k * a.L; }
  __device__ __forceinline__ int64_t trace_index(const KArgs &a, int k) const { return (wbase >> 6) * a.ipt + k; }
};

// Inputs of the next step are loaded while the current step computes
// (software pipelining).  The loads are issued unconditionally so that the
// compiler can count them exactly and wait only for the ones it needs: a lane
// that does not need step k's inputs loads the wave's first item of step
// k-1 instead, a line the wave has just fetched, which costs no HBM traffic.
template <class R>
__device__ __forceinline__ void prefetch(const KArgs &a, const LaneGeom &g, int k, bool want, float (&xn)[R::kIn]) {
  int64_t i = g.item(a, k);
  if (!(want && k < a.ipt && g.active(a, k))) {
    i = g.wbase + (int64_t)(k - 1) * a.L;
    if (i >= a.n) i = a.n - 1;
  }
  load_inputs<R>(a, i, xn);
}

// Inputs of the first step (before the loop; conditional).
template <class R>
__device__ __forceinline__ void load_first(const KArgs &a, const LaneGeom &g, bool want, float (&x)[R::kIn]) {
  if (want && g.active(a, 0)) load_inputs<R>(a, g.item(a, 0), x);
}

// Runs step(k, x_k, x_{k+1}) for k = 0, 1, ... while it returns true.
template <int N, class Step>
__device__ __forceinline__ void step_loop(int ipt, float (&xa)[N], float (&xb)[N], Step step) {
  for (int k = 0; k < ipt; k += 2) {
    if (!step(k, xa, xb)) break;
    if (k + 1 >= ipt || !step(k + 1, xb, xa)) break;
  }
}

// --------------------------------------------------------------- exact path

// The counted variants (kStats, k_perfo) run a grid of at most
// kCountedGrid workgroups that stride over the workgroups of the full grid:
// each physical workgroup adds into the caller's counters once, since
// same-address atomics from tens of thousands of workgroups serialize.
constexpr unsigned kCountedGrid = 2048;

template <class R, bool kStats>
__global__ void __launch_bounds__(256) k_exact(KArgs a) {
  __shared__ unsigned long long sums[4];
  StatsSink sink{kStats ? a.counters : nullptr, sums};
  sink.begin();
  WaveStats st;
  auto run_block = [&](int64_t b) {
    const LaneGeom g(b);
    float xa[R::kIn], xb[R::kIn];
    load_first<R>(a, g, true, xa);
    step_loop(a.ipt, xa, xb, [&](int k, float (&x)[R::kIn], float (&xn)[R::kIn]) {
      if (!g.wave_has(a, k)) return false;
      const bool active = g.active(a, k);
      prefetch<R>(a, g, k + 1, true, xn);
      if (active) {
        float y[R::kOut];
        eval_at<R>(x, g.item(a, k), y);
        store_outputs<R>(a, g.item(a, k), y);
      }
      if (kStats) {
        st.add(popc(ballot(active)), 0, false);
        if (a.trace && lane_id() == 0) a.trace[g.trace_index(a, k)] = trace_word(0, 0, -1, false, false);
      }
      return true;
    });
  };
  if (kStats) {
    const int64_t blocks = (a.L + blockDim.x - 1) / blockDim.x;
    for (int64_t b = blockIdx.x; b < blocks; b += gridDim.x) run_block(b);
  } else if (a.ipt == 1) {
    // one item per lane: no next step to prefetch
    const LaneGeom g;
    if (g.active(a, 0)) {
      float x[R::kIn], y[R::kOut];
      load_inputs<R>(a, g.item(a, 0), x);
      eval_at<R>(x, g.item(a, 0), y);
      store_outputs<R>(a, g.item(a, 0), y);
    }
  } else {
    run_block(blockIdx.x);  // the uncounted grid is the full grid
  }
  sink.end(st);
}

// Regions that evaluate a pair of items at once (packed arithmetic).
template <class R, class = void>
struct IsPaired : std::false_type {};
template <class R>
struct IsPaired<R, std::void_t<decltype(R::kPaired)>> : std::bool_constant<R::kPaired> {};

// Exact path of a paired region, uncounted, items per lane >= 2: steps k and
// k + 1 of a lane go through one packed evaluation.  Same lanes and items as
// k_exact; an odd last step is paired with a copy of itself.
template <class R>
__global__ void __launch_bounds__(256) k_exact_pairs(KArgs a) {
  const LaneGeom g;
  for (int k = 0; k < a.ipt; k += 2) {
    if (!g.wave_has(a, k)) return;
    const bool act0 = g.active(a, k);
    const bool act1 = k + 1 < a.ipt && g.active(a, k + 1);
    float x0[R::kIn], x1[R::kIn];
    if (act0) load_inputs<R>(a, g.item(a, k), x0);
    if (act1) load_inputs<R>(a, g.item(a, k + 1), x1);
    if (act0) {
      if (!act1)
#pragma unroll
        for (int j = 0; j < R::kIn; ++j) x1[j] = x0[j];
      float y0[R::kOut], y1[R::kOut];
      R::eval2(x0, x1, y0, y1);
      store_outputs<R>(a, g.item(a, k), y0);
      if (act1) store_outputs<R>(a, g.item(a, k + 1), y1);
    }
  }
}

// ---------------------------------------------------------------- perforation

struct PerfoRule {
  int kind, param, offset;
  int64_t cut;
  // herded: the step rule is identical for every lane
  __device__ __forceinline__ bool step_skipped(int64_t k) const {
    const int64_t kk = k + offset;
    if (kind == kSmall) return param > 0 && (kk % param) == param - 1;
    if (kind == kLarge) return param > 0 && (kk % param) != 0;
    return false;
  }
  __device__ __forceinline__ bool skipped(int64_t k, int64_t i, int64_t n) const {
    if (kind == kIni) return i < cut;
    if (kind == kFini) return i >= n - cut;
    return step_skipped(k);
  }
};

// Perforation with the per-(wave, step) trace and counters.
template <class R>
__global__ void __launch_bounds__(256) k_perfo(KArgs a, int kind, int param, int offset) {
  __shared__ unsigned long long sums[4];
  StatsSink sink{a.counters, sums};
  sink.begin();
  const PerfoRule rule{kind, param, offset, (kind == kIni || kind == kFini) ? ((int64_t)param * a.n) / 100 : 0};
  WaveStats st;
  const int64_t blocks = (a.L + blockDim.x - 1) / blockDim.x;
  for (int64_t b = blockIdx.x; b < blocks; b += gridDim.x) {
    const LaneGeom g(b);
    float xa[R::kIn], xb[R::kIn];
    load_first<R>(a, g, !rule.skipped(0, g.item(a, 0), a.n), xa);
    step_loop(a.ipt, xa, xb, [&](int k, float (&x)[R::kIn], float (&xn)[R::kIn]) {
      if (!g.wave_has(a, k)) return false;
      const int64_t i = g.item(a, k);
      const bool active = g.active(a, k);
      const bool skip = rule.skipped(k, i, a.n);
      // the next executed step's inputs; dropped steps load nothing
      prefetch<R>(a, g, k + 1, !rule.skipped(k + 1, g.item(a, k + 1), a.n), xn);
      if (active && !skip) {
        float y[R::kOut];
        R::eval(x, y);
        store_outputs<R>(a, i, y);
      }
      if (a.trace || a.counters) {
        const int nact = popc(ballot(active));
        const int nskip = popc(ballot(active && skip));
        st.add(nact, nskip, nskip > 0);
        if (a.trace && lane_id() == 0) a.trace[g.trace_index(a, k)] = trace_word(0, nskip, -1, nskip > 0, false);
      }
      return true;
    });
  }
  sink.end(st);
}

// Perforation without trace or counters.  The region keeps no state, so the
// items a herded pattern keeps -- whole grid-stride steps, i.e. the item
// ranges [kL, (k+1)L) of the kept steps k -- can be evaluated by any lanes:
// one item per lane, workgroups mapped onto the kept ranges, dropped ranges
// never launched.  The outputs are those of k_perfo bit for bit.
// Kept steps repeat with period M: SMALL keeps every position of a period
// but `special`, LARGE keeps only `special`.  The grid is (workgroups per
// step, kept positions per period, periods), so a workgroup finds its step
// without an integer division (one on each wave's path to its first load
// cost the launch 8%).
template <class R>
__global__ void __launch_bounds__(256) k_perfo_dense(KArgs a, int64_t steps, int M, int special, int large) {
  const int r = blockIdx.y;
  const int s = large ? special : (r < special ? r : r + 1);
  const int64_t k = (int64_t)blockIdx.z * M + s;
  if (k >= steps) return;  // past the last step of a partial period
  const int64_t i = k * a.L + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t end = (k + 1) * a.L < a.n ? (k + 1) * a.L : a.n;
  if (i < end) {
    float x[R::kIn], y[R::kOut];
    load_inputs<R>(a, i, x);
    R::eval(x, y);
    store_outputs<R>(a, i, y);
  }
}

// ------------------------------------------------------------------- iACT

template <class R>
constexpr int entry_floats() { return (R::kIn + R::kOut + 3) & ~3; }

// LDS layout of a wave's tables.  With several tables per wave the lanes
// read the same word of different tables at once: tables one float more
// than their size apart (an odd stride) put those words in different banks,
// when that still fits the workgroup's 64 KiB of LDS; otherwise the tables
// are interleaved word by word (word j of entry e of table t at
// (e * entry + j) * tables + t), which needs no pad and is read conflict-free
// at the price of computed addresses.
constexpr int64_t kIactLdsLimit = 65536;
__host__ __device__ inline bool iact_interleaved(int entry, int block, int tsize, int tpw) {
  return tpw > 1 && (int64_t)(block / kWave) * tpw * (tsize * entry + 1) * 4 > kIactLdsLimit;
}
__host__ __device__ inline int iact_table_stride(int entry, int block, int tsize, int tpw) {
  return iact_interleaved(entry, block, tsize, tpw) ? tsize * entry : tsize * entry + 1;
}

// Squared Euclidean distance in FP32 with a fixed rounding sequence:
// t0*t0, then fma(tj, tj, acc).  No other contraction is allowed here.
template <int N, int WS = 1>
__device__ __forceinline__ float dist2(const float (&x)[N], const float *e, int ws = WS) {
#pragma clang fp contract(off)
  float t = x[0] - e[0];
  float acc = t * t;
#pragma unroll
  for (int j = 1; j < N; ++j) {
    const float u = x[j] - e[j * ws];
    acc = __builtin_fmaf(u, u, acc);
  }
  return acc;
}

// kOne: one table per wave (tpw == 1), compiled apart so that the
// compiler sees the table count and insertion slot as wave-uniform values
// (uniform search loop, no per-lane segment arithmetic) and the writer is
// elected on integer keys by a folded DPP max.
template <class R, int LEVEL, bool kInterleaved, bool kOne = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) k_iact(KArgs a, int tsize, float theta,
                                                                                       int tpw) {
  extern __shared__ float lds[];
  __shared__ int tally_mem[6];
  __shared__ unsigned long long sums[4];
  constexpr int E = entry_floats<R>();
  const LaneGeom g;
  const int lane = lane_id();
  const int wib = threadIdx.x >> 6;
  if (kOne) tpw = 1;
  const int lpt = kWave / tpw;  // lanes per table
  const int tab_in_wave = kOne ? 0 : lane / lpt;
  // word j of entry e of this lane's table: tab[(e * E + j) * ws]
  const int ws = kInterleaved ? tpw : 1;
  float *tab = kInterleaved ? lds + (size_t)wib * tpw * tsize * E + tab_in_wave
                            : lds + ((size_t)wib * tpw + tab_in_wave) * iact_table_stride(E, blockDim.x, tsize, tpw);
  StatsSink sink{a.counters, sums};
  sink.begin();
  BlockTally tally{tally_mem};
  if (LEVEL == kBlock) tally.init();
  const float thr2 = theta * theta;
  const int seg0 = tab_in_wave * lpt;
  const uint64_t segmask = kOne || lpt == kWave ? ~0ull : (((1ull << lpt) - 1) << seg0);
  int cnt = 0, ins = 0;  // valid entries of this lane's table, and its next slot (insertions mod size)
  WaveStats st;
  float xa[R::kIn], xb[R::kIn];
  load_first<R>(a, g, true, xa);

  step_loop(a.ipt, xa, xb, [&](int k, float (&x)[R::kIn], float (&xn)[R::kIn]) {
    if (LEVEL != kBlock && !g.wave_has(a, k)) return false;
    if (LEVEL == kBlock && !g.block_has(a, k)) return false;
    const int64_t i = g.item(a, k);
    const bool active = g.active(a, k);
    prefetch<R>(a, g, k + 1, true, xn);
    // read phase: distance to the nearest valid entry of this lane's table
    float md2 = INFINITY;
    if (active)
      for (int e = 0; e < cnt; ++e) md2 = fminf(md2, dist2<R::kIn>(x, tab + e * E * ws, ws));
    const bool hit = active && cnt > 0 && md2 < thr2;
    const uint64_t amask = ballot(active);
    const uint64_t vmask = ballot(hit);
    bool group_approx;
    if (LEVEL == kThread) group_approx = hit;
    else if (LEVEL == kWaveLvl) group_approx = majority(popc(vmask), popc(amask));
    else group_approx = tally.decide(k, popc(vmask), popc(amask));
    const bool lane_approx = active && group_approx && cnt > 0;
    const bool computes = active && !lane_approx;
    float y[R::kOut];
    if (lane_approx) {
      // the nearest entry: lowest slot at the minimum distance (recomputing
      // the identical FP32 distances)
      int arg = 0;
      for (int e = cnt - 1; e >= 0; --e)
        if (dist2<R::kIn>(x, tab + e * E * ws, ws) == md2) arg = e;
#pragma unroll
      for (int o = 0; o < R::kOut; ++o) y[o] = tab[(arg * E + R::kIn + o) * ws];
    }
    if (computes) eval_at<R>(x, i, y);
    if (active) store_outputs<R>(a, i, y);
    // write phase: one writer per table among the lanes that computed
    const uint64_t cmask = ballot(computes);
    int writer0 = -1;
    if (cmask) {
      uint64_t cand;
      if (kOne) {
        // keys: the distance's bits plus one (order-preserving for
        // non-negative floats, +inf included), 0 for lanes that do not compute
        // (the scan runs on every lane, outside the short-circuit below)
        const uint32_t key = computes ? __float_as_uint(md2) + 1u : 0u;
        const uint32_t m = wave_umax(key);
        cand = ballot(computes && key == m);
      } else {
        const float key = computes ? md2 : -1.0f;
        const float m = segment_max(key, lpt);
        cand = ballot(computes && key == m);
      }
      const uint64_t mine = cand & segmask;
      if (mine) {
        if (lane == lowest_lane(mine)) {
          float *slot = tab + ins * E * ws;
#pragma unroll
          for (int j = 0; j < R::kIn; ++j) slot[j * ws] = x[j];
#pragma unroll
          for (int o = 0; o < R::kOut; ++o) slot[(R::kIn + o) * ws] = y[o];
        }
        cnt = cnt < tsize ? cnt + 1 : tsize;
        ins = ins + 1 == tsize ? 0 : ins + 1;
      }
      const uint64_t cand0 = cand & (kOne || lpt == kWave ? ~0ull : ((1ull << lpt) - 1));
      writer0 = cand0 ? lowest_lane(cand0) : -1;
      wave_lds_fence();
    }
    if (amask && (a.trace || a.counters)) {
      const int nact = popc(amask);
      const int napx = popc(ballot(lane_approx));
      const bool wave_approx = LEVEL == kThread ? napx > 0 : group_approx;
      st.add(nact, napx, wave_approx);
      if (a.trace && lane == 0)
        a.trace[g.trace_index(a, k)] = trace_word(popc(vmask), napx, writer0, wave_approx, true);
    }
    return true;
  });
  sink.end(st);
}

// -------------------------------------------------------------------- TAF

// RSD criterion of one lane in FP64 over every output o of the window:
// with s = sum_q w_q and D = sum_q (h w_q - s)^2 (= h^3 var), the test
// var < theta^2 mu^2 is D < h theta^2 s^2, and var == 0 is D == 0, which
// passes whenever theta > 0.  No division is needed.
template <int H, int NO>
__device__ __forceinline__ bool rsd_below(const float (&w)[H][NO], double th2, bool th_pos) {
  bool ok = true;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < H; ++q) s += (double)w[q][o];
    double D = 0.0;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      const double d = (double)H * (double)w[q][o] - s;
      D = __builtin_fma(d, d, D);
    }
    const bool v = D == 0.0 ? th_pos : D < (double)H * th2 * (s * s);
    ok = ok && v;
  }
  return ok;
}

// TAF state carried between launches (caller-owned, zeroed before the
// first one), per logical lane l of the launch's L lanes: the window, word
// (q * NO + o) * L + l (q = H - 1 the newest output), then the window's fill
// and the group's remaining approximate steps as int32[L] each.  A launch
// with a state starts from it and leaves its own end state there, so lane l
// continues its sequence of steps across launches of the same shape.
template <int H, int NO>
struct TafState {
  float *base;
  int64_t L;
  __device__ __forceinline__ float *word(int q, int o) const { return base + ((int64_t)q * NO + o) * L; }
  __device__ __forceinline__ int32_t *fill() const { return (int32_t *)(base + (int64_t)H * NO * L); }
  __device__ __forceinline__ int32_t *rho() const { return fill() + L; }
  __device__ __forceinline__ void load(int64_t l, float (&w)[H][NO], int &f, int &r) const {
#pragma unroll
    for (int q = 0; q < H; ++q)
#pragma unroll
      for (int o = 0; o < NO; ++o) w[q][o] = word(q, o)[l];
    f = fill()[l];
    r = rho()[l];
  }
  __device__ __forceinline__ void store(int64_t l, const float (&w)[H][NO], int f, int r) const {
#pragma unroll
    for (int q = 0; q < H; ++q)
#pragma unroll
      for (int o = 0; o < NO; ++o) word(q, o)[l] = w[q][o];
    fill()[l] = f;
    rho()[l] = r;
  }
};

template <class R, int LEVEL, int H>
__global__ void __launch_bounds__(256) k_taf(KArgs a, int psize, float theta, float *state) {
  __shared__ int tally_mem[6];
  __shared__ unsigned long long sums[4];
  const LaneGeom g;
  const int lane = lane_id();
  StatsSink sink{a.counters, sums};
  sink.begin();
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
  const TafState<H, R::kOut> ts{state, a.L};
  if (state && g.l < a.L) ts.load(g.l, win, fill, rho);
  bool prev_stable = false;
  WaveStats st;
  float xa[R::kIn], xb[R::kIn];
  load_first<R>(a, g, true, xa);

  step_loop(a.ipt, xa, xb, [&](int k, float (&x)[R::kIn], float (&xn)[R::kIn]) {
    if (LEVEL != kBlock && !g.wave_has(a, k)) return false;
    if (LEVEL == kBlock && !g.block_has(a, k)) return false;
    const int64_t i = g.item(a, k);
    const bool active = g.active(a, k);
    const bool stable = rho > 0;
    const bool lane_approx = active && stable;
    const bool computes = active && !stable;
    // Inputs of step k+1 are needed unless it is certainly approximate
    // (this step is approximate with more to come).  At wave level, the
    // first accurate step after an approximate run is the step whose vote
    // most likely passes again: its prefetch waits for the vote, so that a
    // passing vote loads nothing.  Elsewhere step k+1's loads are issued
    // before step k computes, and a passing vote leaves them unused.
    const bool late = LEVEL == kWaveLvl && !stable && prev_stable;
    prev_stable = stable;
    if (!late) prefetch<R>(a, g, k + 1, !stable || rho == 1, xn);
    bool crit = false, voted = false;
    if (lane_approx) store_outputs<R>(a, i, win[H - 1]);
    if (computes) {
      float y[R::kOut];
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
        crit = rsd_below<H, R::kOut>(win, th2, th > 0.0);
      }
    }
    const uint64_t amask = ballot(active);
    const uint64_t vmask = ballot(crit);
    const bool any_vote = ballot(voted) != 0;
    bool wave_approx;
    bool pass = false;
    if (LEVEL == kThread) {
      pass = crit;
      wave_approx = ballot(lane_approx) != 0;
    } else if (LEVEL == kWaveLvl) {
      pass = any_vote && majority(popc(vmask), popc(amask));
      wave_approx = stable && amask != 0;
    } else {
      // every wave of the block takes part in the tally at every step; the
      // result only matters after an accurate step whose windows were full
      // (before that no lane's criterion holds, so the majority fails)
      pass = tally.decide(k, popc(vmask), popc(amask)) && !stable;
      wave_approx = stable && amask != 0;
    }
    if (late) prefetch<R>(a, g, k + 1, !pass, xn);
    if (stable) rho -= 1;
    else if (pass) rho = psize;
    if (amask && (a.trace || a.counters)) {
      const int nact = popc(amask);
      const int napx = popc(ballot(lane_approx));
      st.add(nact, napx, wave_approx);
      if (a.trace && lane == 0)
        a.trace[g.trace_index(a, k)] = trace_word(any_vote ? popc(vmask) : 0, napx, -1, wave_approx, any_vote);
    }
    return true;
  });
  if (state && g.l < a.L) ts.store(g.l, win, fill, rho);
  sink.end(st);
}

// Wave-level TAF as a loop over runs: one accurate step (region, window,
// vote), then, if the wave votes to approximate, psize approximate steps
// that only store the last output.  The inputs of the next accurate step are
// loaded right after the vote: before the psize stores of a run, or, when
// the vote fails, before the next step.  Only when the previous vote failed
// is the next step's load issued speculatively before the region computes
// (the vote is then likely to fail again); a pass wastes that load once.
// Same decisions as k_taf at wave level.  kState: a launch with a
// persistent state (compiled apart, so that the launch-scoped path carries
// none of its code).
template <class R, int H, bool kState>
__global__ void __launch_bounds__(256) k_taf_wave(KArgs a, int psize, float theta, float *state) {
  __shared__ unsigned long long sums[4];
  const LaneGeom g;
  const int lane = lane_id();
  StatsSink sink{a.counters, sums};
  sink.begin();
  const double th = (double)theta;
  const double th2 = th * th;
  float win[H][R::kOut];  // win[H-1] is the newest accurate output
#pragma unroll
  for (int q = 0; q < H; ++q)
#pragma unroll
    for (int o = 0; o < R::kOut; ++o) win[q][o] = 0.0f;
  int fill = 0;
  bool prev_pass = false;
  WaveStats st;
  // with a state: the window, and the approximate steps still owed to the
  // previous launch's last passing vote (the same for every lane of a wave)
  const TafState<H, R::kOut> ts{state, a.L};
  int owed = 0;
  if (kState && g.l < a.L) ts.load(g.l, win, fill, owed);
  owed = __builtin_amdgcn_readfirstlane(owed);
  int k = 0;
  for (; k < owed && k < a.ipt && g.wave_has(a, k); ++k) {
    const bool act = g.active(a, k);
    if (act) store_outputs<R>(a, g.item(a, k), win[H - 1]);
    if (a.trace || a.counters) {
      const int nact = popc(ballot(act));
      st.add(nact, nact, true);
      if (a.trace && lane == 0) a.trace[g.trace_index(a, k)] = trace_word(0, nact, -1, true, false);
    }
  }
  int left = owed - k > 0 ? owed - k : 0;  // still owed when the launch ends
  float x[R::kIn], xn[R::kIn];
#pragma unroll
  for (int j = 0; j < R::kIn; ++j) xn[j] = 0.0f;
  if (k < a.ipt && g.active(a, k)) load_inputs<R>(a, g.item(a, k), xn);
  while (k < a.ipt && g.wave_has(a, k)) {
#pragma unroll
    for (int j = 0; j < R::kIn; ++j) x[j] = xn[j];
    const bool active = g.active(a, k);
    const int64_t i = g.item(a, k);
    if (!prev_pass && k + 1 < a.ipt && g.active(a, k + 1)) load_inputs<R>(a, g.item(a, k + 1), xn);
    bool crit = false, voted = false;
    if (active) {
      float y[R::kOut];
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
        crit = rsd_below<H, R::kOut>(win, th2, th > 0.0);
      }
    }
    const uint64_t amask = ballot(active);
    const uint64_t vmask = ballot(crit);
    const bool any_vote = ballot(voted) != 0;
    const bool pass = any_vote && majority(popc(vmask), popc(amask));
    const int next = pass ? k + psize + 1 : k + 1;
    if ((prev_pass || pass) && next < a.ipt && g.active(a, next)) load_inputs<R>(a, g.item(a, next), xn);
    if (a.trace || a.counters) {
      st.add(popc(amask), 0, false);
      if (a.trace && lane == 0)
        a.trace[g.trace_index(a, k)] = trace_word(any_vote ? popc(vmask) : 0, 0, -1, false, any_vote);
    }
    left = 0;
    if (pass) {
      int kk = k + 1;
      for (; kk < next && kk < a.ipt && g.wave_has(a, kk); ++kk) {
        const bool act = g.active(a, kk);
        if (act) store_outputs<R>(a, g.item(a, kk), win[H - 1]);
        if (a.trace || a.counters) {
          const int nact = popc(ballot(act));
          st.add(nact, nact, true);
          if (a.trace && lane == 0) a.trace[g.trace_index(a, kk)] = trace_word(0, nact, -1, true, false);
        }
      }
      left = next - kk;
    }
    prev_pass = pass;
    k = next;
  }
  if (kState && g.l < a.L) ts.store(g.l, win, fill, left);
  sink.end(st);
}

// ------------------------------------------------------------------ probe

__global__ void __launch_bounds__(256) k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

// VALU issue rate: 8 independent FMA chains per lane.  With kScalar the
// multiplier and addend stay wave-uniform (scalar-register operands); else
// each lane holds its own copy (a + 0 * lane is not folded: it is -0 or NaN
// for some a), so every operand is a vector register.
template <bool kScalar>
__global__ void __launch_bounds__(256) k_probe_valu(float *out, int iters, float a, float b) {
  const float lanef = (float)threadIdx.x;
  const float av = kScalar ? a : a + 0.0f * lanef, bv = kScalar ? b : b + 0.0f * lanef;
  float r[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = lanef * 1e-3f + (float)j;
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int j = 0; j < 8; ++j) r[j] = __builtin_fmaf(r[j], av, bv);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += r[j];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// --------------------------------------------------------------- launchers

static inline dim3 grid_for(const KArgs &a, int block) { return dim3((unsigned)((a.L + block - 1) / block)); }
static inline dim3 counted_grid(const KArgs &a, int block) {
  const dim3 g = grid_for(a, block);
  return dim3(g.x < kCountedGrid ? g.x : kCountedGrid);
}

static_assert(entry_floats<RegionBSPriceRef>() == entry_floats<RegionBSPrice>(), "source-item entries");

int64_t iact_lds_bytes(int region, int block, int table_size, int tables_per_wave) {
  const int E = region == 1 ? entry_floats<RegionBSPriceGrad>() : entry_floats<RegionBSPrice>();
  return (int64_t)(block / kWave) * tables_per_wave * iact_table_stride(E, block, table_size, tables_per_wave) *
         (int64_t)sizeof(float);
}

// (region, column type) -> region type.  Regions: 0 price, 1 price and
// Jacobian, 2 price in FP16, 3 price at BF16 precision, 5 price and source
// item (exact and iACT only).  Column types: 0 FP32, 1 FP16, 2 BF16.  The
// half-precision bodies pair with FP32 columns or with columns of their own
// type; the Jacobian and source-item regions take FP32 columns only.
bool region_dtype_supported(int region, int dtype) {
  switch (region) {
    case 0: return dtype >= 0 && dtype <= 2;
    case 1: return dtype == 0;
    case 5: return dtype == 0;
    case 2: return dtype == 0 || dtype == 1;
    case 3: return dtype == 0 || dtype == 2;
    default: return false;
  }
}

template <bool kIndexRegions = false, class F>
static hipError_t with_region(int region, int dtype, const F &f) {
  if constexpr (kIndexRegions) {
    if (region == 5 && dtype == 0) return f.template go<RegionBSPriceRef>();
  }
  switch (region * 4 + dtype) {
    case 0: return f.template go<RegionBSPrice>();
    case 1: return f.template go<WithIo<RegionBSPrice, IoF16>>();
    case 2: return f.template go<WithIo<RegionBSPrice, IoBF16>>();
    case 4: return f.template go<RegionBSPriceGrad>();
    case 8: return f.template go<RegionBSPriceF16>();
    case 9: return f.template go<WithIo<RegionBSPriceF16, IoF16>>();
    case 12: return f.template go<RegionBSPriceBF16>();
    case 14: return f.template go<WithIo<RegionBSPriceBF16, IoBF16>>();
    default: return hipErrorInvalidValue;
  }
}

struct ExactL {
  const LaunchCfg &c;
  const KArgs &a;
  template <class R>
  hipError_t go() const {
    if (a.ipt > 1) return run<Streamed<R>>();
    return run<R>();
  }
  template <class R>
  hipError_t run() const {
    if (a.trace || a.counters)
      hipLaunchKernelGGL((k_exact<R, true>), counted_grid(a, c.block), dim3(c.block), 0, c.stream, a);
    else if constexpr (IsPaired<R>::value) {
      if (a.ipt >= 2)
        hipLaunchKernelGGL((k_exact_pairs<R>), grid_for(a, c.block), dim3(c.block), 0, c.stream, a);
      else
        hipLaunchKernelGGL((k_exact<R, false>), grid_for(a, c.block), dim3(c.block), 0, c.stream, a);
    } else {
      hipLaunchKernelGGL((k_exact<R, false>), grid_for(a, c.block), dim3(c.block), 0, c.stream, a);
    }
    return hipGetLastError();
  }
};

hipError_t launch_exact(const LaunchCfg &c, const KArgs &a) {
  return with_region<true>(c.region, c.dtype, ExactL{c, a});
}

// A dispatch's grid size is a 32-bit count of lanes per dimension; the
// second and third dimensions are kept within 65535 workgroups.
constexpr int64_t kMaxGridLanes = 0xFFFFFFFFll;
constexpr int64_t kMaxGridYZ = 65535;

struct PerfoL {
  const LaunchCfg &c;
  const KArgs &a;
  int kind, param, offset;
  // the per-(wave, step) kernel on at most kCountedGrid workgroups
  template <class R>
  hipError_t counted_launch() const {
    hipLaunchKernelGGL((k_perfo<R>), counted_grid(a, c.block), dim3(c.block), 0, c.stream, a, kind, param, offset);
    return hipGetLastError();
  }
  template <class R>
  hipError_t go() const {
    // the dense paths launch one lane per kept item, unless that grid
    // would exceed the dispatch's 32-bit lane count
    auto counted = [&] { return counted_launch<R>(); };
    if (a.trace || a.counters || param == 0) return counted();
    if (kind == kIni || kind == kFini) {
      // a contiguous kept range: the exact kernel over it, one item per lane
      const int64_t cut = ((int64_t)param * a.n) / 100;
      KArgs b = a;
      const int64_t lo = kind == kIni ? cut : 0;
      const int64_t esz = sizeof(typename R::io::elem);
      b.n = a.n - cut;
      b.ipt = 1;
      b.L = ((b.n + 63) / 64) * 64;
      for (int j = 0; j < R::kIn; ++j) b.in[j] = (const char *)a.in[j] + lo * esz;
      for (int o = 0; o < R::kOut; ++o) b.out[o] = (char *)a.out[o] + lo * esz;
      if (b.n == 0) return hipSuccess;
      if ((int64_t)grid_for(b, c.block).x * c.block > kMaxGridLanes) return counted();
      hipLaunchKernelGGL((k_exact<R, false>), grid_for(b, c.block), dim3(c.block), 0, c.stream, b);
      return hipGetLastError();
    }
    // SMALL / LARGE: kept steps repeat with period M
    const int M = param;
    const int off = (int)(offset % M);
    const int special = kind == kSmall ? ((M - 1 - off) % M + M) % M : ((M - off) % M + M) % M;
    const int kept_per_period = kind == kSmall ? M - 1 : 1;
    if (kept_per_period == 0) return hipSuccess;  // SMALL with M = 1 drops every step
    const int64_t steps = (a.n + a.L - 1) / a.L;  // steps that hold items
    // kept steps below `steps`
    int64_t kept = (steps / M) * kept_per_period;
    for (int64_t st = (steps / M) * M; st < steps; ++st) {
      const int pos = (int)(st % M);
      kept += kind == kSmall ? pos != special : pos == special;
    }
    if (kept == 0) return hipSuccess;
    const int64_t bps = (a.L + c.block - 1) / c.block;
    const int64_t periods = (steps + M - 1) / M;
    if (bps * c.block > kMaxGridLanes || periods > kMaxGridYZ || kept_per_period > kMaxGridYZ) return counted();
    hipLaunchKernelGGL((k_perfo_dense<R>), dim3((unsigned)bps, (unsigned)kept_per_period, (unsigned)periods),
                       dim3(c.block), 0, c.stream, a, steps, M, special, kind == kLarge ? 1 : 0);
    return hipGetLastError();
  }
};

hipError_t launch_perfo(const LaunchCfg &c, const KArgs &a, int kind, int param, int offset) {
  return with_region(c.region, c.dtype, PerfoL{c, a, kind, param, offset});
}

struct IactL {
  const LaunchCfg &c;
  const KArgs &a;
  int level, t;
  float thr;
  int tpw;
  template <class R0>
  hipError_t go() const {
    using R = Streamed<R0>;
    const size_t lds = (size_t)iact_lds_bytes(c.region, c.block, t, tpw);
    if (tpw == 1) return launch<R, false, true>(lds);
    if (iact_interleaved(entry_floats<R>(), c.block, t, tpw)) return launch<R, true, false>(lds);
    return launch<R, false, false>(lds);
  }
  template <class R, bool kIl, bool kOne>
  hipError_t launch(size_t lds) const {
    const dim3 g = grid_for(a, c.block), b(c.block);
    switch (level) {
      case kThread: hipLaunchKernelGGL((k_iact<R, kThread, kIl, kOne>), g, b, lds, c.stream, a, t, thr, tpw); break;
      case kWaveLvl: hipLaunchKernelGGL((k_iact<R, kWaveLvl, kIl, kOne>), g, b, lds, c.stream, a, t, thr, tpw); break;
      default: hipLaunchKernelGGL((k_iact<R, kBlock, kIl, kOne>), g, b, lds, c.stream, a, t, thr, tpw); break;
    }
    return hipGetLastError();
  }
};

hipError_t launch_iact(const LaunchCfg &c, const KArgs &a, int level, int table_size, float threshold,
                       int tables_per_wave) {
  return with_region<true>(c.region, c.dtype, IactL{c, a, level, table_size, threshold, tables_per_wave});
}

template <class R, int LEVEL, int H>
static void taf_go(const LaunchCfg &c, const KArgs &a, int p, float thr, float *st) {
  if constexpr (LEVEL == kWaveLvl) {
    if (st)
      hipLaunchKernelGGL((k_taf_wave<R, H, true>), grid_for(a, c.block), dim3(c.block), 0, c.stream, a, p, thr, st);
    else
      hipLaunchKernelGGL((k_taf_wave<R, H, false>), grid_for(a, c.block), dim3(c.block), 0, c.stream, a, p, thr, st);
  } else {
    hipLaunchKernelGGL((k_taf<R, LEVEL, H>), grid_for(a, c.block), dim3(c.block), 0, c.stream, a, p, thr, st);
  }
}

template <class R, int LEVEL>
static void taf_h(const LaunchCfg &c, const KArgs &a, int h, int p, float thr, float *st) {
  switch (h) {
    case 1: taf_go<R, LEVEL, 1>(c, a, p, thr, st); break;
    case 2: taf_go<R, LEVEL, 2>(c, a, p, thr, st); break;
    case 3: taf_go<R, LEVEL, 3>(c, a, p, thr, st); break;
    case 4: taf_go<R, LEVEL, 4>(c, a, p, thr, st); break;
    case 5: taf_go<R, LEVEL, 5>(c, a, p, thr, st); break;
    case 6: taf_go<R, LEVEL, 6>(c, a, p, thr, st); break;
    case 7: taf_go<R, LEVEL, 7>(c, a, p, thr, st); break;
    default: taf_go<R, LEVEL, 8>(c, a, p, thr, st); break;
  }
}

struct TafL {
  const LaunchCfg &c;
  const KArgs &a;
  int level, h, p;
  float thr;
  float *st;
  template <class R0>
  hipError_t go() const {
    using R = Streamed<R0>;
    switch (level) {
      case kThread: taf_h<R, kThread>(c, a, h, p, thr, st); break;
      case kWaveLvl: taf_h<R, kWaveLvl>(c, a, h, p, thr, st); break;
      default: taf_h<R, kBlock>(c, a, h, p, thr, st); break;
    }
    return hipGetLastError();
  }
};

hipError_t launch_taf(const LaunchCfg &c, const KArgs &a, int level, int history_size, int prediction_size,
                      float threshold, void *state) {
  return with_region(c.region, c.dtype,
                     TafL{c, a, level, history_size, prediction_size, threshold, static_cast<float *>(state)});
}

int64_t taf_state_bytes(int n_out, int64_t lanes, int history_size) {
  return lanes * ((int64_t)history_size * n_out + 2) * 4;
}

hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t stream) {
  const int64_t n4 = bytes / 16;
  int64_t blocks = (n4 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, stream, (const float4 *)src, (float4 *)dst, n4);
  return hipGetLastError();
}

hipError_t launch_probe_valu(float *out, int workgroups, int iters, bool scalar_operand, hipStream_t stream) {
  if (scalar_operand)
    hipLaunchKernelGGL(k_probe_valu<true>, dim3(workgroups), dim3(256), 0, stream, out, iters, 0.999f, 1e-3f);
  else
    hipLaunchKernelGGL(k_probe_valu<false>, dim3(workgroups), dim3(256), 0, stream, out, iters, 0.999f, 1e-3f);
  return hipGetLastError();
}

}  // namespace hpac

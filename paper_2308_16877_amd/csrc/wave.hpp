// Wavefront primitives for gfx950 (64-lane waves): votes, reductions and the
// intra-wave LDS ordering used by the approximation kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpac {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// 64-bit ballot of a per-lane predicate (inactive lanes contribute 0).
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc(uint64_t m) { return __popcll(m); }

// Index of the lowest set bit; m must be non-zero.
__device__ __forceinline__ int lowest_lane(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }

// Majority rule of the paper's hierarchical decisions: more than half of the
// active lanes (a tie computes).
__device__ __forceinline__ bool majority(int votes, int active) { return 2 * votes > active; }

// One DPP step of a max-scan: v = max(v, v of the lane selected by CTRL),
// lanes with no source keep v (the shifted-in value is -inf).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_max(float v) {
  const int s = __builtin_amdgcn_update_dpp(__float_as_int(-INFINITY), __float_as_int(v), CTRL, ROW_MASK, 0xf, false);
  return fmaxf(v, __int_as_float(s));
}

// Maximum of v over the whole wave, returned to every lane.  DPP row shifts
// scan each row of 16 lanes, row broadcasts carry rows 0->1, 2->3 and then
// 1->2,3, so lane 63 ends with the wave maximum; no LDS crossbar is used.
__device__ __forceinline__ float wave_max(float v) {
  v = dpp_max<0x111, 0xf>(v);  // row_shr:1
  v = dpp_max<0x112, 0xf>(v);  // row_shr:2
  v = dpp_max<0x114, 0xf>(v);  // row_shr:4
  v = dpp_max<0x118, 0xf>(v);  // row_shr:8
  v = dpp_max<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_max<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// One DPP step of an unsigned max-scan, v = max(v, v of the lane CTRL
// selects); lanes with no source, and rows ROW_MASK leaves out, see 0, the
// scan's identity.  The compiler folds the DPP move into the max.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_umax(uint32_t v) {
  const uint32_t s = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, true);
  return v > s ? v : s;
}

// Maximum of an unsigned key over the wave, returned to every lane (the
// same scan as wave_max, one instruction per step).
__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
  v = dpp_umax<0x111, 0xf>(v);  // row_shr:1
  v = dpp_umax<0x112, 0xf>(v);  // row_shr:2
  v = dpp_umax<0x114, 0xf>(v);  // row_shr:4
  v = dpp_umax<0x118, 0xf>(v);  // row_shr:8
  v = dpp_umax<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_umax<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Maximum of v over aligned segments of `seg` lanes (seg a power of two up to
// 64), returned to every lane of the segment.
__device__ __forceinline__ float segment_max(float v, int seg) {
  if (seg == kWave) return wave_max(v);
  for (int off = 1; off < seg; off <<= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
  return v;
}

// Orders a lane's LDS write before every lane's later LDS reads within the
// same wave: a wavefront-scope release/acquire fence plus a wave barrier so
// the compiler keeps the accesses in program order.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace hpac

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

// Maximum of v over aligned segments of `seg` lanes (seg a power of two up to
// 64), returned to every lane of the segment.  Butterfly over xor offsets.
__device__ __forceinline__ float segment_max(float v, int seg) {
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

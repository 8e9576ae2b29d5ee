// Launchers of the Binomial Options kernels (binomial_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpac {

struct BoArgs {
  const float *in[5];  // S, K, T, r, v
  float *out[2];       // call, put
  int64_t n;           // options
  int64_t L;           // decision units (waves), a multiple of 64
  int32_t ipt;         // options per unit
  int32_t steps;       // time steps of the tree
  bool american;
  // technique parameters
  int32_t tsize;       // iACT table size
  float threshold;     // iACT distance / TAF RSD threshold
  int32_t hsize, psize;  // TAF
  int32_t kind, param, offset;  // perforation
  int32_t kept_per_period, special;  // dense small/large perforation (set by the launcher)
  uint32_t *trace;     // optional, L * ipt words
  unsigned long long *counters;  // optional, 4
};

int64_t bo_units(int64_t n, int ipt);
int bo_nodes_per_lane(int steps);  // 0 if the tree does not fit
// tech: 0 exact, 1 iACT, 2 TAF, 3 perforation
hipError_t launch_binomial(const BoArgs &a, int tech, int block, hipStream_t stream);

}  // namespace hpac

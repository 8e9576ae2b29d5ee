// Internal interface between the C ABI (argument checking, dispatch) and the
// kernel launchers.  Not installed; the public interface is include/hpac.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpac {

constexpr int kMaxIn = 8;
constexpr int kMaxOut = 16;

// Kernel arguments of one region launch (passed by value).
struct KArgs {
  const void *in[kMaxIn];  // columns of the region's element type
  void *out[kMaxOut];
  int64_t n;     // items
  int64_t L;     // logical lanes (multiple of 64)
  int32_t ipt;   // items per lane
  uint32_t *trace;
  unsigned long long *counters;
};

struct LaunchCfg {
  int region;
  int dtype;
  int block;  // workgroup lanes
  hipStream_t stream;
};

// Each returns hipSuccess or the launch error; arguments are already valid.
hipError_t launch_exact(const LaunchCfg &c, const KArgs &a);
hipError_t launch_iact(const LaunchCfg &c, const KArgs &a, int level, int table_size, float threshold,
                       int tables_per_wave);
hipError_t launch_taf(const LaunchCfg &c, const KArgs &a, int level, int history_size, int prediction_size,
                      float threshold, void *state);
// Bytes of a persistent TAF state: the window and two int32 per lane.
int64_t taf_state_bytes(int n_out, int64_t lanes, int history_size);
hipError_t launch_perfo(const LaunchCfg &c, const KArgs &a, int kind, int param, int offset);
hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t stream);
hipError_t launch_probe_valu(float *out, int workgroups, int iters, bool scalar_operand, hipStream_t stream);

// Bytes of LDS one iACT workgroup needs.
int64_t iact_lds_bytes(int region, int block, int table_size, int tables_per_wave);

// Whether (region, dtype) is provided.
bool region_dtype_supported(int region, int dtype);

}  // namespace hpac

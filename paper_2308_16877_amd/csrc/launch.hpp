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
                      float threshold);
hipError_t launch_perfo(const LaunchCfg &c, const KArgs &a, int kind, int param, int offset);
hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t stream);

// Bytes of LDS one iACT workgroup needs.
int64_t iact_lds_bytes(int region, int block, int table_size, int tables_per_wave);

// Whether (region, dtype) is provided.
bool region_dtype_supported(int region, int dtype);

}  // namespace hpac

namespace hpac {

// Greeks backward: grad_in[j] = gC * dC/dx_j + gP * dP/dx_j for the five
// inputs, from a saved Jacobian (10 columns) or recomputed from the inputs.
// gC or gP may be null (treated as zero).
struct VjpArgs {
  int64_t n;
  const float *jac[10];  // used by the saved-Jacobian kernel
  const float *in[5];    // used by the recomputing kernel
  const float *gC, *gP;
  float *gin[5];
};
hipError_t launch_bs_vjp(const VjpArgs &a, hipStream_t stream);
hipError_t launch_bs_adjoint(const VjpArgs &a, hipStream_t stream);

}  // namespace hpac

namespace hpac {

// MLP surrogate (parameters: one FP32 array, see mlp_kernels.hip).
struct MlpArgs {
  int64_t n;
  const float *in[5];
  float *out[2];
  const float *params;
  float in_center[5], in_scale[5], out_mean[2], out_scale[2];
  float box_lo[5], box_hi[5];
  int32_t *queue;
  int32_t *queue_count;
};
struct MlpGradArgs {
  int64_t n;
  const float *x[5];
  const float *t[2];
  const float *params;
  float in_center[5], in_scale[5], out_mean[2], out_scale[2];
  float inv_count;  // 1 / number of items the loss averages over
  float *grad_partials;
  float *loss_partials;
};
struct AdamArgs {
  const float *grad_partials;
  int64_t blocks;
  float *params, *m, *v;
  float lr, beta1, beta2, eps, bc1, bc2;
};
int mlp_num_params();
hipError_t launch_mlp_infer(const MlpArgs &a, hipStream_t stream);
hipError_t launch_mlp_grad(const MlpGradArgs &a, hipStream_t stream);
hipError_t launch_mlp_adam(const AdamArgs &a, hipStream_t stream);

}  // namespace hpac

namespace hpac {

// Lagrangian hydro (hydro_kernels.hip).  Region modes:
constexpr int kHgExact = 0, kHgTafWave = 1, kHgTafThread = 2, kHgPerfo = 3;
constexpr int kEosExact = 0, kEosTafWave = 1, kEosTafThread = 2;

struct HydroArgs {
  int n;                  // elements per side
  int64_t E, Nn, W;       // elements, nodes, waves of the element loop (one element per lane)
  float h;                // initial edge of an element
  float gamma, cq, cl, khg;
  double gamma_d, cfl, growth, dvmax;
  float *x[3], *u[3], *un[3];
  float *mnode, *e, *p, *q, *c, *vol, *mass, *force, *fhg;
  float *weos;
  int32_t *rho_eos, *z_eos;
  float *whg;
  int32_t *rho_hg, *z_hg;
  double *clock, *dt_partials;
  int8_t *dec_eos, *dec_hg;
  // technique of this step
  int eos_h, eos_p;
  float eos_theta;
  int hg_h, hg_p;
  float hg_theta;
  int perfo_kind, perfo_param;
  int hg_ipt;      // items per lane of the force kernel's element loop
  int64_t hg_L;    // its logical lanes
  int32_t step;    // timestep index (perforation offset)
};
int64_t hydro_lanes(int64_t E, int ipt);
int64_t hydro_partials(int64_t E);
hipError_t launch_hydro_init(const HydroArgs &a, double e_origin, double dt0, hipStream_t stream);
hipError_t launch_hydro_step(const HydroArgs &a, int hg_mode, int eos_mode, hipStream_t stream);

}  // namespace hpac

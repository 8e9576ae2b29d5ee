// Launchers of the Lagrangian hydro kernels (hydro_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpac {

// Lagrangian hydro (hydro_kernels.hip).  Region modes (kHgNone: no
// hourglass force, a step that herded perforation drops as a whole):
constexpr int kHgExact = 0, kHgTafWave = 1, kHgTafThread = 2, kHgPerfo = 3, kHgNone = 4, kHgTafBlock = 5;
constexpr int kEosExact = 0, kEosTafWave = 1, kEosTafThread = 2, kEosTafBlock = 3;
constexpr int kHydroBlock = 256;  // elements of a workgroup, the block-level decision group

// Division by a fixed divisor d >= 1 of dividends below 2^31 as one 64-bit
// multiply and a shift (Granlund and Montgomery's round-up method): with
// l = ceil(log2 d) and M = ceil(2^(31+l) / d), M d = 2^(31+l) + e with
// 0 <= e < d <= 2^l, so x M / 2^(31+l) exceeds x / d by less than 1/d and
// floors to the same integer.  Element and node indices of a mesh of up to
// 1000 elements per side are below 2^31.
struct DivBy {
  uint64_t M;
  int s;
  int32_t d;
  static constexpr DivBy of(int32_t d) {
    int l = 0;
    while ((int64_t(1) << l) < d) ++l;
    return DivBy{((uint64_t(1) << (31 + l)) + (uint64_t)d - 1) / (uint64_t)d, 31 + l, d};
  }
  __host__ __device__ constexpr uint32_t quo(uint32_t x) const { return (uint32_t)(((uint64_t)x * M) >> s); }
};
static_assert(DivBy::of(1).quo(0x7fffffffu) == 0x7fffffffu && DivBy::of(2).quo(0x7fffffffu) == 0x3fffffffu);
static_assert(DivBy::of(3).quo(0x7fffffffu) == 0x7fffffffu / 3 && DivBy::of(3).quo(5) == 1 && DivBy::of(3).quo(6) == 2);
static_assert(DivBy::of(90).quo(728999) == 8099 && DivBy::of(90).quo(8099) == 89 && DivBy::of(91).quo(753571) == 8281 && DivBy::of(91).quo(753570) == 8280);
static_assert(DivBy::of(1000).quo(999999999) == 999999 && DivBy::of(1001).quo(1003003000) == 1002000);
static_assert(DivBy::of(0x7fffffff).quo(0x7ffffffeu) == 0 && DivBy::of(0x7fffffff).quo(0x7fffffffu) == 1);

struct HydroArgs {
  int n;                  // elements per side
  DivBy dn, dm;           // division by n and by n + 1 (nodes per side)
  int64_t E, Nn, W;       // elements, nodes, waves of the element loop (one element per lane)
  float h;                // initial edge of an element
  float gamma, cq, cl, khg;
  double gamma_d, cfl, growth, dvmax;
  float *x[3], *u[3], *un[3];
  float *mnode, *e, *p, *q, *c, *vol, *mass, *force;
  float *weos;
  int32_t *rho_eos, *z_eos;
  float *whg;
  int32_t *rho_hg, *z_hg;
  double *clock, *dt_partials;
  int32_t *status;        // numeric-failure flags (bits as hpac.h's HPAC_HYDRO_BAD_*)
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
constexpr int32_t kHydroBadVolume = 1, kHydroBadDt = 2;
int64_t hydro_lanes(int64_t E, int ipt);
int64_t hydro_partials(int64_t E);
// Size of the library's own partial-minimum array (the allocation-free
// step's scratch): enough for meshes of up to 256^3 elements.
constexpr int64_t kHydroScratchPartials = 65536;
// Device address of that array on `stream`'s device (the current device for
// the null stream), looked up on the first call per device.
hipError_t hydro_scratch(hipStream_t stream, double **ptr);
hipError_t launch_hydro_init(const HydroArgs &a, double e_origin, double dt0, hipStream_t stream);
hipError_t launch_hydro_step(const HydroArgs &a, int hg_mode, int eos_mode, hipStream_t stream);

}  // namespace hpac

// C ABI of the approximated-region library: argument checking (no HIP call
// is made before all arguments pass), dispatch to the kernel launchers, and
// the thread-local error message.  Declarations and semantics: hpac.h.
#include "../../include/hpac.h"
#include "launch.hpp"
#include "launch_binomial.hpp"
#include "launch_greeks.hpp"
#include "launch_hydro.hpp"
#include "launch_mlp.hpp"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

static_assert(hpac::kHydroBadVolume == HPAC_HYDRO_BAD_VOLUME && hpac::kHydroBadDt == HPAC_HYDRO_BAD_DT,
              "hydro flag bits");
static_assert((((int64_t)HPAC_HYDRO_NOALLOC_MAX_N * HPAC_HYDRO_NOALLOC_MAX_N * HPAC_HYDRO_NOALLOC_MAX_N + 63) / 64 * 64 +
               255) / 256 <= hpac::kHydroScratchPartials,
              "the allocation-free hydro step's scratch array holds the largest mesh it accepts");

namespace {

thread_local char g_err[512] = "no error";

hpac_status fail(hpac_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

struct RegionShape {
  int n_in, n_out;
};

bool region_shape(int region, RegionShape *s) {
  switch (region) {
    case HPAC_REGION_BS_PRICE:
    case HPAC_REGION_BS_PRICE_F16:
    case HPAC_REGION_BS_PRICE_BF16: *s = {5, 2}; return true;
    case HPAC_REGION_BS_PRICE_GRAD: *s = {5, 12}; return true;
    case HPAC_REGION_BS_PRICE_REF: *s = {5, 3}; return true;
    default: return false;
  }
}

constexpr int64_t kMaxItems = (int64_t)1 << 40;
constexpr int32_t kMaxIpt = 65536;
// A dispatch's grid size is a 32-bit count of work-items.
constexpr int64_t kMaxWorkItems = 0xFFFFFFFFll;

int64_t num_lanes(int64_t n, int32_t ipt) {
  const int64_t per = (n + ipt - 1) / ipt;
  return ((per + 63) / 64) * 64;
}

// Validates the launch description and fills the kernel arguments.
hpac_status check_io(const char *fn, const hpac_region_io *io, hpac::KArgs *a, hpac::LaunchCfg *c) {
  if (!io) return fail(HPAC_EINVAL, "%s: io is NULL", fn);
  RegionShape rs;
  if (!region_shape(io->region, &rs)) return fail(HPAC_EINVAL, "%s: unknown region %d", fn, io->region);
  if (io->dtype < HPAC_F32 || io->dtype > HPAC_BF16) return fail(HPAC_EINVAL, "%s: unknown dtype %d", fn, io->dtype);
  if (!hpac::region_dtype_supported(io->region, io->dtype))
    return fail(HPAC_EUNSUPPORTED, "%s: region %d does not take columns of dtype %d", fn, io->region, io->dtype);
  const uintptr_t align = io->dtype == HPAC_F32 ? 4 : 2;
  if (io->n < 0 || io->n > kMaxItems) return fail(HPAC_EINVAL, "%s: n = %lld out of range [0, 2^40]", fn, (long long)io->n);
  if (io->region == HPAC_REGION_BS_PRICE_REF && io->n > INT32_MAX)
    return fail(HPAC_EINVAL, "%s: the source-item region indexes at most 2^31-1 items", fn);
  if (io->n_in != rs.n_in || io->n_out != rs.n_out)
    return fail(HPAC_EINVAL, "%s: region %d takes %d inputs and %d outputs, got %d and %d", fn, io->region, rs.n_in,
                rs.n_out, io->n_in, io->n_out);
  if (io->items_per_lane < 1 || io->items_per_lane > kMaxIpt)
    return fail(HPAC_EINVAL, "%s: items_per_lane = %d out of range [1, %d]", fn, io->items_per_lane, kMaxIpt);
  const int block = io->block_size == 0 ? 256 : io->block_size;
  if (block < 64 || block > 256 || block % 64)
    return fail(HPAC_EINVAL, "%s: block_size = %d must be 64, 128, 192 or 256", fn, io->block_size);
  if (io->n > 0) {
    if (!io->in || !io->out) return fail(HPAC_EINVAL, "%s: NULL column array", fn);
    for (int j = 0; j < rs.n_in; ++j) {
      if (!io->in[j]) return fail(HPAC_EINVAL, "%s: input column %d is NULL", fn, j);
      if ((uintptr_t)io->in[j] % align) return fail(HPAC_EINVAL, "%s: input column %d is misaligned", fn, j);
    }
    for (int o = 0; o < rs.n_out; ++o) {
      if (!io->out[o]) return fail(HPAC_EINVAL, "%s: output column %d is NULL", fn, o);
      if ((uintptr_t)io->out[o] % align) return fail(HPAC_EINVAL, "%s: output column %d is misaligned", fn, o);
    }
  }
  if ((num_lanes(io->n, io->items_per_lane) + block - 1) / block * block > kMaxWorkItems)
    return fail(HPAC_EINVAL, "%s: %lld items at %d items per lane need a grid of more than 2^32-1 lanes; raise "
                "items_per_lane", fn, (long long)io->n, io->items_per_lane);
  if ((uintptr_t)io->trace % 4) return fail(HPAC_EINVAL, "%s: trace is not 4-byte aligned", fn);
  if ((uintptr_t)io->counters % 8) return fail(HPAC_EINVAL, "%s: counters are not 8-byte aligned", fn);
  for (int j = 0; j < hpac::kMaxIn; ++j) a->in[j] = j < rs.n_in && io->n > 0 ? io->in[j] : nullptr;
  for (int o = 0; o < hpac::kMaxOut; ++o) a->out[o] = o < rs.n_out && io->n > 0 ? io->out[o] : nullptr;
  a->n = io->n;
  a->ipt = io->items_per_lane;
  a->L = num_lanes(io->n, io->items_per_lane);
  a->trace = io->trace;
  a->counters = (unsigned long long *)io->counters;
  c->region = io->region;
  c->dtype = io->dtype;
  c->block = block;
  c->stream = (hipStream_t)io->stream;
  return HPAC_OK;
}

// Binomial Options: the io description plus the tree.
hpac_status check_bo(const char *fn, const hpac_region_io *io, int32_t steps, int32_t american, hpac::BoArgs *a,
                     int *block) {
  if (!io) return fail(HPAC_EINVAL, "%s: io is NULL", fn);
  if (io->region != HPAC_REGION_BINOMIAL)
    return fail(HPAC_EINVAL, "%s: region must be HPAC_REGION_BINOMIAL, got %d", fn, io->region);
  if (io->dtype != HPAC_F32) return fail(HPAC_EUNSUPPORTED, "%s: the binomial region takes FP32 columns", fn);
  if (io->n_in != 5 || io->n_out != 2) return fail(HPAC_EINVAL, "%s: the binomial region takes 5 inputs and 2 outputs", fn);
  if (io->n < 0 || io->n > ((int64_t)1 << 31))
    return fail(HPAC_EINVAL, "%s: n = %lld out of range [0, 2^31]", fn, (long long)io->n);
  if (io->items_per_lane < 1 || io->items_per_lane > kMaxIpt)
    return fail(HPAC_EINVAL, "%s: items_per_lane = %d out of range [1, %d]", fn, io->items_per_lane, kMaxIpt);
  const int b = io->block_size == 0 ? 256 : io->block_size;
  if (b < 64 || b > 256 || b % 64) return fail(HPAC_EINVAL, "%s: block_size = %d must be 64, 128, 192 or 256", fn, b);
  if (hpac::bo_units(io->n, io->items_per_lane) * 64 > kMaxWorkItems)
    return fail(HPAC_EINVAL, "%s: %lld options at %d per unit need a grid of more than 2^32-1 lanes; raise "
                "items_per_lane", fn, (long long)io->n, io->items_per_lane);
  if (steps < 1 || hpac::bo_nodes_per_lane(steps) == 0)
    return fail(HPAC_EINVAL, "%s: steps = %d out of range [1, 1023]", fn, steps);
  if (american != 0 && american != 1) return fail(HPAC_EINVAL, "%s: american must be 0 or 1", fn);
  if (io->n > 0) {
    if (!io->in || !io->out) return fail(HPAC_EINVAL, "%s: NULL column array", fn);
    for (int j = 0; j < 5; ++j)
      if (!io->in[j] || (uintptr_t)io->in[j] % 4) return fail(HPAC_EINVAL, "%s: input column %d is NULL or misaligned", fn, j);
    for (int o = 0; o < 2; ++o)
      if (!io->out[o] || (uintptr_t)io->out[o] % 4)
        return fail(HPAC_EINVAL, "%s: output column %d is NULL or misaligned", fn, o);
  }
  if ((uintptr_t)io->trace % 4) return fail(HPAC_EINVAL, "%s: trace is not 4-byte aligned", fn);
  if ((uintptr_t)io->counters % 8) return fail(HPAC_EINVAL, "%s: counters are not 8-byte aligned", fn);
  *a = hpac::BoArgs{};
  for (int j = 0; j < 5; ++j) a->in[j] = io->n > 0 ? (const float *)io->in[j] : nullptr;
  for (int o = 0; o < 2; ++o) a->out[o] = io->n > 0 ? (float *)io->out[o] : nullptr;
  a->n = io->n;
  a->ipt = io->items_per_lane;
  a->L = hpac::bo_units(io->n, io->items_per_lane);
  a->steps = steps;
  a->american = american != 0;
  a->trace = io->trace;
  a->counters = (unsigned long long *)io->counters;
  *block = b;
  return HPAC_OK;
}

hpac_status check_level(const char *fn, int32_t level) {
  if (level != HPAC_LEVEL_THREAD && level != HPAC_LEVEL_WAVE && level != HPAC_LEVEL_BLOCK)
    return fail(HPAC_EINVAL, "%s: unknown level %d", fn, level);
  return HPAC_OK;
}

hpac_status check_threshold(const char *fn, float t) {
  if (!(t >= 0.0f) || !isfinite(t)) return fail(HPAC_EINVAL, "%s: threshold must be finite and >= 0", fn);
  return HPAC_OK;
}

hpac_status hip_status(const char *fn, hipError_t e) {
  if (e != hipSuccess) return fail(HPAC_EHIP, "%s: %s", fn, hipGetErrorString(e));
  return HPAC_OK;
}

}  // namespace

extern "C" {

int32_t hpac_abi_version(void) { return 3; }

const char *hpac_last_error(void) { return g_err; }

int64_t hpac_taf_state_bytes(int32_t region, int64_t n, int32_t items_per_lane, int32_t history_size) {
  RegionShape rs;
  if (!region_shape(region, &rs) || region == HPAC_REGION_BS_PRICE_REF || n < 0 || n > kMaxItems ||
      items_per_lane < 1 || items_per_lane > kMaxIpt || history_size < 1 || history_size > 8)
    return -1;
  return hpac::taf_state_bytes(rs.n_out, num_lanes(n, items_per_lane), history_size);
}

int64_t hpac_num_lanes(int64_t n, int32_t items_per_lane) {
  if (n < 0 || n > kMaxItems || items_per_lane < 1 || items_per_lane > kMaxIpt) return -1;
  return num_lanes(n, items_per_lane);
}

int64_t hpac_trace_entries(int64_t n, int32_t items_per_lane) {
  const int64_t L = hpac_num_lanes(n, items_per_lane);
  return L < 0 ? -1 : (L / 64) * items_per_lane;
}

hpac_status hpac_exact(const hpac_region_io *io) {
  hpac::KArgs a;
  hpac::LaunchCfg c;
  hpac_status s = check_io("hpac_exact", io, &a, &c);
  if (s != HPAC_OK || a.n == 0) return s;
  return hip_status("hpac_exact", hpac::launch_exact(c, a));
}

hpac_status hpac_iact(const hpac_region_io *io, int32_t table_size, float threshold, int32_t tables_per_wave,
                      int32_t level) {
  const char *fn = "hpac_iact";
  hpac::KArgs a;
  hpac::LaunchCfg c;
  hpac_status s = check_io(fn, io, &a, &c);
  if (s != HPAC_OK) return s;
  if (table_size < 1 || table_size > 32) return fail(HPAC_EINVAL, "%s: table_size = %d out of range [1, 32]", fn, table_size);
  if ((s = check_threshold(fn, threshold)) != HPAC_OK) return s;
  if (tables_per_wave < 1 || tables_per_wave > 64 || 64 % tables_per_wave)
    return fail(HPAC_EINVAL, "%s: tables_per_wave = %d must divide 64", fn, tables_per_wave);
  if ((s = check_level(fn, level)) != HPAC_OK) return s;
  const int64_t lds = hpac::iact_lds_bytes(c.region, c.block, table_size, tables_per_wave);
  if (lds > 65536)
    return fail(HPAC_EUNSUPPORTED, "%s: tables need %lld bytes of LDS per workgroup (limit 65536); use a smaller block",
                fn, (long long)lds);
  if (a.n == 0) return HPAC_OK;
  return hip_status(fn, hpac::launch_iact(c, a, level, table_size, threshold, tables_per_wave));
}

hpac_status hpac_taf(const hpac_region_io *io, int32_t history_size, int32_t prediction_size, float rsd_threshold,
                     int32_t level, void *persistent_state) {
  const char *fn = "hpac_taf";
  hpac::KArgs a;
  hpac::LaunchCfg c;
  hpac_status s = check_io(fn, io, &a, &c);
  if (s != HPAC_OK) return s;
  if (io->region == HPAC_REGION_BS_PRICE_REF)
    return fail(HPAC_EUNSUPPORTED, "%s: the source-item region is provided for hpac_exact and hpac_iact", fn);
  if (history_size < 1 || history_size > 8)
    return fail(HPAC_EINVAL, "%s: history_size = %d out of range [1, 8]", fn, history_size);
  if (prediction_size < 1) return fail(HPAC_EINVAL, "%s: prediction_size = %d must be >= 1", fn, prediction_size);
  if ((s = check_threshold(fn, rsd_threshold)) != HPAC_OK) return s;
  if ((s = check_level(fn, level)) != HPAC_OK) return s;
  if ((uintptr_t)persistent_state % 4) return fail(HPAC_EINVAL, "%s: persistent_state is misaligned", fn);
  if (a.n == 0) return HPAC_OK;
  return hip_status(fn, hpac::launch_taf(c, a, level, history_size, prediction_size, rsd_threshold,
                                         persistent_state));
}

hpac_status hpac_perfo(const hpac_region_io *io, int32_t kind, int32_t param, int32_t offset) {
  const char *fn = "hpac_perfo";
  hpac::KArgs a;
  hpac::LaunchCfg c;
  hpac_status s = check_io(fn, io, &a, &c);
  if (s != HPAC_OK) return s;
  if (io->region == HPAC_REGION_BS_PRICE_REF)
    return fail(HPAC_EUNSUPPORTED, "%s: the source-item region is provided for hpac_exact and hpac_iact", fn);
  if (kind < HPAC_PERFO_SMALL || kind > HPAC_PERFO_FINI) return fail(HPAC_EINVAL, "%s: unknown kind %d", fn, kind);
  if (param < 0) return fail(HPAC_EINVAL, "%s: param = %d must be >= 0", fn, param);
  if ((kind == HPAC_PERFO_INI || kind == HPAC_PERFO_FINI) && param > 100)
    return fail(HPAC_EINVAL, "%s: percentage %d out of range [0, 100]", fn, param);
  if (offset < 0) return fail(HPAC_EINVAL, "%s: offset = %d must be >= 0", fn, offset);
  if (a.n == 0) return HPAC_OK;
  return hip_status(fn, hpac::launch_perfo(c, a, kind, param, offset));
}

static hpac_status check_vjp(const char *fn, int64_t n, const void *const *cols, int ncols, const float *gC,
                             const float *gP, void *const *grad_in, hpac::VjpArgs *a) {
  if (n < 0 || n > kMaxItems) return fail(HPAC_EINVAL, "%s: n = %lld out of range [0, 2^40]", fn, (long long)n);
  a->n = n;
  a->gC = gC;
  a->gP = gP;
  if (n == 0) return HPAC_OK;
  if (!cols || !grad_in) return fail(HPAC_EINVAL, "%s: NULL column array", fn);
  for (int j = 0; j < ncols; ++j)
    if (!cols[j] || (uintptr_t)cols[j] % 4) return fail(HPAC_EINVAL, "%s: column %d is NULL or misaligned", fn, j);
  for (int j = 0; j < 5; ++j)
    if (!grad_in[j] || (uintptr_t)grad_in[j] % 4)
      return fail(HPAC_EINVAL, "%s: gradient column %d is NULL or misaligned", fn, j);
  if ((uintptr_t)gC % 4 || (uintptr_t)gP % 4) return fail(HPAC_EINVAL, "%s: upstream gradient misaligned", fn);
  for (int j = 0; j < 5; ++j) a->gin[j] = (float *)grad_in[j];
  return HPAC_OK;
}

hpac_status hpac_bs_vjp(int64_t n, const void *const *jacobian, const float *grad_call, const float *grad_put,
                        void *const *grad_in, void *stream) {
  const char *fn = "hpac_bs_vjp";
  hpac::VjpArgs a = {};
  hpac_status s = check_vjp(fn, n, jacobian, 10, grad_call, grad_put, grad_in, &a);
  if (s != HPAC_OK || n == 0) return s;
  for (int j = 0; j < 10; ++j) a.jac[j] = (const float *)jacobian[j];
  return hip_status(fn, hpac::launch_bs_vjp(a, (hipStream_t)stream));
}

hpac_status hpac_bs_vjp_ref(int64_t n, const void *const *in, const int32_t *source, const float *grad_call,
                            const float *grad_put, void *const *grad_in, void *stream) {
  const char *fn = "hpac_bs_vjp_ref";
  hpac::VjpArgs a = {};
  if (n > INT32_MAX) return fail(HPAC_EINVAL, "%s: at most 2^31-1 items (int32 source indices)", fn);
  hpac_status s = check_vjp(fn, n, in, 5, grad_call, grad_put, grad_in, &a);
  if (s != HPAC_OK || n == 0) return s;
  if (!source || (uintptr_t)source % 4) return fail(HPAC_EINVAL, "%s: source is NULL or misaligned", fn);
  for (int j = 0; j < 5; ++j) a.in[j] = (const float *)in[j];
  a.src = source;
  return hip_status(fn, hpac::launch_bs_vjp_ref(a, (hipStream_t)stream));
}

hpac_status hpac_bs_adjoint(int64_t n, const void *const *in, const float *grad_call, const float *grad_put,
                            void *const *grad_in, void *stream) {
  const char *fn = "hpac_bs_adjoint";
  hpac::VjpArgs a = {};
  hpac_status s = check_vjp(fn, n, in, 5, grad_call, grad_put, grad_in, &a);
  if (s != HPAC_OK || n == 0) return s;
  for (int j = 0; j < 5; ++j) a.in[j] = (const float *)in[j];
  return hip_status(fn, hpac::launch_bs_adjoint(a, (hipStream_t)stream));
}

static hpac_status copy_norm(const char *fn, const hpac_mlp_norm *norm, float *c, float *s, float *mu,
                             float *sc, float *sh) {
  if (!norm) return fail(HPAC_EINVAL, "%s: norm is NULL", fn);
  for (int j = 0; j < 5; ++j) {
    if (!isfinite(norm->in_center[j]) || !isfinite(norm->in_scale[j]))
      return fail(HPAC_EINVAL, "%s: input normalisation must be finite", fn);
    c[j] = norm->in_center[j];
    s[j] = norm->in_scale[j];
  }
  for (int o = 0; o < 2; ++o) {
    if (!isfinite(norm->out_mean[o]) || !isfinite(norm->out_scale[o]) || norm->out_scale[o] == 0.0f)
      return fail(HPAC_EINVAL, "%s: output normalisation must be finite with a non-zero scale", fn);
    if (!isfinite(norm->out_shift[o]) || !(norm->out_shift[o] >= 0.0f))
      return fail(HPAC_EINVAL, "%s: output shifts must be finite and >= 0", fn);
    mu[o] = norm->out_mean[o];
    sc[o] = norm->out_scale[o];
    sh[o] = norm->out_shift[o];
  }
  return HPAC_OK;
}

hpac_status hpac_surrogate(const hpac_region_io *io, const float *params, const hpac_mlp_norm *norm,
                           const float *box_lo, const float *box_hi, int32_t *queue, int32_t *queue_count) {
  const char *fn = "hpac_surrogate";
  hpac::KArgs ka;
  hpac::LaunchCfg c;
  hpac_status s = check_io(fn, io, &ka, &c);
  if (s != HPAC_OK) return s;
  if (io->region != HPAC_REGION_BS_PRICE || io->dtype != HPAC_F32)
    return fail(HPAC_EUNSUPPORTED, "%s: the surrogate replaces HPAC_REGION_BS_PRICE with FP32 columns", fn);
  if (io->n > 2147483647) return fail(HPAC_EINVAL, "%s: at most 2^31-1 items per call (int32 queue)", fn);
  if (!box_lo || !box_hi) return fail(HPAC_EINVAL, "%s: NULL box", fn);
  hpac::MlpArgs a = {};
  s = copy_norm(fn, norm, a.in_center, a.in_scale, a.out_mean, a.out_scale, a.out_shift);
  if (s != HPAC_OK) return s;
  for (int j = 0; j < 5; ++j) {
    a.box_lo[j] = box_lo[j];
    a.box_hi[j] = box_hi[j];
  }
  if (io->n == 0) return HPAC_OK;
  if (!params || (uintptr_t)params % 4) return fail(HPAC_EINVAL, "%s: params NULL or misaligned", fn);
  if (!queue || !queue_count || (uintptr_t)queue % 4 || (uintptr_t)queue_count % 4)
    return fail(HPAC_EINVAL, "%s: queue or queue_count NULL or misaligned", fn);
  a.n = io->n;
  for (int j = 0; j < 5; ++j) a.in[j] = (const float *)io->in[j];
  for (int o = 0; o < 2; ++o) a.out[o] = (float *)io->out[o];
  a.params = params;
  a.queue = queue;
  a.queue_count = queue_count;
  return hip_status(fn, hpac::launch_mlp_infer(a, (hipStream_t)io->stream));
}

int64_t hpac_mlp_grad_blocks(int64_t batch) { return batch < 0 ? -1 : (batch + 63) / 64; }

hpac_status hpac_mlp_grad(int64_t batch, const float *const *x, const float *const *t, const float *params,
                          const hpac_mlp_norm *norm, int64_t loss_count, float *grad_partials, float *loss_partials,
                          void *stream) {
  const char *fn = "hpac_mlp_grad";
  if (batch < 0 || (batch + 63) / 64 * 64 > kMaxWorkItems)
    return fail(HPAC_EINVAL, "%s: batch = %lld out of range [0, 2^32 - 64]", fn, (long long)batch);
  if (loss_count < 1) return fail(HPAC_EINVAL, "%s: loss_count must be >= 1", fn);
  hpac::MlpGradArgs a = {};
  hpac_status s = copy_norm(fn, norm, a.in_center, a.in_scale, a.out_mean, a.out_scale, a.out_shift);
  if (s != HPAC_OK || batch == 0) return s;
  if (!x || !t || !params || !grad_partials || !loss_partials) return fail(HPAC_EINVAL, "%s: NULL pointer", fn);
  for (int j = 0; j < 5; ++j)
    if (!x[j] || (uintptr_t)x[j] % 4) return fail(HPAC_EINVAL, "%s: input column %d NULL or misaligned", fn, j);
  for (int o = 0; o < 2; ++o)
    if (!t[o] || (uintptr_t)t[o] % 4) return fail(HPAC_EINVAL, "%s: target column %d NULL or misaligned", fn, o);
  a.n = batch;
  for (int j = 0; j < 5; ++j) a.x[j] = x[j];
  for (int o = 0; o < 2; ++o) a.t[o] = t[o];
  a.params = params;
  a.inv_count = 1.0f / (float)loss_count;
  a.grad_partials = grad_partials;
  a.loss_partials = loss_partials;
  return hip_status(fn, hpac::launch_mlp_grad(a, (hipStream_t)stream));
}

hpac_status hpac_mlp_adam(const float *grad_partials, int64_t blocks, float *params, float *m, float *v, float lr,
                          float beta1, float beta2, float eps, int32_t step, void *stream) {
  const char *fn = "hpac_mlp_adam";
  if (blocks < 1 || !grad_partials || !params || !m || !v) return fail(HPAC_EINVAL, "%s: NULL pointer or no blocks", fn);
  if (step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(HPAC_EINVAL, "%s: hyper-parameters out of range", fn);
  hpac::AdamArgs a = {};
  a.grad_partials = grad_partials;
  a.blocks = blocks;
  a.params = params;
  a.m = m;
  a.v = v;
  a.lr = lr;
  a.beta1 = beta1;
  a.beta2 = beta2;
  a.eps = eps;
  a.bc1 = (float)(1.0 - pow((double)beta1, (double)step));
  a.bc2 = (float)(1.0 - pow((double)beta2, (double)step));
  return hip_status(fn, hpac::launch_mlp_adam(a, (hipStream_t)stream));
}

// ------------------------------------------------------------------ binomial

int64_t hpac_bo_units(int64_t n, int32_t items_per_lane) {
  if (n < 0 || n > ((int64_t)1 << 31) || items_per_lane < 1 || items_per_lane > kMaxIpt) return -1;
  return hpac::bo_units(n, items_per_lane);
}

static hpac_status bo_launch(const char *fn, const hpac_region_io *io, const hpac::BoArgs &a, int tech, int block) {
  if (a.n == 0) return HPAC_OK;
  return hip_status(fn, hpac::launch_binomial(a, tech, block, (hipStream_t)io->stream));
}

hpac_status hpac_bo_exact(const hpac_region_io *io, int32_t steps, int32_t american) {
  const char *fn = "hpac_bo_exact";
  hpac::BoArgs a;
  int block;
  const hpac_status st = check_bo(fn, io, steps, american, &a, &block);
  return st != HPAC_OK ? st : bo_launch(fn, io, a, 0, block);
}

hpac_status hpac_bo_iact(const hpac_region_io *io, int32_t steps, int32_t american, int32_t table_size,
                         float threshold) {
  const char *fn = "hpac_bo_iact";
  hpac::BoArgs a;
  int block;
  hpac_status st = check_bo(fn, io, steps, american, &a, &block);
  if (st == HPAC_OK) st = check_threshold(fn, threshold);
  if (st != HPAC_OK) return st;
  if (table_size < 1 || table_size > 32) return fail(HPAC_EINVAL, "%s: table_size = %d out of range [1, 32]", fn, table_size);
  a.tsize = table_size;
  a.threshold = threshold;
  return bo_launch(fn, io, a, 1, block);
}

hpac_status hpac_bo_taf(const hpac_region_io *io, int32_t steps, int32_t american, int32_t history_size,
                        int32_t prediction_size, float rsd_threshold) {
  const char *fn = "hpac_bo_taf";
  hpac::BoArgs a;
  int block;
  hpac_status st = check_bo(fn, io, steps, american, &a, &block);
  if (st == HPAC_OK) st = check_threshold(fn, rsd_threshold);
  if (st != HPAC_OK) return st;
  if (history_size < 1 || history_size > 8)
    return fail(HPAC_EINVAL, "%s: history_size = %d out of range [1, 8]", fn, history_size);
  if (prediction_size < 1) return fail(HPAC_EINVAL, "%s: prediction_size = %d must be >= 1", fn, prediction_size);
  a.hsize = history_size;
  a.psize = prediction_size;
  a.threshold = rsd_threshold;
  return bo_launch(fn, io, a, 2, block);
}

hpac_status hpac_bo_perfo(const hpac_region_io *io, int32_t steps, int32_t american, int32_t kind, int32_t param,
                          int32_t offset) {
  const char *fn = "hpac_bo_perfo";
  hpac::BoArgs a;
  int block;
  const hpac_status st = check_bo(fn, io, steps, american, &a, &block);
  if (st != HPAC_OK) return st;
  if (kind < HPAC_PERFO_SMALL || kind > HPAC_PERFO_FINI) return fail(HPAC_EINVAL, "%s: unknown kind %d", fn, kind);
  if (param < 0) return fail(HPAC_EINVAL, "%s: param = %d must be >= 0", fn, param);
  if ((kind == HPAC_PERFO_INI || kind == HPAC_PERFO_FINI) && param > 100)
    return fail(HPAC_EINVAL, "%s: percentage %d out of range [0, 100]", fn, param);
  if (offset < 0) return fail(HPAC_EINVAL, "%s: offset = %d must be >= 0", fn, offset);
  a.kind = kind;
  a.param = param;
  a.offset = offset;
  return bo_launch(fn, io, a, 3, block);
}

// ------------------------------------------------------------------ hydro

static bool aligned4(const void *p) { return p && (uintptr_t)p % 4 == 0; }

static hpac_status check_hydro_params(const char *fn, const hpac_hydro_params *P) {
  if (!P) return fail(HPAC_EINVAL, "%s: params is NULL", fn);
  if (P->n < 1 || P->n > 1000) return fail(HPAC_EINVAL, "%s: n = %d out of range [1, 1000]", fn, P->n);
  const double v[] = {P->side, P->gamma, P->cq, P->cl, P->khg, P->cfl, P->growth, P->dvmax, P->dt0};
  for (double x : v)
    if (!isfinite(x)) return fail(HPAC_EINVAL, "%s: non-finite parameter", fn);
  if (!(P->side > 0) || !(P->gamma > 1) || P->cq < 0 || P->cl < 0 || P->khg < 0 || !(P->cfl > 0) ||
      !(P->growth >= 1) || !(P->dvmax > 0) || !(P->dt0 > 0))
    return fail(HPAC_EINVAL, "%s: parameter out of range", fn);
  return HPAC_OK;
}

static hpac_status check_hydro_state(const char *fn, const hpac_hydro_state *S, bool own_partials = true) {
  if (!S) return fail(HPAC_EINVAL, "%s: state is NULL", fn);
  for (int d = 0; d < 3; ++d)
    if (!aligned4(S->x[d]) || !aligned4(S->u[d]) || !aligned4(S->unew[d]))
      return fail(HPAC_EINVAL, "%s: node coordinate or velocity %d is NULL or misaligned", fn, d);
  const float *f[] = {S->mnode, S->e, S->p, S->q, S->c, S->vol, S->mass, S->force};
  for (const float *x : f)
    if (!aligned4(x)) return fail(HPAC_EINVAL, "%s: a mesh field is NULL or misaligned", fn);
  if (!S->clock || (uintptr_t)S->clock % 8) return fail(HPAC_EINVAL, "%s: clock is NULL or misaligned", fn);
  if (own_partials && (!S->dt_partials || (uintptr_t)S->dt_partials % 8))
    return fail(HPAC_EINVAL, "%s: dt_partials is NULL or misaligned", fn);
  if (!aligned4(S->status)) return fail(HPAC_EINVAL, "%s: status is NULL or misaligned", fn);
  return HPAC_OK;
}

static hpac::HydroArgs hydro_args(const hpac_hydro_params *P, const hpac_hydro_state *S) {
  hpac::HydroArgs a = {};
  a.n = P->n;
  a.dn = hpac::DivBy::of(P->n);
  a.dm = hpac::DivBy::of(P->n + 1);
  a.E = (int64_t)P->n * P->n * P->n;
  a.Nn = (int64_t)(P->n + 1) * (P->n + 1) * (P->n + 1);
  a.W = hpac::hydro_lanes(a.E, 1) / 64;
  a.h = (float)(P->side / P->n);
  a.gamma = (float)P->gamma;
  a.gamma_d = P->gamma;
  a.cq = (float)P->cq;
  a.cl = (float)P->cl;
  a.khg = (float)P->khg;
  a.cfl = P->cfl;
  a.growth = P->growth;
  a.dvmax = P->dvmax;
  for (int d = 0; d < 3; ++d) {
    a.x[d] = S->x[d];
    a.u[d] = S->u[d];
    a.un[d] = S->unew[d];
  }
  a.mnode = S->mnode;
  a.e = S->e;
  a.p = S->p;
  a.q = S->q;
  a.c = S->c;
  a.vol = S->vol;
  a.mass = S->mass;
  a.force = S->force;
  a.weos = S->weos;
  a.rho_eos = S->rho_eos;
  a.z_eos = S->z_eos;
  a.whg = S->whg;
  a.rho_hg = S->rho_hg;
  a.z_hg = S->z_hg;
  a.clock = S->clock;
  a.dt_partials = S->dt_partials;
  a.status = S->status;
  a.hg_ipt = 1;
  a.hg_L = hpac::hydro_lanes(a.E, 1);
  return a;
}

int64_t hpac_hydro_waves(int32_t n) {
  if (n < 1 || n > 1000) return -1;
  return hpac::hydro_lanes((int64_t)n * n * n, 1) / 64;
}

int64_t hpac_hydro_groups(int32_t n, int32_t level) {
  if (n < 1 || n > 1000) return -1;
  if (level == HPAC_LEVEL_THREAD) return (int64_t)n * n * n;
  if (level == HPAC_LEVEL_WAVE) return hpac::hydro_lanes((int64_t)n * n * n, 1) / 64;
  if (level == HPAC_LEVEL_BLOCK) return ((int64_t)n * n * n + hpac::kHydroBlock - 1) / hpac::kHydroBlock;
  return -1;
}

int64_t hpac_hydro_partials(int32_t n) {
  if (n < 1 || n > 1000) return -1;
  return hpac::hydro_partials((int64_t)n * n * n);
}

hpac_status hpac_hydro_init(const hpac_hydro_params *params, double e_origin, const hpac_hydro_state *state,
                            void *stream) {
  const char *fn = "hpac_hydro_init";
  hpac_status st = check_hydro_params(fn, params);
  if (st == HPAC_OK) st = check_hydro_state(fn, state);
  if (st != HPAC_OK) return st;
  if (!isfinite(e_origin) || e_origin < 0) return fail(HPAC_EINVAL, "%s: e_origin must be finite and >= 0", fn);
  if ((state->rho_eos == NULL) != (state->z_eos == NULL) || (state->rho_hg == NULL) != (state->z_hg == NULL))
    return fail(HPAC_EINVAL, "%s: a countdown array without its push-count array", fn);
  if ((state->rho_eos && !aligned4(state->rho_eos)) ||
      (state->z_eos && !aligned4(state->z_eos)) || (state->rho_hg && !aligned4(state->rho_hg)) ||
      (state->z_hg && !aligned4(state->z_hg)))
    return fail(HPAC_EINVAL, "%s: misaligned optional field", fn);
  const hpac::HydroArgs a = hydro_args(params, state);
  return hip_status(fn, hpac::launch_hydro_init(a, e_origin, params->dt0, (hipStream_t)stream));
}

// Checks of a hydro step's arguments and its kernel arguments and modes.
static hpac_status hydro_prepare(const char *fn, const hpac_hydro_params *params, const hpac_hydro_tech *tech,
                                 int32_t step, const hpac_hydro_state *state, int8_t *dec_eos, int8_t *dec_hg,
                                 hpac::HydroArgs *out, int *hg_mode, int *eos_mode_out,
                                 bool own_partials = true) {
  hpac_status st = check_hydro_params(fn, params);
  if (st == HPAC_OK) st = check_hydro_state(fn, state, own_partials);
  if (st != HPAC_OK) return st;
  if (!tech) return fail(HPAC_EINVAL, "%s: tech is NULL", fn);
  if (step < 0) return fail(HPAC_EINVAL, "%s: step = %d must be >= 0", fn, step);
  const hpac_hydro_tech &T = *tech;
  if (T.eos_history < 0 || T.eos_history > 8 || T.hg_history < 0 || T.hg_history > 8)
    return fail(HPAC_EINVAL, "%s: history sizes must be in [0, 8]", fn);
  if ((T.eos_history && T.eos_prediction < 1) || (T.hg_history && T.hg_prediction < 1))
    return fail(HPAC_EINVAL, "%s: prediction sizes must be >= 1", fn);
  auto level_ok = [](int32_t lv) {
    return lv == HPAC_LEVEL_WAVE || lv == HPAC_LEVEL_THREAD || lv == HPAC_LEVEL_BLOCK;
  };
  if ((T.eos_history && !level_ok(T.eos_level)) || (T.hg_history && !level_ok(T.hg_level)))
    return fail(HPAC_EINVAL, "%s: hydro TAF levels are HPAC_LEVEL_THREAD, _WAVE or _BLOCK", fn);
  if (!(T.eos_threshold >= 0.0f) || !isfinite(T.eos_threshold) || !(T.hg_threshold >= 0.0f) ||
      !isfinite(T.hg_threshold))
    return fail(HPAC_EINVAL, "%s: thresholds must be finite and >= 0", fn);
  if (T.perfo_kind < HPAC_PERFO_SMALL || T.perfo_kind > HPAC_PERFO_FINI || T.perfo_param < 0)
    return fail(HPAC_EINVAL, "%s: bad perforation kind or parameter", fn);
  if ((T.perfo_kind == HPAC_PERFO_INI || T.perfo_kind == HPAC_PERFO_FINI) && T.perfo_param > 100)
    return fail(HPAC_EINVAL, "%s: perforation percentage %d > 100", fn, T.perfo_param);
  if (T.perfo_param && (T.perfo_items_per_lane < 1 || T.perfo_items_per_lane > 64))
    return fail(HPAC_EINVAL, "%s: perfo_items_per_lane must be in [1, 64]", fn);
  if (T.hg_history && T.perfo_param) return fail(HPAC_EINVAL, "%s: TAF and perforation on the hourglass region", fn);
  if (T.eos_history && (!aligned4(state->weos) || !aligned4(state->rho_eos) || !aligned4(state->z_eos)))
    return fail(HPAC_EINVAL, "%s: EOS TAF needs weos, rho_eos and z_eos", fn);
  if (T.hg_history && (!aligned4(state->whg) || !aligned4(state->rho_hg) || !aligned4(state->z_hg)))
    return fail(HPAC_EINVAL, "%s: hourglass TAF needs whg, rho_hg and z_hg", fn);
  hpac::HydroArgs a = hydro_args(params, state);
  a.step = step;
  a.dec_eos = T.eos_history ? dec_eos : nullptr;
  a.dec_hg = T.hg_history ? dec_hg : nullptr;
  a.eos_h = T.eos_history;
  a.eos_p = T.eos_prediction;
  a.eos_theta = T.eos_threshold;
  a.hg_h = T.hg_history;
  a.hg_p = T.hg_prediction;
  a.hg_theta = T.hg_threshold;
  a.perfo_kind = T.perfo_kind;
  a.perfo_param = T.perfo_param;
  int mode = hpac::kHgExact;
  if (T.hg_history) {
    mode = T.hg_level == HPAC_LEVEL_THREAD ? hpac::kHgTafThread
         : T.hg_level == HPAC_LEVEL_BLOCK  ? hpac::kHgTafBlock
                                           : hpac::kHgTafWave;
  } else if (T.perfo_param) {
    mode = hpac::kHgPerfo;
    a.hg_ipt = T.perfo_items_per_lane;
    a.hg_L = hpac::hydro_lanes(a.E, a.hg_ipt);
  }
  int eos_mode = hpac::kEosExact;
  if (T.eos_history)
    eos_mode = T.eos_level == HPAC_LEVEL_THREAD ? hpac::kEosTafThread
             : T.eos_level == HPAC_LEVEL_BLOCK  ? hpac::kEosTafBlock
                                                : hpac::kEosTafWave;
  *out = a;
  *hg_mode = mode;
  *eos_mode_out = eos_mode;
  return HPAC_OK;
}

hpac_status hpac_hydro_step(const hpac_hydro_params *params, const hpac_hydro_tech *tech, int32_t step,
                            const hpac_hydro_state *state, int8_t *dec_eos, int8_t *dec_hg, void *stream) {
  const char *fn = "hpac_hydro_step";
  hpac::HydroArgs a;
  int mode = 0, eos_mode = 0;
  const hpac_status st = hydro_prepare(fn, params, tech, step, state, dec_eos, dec_hg, &a, &mode, &eos_mode);
  if (st != HPAC_OK) return st;
  return hip_status(fn, hpac::launch_hydro_step(a, mode, eos_mode, (hipStream_t)stream));
}

hpac_status hpac_hydro_step_noalloc(const hpac_hydro_params *params, const hpac_hydro_tech *tech, int32_t step,
                                    const hpac_hydro_state *state, int8_t *dec_eos, int8_t *dec_hg, void *stream) {
  const char *fn = "hpac_hydro_step_noalloc";
  if (params && params->n > HPAC_HYDRO_NOALLOC_MAX_N)
    return fail(HPAC_EINVAL, "%s: n = %d exceeds the %d elements per side the library's scratch array holds", fn,
                params->n, HPAC_HYDRO_NOALLOC_MAX_N);
  hpac::HydroArgs a;
  int mode = 0, eos_mode = 0;
  const hpac_status st = hydro_prepare(fn, params, tech, step, state, dec_eos, dec_hg, &a, &mode, &eos_mode, false);
  if (st != HPAC_OK) return st;
  if (hpac::hydro_partials(a.E) > hpac::kHydroScratchPartials)
    return fail(HPAC_EINVAL, "%s: the mesh needs more partial minima than the scratch array holds", fn);
  hipError_t e = hpac::hydro_scratch((hipStream_t)stream, &a.dt_partials);
  if (e == hipSuccess) e = hpac::launch_hydro_step(a, mode, eos_mode, (hipStream_t)stream);
  return hip_status(fn, e);
}

hpac_status hpac_hydro_run(const hpac_hydro_params *params, const hpac_hydro_tech *tech, int32_t first_step,
                           int32_t steps, const hpac_hydro_state *state, void *stream) {
  const char *fn = "hpac_hydro_run";
  if (steps < 0) return fail(HPAC_EINVAL, "%s: steps = %d must be >= 0", fn, steps);
  if ((int64_t)first_step + steps > INT32_MAX) return fail(HPAC_EINVAL, "%s: step indices overflow int32", fn);
  hpac::HydroArgs a;
  int mode = 0, eos_mode = 0;
  const hpac_status st = hydro_prepare(fn, params, tech, first_step, state, nullptr, nullptr, &a, &mode, &eos_mode);
  if (st != HPAC_OK) return st;
  for (int32_t k = 0; k < steps; ++k) {
    a.step = first_step + k;
    const hipError_t e = hpac::launch_hydro_step(a, mode, eos_mode, (hipStream_t)stream);
    if (e != hipSuccess) return hip_status(fn, e);
    for (int d = 0; d < 3; ++d) {  // the new velocities are the next step's old ones
      float *t = a.u[d];
      a.u[d] = a.un[d];
      a.un[d] = t;
    }
  }
  return HPAC_OK;
}

hpac_status hpac_hydro_check(const hpac_hydro_state *state, void *stream) {
  const char *fn = "hpac_hydro_check";
  if (!state || !aligned4(state->status)) return fail(HPAC_EINVAL, "%s: status is NULL or misaligned", fn);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  int32_t flags = 0;
  if (e == hipSuccess) e = hipMemcpy(&flags, state->status, sizeof flags, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_status(fn, e);
  if (flags)
    return fail(HPAC_ENUMERIC, "%s: the hydro left its numeric domain:%s%s", fn,
                flags & HPAC_HYDRO_BAD_VOLUME ? " a non-positive element volume (tangled mesh)" : "",
                flags & HPAC_HYDRO_BAD_DT ? " a time step that is not finite and positive" : "");
  return HPAC_OK;
}

hpac_status hpac_probe_copy(const void *src, void *dst, int64_t bytes, void *stream) {
  const char *fn = "hpac_probe_copy";
  if (bytes < 0 || bytes % 16) return fail(HPAC_EINVAL, "%s: bytes must be a non-negative multiple of 16", fn);
  if (bytes > 0 && (!src || !dst)) return fail(HPAC_EINVAL, "%s: NULL buffer", fn);
  if ((uintptr_t)src % 16 || (uintptr_t)dst % 16) return fail(HPAC_EINVAL, "%s: buffers must be 16-byte aligned", fn);
  if (bytes == 0) return HPAC_OK;
  return hip_status(fn, hpac::launch_copy(src, dst, bytes, (hipStream_t)stream));
}

hpac_status hpac_probe_valu(float *out, int32_t workgroups, int32_t iters, int32_t scalar_operand, void *stream) {
  const char *fn = "hpac_probe_valu";
  if (workgroups < 1 || workgroups > 65536 || iters < 1 || iters > 65536)
    return fail(HPAC_EINVAL, "%s: workgroups and iters must be in [1, 65536]", fn);
  if (!out || (uintptr_t)out % 4) return fail(HPAC_EINVAL, "%s: out must be a 4-byte aligned device buffer", fn);
  return hip_status(fn, hpac::launch_probe_valu(out, workgroups, iters, scalar_operand != 0, (hipStream_t)stream));
}

}  // extern "C"

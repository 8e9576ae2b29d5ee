/*
 * hpac.h -- C ABI of the MI355X (gfx950) approximated-region library.
 *
 * The library executes a data-parallel code region over n items on the GPU
 * and applies one of the approximation techniques of HPAC-Offload
 * (Fink, Parasyris, Georgakoudis, Menon, arXiv 2308.16877): input
 * memoization (iACT), output memoization (TAF) and loop perforation, with the
 * approximate-or-compute decision taken per hierarchy group (section 3.1.2),
 * by default per 64-lane wavefront.
 *
 * Conventions shared by every entry point:
 *  - All column pointers are DEVICE pointers owned by the caller.  The
 *    library never allocates, frees or retains device memory; its only state
 *    is in registers and LDS for the duration of one launch (section 3.1.1).
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  Nothing is synchronised; a kernel fault surfaces at the
 *    caller's next synchronisation of that stream.
 *  - Every entry point returns an hpac_status.  HPAC_EINVAL is returned
 *    before any HIP call is made, so argument checking works on a host
 *    without a GPU.  hpac_last_error() returns a thread-local message for the
 *    last non-OK status of the calling thread.
 *  - No C++ exception crosses this interface.
 *  - Item -> lane mapping (sections 3.1.3, 3.3; items per thread, Table 2):
 *    L = 64 * ceil(ceil(n / items_per_lane) / 64) logical lanes; lane l at
 *    grid-stride step k (0 <= k < items_per_lane) owns item i = l + k * L and
 *    is active iff i < n.  Wave w holds lanes 64w .. 64w + 63.  The
 *    approximation state (tables, windows, countdowns) of a lane, wave or
 *    block lives for one launch and evolves over its steps k in order, so
 *    results depend on items_per_lane (and, at block level, on block_size).
 *  - Majority rule (section 3.3): a group approximates iff more than half of
 *    its active lanes meet the technique's criterion; a tie computes.
 *  - A threshold (or perforation parameter) of 0 reproduces the exact
 *    region bit for bit.
 */
#ifndef HPAC_H
#define HPAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hpac_status;
#define HPAC_OK 0
#define HPAC_EINVAL (-1)       /* an argument is out of range or NULL       */
#define HPAC_EUNSUPPORTED (-2) /* valid request the library does not provide */
#define HPAC_EHIP (-3)         /* the HIP runtime reported an error         */
#define HPAC_ENUMERIC (-4)     /* the computation left its numeric domain   */

/* Regions.  Inputs and outputs are structure-of-arrays columns of n
 * elements (the column-major, stride-n array sections of section 3.2).
 *
 * HPAC_REGION_BS_PRICE: European call and put under Black-Scholes-Merton
 *   (the paper's Black-Scholes benchmark, section 4 and Table 1).
 *   in  (5): S spot, K strike, T years to expiry, r riskless rate, v volatility
 *   out (2): call, put.  Domain: S, K, T, v > 0.
 * HPAC_REGION_BS_PRICE_GRAD: the same prices plus their Jacobian.
 *   in  (5): as above.  out (12): call, put, then dC/d(S, K, T, r, v) and
 *   dP/d(S, K, T, r, v).  Under iACT the memoized outputs are all 12
 *   columns, so a reused entry also reuses its gradients. */
#define HPAC_REGION_BS_PRICE 0
#define HPAC_REGION_BS_PRICE_GRAD 1
/* HPAC_REGION_BS_PRICE_REF: the prices plus the item that produced them.
 *   in (5): as above.  out (3): call, put (FP32), then an int32 column: the
 *   item's own index where the region was evaluated, the source item of the
 *   reused entry where iACT approximated (its inputs were stored with the
 *   entry).  hpac_bs_vjp_ref recomputes the derivatives at the source item,
 *   which reuses the memoized gradient by reference (4 bytes per item instead
 *   of ten Jacobian columns).  Taken by hpac_exact and hpac_iact only (other
 *   techniques return HPAC_EUNSUPPORTED); n <= 2^31 - 1. */
#define HPAC_REGION_BS_PRICE_REF 5
/* Reduced-precision bodies of HPAC_REGION_BS_PRICE (same inputs and outputs):
 *   _F16  every operation in FP16;
 *   _BF16 every operation at BF16 precision (inputs and each result rounded
 *         to the nearest BF16). */
#define HPAC_REGION_BS_PRICE_F16 2
#define HPAC_REGION_BS_PRICE_BF16 3
/* HPAC_REGION_BINOMIAL: the paper's Binomial Options region (section 4,
 * Table 1): call and put on a Cox-Ross-Rubinstein tree (see hpac_bo_*,
 * which alone take it).  in (5) and out (2) as HPAC_REGION_BS_PRICE, FP32. */
#define HPAC_REGION_BINOMIAL 4

/* Element type of every column of a call (both inputs and outputs).
 * HPAC_REGION_BS_PRICE takes any of the three; _F16 takes F32 or F16; _BF16
 * takes F32 or BF16; _GRAD takes F32.  Other pairs return HPAC_EUNSUPPORTED.
 * Half-precision columns must be 2-byte aligned, FP32 columns 4-byte. */
#define HPAC_F32 0
#define HPAC_F16 1
#define HPAC_BF16 2

/* Decision hierarchy (section 3.1.2, the level clause of section 3.2). */
#define HPAC_LEVEL_THREAD 0 /* each lane decides alone                     */
#define HPAC_LEVEL_WAVE 1   /* 64-lane wavefront decides by majority       */
#define HPAC_LEVEL_BLOCK 2  /* the workgroup decides by majority           */

/* Perforation kinds (section 2.3; runtime in section 3.3). */
#define HPAC_PERFO_SMALL 0 /* skip step k iff (k + offset) mod M == M - 1 */
#define HPAC_PERFO_LARGE 1 /* run step k only iff (k + offset) mod M == 0 */
#define HPAC_PERFO_INI 2   /* skip items i < floor(p * n / 100)            */
#define HPAC_PERFO_FINI 3  /* skip items i >= n - floor(p * n / 100)       */

/* Counters, accumulated with atomics when hpac_region_io.counters != NULL
 * (the caller zeroes them): */
#define HPAC_CNT_LANE_STEPS 0        /* items visited (active lane-steps)  */
#define HPAC_CNT_APPROX_LANE_STEPS 1 /* items approximated or skipped      */
#define HPAC_CNT_APPROX_WAVE_STEPS 2 /* wave-steps taken approximately     */
#define HPAC_CNT_WAVE_STEPS 3        /* wave-steps with an active lane     */
#define HPAC_NUM_COUNTERS 4

/* Trace record, one uint32 per (wave w, step k) at trace[w * ipt + k] when
 * hpac_region_io.trace != NULL (hpac_trace_entries() entries):
 *   bits  0..6   lanes whose criterion held at this step's vote
 *   bits  8..14  lanes that took the approximate path
 *   bits 16..21  iACT writer lane (table 0 of the wave); bit 22 set if valid
 *   bit  24      the wave's decision was approximate (perforation: skipped)
 *   bit  25      a vote was taken at this step
 *   bit  31      the wave had an active lane at this step (else all zero)  */
#define HPAC_TRACE_VOTES(t) ((t) & 0x7Fu)
#define HPAC_TRACE_NAPPROX(t) (((t) >> 8) & 0x7Fu)
#define HPAC_TRACE_WRITER(t) (((t) >> 16) & 0x3Fu)
#define HPAC_TRACE_WRITER_VALID(t) (((t) >> 22) & 1u)
#define HPAC_TRACE_APPROX(t) (((t) >> 24) & 1u)
#define HPAC_TRACE_VOTED(t) (((t) >> 25) & 1u)
#define HPAC_TRACE_ACTIVE(t) (((t) >> 31) & 1u)

/* One launch of a region over n items. */
typedef struct hpac_region_io {
  int32_t region;          /* HPAC_REGION_*                                  */
  int32_t dtype;           /* HPAC_F32                                       */
  int64_t n;               /* items, 0 <= n <= 2^40; n == 0 launches nothing */
  const void *const *in;   /* host array of n_in device column pointers     */
  int32_t n_in;            /* must equal the region's input count           */
  void *const *out;        /* host array of n_out device column pointers    */
  int32_t n_out;           /* must equal the region's output count          */
  int32_t items_per_lane;  /* 1 .. 65536                                     */
  int32_t block_size;      /* workgroup lanes: 64, 128, 192 or 256; 0 = 256  */
  void *stream;            /* hipStream_t; NULL = null stream                */
  uint32_t *trace;         /* optional device buffer, see above              */
  uint64_t *counters;      /* optional device uint64[HPAC_NUM_COUNTERS]      */
} hpac_region_io;

/* Exact region: every item is evaluated.  Outputs are bitwise those that
 * every technique produces on its accurate path. */
hpac_status hpac_exact(const hpac_region_io *io);

/* iACT input memoization (sections 2.3, 3.1.4, 3.2, 3.3).
 * table_size: entries per table, 1..32 (the tSize clause argument).
 * threshold:  Euclidean distance threshold over the region's inputs in
 *             their own units, finite, >= 0 (FP32, as the 0.5f of the
 *             clause).  A lane's criterion: its table is non-empty and the
 *             squared distance to its nearest entry, computed in FP32 as
 *             t0*t0 then fma(tj, tj, acc) for j = 1.., with tj = x_j - e_j,
 *             is below threshold*threshold (FP32).  Nearest: lowest slot
 *             among equal distances.
 * tables_per_wave: tables shared by 64 / tables_per_wave consecutive lanes
 *             (the tPerWarp clause argument); must divide 64.  The tables
 *             of a workgroup live in its LDS and must fit in 64 KiB
 *             (HPAC_EUNSUPPORTED otherwise); with many tables per wave,
 *             smaller workgroups (io->block_size) let more of them share a
 *             CU and run faster.
 * level:      HPAC_LEVEL_*.
 * Approximate lanes return their nearest entry's outputs without evaluating
 * the region.  Write phase: in each table, among its lanes that evaluated
 * the region this step, the one whose nearest-entry distance is largest
 * (infinite for an empty table; lowest lane on ties) stores its inputs and
 * outputs at slot (insertions mod table_size), round robin.  Tables start
 * empty at every launch. */
hpac_status hpac_iact(const hpac_region_io *io, int32_t table_size, float threshold,
                      int32_t tables_per_wave, int32_t level);

/* TAF output memoization (sections 2.3, 3.1.3, 3.2, 3.3).
 * history_size:    window of a lane's last accurate outputs, 1..8 (hSize).
 * prediction_size: steps approximated after a passing vote, >= 1 (pSize).
 * rsd_threshold:   finite, >= 0 (FP32).  After each accurate step that
 *   leaves the window full, a lane's criterion is RSD < rsd_threshold, with
 *   RSD = sigma/|mu| (population) maximised over the region's outputs,
 *   RSD = 0 when sigma = 0 and +inf when mu = 0 < sigma, evaluated in FP64
 *   as var == 0 ? threshold > 0 : var < threshold^2 * mu^2.  A passing group
 *   approximates its next prediction_size steps: each active lane writes its
 *   last accurate output and reads no input.  The window slides over
 *   accurate steps only and is never reset within a launch.
 * persistent_state: NULL keeps the state within the launch (the paper's
 *   kernel-scoped state, section 3.1.1).  Otherwise a device buffer of
 *   hpac_taf_state_bytes(region, n, items_per_lane, history_size) bytes,
 *   4-byte aligned, owned by the caller and zeroed before the first launch:
 *   each lane's window and fill and its group's remaining approximate steps
 *   are read from it at the start and written back at the end, so that a
 *   sequence of launches of the same shape (region, n, items_per_lane,
 *   block_size, level, history_size) continues each lane's sequence of
 *   steps -- output memoization across calls, as across the timesteps of a
 *   simulation.  Launches that share a state must not overlap. */
hpac_status hpac_taf(const hpac_region_io *io, int32_t history_size, int32_t prediction_size,
                     float rsd_threshold, int32_t level, void *persistent_state);
/* Bytes of a persistent TAF state for that launch shape (the window of
 * history_size outputs and two int32 per logical lane); -1 if an argument
 * is out of range. */
int64_t hpac_taf_state_bytes(int32_t region, int64_t n, int32_t items_per_lane, int32_t history_size);

/* Herded loop perforation (sections 2.3, 3.1.5, 3.3): every lane drops the
 * same steps, so control flow stays uniform across each wave.
 * kind: HPAC_PERFO_*.  param: M >= 0 for SMALL/LARGE, percent 0..100 for
 * INI/FINI; 0 = no perforation.  offset >= 0 is added to the step index.
 * A dropped item reads no input and writes no output (its output columns
 * keep their previous contents). */
hpac_status hpac_perfo(const hpac_region_io *io, int32_t kind, int32_t param, int32_t offset);

/* Greeks backward (the adjoint of HPAC_REGION_BS_PRICE_GRAD's prices).
 * For i < n and each input j in (S, K, T, r, v):
 *   grad_in[j][i] = grad_call[i] * dC/dx_j + grad_put[i] * dP/dx_j.
 * hpac_bs_vjp takes the derivatives from a saved Jacobian: the 10 columns
 * 2..11 written by the forward region (dC/dx then dP/dx), so derivatives that
 * iACT reused in the forward pass are reused here too.
 * hpac_bs_adjoint recomputes them from the 5 input columns instead.
 * grad_call or grad_put may be NULL (taken as zero).  All pointers are
 * device pointers of n floats; grad_in is a host array of 5 of them.
 * Asynchronous on `stream`; n == 0 launches nothing. */
hpac_status hpac_bs_vjp(int64_t n, const void *const *jacobian, const float *grad_call, const float *grad_put,
                        void *const *grad_in, void *stream);
hpac_status hpac_bs_adjoint(int64_t n, const void *const *in, const float *grad_call, const float *grad_put,
                            void *const *grad_in, void *stream);
/* The same contraction for a forward on HPAC_REGION_BS_PRICE_REF: item i
 * takes the derivatives of item source[i] (device int32 column of n),
 * recomputed from in[5] at that item; equal bit for bit to hpac_bs_vjp of
 * the Jacobian HPAC_REGION_BS_PRICE_GRAD would have saved under the same
 * technique.  An index outside [0, n) yields NaN gradients for that item
 * (nothing is read for it).  n <= 2^31 - 1. */
hpac_status hpac_bs_vjp_ref(int64_t n, const void *const *in, const int32_t *source, const float *grad_call,
                            const float *grad_put, void *const *grad_in, void *stream);

/* ------------------------------------------------------------------------
 * MLP surrogate: a further approximation technique for HPAC_REGION_BS_PRICE
 * (a learned model standing in for the region inside the box it was trained
 * on; the exact region is the fallback outside it and the yardstick of
 * its error).  Network 5 -> 64 -> 64 -> 2, GELU (tanh form) on both hidden
 * layers.  Parameters: one device array of HPAC_MLP_NUM_PARAMS floats,
 *   W1[64][5], b1[64], W2[64][64], b2[64], W3[2][64], b3[2]
 * (row = output unit), kept in FP32; the kernels use the weights rounded to
 * BF16 (nearest, ties to even) and the biases in FP32.
 * Normalisation (host values): the network sees xh_j = (x_j - in_center[j])
 * * in_scale[j]; its outputs yh map back to v_o = yh_o * out_scale[o] +
 * out_mean[o], and the result is y_o = v_o when out_shift[o] = 0, or
 * y_o = exp(v_o) - out_shift[o] when out_shift[o] > 0: the network then
 * models log(y_o + out_shift[o]), whose errors are relative to y_o +
 * out_shift[o] (prices near zero keep small absolute errors).
 * ------------------------------------------------------------------------ */
#define HPAC_MLP_NUM_PARAMS 4674
typedef struct hpac_mlp_norm {
  float in_center[5];
  float in_scale[5];
  float out_mean[2];
  float out_scale[2];
  float out_shift[2]; /* >= 0, finite */
} hpac_mlp_norm;

/* Surrogate inference over io->n items (region HPAC_REGION_BS_PRICE, FP32
 * columns; items_per_lane, trace and counters are ignored).  An item with
 * box_lo[j] <= x_j <= box_hi[j] for all five inputs (host arrays) gets the
 * network's outputs, computed with BF16 MFMA and FP32 accumulation, the layer
 * inputs rounded to BF16; every other item is appended to `queue` (device,
 * n int32 entries, order unspecified) and gets the exact region's outputs.
 * *queue_count (device int32) is set to the number queued.  Three launches
 * on io->stream. */
hpac_status hpac_surrogate(const hpac_region_io *io, const float *params, const hpac_mlp_norm *norm,
                           const float *box_lo, const float *box_hi, int32_t *queue, int32_t *queue_count);

/* Training step, part 1: the gradient of L = 1/(2 N) sum_i sum_o
 * (yh_o(x_i) - (g_o(t_o,i) - out_mean[o]) / out_scale[o])^2 over the `batch`
 * items, g_o(t) = t, or log(t + out_shift[o]) when out_shift[o] > 0 (targets
 * t are region outputs, transformed by the kernel)
 * (columns x[5], targets t[2], device) with respect to every parameter, with
 * FP32 activations and BF16-rounded weights (the rounding is passed through
 * as the identity), N = loss_count.  Writes one partial gradient per 64 items:
 * grad_partials[b * HPAC_MLP_NUM_PARAMS + p] and the partial sum of squared
 * errors loss_partials[b], b < hpac_mlp_grad_blocks(batch). */
int64_t hpac_mlp_grad_blocks(int64_t batch);
hpac_status hpac_mlp_grad(int64_t batch, const float *const *x, const float *const *t, const float *params,
                          const hpac_mlp_norm *norm, int64_t loss_count, float *grad_partials, float *loss_partials,
                          void *stream);

/* Training step, part 2: Adam (Kingma and Ba) on the FP32 parameters with
 * the sum of `blocks` partial gradients; m and v are the caller's moment
 * arrays (zero at step 1); step >= 1 is the bias-correction step. */
hpac_status hpac_mlp_adam(const float *grad_partials, int64_t blocks, float *params, float *m, float *v, float lr,
                          float beta1, float beta2, float eps, int32_t step, void *stream);

/* ------------------------------------------------------------------------
 * Lagrangian hydrodynamics with approximated regions across timesteps.
 *
 * The paper's hydrodynamics workload is a Sedov blast on volumetric
 * elements whose quantity of interest is the final energy at the origin,
 * with the hourglass-force computation among the approximated kernels
 * (section 4, Table 1 and 4.1).  This is a staggered-grid scheme of our own
 * from published methods (FP32 state, FP64 time step): exact trilinear
 * hexahedron volume and gradient, viscous Flanagan-Belytschko hourglass
 * control, compatible total-energy update, ideal gas with von
 * Neumann-Richtmyer viscosity; n^3 elements on [0, side]^3 with symmetry
 * planes x=0, y=0, z=0, unit initial density, at rest, specific energy
 * e_origin in the element at the origin.
 *
 * Two per-element regions take the paper's techniques with one element per
 * lane (a wave is 64 consecutive elements, a TAF step is a timestep, TAF
 * state persists in the caller's buffers between calls):
 *  - hourglass region (24 corner forces, added to the element's corner
 *    forces): TAF (history 1..8; an approximated element adds its last
 *    accurate forces, the newest slot of its window) or herded perforation (section 3.1.5) of the
 *    element loop at perfo_items_per_lane, offset = timestep (a skipped
 *    iteration adds nothing);
 *  - EOS region (e, p, q, c): TAF; approximated elements keep their values.
 * TAF decides per element (thread level), per wave (majority of its 64
 * elements) or per workgroup (block level: majority of 256 consecutive
 * elements), the levels of section 3.1.2.
 * Layouts: element fields n^3 floats, element z = i + n (j + n k); node
 * fields (n+1)^3 floats, node i + (n+1) (j + (n+1) k); force is
 * [(corner * 3 + dim) * n^3 + z] with corner a + 2b + 4c for node
 * (i+a, j+b, k+c); windows are [(slot * outputs + o) * n^3 + z];
 * per-group ints have hpac_hydro_groups(n, level) entries.  All device memory, owned
 * by the caller.  Calls are asynchronous on `stream`; the time step stays
 * on the device (clock), so a step never waits for the host.
 * ------------------------------------------------------------------------ */
typedef struct hpac_hydro_params {
  int32_t n;     /* elements per side, 1..1000 */
  double side;   /* edge of the domain */
  double gamma;  /* ratio of specific heats */
  double cq, cl; /* quadratic and linear viscosity coefficients */
  double khg;    /* hourglass coefficient */
  double cfl;    /* Courant factor */
  double growth; /* largest ratio of consecutive time steps */
  double dvmax;  /* largest relative volume change per step */
  double dt0;    /* time step taken as "previous" by the first step */
} hpac_hydro_params;

typedef struct hpac_hydro_state {
  float *x[3], *u[3], *unew[3]; /* node positions, velocities, velocities after a step */
  float *mnode;                 /* node masses */
  float *e, *p, *q, *c;         /* element specific energy, pressure, viscosity, sound speed */
  float *vol, *mass;            /* element volume at the last force evaluation, mass */
  float *force;                 /* corner forces, 24 n^3 */
  float *weos;                  /* EOS window, eos_history * 4 n^3 (EOS TAF only) */
  int32_t *rho_eos, *z_eos;     /* per decision group: countdown, pushes (EOS TAF only) */
  float *whg;                   /* hourglass window, hg_history * 24 n^3 (hourglass TAF only) */
  int32_t *rho_hg, *z_hg;
  double *clock;                /* [0] time, [1] last time step */
  double *dt_partials;          /* hpac_hydro_partials(n) doubles */
  int32_t *status;              /* numeric-failure flags, HPAC_HYDRO_BAD_* (one int32) */
} hpac_hydro_state;

/* Numeric-failure flags, OR-ed into *state->status by the step kernels
 * (zeroed by hpac_hydro_init) when an element's volume is not positive
 * (a tangled mesh: too large a Courant factor or time step) or the step's
 * time step is not finite and positive.  The step carries on (no index
 * depends on the values, so a failed run cannot fault); the caller learns
 * of the failure at its next read of the flags: hpac_hydro_check, or a
 * copy of *status after the stream has passed the step. */
#define HPAC_HYDRO_BAD_VOLUME 1
#define HPAC_HYDRO_BAD_DT 2

typedef struct hpac_hydro_tech {
  int32_t eos_history, eos_prediction; /* EOS TAF; history 0 = exact */
  float eos_threshold;
  int32_t eos_level;                   /* HPAC_LEVEL_THREAD, _WAVE or _BLOCK */
  int32_t hg_history, hg_prediction;   /* hourglass TAF; history 0 = none */
  float hg_threshold;
  int32_t hg_level;
  int32_t perfo_kind;                  /* hourglass perforation, HPAC_PERFO_* */
  int32_t perfo_param;                 /* 0 = none */
  int32_t perfo_items_per_lane;        /* 1..64 */
} hpac_hydro_tech;

/* Waves of the element loop, TAF decision groups at `level` (elements,
 * waves or 256-element blocks: the size of dec_*; rho_* and z_* always have
 * one entry per element), and
 * entries of dt_partials; -1 if an argument is invalid. */
int64_t hpac_hydro_waves(int32_t n);
int64_t hpac_hydro_groups(int32_t n, int32_t level);
int64_t hpac_hydro_partials(int32_t n);

/* Initial state (every non-NULL field of *state is written; rho_* / z_* are
 * zeroed over hpac_hydro_groups(n, THREAD) entries, so they must have that
 * many when given; windows are only read after they are written). */
hpac_status hpac_hydro_init(const hpac_hydro_params *params, double e_origin, const hpac_hydro_state *state,
                            void *stream);

/* One timestep with index `step` (the perforation offset).  On return, in
 * stream order, the velocities after the step are in state->unew: swap u
 * and unew before the next call.  dec_eos / dec_hg (optional, device int8
 * per decision group): 0 the group computed the region this step, 1 it
 * approximated.
 * Fields a technique needs must be non-NULL (HPAC_EINVAL otherwise). */
hpac_status hpac_hydro_step(const hpac_hydro_params *params, const hpac_hydro_tech *tech, int32_t step,
                            const hpac_hydro_state *state, int8_t *dec_eos, int8_t *dec_hg, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * timestep as hpac_hydro_step, with the time-step reduction's partial minima
 * kept in the library's own device array (512 KiB, allocated with the
 * library's code object on each GPU it runs on and held until the process
 * ends) instead of state->dt_partials, which is ignored and may be NULL.
 * Meshes of n <= HPAC_HYDRO_NOALLOC_MAX_N elements per side; larger n is
 * rejected with HPAC_EINVAL.  The call allocates nothing.  The array is
 * shared by every call on that GPU: calls that overlap on one GPU (on
 * different streams, or from several threads) race on it, so serialise them;
 * each call writes every entry it reads before reading it. */
#define HPAC_HYDRO_NOALLOC_MAX_N 256
hpac_status hpac_hydro_step_noalloc(const hpac_hydro_params *params, const hpac_hydro_tech *tech, int32_t step,
                                    const hpac_hydro_state *state, int8_t *dec_eos, int8_t *dec_hg, void *stream);

/* `steps` (>= 0) timesteps with indices first_step, first_step + 1, ...:
 * the same launches as that many hpac_hydro_step calls with u and unew
 * swapped between them, issued from one host loop (no decision records).
 * On return, in stream order, the latest velocities are in state->unew if
 * `steps` is odd and in state->u if it is even. */
hpac_status hpac_hydro_run(const hpac_hydro_params *params, const hpac_hydro_tech *tech, int32_t first_step,
                           int32_t steps, const hpac_hydro_state *state, void *stream);

/* Waits for `stream`, then reads *state->status: HPAC_OK if no flag is set,
 * HPAC_ENUMERIC (the message names the flags) otherwise.  The one hydro call
 * that waits for the device. */
hpac_status hpac_hydro_check(const hpac_hydro_state *state, void *stream);

/* ------------------------------------------------------------------------
 * Binomial Options.  One wavefront prices one option on an N-step
 * Cox-Ross-Rubinstein tree (dt = T/N, u = exp(v sqrt(dt)), d = 1/u,
 * p = (exp(r dt) - d) / (u - d); American: each node takes the larger of
 * its continuation and exercise values), 1 <= N <= 1023.  The paper's
 * benchmark has one group of threads per option and decides per option
 * (section 4.1); here the wavefront is that group and the decision unit:
 * unit u of hpac_bo_units(n, io->items_per_lane) units processes options
 * u + k * units, k < items_per_lane, and decides alone for each (the thread
 * level of section 3.1.2 with the wavefront as the thread).  io->region must
 * be HPAC_REGION_BINOMIAL and io->dtype HPAC_F32; io->block_size (64..256)
 * sets the units per workgroup.  io->trace, if given, receives one word per
 * (unit, k) at trace[unit * items_per_lane + k] (bit 31 visited, bit 24
 * approximated or skipped, bit 25 voted or inserted, bit 0 criterion held);
 * io->counters as for the other techniques, per option.
 *   iACT: a table of table_size (1..32) entries per unit, in FP32 with the
 *     squared-distance rounding of hpac_iact; the nearest entry (lowest slot
 *     on ties) is reused when its distance is below the threshold; a unit
 *     that computed inserts its option round-robin.
 *   TAF: per unit, a window of its last history_size (1..8) accurate
 *     outputs, FP64 RSD test, prediction_size approximate options after a
 *     passing test.
 *   Perforation: herded over the unit's option loop as in hpac_perfo; a
 *     skipped option is neither read nor written.
 * ------------------------------------------------------------------------ */
int64_t hpac_bo_units(int64_t n, int32_t items_per_lane);
hpac_status hpac_bo_exact(const hpac_region_io *io, int32_t steps, int32_t american);
hpac_status hpac_bo_iact(const hpac_region_io *io, int32_t steps, int32_t american, int32_t table_size,
                         float threshold);
hpac_status hpac_bo_taf(const hpac_region_io *io, int32_t steps, int32_t american, int32_t history_size,
                        int32_t prediction_size, float rsd_threshold);
hpac_status hpac_bo_perfo(const hpac_region_io *io, int32_t steps, int32_t american, int32_t kind, int32_t param,
                          int32_t offset);

/* Number of logical lanes L for n items at items_per_lane (see above);
 * -1 on invalid arguments. */
int64_t hpac_num_lanes(int64_t n, int32_t items_per_lane);

/* Entries a trace buffer needs: (L / 64) * items_per_lane; -1 if invalid. */
int64_t hpac_trace_entries(int64_t n, int32_t items_per_lane);

/* Measurement helper, not part of the method: copies `bytes` (a multiple of
 * 16) from src to dst with a plain streaming kernel on `stream`.  Used to
 * calibrate hardware byte counters against a transfer of known size. */
hpac_status hpac_probe_copy(const void *src, void *dst, int64_t bytes, void *stream);

/* Measurement helper, not part of the method: `workgroups` (1..65536)
 * workgroups of 256 lanes each issue `iters` (1..65536) x 64 independent
 * FP32 fused multiply-adds, on 8 chains per lane; with scalar_operand != 0
 * the multiplier and addend are wave-uniform kernel arguments (scalar
 * register operands), else per-lane copies of them (vector registers).
 * Each lane writes one float to out (workgroups * 256 floats, device), so
 * the caller can time the launch: lane-FMAs = workgroups * 256 * iters * 64. */
hpac_status hpac_probe_valu(float *out, int32_t workgroups, int32_t iters, int32_t scalar_operand, void *stream);

/* Thread-local message describing the last non-OK status; never NULL. */
const char *hpac_last_error(void);

/* ABI version of this header: 2 (the hydro state gained `status`). */
int32_t hpac_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HPAC_H */

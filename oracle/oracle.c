/*
 * CPU oracle for the approximated-region hot path of HPAC-Offload
 * (Fink, Parasyris, Georgakoudis, Menon; arXiv 2308.16877).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or constant with the GPU library; the two meet only
 * through data (the seeded inputs and the outputs being compared).
 *
 * Layers:
 *   R  exact regions in FP64 (Black-Scholes-Merton price and its Jacobian)
 *   E  the approximation engine: item->lane mapping, group votes, iACT input
 *      memoization, TAF output memoization, loop perforation, emulating the
 *      64-lane wavefront grouping of the GPU design
 *   M  the MAPE quality metric
 *
 * Floating point: FP64 throughout, except where a floating-point value
 * decides an integer and the GPU takes that decision in FP32: the iACT
 * squared distance, its threshold comparison, its arg-min and its writer
 * election are evaluated here in FP32 with a fixed operation order
 * (sub, mul, then fmaf) so both sides take bit-identical decisions.
 * Build with -ffp-contract=off so the compiler adds no fusion of its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_WAVE 64

/* ------------------------------------------------------------------------ */
/* R1: European call and put under Black-Scholes-Merton, no dividends.       */
/* The paper's Black-Scholes benchmark prices a portfolio of European        */
/* options analytically (section 4, Table 1).  N(x) = erfc(-x/sqrt2)/2.      */
/* ------------------------------------------------------------------------ */

static double or_ncdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

static double or_npdf(double x) { return exp(-0.5 * x * x) / sqrt(2.0 * M_PI); }

/* Price one option.  Outputs: call, put, and the two tolerance scales
 * |S N(d1)| + |D N(d2)| and |D N(-d2)| + |S N(-d1)| (the sums of the
 * absolute values of each price's two terms). */
static void or_bs_one(double S, double K, double T, double r, double v,
                      double *C, double *P, double *sC, double *sP) {
  double sqT = sqrt(T);
  double vs = v * sqT;
  double d1 = (log(S / K) + (r + 0.5 * v * v) * T) / vs;
  double d2 = d1 - vs;
  double D = K * exp(-r * T);
  double a = S * or_ncdf(d1), b = D * or_ncdf(d2);
  double c = D * or_ncdf(-d2), d = S * or_ncdf(-d1);
  *C = a - b;
  *P = c - d;
  if (sC) *sC = fabs(a) + fabs(b);
  if (sP) *sP = fabs(c) + fabs(d);
}

void or_bs_price(int64_t n, const double *S, const double *K, const double *T,
                 const double *r, const double *v, double *C, double *P,
                 double *scaleC, double *scaleP) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    or_bs_one(S[i], K[i], T[i], r[i], v[i], &C[i], &P[i],
              scaleC ? &scaleC[i] : NULL, scaleP ? &scaleP[i] : NULL);
}

/* R2: Jacobian of (C, P) with respect to (S, K, T, r, v), closed forms.
 * J is 10 columns of n: rows C then P, each in input order S, K, T, r, v.
 * Call row: dC/dS = N(d1), dC/dK = -e^{-rT} N(d2),
 *           dC/dT = S phi(d1) v / (2 sqrt T) + r K e^{-rT} N(d2),
 *           dC/dr = K T e^{-rT} N(d2), dC/dv = S phi(d1) sqrt T.
 * Put row (the derivative of parity P = C - S + K e^{-rT}, with 1 - N(x)
 * written as N(-x) so that no entry loses its relative accuracy):
 *           dP/dS = -N(-d1), dP/dK = e^{-rT} N(-d2),
 *           dP/dT = S phi(d1) v / (2 sqrt T) - r K e^{-rT} N(-d2),
 *           dP/dr = -K T e^{-rT} N(-d2), dP/dv = S phi(d1) sqrt T. */
void or_bs_jacobian(int64_t n, const double *S_, const double *K_, const double *T_,
                    const double *r_, const double *v_, double *const *J) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double S = S_[i], K = K_[i], T = T_[i], r = r_[i], v = v_[i];
    double sqT = sqrt(T), vs = v * sqT;
    double d1 = (log(S / K) + (r + 0.5 * v * v) * T) / vs, d2 = d1 - vs;
    double disc = exp(-r * T), D = K * disc;
    double Nd2 = or_ncdf(d2), Nmd2 = or_ncdf(-d2), pd1 = or_npdf(d1);
    double theta = S * pd1 * v / (2.0 * sqT);
    J[0][i] = or_ncdf(d1);
    J[1][i] = -disc * Nd2;
    J[2][i] = theta + r * D * Nd2;
    J[3][i] = K * T * disc * Nd2;
    J[4][i] = S * pd1 * sqT;
    J[5][i] = -or_ncdf(-d1);
    J[6][i] = disc * Nmd2;
    J[7][i] = theta - r * D * Nmd2;
    J[8][i] = -K * T * disc * Nmd2;
    J[9][i] = S * pd1 * sqT;
  }
}

/* ------------------------------------------------------------------------ */
/* E0: item -> lane mapping.  Grid-stride loop (sections 3.1.3 and 3.3):    */
/* L logical lanes, a multiple of 64, enough that each lane handles at most  */
/* ipt items ("items per thread", Table 2).  Lane l at step k owns item      */
/* i = l + k L and is active iff i < n.  Wave w holds lanes 64w .. 64w+63.    */
/* ------------------------------------------------------------------------ */

int64_t or_num_lanes(int64_t n, int32_t ipt) {
  int64_t per = (n + ipt - 1) / ipt;
  return ((per + OR_WAVE - 1) / OR_WAVE) * OR_WAVE;
}

/* Majority rule (section 3.3): the group approximates iff more than half of
 * its active lanes meet the criterion; a tie goes to the accurate path. */
static int or_majority(int votes, int active) { return 2 * votes > active; }

/* Per-(wave, step) record shared by the engines.  dec: -1 no active lane,
 * 0 accurate, 1 approximate (for thread level: 1 if any lane approximated).
 * votes: lanes whose criterion held (iACT: hit; TAF: RSD below threshold;
 * -1 when no vote was taken).  writer: iACT table-0 writer lane or -1.
 * fragile: 1 if flipping the lanes whose statistic lies within the band of
 * the threshold could change the group decision. */
typedef struct {
  int8_t *dec;
  int16_t *votes;
  int16_t *writer;
  uint8_t *fragile;
  int16_t *napprox; /* lanes that took the approximate path */
} or_trace;

static void or_trace_init(const or_trace *t, int64_t entries) {
  for (int64_t e = 0; e < entries; ++e) {
    if (t->dec) t->dec[e] = -1;
    if (t->votes) t->votes[e] = -1;
    if (t->writer) t->writer[e] = -1;
    if (t->fragile) t->fragile[e] = 0;
    if (t->napprox) t->napprox[e] = 0;
  }
}

/* ------------------------------------------------------------------------ */
/* E1: iACT approximate input memoization (section 2.3; GPU form 3.1.4, 3.3) */
/* Tables are shared by groups of 64/g consecutive lanes of a wave          */
/* (g = tables per wave).  Read phase: each lane finds its nearest valid    */
/* entry (Euclidean distance over the inputs; squared distance in FP32).    */
/* Criterion: table non-empty and distance below the threshold.  Decision:  */
/* per group of `group` lanes by majority (group 1 = thread level).  A lane  */
/* of an approximating group returns its nearest entry's outputs; a lane    */
/* whose table is empty cannot and computes.  Write phase: in each table    */
/* that had computing lanes, the computing lane farthest from every stored  */
/* entry (+inf for an empty table; lowest lane on ties) inserts its inputs  */
/* and outputs at the round-robin slot.                                     */
/* ------------------------------------------------------------------------ */

static float or_dist2_f32(const float *a, const float *b, int d) {
  float t = a[0] - b[0];
  float acc = t * t;
  for (int j = 1; j < d; ++j) {
    float u = a[j] - b[j];
    acc = fmaf(u, u, acc);
  }
  return acc;
}

/* The plain definition: the squared Euclidean distance in FP64 of the two
 * FP32 points, summed over the coordinates in order. */
static double or_dist2_f64(const float *a, const float *b, int d) {
  double acc = 0.0;
  for (int j = 0; j < d; ++j) {
    double u = (double)a[j] - (double)b[j];
    acc += u * u;
  }
  return acc;
}

#define OR_MAX_IN 8
#define OR_MAX_OUT 16
#define OR_MAX_T 64

/* dist_fp64 selects the reading of the distance: 0 = the squared distance,
 * its threshold and their comparison in FP32 with the fixed rounding order
 * of or_dist2_f32 (the precision the GPU decides in); 1 = the plain FP64
 * definition (or_dist2_f64, compared with theta^2 in FP64).  With fragile
 * != NULL, a (wave, step) is marked where a statistic lies so close to the
 * point where a choice changes that the other precision could choose
 * differently: (i) lanes whose distance is within band * theta of theta
 * could flip their group's majority, (ii) a table's two farthest computing
 * lanes (writer candidates) are within `band` relative of each other, or
 * (iii) an approximating lane's two nearest entries with different outputs
 * are within `band` relative of each other. */
int or_iact(int64_t n, int32_t ipt, int32_t group, int32_t n_in,
            const float *const *x, int32_t n_out, const double *const *ysrc,
            const double *const *ssrc, int32_t tsize, float theta,
            int32_t tables_per_wave, double *const *out, double *const *oscale,
            int8_t *dec, int16_t *votes, int16_t *writer, int16_t *napprox,
            int64_t *n_evals, int32_t dist_fp64, double band, uint8_t *fragile) {
  if (n_in < 1 || n_in > OR_MAX_IN || n_out < 1 || n_out > OR_MAX_OUT) return -1;
  if (tsize < 1 || tsize > OR_MAX_T) return -1;
  if (tables_per_wave < 1 || OR_WAVE % tables_per_wave) return -1;
  if (group < 1 || (group != 1 && group % OR_WAVE)) return -1;
  int64_t L = or_num_lanes(n, ipt);
  int64_t nwaves = L / OR_WAVE;
  or_trace tr = {dec, votes, writer, fragile, napprox};
  or_trace_init(&tr, nwaves * ipt);
  const float thr2_f32 = theta * theta;
  const double thr2_f64 = (double)theta * (double)theta;
  const double th = (double)theta;
  const int lanes_per_table = OR_WAVE / tables_per_wave;
  /* Decision groups never straddle a work unit: a unit is one wave for
   * thread and wave level, one block of `group` lanes for block level. */
  const int64_t unit = group > OR_WAVE ? group : OR_WAVE;
  const int64_t nunits = (L + unit - 1) / unit;
  int64_t evals = 0;

#pragma omp parallel for schedule(dynamic, 16) reduction(+ : evals)
  for (int64_t u = 0; u < nunits; ++u) {
    const int64_t l0 = u * unit;
    const int64_t nl = (l0 + unit <= L) ? unit : (L - l0);
    const int ntab = (int)(nl / OR_WAVE) * tables_per_wave;
    /* table storage, per table: entries of (x, y, scale) */
    float *tx = calloc((size_t)ntab * tsize * n_in, sizeof(float));
    double *ty = calloc((size_t)ntab * tsize * n_out, sizeof(double));
    double *ts = calloc((size_t)ntab * tsize * n_out, sizeof(double));
    int *tcount = calloc(ntab, sizeof(int));
    int64_t *tins = calloc(ntab, sizeof(int64_t));
    double *md2 = malloc(nl * sizeof(double)); /* an FP32 value in FP32 mode */
    double *sec = malloc(nl * sizeof(double)); /* second-nearest entry with other outputs */
    int *arg = malloc(nl * sizeof(int));
    int *hit = malloc(nl * sizeof(int));
    int *computes = malloc(nl * sizeof(int));
    int *gdec = calloc((nl + group - 1) / group, sizeof(int));
    float xi[OR_MAX_IN];

    for (int32_t k = 0; k < ipt; ++k) {
      /* read phase */
      for (int64_t j = 0; j < nl; ++j) {
        int64_t i = l0 + j + (int64_t)k * L;
        hit[j] = 0; md2[j] = INFINITY; sec[j] = INFINITY; arg[j] = -1; computes[j] = 0;
        if (i >= n) continue;
        int tb = (int)(j / lanes_per_table);
        for (int d = 0; d < n_in; ++d) xi[d] = x[d][i];
        for (int e = 0; e < tcount[tb]; ++e) {
          const float *ex = &tx[((size_t)tb * tsize + e) * n_in];
          double d2 = dist_fp64 ? or_dist2_f64(xi, ex, n_in) : (double)or_dist2_f32(xi, ex, n_in);
          if (d2 < md2[j]) { md2[j] = d2; arg[j] = e; }
        }
        if (fragile && arg[j] >= 0) {
          /* the nearest entry whose outputs differ from the chosen one's */
          const double *ya = &ty[((size_t)tb * tsize + arg[j]) * n_out];
          for (int e = 0; e < tcount[tb]; ++e) {
            const double *ye = &ty[((size_t)tb * tsize + e) * n_out];
            int same = 1;
            for (int o = 0; o < n_out; ++o) same &= ye[o] == ya[o];
            if (same) continue;
            const float *ex = &tx[((size_t)tb * tsize + e) * n_in];
            double d2 = dist_fp64 ? or_dist2_f64(xi, ex, n_in) : (double)or_dist2_f32(xi, ex, n_in);
            if (d2 < sec[j]) sec[j] = d2;
          }
        }
        hit[j] = tcount[tb] > 0 && (dist_fp64 ? md2[j] < thr2_f64 : (float)md2[j] < thr2_f32);
      }
      /* decision per group, then each lane's path */
      for (int64_t g0 = 0; g0 < nl; g0 += group) {
        int act = 0, yes = 0;
        for (int64_t j = g0; j < g0 + group && j < nl; ++j) {
          if (l0 + j + (int64_t)k * L < n) { act++; yes += hit[j]; }
        }
        if (!act) continue;
        int approx = or_majority(yes, act);
        gdec[g0 / group] = approx;
        if (fragile && th > 0.0) {
          /* (i): lanes whose distance lies within band * theta of theta */
          int near_yes = 0, near_no = 0;
          for (int64_t j = g0; j < g0 + group && j < nl; ++j) {
            if (l0 + j + (int64_t)k * L >= n || arg[j] < 0) continue;
            if (fabs(sqrt(md2[j]) - th) <= band * th) { if (hit[j]) near_yes++; else near_no++; }
          }
          int flip = group == 1 ? near_yes + near_no > 0
                                : or_majority(yes - near_yes, act) != or_majority(yes + near_no, act);
          for (int64_t wl = g0 / OR_WAVE; flip && wl * OR_WAVE < g0 + group && wl * OR_WAVE < nl; ++wl)
            fragile[(l0 / OR_WAVE + wl) * ipt + k] = 1;
        }
        for (int64_t j = g0; j < g0 + group && j < nl; ++j) {
          int64_t i = l0 + j + (int64_t)k * L;
          if (i >= n) continue;
          int tb = (int)(j / lanes_per_table);
          int lane_approx = group == 1 ? hit[j] : approx;
          if (fragile && lane_approx && arg[j] >= 0 && sqrt(sec[j]) - sqrt(md2[j]) <= band * sqrt(sec[j]))
            fragile[((l0 + j) / OR_WAVE) * ipt + k] = 1; /* (iii) */
          if (lane_approx && arg[j] >= 0) {
            for (int o = 0; o < n_out; ++o) {
              out[o][i] = ty[((size_t)tb * tsize + arg[j]) * n_out + o];
              if (oscale) oscale[o][i] = ts[((size_t)tb * tsize + arg[j]) * n_out + o];
            }
          } else {
            computes[j] = 1;
            evals++;
            for (int o = 0; o < n_out; ++o) {
              out[o][i] = ysrc[o][i];
              if (oscale) oscale[o][i] = ssrc ? ssrc[o][i] : 0.0;
            }
          }
        }
      }
      /* write phase: one writer per table among its computing lanes */
      int64_t w_first = l0 / OR_WAVE;
      for (int tb = 0; tb < ntab; ++tb) {
        int64_t j0 = (int64_t)tb * lanes_per_table;
        int64_t best = -1, second = -1;
        for (int64_t j = j0; j < j0 + lanes_per_table; ++j) {
          if (!computes[j]) continue;
          if (best < 0 || md2[j] > md2[best]) { second = best; best = j; }
          else if (second < 0 || md2[j] > md2[second]) second = j;
        }
        /* (ii): two writer candidates at finite distances within band */
        if (fragile && second >= 0 && isfinite(md2[best]) &&
            sqrt(md2[best]) - sqrt(md2[second]) <= band * sqrt(md2[best]))
          fragile[((l0 + j0) / OR_WAVE) * ipt + k] = 1;
        if (best >= 0) {
          int64_t i = l0 + best + (int64_t)k * L;
          int slot = (int)(tins[tb] % tsize);
          for (int d = 0; d < n_in; ++d) tx[((size_t)tb * tsize + slot) * n_in + d] = x[d][i];
          for (int o = 0; o < n_out; ++o) {
            ty[((size_t)tb * tsize + slot) * n_out + o] = out[o][i];
            ts[((size_t)tb * tsize + slot) * n_out + o] = oscale ? oscale[o][i] : 0.0;
          }
          if (tcount[tb] < tsize) tcount[tb]++;
          tins[tb]++;
        }
        if (writer && tb % tables_per_wave == 0) {
          int64_t w = w_first + tb / tables_per_wave;
          writer[w * ipt + k] = best < 0 ? -1 : (int16_t)(best - (int64_t)(tb / tables_per_wave) * OR_WAVE);
        }
      }
      /* per-wave record: for wave and block level the group decision, for
       * thread level whether any lane approximated */
      for (int64_t wl = 0; wl < nl / OR_WAVE; ++wl) {
        int64_t w = w_first + wl;
        int act = 0, yes = 0, na = 0;
        for (int64_t j = wl * OR_WAVE; j < (wl + 1) * OR_WAVE; ++j) {
          if (l0 + j + (int64_t)k * L >= n) continue;
          act++; yes += hit[j]; na += !computes[j];
        }
        if (!act) continue;
        if (dec) dec[w * ipt + k] = (int8_t)(group == 1 ? (na > 0) : gdec[wl * OR_WAVE / group]);
        if (votes) votes[w * ipt + k] = (int16_t)yes;
        if (napprox) napprox[w * ipt + k] = (int16_t)na;
      }
    }
    free(tx); free(ty); free(ts); free(tcount); free(tins);
    free(md2); free(sec); free(arg); free(hit); free(computes); free(gdec);
  }
  if (n_evals) *n_evals = evals;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* E2: TAF output memoization (section 2.3; GPU form 3.1.3, 3.3).  Each     */
/* lane keeps a sliding window of its last h accurate outputs across its    */
/* grid-stride steps.  After each accurate step with a full window, the     */
/* lane's criterion is RSD < theta, RSD = sigma/|mu| (population sigma),    */
/* taken as the maximum over the region's outputs; RSD = 0 when sigma = 0   */
/* and +inf when mu = 0 < sigma.  When the group's majority holds, the      */
/* group is in the stable regime for the next p steps: each active lane    */
/* returns its last accurately computed output without evaluating the       */
/* region.  The window is not reset by a stable regime.                     */
/* `band` marks lanes whose RSD lies within band*theta of theta.            */
/* State across launches (st non-NULL): each lane's window, fill, last       */
/* output (and its tolerance scale) and its group's remaining approximate    */
/* steps are read from st at the start and written back at the end, so a    */
/* launch continues every lane's sequence of steps where the previous        */
/* launch of the same shape left it (a state of zeros is a fresh start).     */
/* ------------------------------------------------------------------------ */

static double or_rsd(const double *w, int h) {
  double mu = 0.0;
  for (int q = 0; q < h; ++q) mu += w[q];
  mu /= h;
  double var = 0.0;
  for (int q = 0; q < h; ++q) var += (w[q] - mu) * (w[q] - mu);
  var /= h;
  double sigma = sqrt(var);
  if (sigma == 0.0) return 0.0;
  if (mu == 0.0) return INFINITY;
  return sigma / fabs(mu);
}

#define OR_MAX_H 64

/* A launch's TAF state, per logical lane l of L (the oracle's own layout):
 * win[(l * n_out + o) * h + q] (q = 0 the oldest of the fill entries),
 * last and lasts [l * n_out + o], fill[l], rho[l] (the group's countdown,
 * the same for every lane of a group). */
typedef struct {
  double *win, *last, *lasts;
  int32_t *fill, *rho;
} or_taf_state;

int or_taf(int64_t n, int32_t ipt, int32_t group, int32_t n_out,
           const double *const *ysrc, const double *const *ssrc, int32_t hsize,
           int32_t psize, float theta, double band, double *const *out,
           double *const *oscale, int8_t *dec, int16_t *votes, uint8_t *fragile,
           int16_t *napprox, int64_t *n_evals, const or_taf_state *st) {
  if (n_out < 1 || n_out > OR_MAX_OUT || hsize < 1 || hsize > OR_MAX_H || psize < 1) return -1;
  if (group < 1 || (group != 1 && group % OR_WAVE)) return -1;
  int64_t L = or_num_lanes(n, ipt);
  int64_t nwaves = L / OR_WAVE;
  or_trace tr = {dec, votes, NULL, fragile, napprox};
  or_trace_init(&tr, nwaves * ipt);
  const double th = (double)theta;
  const int64_t unit = group > OR_WAVE ? group : OR_WAVE;
  const int64_t nunits = (L + unit - 1) / unit;
  int64_t evals = 0;

#pragma omp parallel for schedule(dynamic, 16) reduction(+ : evals)
  for (int64_t u = 0; u < nunits; ++u) {
    const int64_t l0 = u * unit;
    const int64_t nl = (l0 + unit <= L) ? unit : (L - l0);
    const int64_t ngroups = (nl + group - 1) / group;
    /* window[j][o][q], q = 0 oldest */
    double *win = calloc((size_t)nl * n_out * hsize, sizeof(double));
    double *last = calloc((size_t)nl * n_out, sizeof(double));
    double *lasts = calloc((size_t)nl * n_out, sizeof(double));
    int *fill = calloc(nl, sizeof(int));
    int *rho = calloc(ngroups, sizeof(int));
    int *crit = calloc(nl, sizeof(int));
    int *near = calloc(nl, sizeof(int));
    int *took = calloc(nl, sizeof(int));
    int *voted = calloc(nl, sizeof(int));
    if (st) {
      for (int64_t j = 0; j < nl; ++j) {
        const int64_t l = l0 + j;
        for (int o = 0; o < n_out; ++o) {
          for (int q = 0; q < hsize; ++q)
            win[((size_t)j * n_out + o) * hsize + q] = st->win[((size_t)l * n_out + o) * hsize + q];
          last[j * n_out + o] = st->last[l * n_out + o];
          lasts[j * n_out + o] = st->lasts[l * n_out + o];
        }
        fill[j] = st->fill[l];
      }
      for (int64_t gi = 0; gi < ngroups; ++gi) rho[gi] = st->rho[l0 + gi * group];
    }

    for (int32_t k = 0; k < ipt; ++k) {
      for (int64_t gi = 0; gi < ngroups; ++gi) {
        int64_t g0 = gi * group, g1 = g0 + group < nl ? g0 + group : nl;
        int act = 0;
        for (int64_t j = g0; j < g1; ++j) {
          took[j] = 0; crit[j] = 0; near[j] = 0; voted[j] = 0;
          if (l0 + j + (int64_t)k * L < n) act++;
        }
        if (!act) continue;
        if (rho[gi] > 0) {
          for (int64_t j = g0; j < g1; ++j) {
            int64_t i = l0 + j + (int64_t)k * L;
            if (i >= n) continue;
            took[j] = 1;
            for (int o = 0; o < n_out; ++o) {
              out[o][i] = last[j * n_out + o];
              if (oscale) oscale[o][i] = lasts[j * n_out + o];
            }
          }
          rho[gi]--;
          continue;
        }
        int yes = 0, full = 1, near_yes = 0, near_no = 0;
        for (int64_t j = g0; j < g1; ++j) {
          int64_t i = l0 + j + (int64_t)k * L;
          if (i >= n) continue;
          evals++;
          double *wj = &win[(size_t)j * n_out * hsize];
          for (int o = 0; o < n_out; ++o) {
            double y = ysrc[o][i];
            out[o][i] = y;
            if (oscale) oscale[o][i] = ssrc ? ssrc[o][i] : 0.0;
            last[j * n_out + o] = y;
            lasts[j * n_out + o] = ssrc ? ssrc[o][i] : 0.0;
            double *wo = &wj[o * hsize];
            if (fill[j] < hsize) {
              wo[fill[j]] = y;
            } else {
              for (int q = 0; q + 1 < hsize; ++q) wo[q] = wo[q + 1];
              wo[hsize - 1] = y;
            }
          }
          if (fill[j] < hsize) fill[j]++;
          if (fill[j] < hsize) { full = 0; continue; }
          double rsd = 0.0;
          for (int o = 0; o < n_out; ++o) {
            double ro = or_rsd(&wj[o * hsize], hsize);
            if (ro > rsd || isnan(ro)) rsd = ro;
          }
          crit[j] = rsd < th;
          yes += crit[j];
          if (th > 0.0 && fabs(rsd - th) <= band * th) {
            near[j] = 1;
            if (crit[j]) near_yes++; else near_no++;
          }
        }
        if (!full) continue;
        for (int64_t j = g0; j < g1; ++j) voted[j] = l0 + j + (int64_t)k * L < n;
        int approx = group == 1 ? crit[g0] : or_majority(yes, act);
        if (approx) rho[gi] = psize;
        if (fragile) {
          int flip = group == 1 ? near[g0]
                                : or_majority(yes - near_yes, act) != or_majority(yes + near_no, act);
          if (flip) fragile[((l0 + g0) / OR_WAVE) * ipt + k] = 1;
          for (int64_t wl = g0 / OR_WAVE + 1; flip && wl * OR_WAVE < g1; ++wl)
            fragile[(l0 / OR_WAVE + wl) * ipt + k] = 1;
        }
      }
      /* per-wave decisions for this step */
      for (int64_t wl = 0; wl < nl / OR_WAVE; ++wl) {
        int64_t w = l0 / OR_WAVE + wl;
        int act = 0, na = 0;
        for (int64_t j = wl * OR_WAVE; j < (wl + 1) * OR_WAVE; ++j) {
          if (l0 + j + (int64_t)k * L >= n) continue;
          act++; na += took[j];
        }
        if (!act) continue;
        if (dec) dec[w * ipt + k] = na > 0;
        if (napprox) napprox[w * ipt + k] = (int16_t)na;
        if (votes) {
          int nv = 0, wy = 0;
          for (int64_t j = wl * OR_WAVE; j < (wl + 1) * OR_WAVE; ++j) { nv += voted[j]; wy += voted[j] && crit[j]; }
          votes[w * ipt + k] = nv ? (int16_t)wy : -1;
        }
      }
    }
    if (st) {
      for (int64_t j = 0; j < nl; ++j) {
        const int64_t l = l0 + j;
        for (int o = 0; o < n_out; ++o) {
          for (int q = 0; q < hsize; ++q)
            st->win[((size_t)l * n_out + o) * hsize + q] = win[((size_t)j * n_out + o) * hsize + q];
          st->last[l * n_out + o] = last[j * n_out + o];
          st->lasts[l * n_out + o] = lasts[j * n_out + o];
        }
        st->fill[l] = fill[j];
        st->rho[l] = rho[j / group];
      }
    }
    free(win); free(last); free(lasts); free(fill); free(rho);
    free(crit); free(near); free(took); free(voted);
  }
  if (n_evals) *n_evals = evals;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* E3: loop perforation (section 2.3; herded form 3.1.5; runtime 3.3).      */
/* kind 0 small: skip step k iff (k + offset) mod M = M - 1.                */
/* kind 1 large: execute step k iff (k + offset) mod M = 0.                 */
/* kind 2 ini:  skip items i < floor(p n / 100).                            */
/* kind 3 fini: skip items i >= n - floor(p n / 100).                       */
/* Herded: the pattern depends on the step only, identical for every lane.  */
/* A skipped item is neither read nor written.  param 0 = no perforation.   */
/* ------------------------------------------------------------------------ */

int or_perfo(int64_t n, int32_t ipt, int32_t n_out, const double *const *ysrc,
             const double *const *ssrc, int32_t kind, int32_t param,
             int32_t offset, double *const *out, double *const *oscale,
             int8_t *dec, int64_t *n_evals) {
  if (kind < 0 || kind > 3 || param < 0) return -1;
  if ((kind == 2 || kind == 3) && param > 100) return -1;
  int64_t L = or_num_lanes(n, ipt);
  int64_t nwaves = L / OR_WAVE;
  or_trace tr = {dec, NULL, NULL, NULL, NULL};
  or_trace_init(&tr, nwaves * ipt);
  const int64_t cut = (kind >= 2) ? ((int64_t)param * n) / 100 : 0;
  int64_t evals = 0;
#pragma omp parallel for schedule(static) reduction(+ : evals)
  for (int64_t w = 0; w < nwaves; ++w) {
    for (int32_t k = 0; k < ipt; ++k) {
      int64_t kk = (int64_t)k + offset;
      int skip_step = 0;
      if (param > 0 && kind == 0) skip_step = (kk % param) == param - 1;
      if (param > 0 && kind == 1) skip_step = (kk % param) != 0;
      int any = 0, nsk = 0;
      for (int j = 0; j < OR_WAVE; ++j) {
        int64_t i = w * OR_WAVE + j + (int64_t)k * L;
        if (i >= n) continue;
        any = 1;
        int skip = skip_step;
        if (kind == 2) skip = i < cut;
        if (kind == 3) skip = i >= n - cut;
        if (skip) { nsk++; continue; }
        evals++;
        for (int o = 0; o < n_out; ++o) {
          out[o][i] = ysrc[o][i];
          if (oscale) oscale[o][i] = ssrc ? ssrc[o][i] : 0.0;
        }
      }
      if (any && dec) dec[w * ipt + k] = nsk > 0;
    }
  }
  if (n_evals) *n_evals = evals;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* M: mean absolute percentage error (section 4, the MAPE equation), as a   */
/* fraction.  The denominator is floored: max(|O_ac|, tau), so that outputs */
/* that are zero or vanishingly small do not make the mean diverge.         */
/* Also returns how many entries were floored and the MAPE over the rest.   */
/* ------------------------------------------------------------------------ */

void or_mape(int64_t m, const double *exact, const double *approx, double tau,
             double *mape, int64_t *n_floored, double *mape_rest) {
  double s = 0.0, sr = 0.0;
  int64_t nf = 0;
  for (int64_t e = 0; e < m; ++e) {
    double a = fabs(exact[e]);
    double err = fabs(exact[e] - approx[e]);
    if (a < tau) {
      nf++;
      s += err / tau;
    } else {
      s += err / a;
      sr += err / a;
    }
  }
  *mape = m ? s / (double)m : 0.0;
  *n_floored = nf;
  *mape_rest = (m - nf) ? sr / (double)(m - nf) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* R3: the MLP surrogate 5 -> 64 -> 64 -> 2 used as a further approximation  */
/* of the Black-Scholes region.  Inputs are mapped affinely,                */
/* xh_j = (x_j - c_j) * s_j; outputs are mapped back, y_o = yh_o * sc_o +     */
/* mu_o.  Hidden layers use the tanh form of GELU,                          */
/* gelu(x) = x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))).                   */
/* Parameters are one array: W1[64][5], b1[64], W2[64][64], b2[64],          */
/* W3[2][64], b3[2] (row = output unit).  The weights are rounded to BF16    */
/* (round to nearest even) before use; biases are used as given.  With       */
/* round_act the layer inputs (xh, h1, h2) are rounded to BF16 as well.      */
/* act = 0 replaces GELU by the identity (a pin against plain products).     */
/* ------------------------------------------------------------------------ */

#define OR_NH 64
#define OR_P (64 * 5 + 64 + 64 * 64 + 64 + 2 * 64 + 2)
#define OR_OFF_B1 (64 * 5)
#define OR_OFF_W2 (OR_OFF_B1 + 64)
#define OR_OFF_B2 (OR_OFF_W2 + 64 * 64)
#define OR_OFF_W3 (OR_OFF_B2 + 64)
#define OR_OFF_B3 (OR_OFF_W3 + 2 * 64)

int32_t or_mlp_num_params(void) { return OR_P; }

/* nearest BF16 (8 significant bits), ties to even */
double or_bf16(double v) {
  if (v == 0.0 || !isfinite(v)) return v;
  int e;
  double m = frexp(v, &e); /* v = m 2^e, 0.5 <= |m| < 1 */
  double r = nearbyint(ldexp(m, 8));
  return ldexp(r, e - 8);
}

static double or_gelu(double x, int act) {
  if (!act) return x;
  const double k = sqrt(2.0 / M_PI);
  return 0.5 * x * (1.0 + tanh(k * (x + 0.044715 * x * x * x)));
}

static double or_gelu_d(double x, int act) {
  if (!act) return 1.0;
  const double k = sqrt(2.0 / M_PI);
  double u = k * (x + 0.044715 * x * x * x);
  double t = tanh(u);
  return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * k * (1.0 + 3.0 * 0.044715 * x * x);
}

typedef struct {
  double xh[5], z1[OR_NH], h1[OR_NH], z2[OR_NH], h2[OR_NH], yh[2];
} or_mlp_act;

static void or_mlp_fwd1(const double *w, const double *xin, const double *c, const double *s, int round_act,
                        int act, or_mlp_act *A) {
  for (int j = 0; j < 5; ++j) {
    A->xh[j] = (xin[j] - c[j]) * s[j];
    if (round_act) A->xh[j] = or_bf16(A->xh[j]);
  }
  for (int o = 0; o < OR_NH; ++o) {
    double z = w[OR_OFF_B1 + o];
    for (int j = 0; j < 5; ++j) z += or_bf16(w[o * 5 + j]) * A->xh[j];
    A->z1[o] = z;
    A->h1[o] = or_gelu(z, act);
    if (round_act) A->h1[o] = or_bf16(A->h1[o]);
  }
  for (int o = 0; o < OR_NH; ++o) {
    double z = w[OR_OFF_B2 + o];
    for (int j = 0; j < OR_NH; ++j) z += or_bf16(w[OR_OFF_W2 + o * OR_NH + j]) * A->h1[j];
    A->z2[o] = z;
    A->h2[o] = or_gelu(z, act);
    if (round_act) A->h2[o] = or_bf16(A->h2[o]);
  }
  for (int o = 0; o < 2; ++o) {
    double z = w[OR_OFF_B3 + o];
    for (int j = 0; j < OR_NH; ++j) z += or_bf16(w[OR_OFF_W3 + o * OR_NH + j]) * A->h2[j];
    A->yh[o] = z;
  }
}

/* y (2 columns) = the surrogate's outputs for n items; x is 5 columns.  The
 * output map: v = yh sc + mu, and y = v, or exp(v) - sh where sh > 0 (the
 * network then models log(y + sh)). */
void or_mlp_forward(int64_t n, const double *const *x, const double *w, const double *c, const double *s,
                    const double *mu, const double *sc, const double *sh, int32_t round_act, int32_t act,
                    double *const *y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double xin[5];
    or_mlp_act A;
    for (int j = 0; j < 5; ++j) xin[j] = x[j][i];
    or_mlp_fwd1(w, xin, c, s, round_act, act, &A);
    for (int o = 0; o < 2; ++o) {
      const double v = A.yh[o] * sc[o] + mu[o];
      y[o][i] = sh[o] > 0.0 ? exp(v) - sh[o] : v;
    }
  }
}

/* Mean squared error over the n items and 2 outputs in the normalised output
 * space, L = 1/(2n) sum_i sum_o (yh_o - (g_o(t_o) - mu_o)/sc_o)^2, g_o(t) = t,
 * or log(t + sh_o) where sh_o > 0, with FP64 activations, and its gradient
 * with respect to every parameter (through the BF16 rounding of the weights
 * as if it were the identity). */
double or_mlp_loss_grad(int64_t n, const double *const *x, const double *const *t, const double *w,
                        const double *c, const double *s, const double *mu, const double *sc, const double *sh,
                        int32_t act, double *grad) {
  double loss = 0.0;
  for (int p = 0; p < OR_P; ++p) grad[p] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double xin[5], dy[2], dz2[OR_NH], dz1[OR_NH];
    or_mlp_act A;
    for (int j = 0; j < 5; ++j) xin[j] = x[j][i];
    or_mlp_fwd1(w, xin, c, s, 0, act, &A);
    for (int o = 0; o < 2; ++o) {
      const double g = sh[o] > 0.0 ? log(t[o][i] + sh[o]) : t[o][i];
      double e = A.yh[o] - (g - mu[o]) / sc[o];
      loss += e * e;
      dy[o] = 2.0 * e / (2.0 * (double)n);
      grad[OR_OFF_B3 + o] += dy[o];
      for (int j = 0; j < OR_NH; ++j) grad[OR_OFF_W3 + o * OR_NH + j] += dy[o] * A.h2[j];
    }
    for (int j = 0; j < OR_NH; ++j) {
      double dh = 0.0;
      for (int o = 0; o < 2; ++o) dh += or_bf16(w[OR_OFF_W3 + o * OR_NH + j]) * dy[o];
      dz2[j] = dh * or_gelu_d(A.z2[j], act);
      grad[OR_OFF_B2 + j] += dz2[j];
    }
    for (int o = 0; o < OR_NH; ++o)
      for (int j = 0; j < OR_NH; ++j) grad[OR_OFF_W2 + o * OR_NH + j] += dz2[o] * A.h1[j];
    for (int j = 0; j < OR_NH; ++j) {
      double dh = 0.0;
      for (int o = 0; o < OR_NH; ++o) dh += or_bf16(w[OR_OFF_W2 + o * OR_NH + j]) * dz2[o];
      dz1[j] = dh * or_gelu_d(A.z1[j], act);
      grad[OR_OFF_B1 + j] += dz1[j];
    }
    for (int o = 0; o < OR_NH; ++o)
      for (int j = 0; j < 5; ++j) grad[o * 5 + j] += dz1[o] * A.xh[j];
  }
  return loss / (2.0 * (double)n);
}

double or_mlp_gelu(double x) { return or_gelu(x, 1); }

/* ------------------------------------------------------------------------ */
/* Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization",        */
/* ICLR 2015, Algorithm 1) in FP64: the surrogate's optimiser.  The          */
/* gradient is the sum of `blocks` partial gradients of p parameters each    */
/* (partials[b * p + q]); t >= 1 is the step number of the bias correction. */
/*   m <- beta1 m + (1 - beta1) g;  v <- beta2 v + (1 - beta2) g^2           */
/*   w <- w - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps)      */
/* ------------------------------------------------------------------------ */
void or_adam(int64_t p, int64_t blocks, const double *partials, double *w, double *m, double *v, double lr,
             double beta1, double beta2, double eps, int32_t t) {
  const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
  for (int64_t q = 0; q < p; ++q) {
    double g = 0.0;
    for (int64_t b = 0; b < blocks; ++b) g += partials[b * p + q];
    m[q] = beta1 * m[q] + (1.0 - beta1) * g;
    v[q] = beta2 * v[q] + (1.0 - beta2) * g * g;
    w[q] -= lr * (m[q] / c1) / (sqrt(v[q] / c2) + eps);
  }
}

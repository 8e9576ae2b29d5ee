/*
 * CPU oracle, part 2: a staggered-grid Lagrangian hydrodynamics step on a
 * structured hexahedral mesh (a Sedov point blast), in FP64, with the
 * approximation techniques of the paper applied to two of its per-element
 * regions across timesteps.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c): only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header or constant with the GPU library.
 *
 * The paper evaluates its techniques on a hydrodynamics proxy that models a
 * Sedov blast on volumetric elements, with the final energy at the origin as
 * quantity of interest (section 4, Table 1), and approximates its hourglass
 * force computation (section 4.1, the hydrodynamics results).  That code is
 * not reproduced here: this is a scheme of our own built from published
 * methods, and the GPU library implements the same discretisation.
 *
 * Scheme (one step n -> n+1, time step dt^n in FP64):
 *   mesh     n^3 elements on [0, side]^3, (n+1)^3 nodes; element (i,j,k) has
 *            corners (i+a, j+b, k+c) for a,b,c in {0,1}, local corner index
 *            a + 2b + 4c and reference coordinates s = (2a-1, 2b-1, 2c-1).
 *            Symmetry planes x=0, y=0, z=0; the outer faces are free.
 *   volume   V = sum over the 2x2x2 Gauss points of det J (exact for the
 *            trilinear map), and B = dV/dx_corner (24 values) from the
 *            cofactors of J.
 *   forces   corner force = (p + q) B + hourglass force; the hourglass force
 *            is the viscous Flanagan-Belytschko (1981) form: hourglass base
 *            vectors Gamma (products of reference coordinates), made
 *            orthogonal to linear fields, gamma = Gamma - (1/V) sum_i
 *            (Gamma . x_i) B_i, mode rates h_a = gamma_a . u, force
 *            -(khg/8) rho c V^(2/3) sum_a gamma_a h_a.
 *   momentum node force = sum of its corner forces, gathered over the
 *            adjacent elements in corner order 0..7 (no atomics);
 *            u^{n+1} = u^n + dt F / M; zero normal velocity on the symmetry
 *            planes; x^{n+1} = x^n + dt (u^n + u^{n+1}) / 2.
 *   energy   compatible total-energy update (Caramana, Burton, Shashkov,
 *            Whalen 1998): m (e^{n+1} - e^n) = -dt sum_corners F . u^{n+1/2},
 *            so internal plus kinetic energy is conserved to rounding.
 *   EOS      ideal gas p = (gamma - 1) rho e; von Neumann-Richtmyer
 *            viscosity q = rho (cq du^2 + cl c |du|) under compression,
 *            du = (dV/dt) / (V^{n+1})^(2/3), dV/dt = sum B(x^{n+1}) .
 *            u^{n+1/2} (the volume rate, not a difference of volumes);
 *            c = sqrt(gamma max(p, 0) / rho).
 *   dt       dt^n = min(growth dt^{n-1}, min over elements of
 *            cfl V^(1/3) / sqrt(gamma max(p + q, 0) / rho) and of
 *            dvmax V / |dV/dt|, dV/dt = sum B . u), at time n.
 *
 * Approximated regions (the paper's techniques, applied per element with
 * one item per lane and one launch per timestep, so a wave is 64
 * consecutive elements and the "steps" of TAF are timesteps):
 *   hourglass region: inputs the element's corner coordinates and
 *            velocities, volume, B, density and sound speed; outputs the 24
 *            hourglass corner forces, which the element adds to its corner
 *            forces.  TAF (section 3.1.3): an approximated element adds its
 *            last computed hourglass forces.  Herded perforation (section
 *            3.1.5) with the grid-stride mapping of the element loop and
 *            offset = timestep: a skipped iteration computes and adds
 *            nothing, so the element has no hourglass force that step.
 *   EOS region: inputs e, c, mass, the corner forces and the corner
 *            velocities before and after the step and the new corner
 *            positions; outputs e, p, q, c.  TAF: an approximated element
 *            keeps its previous e, p, q, c.
 * TAF decisions are taken per wave (majority of its lanes) or per element
 * (thread level, section 3.1.2); the state (windows, a countdown and a push
 * count per decision group) persists across timesteps in the state arrays.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HY_WAVE 64
#define HY_BLOCK 256 /* a workgroup of four waves: the team level of section 3.1.2 */
#define HY_MAX_H 16

typedef struct {
  int32_t n;      /* elements per side */
  double side;    /* edge of the cubic domain */
  double gamma;   /* ideal-gas ratio of specific heats */
  double cq, cl;  /* quadratic and linear artificial-viscosity coefficients */
  double khg;     /* hourglass coefficient */
  double cfl;     /* Courant factor */
  double growth;  /* largest ratio of consecutive time steps */
  double dvmax;   /* largest relative volume change of an element in one step */
  double dt0;     /* time step before the first step (the growth cap of step 0) */
} hy_par;

typedef struct {
  double *x[3], *u[3];      /* node positions and velocities (n+1)^3 */
  double *unew[3];          /* scratch: velocities after the step */
  double *mnode;            /* node masses */
  double *e, *p, *q, *c;    /* element specific energy, pressure, viscosity, sound speed */
  double *vol, *mass;       /* element volume (at the last force evaluation), mass */
  double *force;            /* corner forces [(corner*3 + dim) * E + z] */
  double *fhg;              /* last computed hourglass forces, same layout */
  double *weos;             /* EOS TAF window [(slot*4 + o) * E + z] */
  int32_t *rho_eos, *z_eos; /* per decision group: countdown, accurate pushes */
  double *whg;              /* hourglass TAF window [(slot*24 + o) * E + z] */
  int32_t *rho_hg, *z_hg;
  double *clock;            /* [0] time, [1] last time step */
} hy_state;

typedef struct {
  int32_t eos_h, eos_p;  /* EOS TAF: history and prediction sizes (h = 0: exact) */
  double eos_theta;
  int32_t eos_group;     /* lanes per decision: 1 (thread), 64 (wave) or 256 (block level) */
  int32_t hg_h, hg_p;    /* hourglass TAF (h = 0: none) */
  double hg_theta;
  int32_t hg_group;
  int32_t perfo_kind;    /* hourglass perforation: 0 small, 1 large, 2 ini, 3 fini */
  int32_t perfo_param;   /* M for small/large, percent for ini/fini; 0 = none */
  int32_t perfo_ipt;     /* items per lane of the perforated element loop */
  double band;           /* relative band around a threshold for the fragile record */
} hy_tech;

typedef struct {
  int8_t *dec_eos, *dec_hg;     /* per decision group: -1 none, 0 accurate, 1 approximate; NULL = none */
  uint8_t *frag_eos, *frag_hg;  /* per decision group: the vote flips within the band */
} hy_rec;

static inline int64_t hy_elems(const hy_par *P) { return (int64_t)P->n * P->n * P->n; }
static inline int64_t hy_nodes(const hy_par *P) { return (int64_t)(P->n + 1) * (P->n + 1) * (P->n + 1); }

/* node index of corner c of element z */
static inline int64_t hy_corner_node(const hy_par *P, int64_t z, int c) {
  const int64_t n = P->n, m = n + 1;
  const int64_t i = z % n, j = (z / n) % n, k = z / (n * n);
  return (i + (c & 1)) + m * ((j + ((c >> 1) & 1)) + m * (k + ((c >> 2) & 1)));
}

static inline double hy_sgn(int c, int d) { return ((c >> d) & 1) ? 1.0 : -1.0; }

/* Volume of the trilinear hexahedron with corner coordinates xc[c][d] and,
 * if B != NULL, its gradient B[c][d] = dV/dxc[c][d]. */
static double hy_volume(const double xc[8][3], double B[8][3]) {
  const double g = 1.0 / sqrt(3.0);
  double V = 0.0;
  if (B) memset(B, 0, sizeof(double) * 24);
  for (int qp = 0; qp < 8; ++qp) {
    const double xi[3] = {hy_sgn(qp, 0) * g, hy_sgn(qp, 1) * g, hy_sgn(qp, 2) * g};
    double dN[8][3];
    for (int c = 0; c < 8; ++c)
      for (int j = 0; j < 3; ++j) {
        double v = hy_sgn(c, j) / 8.0;
        for (int l = 0; l < 3; ++l)
          if (l != j) v *= 1.0 + hy_sgn(c, l) * xi[l];
        dN[c][j] = v;
      }
    double J[3][3] = {{0}};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int c = 0; c < 8; ++c) J[i][j] += xc[c][i] * dN[c][j];
    double cof[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        cof[i][j] = J[i1][j1] * J[i2][j2] - J[i1][j2] * J[i2][j1];
      }
    V += J[0][0] * cof[0][0] + J[0][1] * cof[0][1] + J[0][2] * cof[0][2];
    if (B)
      for (int c = 0; c < 8; ++c)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) B[c][i] += cof[i][j] * dN[c][j];
  }
  return V;
}

/* Flanagan-Belytschko viscous hourglass forces f[c][d] of one element. */
static void hy_hourglass(const double xc[8][3], const double uc[8][3], const double B[8][3], double V,
                         double rho, double c, double khg, double f[8][3]) {
  double gam[4][8];
  for (int a = 0; a < 4; ++a) {
    double G[8];
    for (int k = 0; k < 8; ++k) {
      const double s0 = hy_sgn(k, 0), s1 = hy_sgn(k, 1), s2 = hy_sgn(k, 2);
      G[k] = a == 0 ? s1 * s2 : a == 1 ? s0 * s2 : a == 2 ? s0 * s1 : s0 * s1 * s2;
    }
    double gx[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 8; ++k) gx[i] += G[k] * xc[k][i];
    for (int k = 0; k < 8; ++k) {
      double s = 0.0;
      for (int i = 0; i < 3; ++i) s += gx[i] * B[k][i];
      gam[a][k] = G[k] - s / V;
    }
  }
  const double coef = -(khg / 8.0) * rho * c * pow(V, 2.0 / 3.0);
  double h[4][3];
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) {
      h[a][i] = 0.0;
      for (int k = 0; k < 8; ++k) h[a][i] += gam[a][k] * uc[k][i];
    }
  for (int k = 0; k < 8; ++k)
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
      for (int a = 0; a < 4; ++a) s += gam[a][k] * h[a][i];
      f[k][i] = coef * s;
    }
}

/* ------------------------------------------------------------------ state */

int hy_init(const hy_par *P, double e_origin, hy_state *S) {
  if (P->n < 1) return -1;
  const int64_t n = P->n, m = n + 1, E = hy_elems(P), Nn = hy_nodes(P);
  const double h = P->side / n;
  for (int64_t k = 0; k < m; ++k)
    for (int64_t j = 0; j < m; ++j)
      for (int64_t i = 0; i < m; ++i) {
        const int64_t v = i + m * (j + m * k);
        S->x[0][v] = h * i;
        S->x[1][v] = h * j;
        S->x[2][v] = h * k;
        for (int d = 0; d < 3; ++d) S->u[d][v] = 0.0;
      }
  const double rho0 = 1.0;
  for (int64_t z = 0; z < E; ++z) {
    double xc[8][3];
    for (int c = 0; c < 8; ++c)
      for (int d = 0; d < 3; ++d) xc[c][d] = S->x[d][hy_corner_node(P, z, c)];
    S->vol[z] = hy_volume(xc, NULL);
    S->mass[z] = rho0 * S->vol[z];
    S->e[z] = z == 0 ? e_origin : 0.0;
    S->q[z] = 0.0;
    S->p[z] = (P->gamma - 1.0) * rho0 * S->e[z];
    S->c[z] = sqrt(P->gamma * fmax(S->p[z], 0.0) / rho0);
    for (int o = 0; o < 24; ++o) S->fhg[o * E + z] = 0.0;
  }
  /* node mass: an eighth of each adjacent element's mass, corner order 0..7 */
  for (int64_t v = 0; v < Nn; ++v) {
    const int64_t i = v % m, j = (v / m) % m, k = v / (m * m);
    double M = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int64_t ei = i - (c & 1), ej = j - ((c >> 1) & 1), ek = k - ((c >> 2) & 1);
      if (ei < 0 || ej < 0 || ek < 0 || ei >= n || ej >= n || ek >= n) continue;
      M += S->mass[ei + n * (ej + n * ek)] / 8.0;
    }
    S->mnode[v] = M;
  }
  /* decision-group state: sized for the finest grouping (one per element) */
  for (int64_t g = 0; g < E; ++g) {
    if (S->rho_eos) S->rho_eos[g] = 0, S->z_eos[g] = 0;
    if (S->rho_hg) S->rho_hg[g] = 0, S->z_hg[g] = 0;
  }
  S->clock[0] = 0.0;
  S->clock[1] = P->dt0;
  return 0;
}

/* ------------------------------------------------------------------- TAF */

/* RSD of the h values w[0], w[stride], ...: population sigma / |mu|, 0 if
 * sigma = 0, +inf if mu = 0 < sigma (section 2.2's TAF criterion). */
static double hy_rsd(const double *w, int h, int64_t stride) {
  double mu = 0.0;
  for (int s = 0; s < h; ++s) mu += w[s * stride];
  mu /= h;
  double var = 0.0;
  for (int s = 0; s < h; ++s) var += (w[s * stride] - mu) * (w[s * stride] - mu);
  var /= h;
  const double sigma = sqrt(var);
  if (sigma == 0.0) return 0.0;
  if (mu == 0.0) return INFINITY;
  return sigma / fabs(mu);
}

/* Push the lane's outputs y[0..nout) into slot z mod h of its window, and
 * return its criterion (RSD below theta) once the window is full (z + 1 >= h),
 * else -1.  *near is set when the statistic lies within band of theta. */
static int hy_taf_push(double *win, int64_t E, int64_t zel, int nout, int h, int32_t pushes, const double *y,
                       double theta, double band, int *near) {
  const int slot = pushes % h;
  for (int o = 0; o < nout; ++o) win[((int64_t)slot * nout + o) * E + zel] = y[o];
  *near = 0;
  if (pushes + 1 < h) return -1;
  double rsd = 0.0;
  for (int o = 0; o < nout; ++o) {
    const double r = hy_rsd(&win[(int64_t)o * E + zel], h, (int64_t)nout * E);
    if (r > rsd || isnan(r)) rsd = r;
  }
  if (theta > 0.0 && fabs(rsd - theta) <= band * theta) *near = 1;
  return rsd < theta;
}

static int hy_majority(int yes, int act) { return 2 * yes > act; }

/* ------------------------------------------------------------------ step */

static int hy_perfo_skip(const hy_tech *T, int64_t item, int64_t E, int32_t k, int32_t offset) {
  const int32_t M = T->perfo_param;
  if (M <= 0) return 0;
  switch (T->perfo_kind) {
    case 0: return (int32_t)(((int64_t)k + offset) % M) == M - 1;
    case 1: return (int32_t)(((int64_t)k + offset) % M) != 0;
    case 2: return item < (int64_t)M * E / 100;
    case 3: return item >= E - (int64_t)M * E / 100;
  }
  return 0;
}

static void hy_gather(const hy_par *P, const hy_state *S, int64_t z, double xc[8][3], double uc[8][3],
                      double *const src[3]) {
  for (int c = 0; c < 8; ++c) {
    const int64_t v = hy_corner_node(P, z, c);
    for (int d = 0; d < 3; ++d) {
      if (xc) xc[c][d] = S->x[d][v];
      if (uc) uc[c][d] = src[d][v];
    }
  }
}

/* Force phase for one element: V, B, pressure and hourglass corner forces.
 * hg: HY_HG_COMPUTE compute the hourglass forces (and remember them),
 * HY_HG_REUSE add the remembered ones, HY_HG_NONE add none.  Returns the
 * element's time-step bound. */
enum { HY_HG_NONE = 0, HY_HG_COMPUTE = 1, HY_HG_REUSE = 2 };
static double hy_force_elem(const hy_par *P, hy_state *S, int64_t z, int hg) {
  const int64_t E = hy_elems(P);
  double xc[8][3], uc[8][3], B[8][3], f[8][3];
  hy_gather(P, S, z, xc, uc, S->u);
  const double V = hy_volume(xc, B);
  S->vol[z] = V;
  const double rho = S->mass[z] / V;
  if (hg == HY_HG_COMPUTE) {
    hy_hourglass(xc, uc, B, V, rho, S->c[z], P->khg, f);
    if (S->fhg)
      for (int k = 0; k < 8; ++k)
        for (int d = 0; d < 3; ++d) S->fhg[(k * 3 + d) * E + z] = f[k][d];
  } else {
    for (int k = 0; k < 8; ++k)
      for (int d = 0; d < 3; ++d) f[k][d] = hg == HY_HG_REUSE ? S->fhg[(k * 3 + d) * E + z] : 0.0;
  }
  const double pq = S->p[z] + S->q[z];
  for (int k = 0; k < 8; ++k)
    for (int d = 0; d < 3; ++d) S->force[(k * 3 + d) * E + z] = pq * B[k][d] + f[k][d];
  const double ceff2 = P->gamma * fmax(pq, 0.0) / rho;
  double bound = ceff2 > 0.0 ? P->cfl * cbrt(V) / sqrt(ceff2) : INFINITY;
  /* relative volume change per step at most dvmax: dV/dt = sum B . u */
  double vdot = 0.0;
  for (int k = 0; k < 8; ++k)
    for (int d = 0; d < 3; ++d) vdot += B[k][d] * uc[k][d];
  if (vdot != 0.0) bound = fmin(bound, P->dvmax * V / fabs(vdot));
  return bound;
}

/* EOS region for one element (accurate path); y = (e, p, q, c).  Returns
 * the element's new volume. */
static double hy_eos_elem(const hy_par *P, const hy_state *S, int64_t z, double dt, double y[4]) {
  const int64_t E = hy_elems(P);
  double xc[8][3], u0[8][3], u1[8][3];
  hy_gather(P, S, z, xc, u0, S->u);
  hy_gather(P, S, z, NULL, u1, S->unew);
  double W = 0.0;
  for (int k = 0; k < 8; ++k)
    for (int d = 0; d < 3; ++d) W += S->force[(k * 3 + d) * E + z] * 0.5 * (u0[k][d] + u1[k][d]);
  double B1[8][3];
  const double V1 = hy_volume(xc, B1);
  double vdot = 0.0;
  for (int k = 0; k < 8; ++k)
    for (int d = 0; d < 3; ++d) vdot += B1[k][d] * 0.5 * (u0[k][d] + u1[k][d]);
  const double m = S->mass[z];
  const double e1 = S->e[z] - dt * W / m;
  const double rho1 = m / V1;
  const double du = vdot / pow(V1, 2.0 / 3.0);
  const double q1 = du < 0.0 ? rho1 * (P->cq * du * du + P->cl * S->c[z] * fabs(du)) : 0.0;
  const double p1 = (P->gamma - 1.0) * rho1 * e1;
  y[0] = e1;
  y[1] = p1;
  y[2] = q1;
  y[3] = sqrt(P->gamma * fmax(p1, 0.0) / rho1);
  return V1;
}

/* One timestep.  step = the timestep index (the perforation offset).
 * Returns -1 for invalid arguments, else the step's numeric-failure flags:
 * 0, or HY_BAD_VOLUME if an element volume (after the force or the EOS
 * phase) was not positive, plus HY_BAD_DT if the time step was not finite
 * and positive.  The step is completed either way. */
#define HY_BAD_VOLUME 1
#define HY_BAD_DT 2
int hy_step(const hy_par *P, const hy_tech *T, int32_t step, hy_state *S, hy_rec *R) {
  const int64_t n = P->n, m = n + 1, E = hy_elems(P), Nn = hy_nodes(P);
  if ((T->eos_h && (T->eos_h > HY_MAX_H || T->eos_p < 1)) || (T->hg_h && (T->hg_h > HY_MAX_H || T->hg_p < 1)))
    return -1;
  if ((T->eos_group != 1 && T->eos_group != HY_WAVE && T->eos_group != HY_BLOCK) ||
      (T->hg_group != 1 && T->hg_group != HY_WAVE && T->hg_group != HY_BLOCK))
    return -1;
  const int64_t GE = T->eos_group, GH = T->hg_group;
  const int64_t NGE = (E + GE - 1) / GE, NGH = (E + GH - 1) / GH;
  if (T->hg_h && T->perfo_param) return -1;
  if (T->perfo_param && T->perfo_ipt < 1) return -1;
  if (T->perfo_kind < 0 || T->perfo_kind > 3) return -1;
  if (R) {
    for (int64_t g = 0; g < NGE; ++g) {
      if (R->dec_eos) R->dec_eos[g] = -1;
      if (R->frag_eos) R->frag_eos[g] = 0;
    }
    for (int64_t g = 0; g < NGH; ++g) {
      if (R->dec_hg) R->dec_hg[g] = -1;
      if (R->frag_hg) R->frag_hg[g] = 0;
    }
  }

  /* 1. forces (hourglass region under TAF, perforation or exact) and the
   * time-step bound of every element */
  double dtmin = INFINITY;
  int bad = 0;
  if (T->perfo_param) {
    const int64_t L = HY_WAVE * (((E + T->perfo_ipt - 1) / T->perfo_ipt + HY_WAVE - 1) / HY_WAVE);
#pragma omp parallel for schedule(static) reduction(min : dtmin) reduction(| : bad)
    for (int64_t l = 0; l < L; ++l)
      for (int32_t k = 0; k < T->perfo_ipt; ++k) {
        const int64_t z = l + (int64_t)k * L;
        if (z >= E) continue;
        const double b = hy_force_elem(P, S, z, hy_perfo_skip(T, z, E, k, step) ? HY_HG_NONE : HY_HG_COMPUTE);
        dtmin = fmin(dtmin, b);
        if (!(S->vol[z] > 0.0)) bad |= HY_BAD_VOLUME;
      }
  } else {
#pragma omp parallel for schedule(static) reduction(min : dtmin) reduction(| : bad)
    for (int64_t g = 0; g < NGH; ++g) {
      const int64_t z0 = g * GH, z1 = z0 + GH < E ? z0 + GH : E;
      const int act = (int)(z1 - z0);
      if (T->hg_h && S->rho_hg[g] > 0) {
        for (int64_t z = z0; z < z1; ++z) {
          dtmin = fmin(dtmin, hy_force_elem(P, S, z, HY_HG_REUSE));
          if (!(S->vol[z] > 0.0)) bad |= HY_BAD_VOLUME;
        }
        S->rho_hg[g]--;
        if (R && R->dec_hg) R->dec_hg[g] = 1;
        continue;
      }
      int yes = 0, voted = 0, near_yes = 0, near_no = 0;
      for (int64_t z = z0; z < z1; ++z) {
        dtmin = fmin(dtmin, hy_force_elem(P, S, z, HY_HG_COMPUTE));
        if (!(S->vol[z] > 0.0)) bad |= HY_BAD_VOLUME;
        if (!T->hg_h) continue;
        double y[24];
        for (int o = 0; o < 24; ++o) y[o] = S->fhg[o * E + z];
        int near;
        const int crit = hy_taf_push(S->whg, E, z, 24, T->hg_h, S->z_hg[g], y, T->hg_theta, T->band, &near);
        if (crit >= 0) {
          voted = 1;
          yes += crit;
          if (near) crit ? near_yes++ : near_no++;
        }
      }
      if (!T->hg_h) continue;
      S->z_hg[g]++;
      if (R && R->dec_hg) R->dec_hg[g] = 0;
      if (voted && hy_majority(yes, act)) S->rho_hg[g] = T->hg_p;
      if (voted && R && R->frag_hg)
        R->frag_hg[g] = hy_majority(yes - near_yes, act) != hy_majority(yes + near_no, act);
    }
  }

  /* 2. time step */
  const double dt = fmin(dtmin, P->growth * S->clock[1]);
  if (!(dt > 0.0) || !isfinite(dt)) bad |= HY_BAD_DT;

  /* 3. nodes: gather corner forces, momentum, boundary conditions, positions */
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < Nn; ++v) {
    const int64_t i = v % m, j = (v / m) % m, k = v / (m * m);
    double F[3] = {0, 0, 0};
    for (int c = 0; c < 8; ++c) {
      const int64_t ei = i - (c & 1), ej = j - ((c >> 1) & 1), ek = k - ((c >> 2) & 1);
      if (ei < 0 || ej < 0 || ek < 0 || ei >= n || ej >= n || ek >= n) continue;
      const int64_t z = ei + n * (ej + n * ek);
      for (int d = 0; d < 3; ++d) F[d] += S->force[(c * 3 + d) * E + z];
    }
    const int64_t idx[3] = {i, j, k};
    for (int d = 0; d < 3; ++d) {
      double un = S->u[d][v] + dt * F[d] / S->mnode[v];
      if (idx[d] == 0) un = 0.0;
      S->unew[d][v] = un;
    }
    for (int d = 0; d < 3; ++d) S->x[d][v] += dt * 0.5 * (S->u[d][v] + S->unew[d][v]);
  }

  /* 4. EOS region per element (TAF or exact) */
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t g = 0; g < NGE; ++g) {
    const int64_t z0 = g * GE, z1 = z0 + GE < E ? z0 + GE : E;
    const int act = (int)(z1 - z0);
    if (T->eos_h && S->rho_eos[g] > 0) {
      S->rho_eos[g]--;
      if (R && R->dec_eos) R->dec_eos[g] = 1;
      continue;
    }
    int yes = 0, voted = 0, near_yes = 0, near_no = 0;
    for (int64_t z = z0; z < z1; ++z) {
      double y[4];
      if (!(hy_eos_elem(P, S, z, dt, y) > 0.0)) bad |= HY_BAD_VOLUME;
      S->e[z] = y[0];
      S->p[z] = y[1];
      S->q[z] = y[2];
      S->c[z] = y[3];
      if (!T->eos_h) continue;
      int near;
      const int crit = hy_taf_push(S->weos, E, z, 4, T->eos_h, S->z_eos[g], y, T->eos_theta, T->band, &near);
      if (crit >= 0) {
        voted = 1;
        yes += crit;
        if (near) crit ? near_yes++ : near_no++;
      }
    }
    if (!T->eos_h) continue;
    S->z_eos[g]++;
    if (R && R->dec_eos) R->dec_eos[g] = 0;
    if (voted && hy_majority(yes, act)) S->rho_eos[g] = T->eos_p;
    if (voted && R && R->frag_eos)
      R->frag_eos[g] = hy_majority(yes - near_yes, act) != hy_majority(yes + near_no, act);
  }

  /* 5. velocities and clock */
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < Nn; ++v)
    for (int d = 0; d < 3; ++d) S->u[d][v] = S->unew[d][v];
  S->clock[0] += dt;
  S->clock[1] = dt;
  return bad;
}

/* Internal and kinetic energy of the state. */
void hy_energy(const hy_par *P, const hy_state *S, double *internal, double *kinetic) {
  const int64_t E = hy_elems(P), Nn = hy_nodes(P);
  double ie = 0.0, ke = 0.0;
  for (int64_t z = 0; z < E; ++z) ie += S->mass[z] * S->e[z];
  for (int64_t v = 0; v < Nn; ++v)
    ke += 0.5 * S->mnode[v] * (S->u[0][v] * S->u[0][v] + S->u[1][v] * S->u[1][v] + S->u[2][v] * S->u[2][v]);
  *internal = ie;
  *kinetic = ke;
}

/* Volume and its gradient of one hexahedron, exported for the pins. */
double hy_hex_volume(const double *xc24, double *B24) {
  double xc[8][3], B[8][3];
  for (int c = 0; c < 8; ++c)
    for (int d = 0; d < 3; ++d) xc[c][d] = xc24[c * 3 + d];
  const double V = hy_volume(xc, B24 ? B : NULL);
  if (B24)
    for (int c = 0; c < 8; ++c)
      for (int d = 0; d < 3; ++d) B24[c * 3 + d] = B[c][d];
  return V;
}

/* Hourglass forces of one hexahedron, exported for the pins. */
void hy_hex_hourglass(const double *xc24, const double *uc24, double rho, double c, double khg, double *f24) {
  double xc[8][3], uc[8][3], B[8][3], f[8][3];
  for (int k = 0; k < 8; ++k)
    for (int d = 0; d < 3; ++d) xc[k][d] = xc24[k * 3 + d], uc[k][d] = uc24[k * 3 + d];
  const double V = hy_volume(xc, B);
  hy_hourglass(xc, uc, B, V, rho, c, khg, f);
  for (int k = 0; k < 8; ++k)
    for (int d = 0; d < 3; ++d) f24[k * 3 + d] = f[k][d];
}

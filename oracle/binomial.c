/*
 * CPU oracle, part 3: the Binomial Options region in FP64.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c): only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header or constant with the GPU library.
 *
 * The paper's Binomial Options benchmark prices a portfolio of American
 * options with a binomial tree, one option per group of threads (section 4,
 * Table 1 and 4.1).  This is the textbook Cox-Ross-Rubinstein tree: with
 * dt = T/N, u = exp(v sqrt(dt)), d = 1/u, growth a = exp(r dt),
 * up-probability p = (a - d)/(u - d):
 *   leaves   S_{N,i} = S u^i d^(N-i), V_{N,i} = payoff(S_{N,i}), i = 0..N;
 *   steps    for n = N-1 .. 0, i = 0..n:
 *            V_{n,i} = (p V_{n+1,i+1} + (1-p) V_{n+1,i}) / a,
 *            American: V_{n,i} = max(V_{n,i}, payoff(S_{n,i}));
 *   price    V_{0,0}.
 * Call payoff max(S - K, 0), put max(K - S, 0).  The node prices of step n
 * follow from those of step n+1 by one multiplication (S_{n,i} =
 * S_{n+1,i} u), in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static double bo_price(double S, double K, double T, double r, double v, int N, int american, int put) {
  const double dt = T / N;
  const double u = exp(v * sqrt(dt)), d = 1.0 / u, a = exp(r * dt);
  const double p = (a - d) / (u - d);
  double *V = malloc(sizeof(double) * (size_t)(N + 1));
  double *X = malloc(sizeof(double) * (size_t)(N + 1));
  for (int i = 0; i <= N; ++i) {
    X[i] = S * pow(u, (double)(2 * i - N));
    V[i] = put ? fmax(K - X[i], 0.0) : fmax(X[i] - K, 0.0);
  }
  for (int n = N - 1; n >= 0; --n) {
    for (int i = 0; i <= n; ++i) {
      X[i] *= u; /* S u^(2i-n) from S u^(2i-n-1) */
      double c = (p * V[i + 1] + (1.0 - p) * V[i]) / a;
      if (american) c = fmax(c, put ? K - X[i] : X[i] - K);
      V[i] = c;
    }
  }
  const double out = V[0];
  free(V);
  free(X);
  return out;
}

/* Call and put prices of n options (FP64 columns) on an N-step tree, and a
 * per-option magnitude S + K e^{-rT} for relative tolerances. */
void or_binomial(int64_t n, const double *S, const double *K, const double *T, const double *r, const double *v,
                 int32_t steps, int32_t american, double *C, double *P, double *scale) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t j = 0; j < n; ++j) {
    C[j] = bo_price(S[j], K[j], T[j], r[j], v[j], steps, american, 0);
    P[j] = bo_price(S[j], K[j], T[j], r[j], v[j], steps, american, 1);
    if (scale) scale[j] = S[j] + K[j] * exp(-r[j] * T[j]);
  }
}

"""Seeded synthetic inputs for the Black-Scholes region.

This module only draws numbers: it holds none of the method's arithmetic and
serves both the GPU library's callers and its CPU checker.  All arrays are
structure-of-arrays float32 columns in the region's input order
(S, K, T, r, v): spot, strike, years to expiry, riskless rate, volatility --
the column-major, stride-n layout of the paper's array sections (3.2).

The paper's Black-Scholes inputs (the PARSEC set) are not available; these
generators stand in for them with the box below and a pool-plus-jitter
structure, so that the inputs repeat approximately the way a portfolio with
repeated contracts does.
"""
import numpy as np

S_BOX = (5.0, 30.0)
K_BOX = (1.0, 100.0)
T_BOX = (0.25, 10.0)
V_BOX = (0.1, 0.5)
RATE = 0.02
BOX_LO = np.array([S_BOX[0], K_BOX[0], T_BOX[0], RATE, V_BOX[0]])
BOX_HI = np.array([S_BOX[1], K_BOX[1], T_BOX[1], RATE, V_BOX[1]])

SEED_POOL, SEED_DRAW, SEED_JITTER, SEED_OUT_OF_BOX, SEED_TRAIN, SEED_INIT = 1001, 1002, 1003, 1004, 1005, 1006


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_box(n, seed):
    """n tuples uniform over the box (float64, shape (5, n)); r is constant."""
    g = _rng(seed)
    S = g.uniform(*S_BOX, n)
    K = g.uniform(*K_BOX, n)
    T = g.uniform(*T_BOX, n)
    v = g.uniform(*V_BOX, n)
    r = np.full(n, RATE)
    return np.stack([S, K, T, r, v])


def _jitter(x, rel, seed):
    """Multiply S, K, T and v by (1 + rel * N(0,1)); r stays exact."""
    if rel == 0.0:
        return x
    g = _rng(seed)
    z = g.standard_normal((4, x.shape[1]))
    y = x.copy()
    for row, j in zip((0, 1, 2, 4), range(4)):
        y[row] = x[row] * (1.0 + rel * z[j])
    return y


def _f32(x):
    return np.ascontiguousarray(x.astype(np.float32))


def portfolio(n, pool_size, sort_by_spot=False, jitter=1e-3,
              seed_pool=SEED_POOL, seed_draw=SEED_DRAW, seed_jitter=SEED_JITTER):
    """Items drawn uniformly from a pool of tuples, each with relative
    Gaussian jitter on S, K, T, v.  Optionally stably sorted by spot."""
    pool = uniform_box(pool_size, seed_pool)
    idx = _rng(seed_draw).integers(0, pool_size, n)
    x = _jitter(pool[:, idx], jitter, seed_jitter)
    if sort_by_spot:
        x = x[:, np.argsort(x[0], kind="stable")]
    return _f32(x)


def periodic(n, period, pool_size=None, jitter=1e-3,
             seed_pool=SEED_POOL, seed_jitter=SEED_JITTER):
    """Structured-locality variant: item i uses pool tuple (i mod period).
    When the lane count is a multiple of the period every lane sees one
    tuple at every step, so output and input memoization both find reuse."""
    pool = uniform_box(pool_size or period, seed_pool)
    idx = np.arange(n) % period
    return _f32(_jitter(pool[:, idx], jitter, seed_jitter))


def grouped(n, run, pool_size=1024, jitter=1e-3,
            seed_pool=SEED_POOL, seed_draw=SEED_DRAW, seed_jitter=SEED_JITTER):
    """Structured-locality variant: runs of `run` consecutive items share a
    pool tuple (before jitter)."""
    pool = uniform_box(pool_size, seed_pool)
    nruns = (n + run - 1) // run
    ridx = _rng(seed_draw).integers(0, pool_size, nruns)
    idx = np.repeat(ridx, run)[:n]
    return _f32(_jitter(pool[:, idx], jitter, seed_jitter))


def constant(n, tup=(20.0, 25.0, 1.0, RATE, 0.3)):
    """Every item is the same tuple."""
    return _f32(np.tile(np.asarray(tup, np.float64)[:, None], (1, n)))


def with_out_of_box(x, frac, seed=SEED_OUT_OF_BOX):
    """Move a fraction of items outside the box: for each chosen item one of
    S, K, T, v is redrawn from (hi, hi + 0.1 (hi - lo)]."""
    g = _rng(seed)
    y = x.astype(np.float64).copy()
    n = y.shape[1]
    m = int(round(frac * n))
    items = g.choice(n, m, replace=False)
    which = g.integers(0, 4, m)
    rows = np.array([0, 1, 2, 4])[which]
    lo, hi = BOX_LO[rows], BOX_HI[rows]
    u = g.uniform(0.0, 1.0, m)
    y[rows, items] = hi + (1.0 - u) * 0.1 * (hi - lo)
    return _f32(y), np.sort(items)

"""Pins for the oracle's exact Black-Scholes region (R1) and its Jacobian (R2).

Each check is independent of the oracle's own formula: a textbook worked
example, the price as a discounted risk-neutral expectation evaluated by
numerical quadrature, no-arbitrage identities and bounds, limits, scaling,
the Black-Scholes PDE through finite differences of the oracle, and central
finite differences for the Jacobian.
"""
import os

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from paper_2308_16877_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_kv(name):
    d = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split("=")
            d[k] = float(v)
    return d


def test_textbook_worked_example():
    g = _read_kv("bs_hull_example.txt")
    C, P, _, _ = oracle.bs_price([g["S"]], [g["K"]], [g["T"]], [g["r"]], [g["sigma"]])
    assert abs(C[0] - g["call"]) <= g["abs_tol"]
    assert abs(P[0] - g["put"]) <= g["abs_tol"]


def _quadrature_price(S, K, T, r, v):
    """Discounted expectation of the payoffs under the risk-neutral
    lognormal law, integrated over the standard normal variable z:
    S_T = S exp((r - v^2/2) T + v sqrt(T) z)."""
    a = (r - 0.5 * v * v) * T
    b = v * np.sqrt(T)
    c = 1.0 / np.sqrt(2.0 * np.pi)

    def payoff_density(z, sign):
        # sign * (S_T - K) * phi(z), with the exponents combined to avoid overflow
        return sign * c * (S * np.exp(a + b * z - 0.5 * z * z) - K * np.exp(-0.5 * z * z))

    z_star = (np.log(K / S) - a) / b  # S_T(z*) = K
    # beyond |z| = 40 + b the integrands are below 1e-300
    hi = max(z_star, b) + 40.0
    lo = min(z_star, 0.0) - 40.0
    kw = dict(epsabs=1e-14, epsrel=1e-12, limit=400)
    call = integrate.quad(payoff_density, z_star, hi, args=(1.0,), points=[b] if z_star < b < hi else None, **kw)[0] \
        if z_star < hi else 0.0
    put = integrate.quad(payoff_density, lo, z_star, args=(-1.0,), **kw)[0] if lo < z_star else 0.0
    disc = np.exp(-r * T)
    return disc * call, disc * put


def test_price_equals_risk_neutral_expectation():
    x = inputs.uniform_box(60, seed=7)
    C, P, sC, sP = oracle.bs_price(*x)
    for i in range(x.shape[1]):
        qc, qp = _quadrature_price(*x[:, i])
        assert abs(C[i] - qc) <= 1e-9 * sC[i] + 1e-12, (i, C[i], qc)
        assert abs(P[i] - qp) <= 1e-9 * sP[i] + 1e-12, (i, P[i], qp)


def test_put_call_parity_and_bounds():
    x = inputs.uniform_box(20000, seed=11)
    S, K, T, r, v = x
    C, P, _, _ = oracle.bs_price(*x)
    D = K * np.exp(-r * T)
    assert np.all(np.abs(C - P - (S - D)) <= 16 * 2.0**-53 * (S + D))
    tol = 1e-12 * (S + D)
    assert np.all(C >= np.maximum(S - D, 0) - tol) and np.all(C <= S + tol)
    assert np.all(P >= np.maximum(D - S, 0) - tol) and np.all(P <= D + tol)


def test_limits_expiry_and_zero_volatility():
    S = np.array([10.0, 25.0, 40.0, 7.0])
    K = np.array([20.0, 25.0 * 0.97, 30.0, 7.5])
    r = np.full(4, 0.02)
    # T -> 0: intrinsic value max(S - K, 0)
    C, P, _, _ = oracle.bs_price(S, K, np.full(4, 1e-12), r, np.full(4, 0.3))
    assert np.allclose(C, np.maximum(S - K, 0), atol=1e-5)
    assert np.allclose(P, np.maximum(K - S, 0), atol=1e-5)
    # v -> 0: max(S - K e^{-rT}, 0)
    T = np.full(4, 2.0)
    D = K * np.exp(-0.02 * T)
    C, P, _, _ = oracle.bs_price(S, K, T, r, np.full(4, 1e-9))
    assert np.allclose(C, np.maximum(S - D, 0), atol=1e-7)
    assert np.allclose(P, np.maximum(D - S, 0), atol=1e-7)


def test_homogeneity_in_spot_and_strike():
    x = inputs.uniform_box(2000, seed=13)
    C, P, sC, sP = oracle.bs_price(*x)
    for lam in (0.5, 3.0):
        y = x.copy()
        y[0] *= lam
        y[1] *= lam
        C2, P2, _, _ = oracle.bs_price(*y)
        assert np.all(np.abs(C2 - lam * C) <= 1e-12 * lam * sC + 1e-300)
        assert np.all(np.abs(P2 - lam * P) <= 1e-12 * lam * sP + 1e-300)


def test_black_scholes_pde_residual():
    """dC/dT = 0.5 v^2 S^2 C_SS + r S C_S - r C (T = time to expiry), by
    central differences of the oracle; also the same for the put."""
    x = inputs.uniform_box(300, seed=17)
    S, K, T, r, v = x
    hs = 1e-3 * S
    ht = 1e-4 * T
    for j in (0, 1):
        f = lambda S_, T_: oracle.bs_price(S_, K, T_, r, v)[j]
        V = f(S, T)
        VS = (f(S + hs, T) - f(S - hs, T)) / (2 * hs)
        VSS = (f(S + hs, T) - 2 * V + f(S - hs, T)) / hs**2
        VT = (f(S, T + ht) - f(S, T - ht)) / (2 * ht)
        res = VT - (0.5 * v * v * S * S * VSS + r * S * VS - r * V)
        scale = 1e-4 * (np.abs(VT) + 0.5 * v * v * S * S * np.abs(VSS) + r * S * np.abs(VS) + r * np.abs(V)) + 1e-8
        assert np.all(np.abs(res) <= scale), np.max(np.abs(res) / scale)


def test_delta_matches_normal_cdf_of_d1():
    """The spot derivative of the call is N(d1) (scipy's normal CDF)."""
    x = inputs.uniform_box(500, seed=19)
    S, K, T, r, v = x
    d1 = (np.log(S / K) + (r + 0.5 * v * v) * T) / (v * np.sqrt(T))
    h = 1e-5 * S
    Cp = oracle.bs_price(S + h, K, T, r, v)[0]
    Cm = oracle.bs_price(S - h, K, T, r, v)[0]
    assert np.allclose((Cp - Cm) / (2 * h), stats.norm.cdf(d1), atol=1e-7)


def test_jacobian_matches_central_differences():
    x = inputs.uniform_box(400, seed=23)
    J = oracle.bs_jacobian(*x)
    for d in range(5):
        h = 1e-6 * np.maximum(np.abs(x[d]), 1.0)
        xp, xm = x.copy(), x.copy()
        xp[d] += h
        xm[d] -= h
        Cp, Pp, sC, sP = oracle.bs_price(*xp)
        Cm, Pm, _, _ = oracle.bs_price(*xm)
        fdC = (Cp - Cm) / (2 * h)
        fdP = (Pp - Pm) / (2 * h)
        tolC = 1e-6 * (np.abs(J[d]) + sC / np.maximum(np.abs(x[d]), 1.0)) + 1e-9
        tolP = 1e-6 * (np.abs(J[5 + d]) + sP / np.maximum(np.abs(x[d]), 1.0)) + 1e-9
        assert np.all(np.abs(fdC - J[d]) <= tolC), (d, np.max(np.abs(fdC - J[d]) / tolC))
        assert np.all(np.abs(fdP - J[5 + d]) <= tolP), (d, np.max(np.abs(fdP - J[5 + d]) / tolP))


def test_scales_bound_the_prices():
    x = inputs.uniform_box(1000, seed=29)
    C, P, sC, sP = oracle.bs_price(*x)
    assert np.all(np.abs(C) <= sC * (1 + 1e-15)) and np.all(np.abs(P) <= sP * (1 + 1e-15))
    assert np.all(sC > 0) and np.all(sP > 0)


def test_put_row_is_the_derivative_of_parity():
    """P = C - S + K e^{-rT}, so the put row equals the call row minus the
    derivative of S - K e^{-rT}."""
    x = inputs.uniform_box(5000, seed=37)
    S, K, T, r, v = x
    J = oracle.bs_jacobian(*x)
    D = K * np.exp(-r * T)
    shift = [np.ones_like(S), -np.exp(-r * T), r * D, T * D, np.zeros_like(S)]
    for j in range(5):
        mag = np.abs(J[j]) + np.abs(shift[j]) + 1e-300
        assert np.all(np.abs(J[5 + j] - (J[j] - shift[j])) <= 1e-14 * mag)

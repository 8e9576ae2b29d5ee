"""GPU parity for the Greeks: the price-and-Jacobian region under exact and
iACT, the backward kernels, and the autograd wrapper, against the oracle's
closed-form Jacobian and central finite differences of its prices.

Tolerance of a Jacobian entry computed in FP32 from FP32 inputs:
1e-5 of its magnitude (for the expiry derivatives, of the magnitude of their
two terms), plus its change under a relative perturbation of 8 FP32 ulps of
each input -- the conditioning of the derivative, estimated by central
differences of the oracle's Jacobian.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, SENTINEL, check_outputs, run, say, to_dev, trace_dec
from paper_2308_16877_amd import hpac, inputs
from paper_2308_16877_amd.greeks import bs_prices

pytestmark = pytest.mark.gpu

EPS_IN = 8 * 2.0 ** -24


def jac_tolerance(x):
    x = np.asarray(x, np.float64)
    J = oracle.bs_jacobian(*x)
    S, K, T, r, v = x
    D = K * np.exp(-r * T)
    mag = np.abs(J)
    mag[[2, 7]] += r * D  # dC/dT, dP/dT: two terms of opposite sign for the put
    tol = 1e-5 * mag
    for j in range(5):
        h = 1e-6 * np.maximum(np.abs(x[j]), 1.0)
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        dJ = (oracle.bs_jacobian(*xp) - oracle.bs_jacobian(*xm)) / (2 * h)
        tol += EPS_IN * np.abs(dJ) * np.abs(x[j])
    return J, tol


def grad_region_reference(x):
    """(values as the FP32 output columns hold them, per-column scale such
    that 1e-5 * scale is the tolerance) for the 12 output columns."""
    C, P, sC, sP = oracle.bs_price(*x)
    J, tolJ = jac_tolerance(x)
    y = np.concatenate([np.stack([C, P]), J]).astype(np.float32).astype(np.float64)
    s = np.concatenate([np.stack([sC, sP]), tolJ / 1e-5])
    return y, s, np.concatenate([np.stack([C, P]), J])


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available()
    hpac.lib()


@pytest.mark.parametrize("n,ipt", [(1, 1), (1000, 3), (65536, 16), (100003, 1)])
def test_jacobian_region_matches_closed_forms(n, ipt):
    say("grad region exact n=%d" % n)
    x = inputs.portfolio(n, 1024)
    y, _, _ = run("exact", to_dev(x), 12, ipt, region=hpac.REGION_BS_PRICE_GRAD)
    yref, scale, _ = grad_region_reference(x)
    check_outputs(y, yref, scale, what="price+jacobian")


def test_jacobian_region_over_the_box():
    x = inputs.uniform_box(100000, seed=41).astype(np.float32)
    y, _, _ = run("exact", to_dev(x), 12, 4, region=hpac.REGION_BS_PRICE_GRAD)
    yref, scale, _ = grad_region_reference(x)
    worst = check_outputs(y, yref, scale, what="price+jacobian box")
    say("  worst err/tol %.3f" % worst)


def test_jacobian_matches_central_differences():
    """Central differences of the oracle's FP64 prices, h = 1e-3 max(|x|, 1):
    agreement within 1e-4 of the entry's magnitude plus the FP32 term."""
    x = inputs.uniform_box(20000, seed=43).astype(np.float32)
    y, _, _ = run("exact", to_dev(x), 12, 1, region=hpac.REGION_BS_PRICE_GRAD)
    xd = x.astype(np.float64)
    J, tolJ = jac_tolerance(x)
    for j in range(5):
        h = 1e-3 * np.maximum(np.abs(xd[j]), 1.0)
        xp, xm = xd.copy(), xd.copy()
        xp[j] += h
        xm[j] -= h
        Cp, Pp, sC, sP = oracle.bs_price(*xp)
        Cm, Pm, _, _ = oracle.bs_price(*xm)
        for row, fd in ((j, (Cp - Cm) / (2 * h)), (5 + j, (Pp - Pm) / (2 * h))):
            # truncation of the central difference: h^2/6 |f'''|, bounded via
            # the oracle's Jacobian differences at the same step
            Jp = oracle.bs_jacobian(*xp)[row]
            Jm = oracle.bs_jacobian(*xm)[row]
            trunc = np.abs(Jp - 2 * J[row] + Jm) / 3.0
            tol = 1e-4 * (np.abs(J[row]) + 1e-6) + trunc + tolJ[row]
            err = np.abs(y[2 + row] - fd)
            assert np.all(err <= tol), (row, float(np.max(err / tol)))


IACT_GRAD_CASES = [
    ("config3_like", lambda: inputs.portfolio(65536, 65536, sort_by_spot=True), 16, 16, 0.05),
    ("periodic2", lambda: inputs.periodic(65536, 2, jitter=1e-3), 16, 16, 0.05),
    ("periodic8_t16", lambda: inputs.periodic(65536, 8, jitter=1e-4), 16, 16, 0.05),
    ("ragged", lambda: inputs.periodic(4099, 4, jitter=1e-4), 5, 4, 0.05),
]


@pytest.mark.parametrize("case", IACT_GRAD_CASES, ids=[c[0] for c in IACT_GRAD_CASES])
def test_iact_memoizes_prices_and_gradients(case):
    name, mk, ipt, t, theta = case
    say("iact grad", name)
    x = mk()
    y, tr, cnt = run("iact", to_dev(x), 12, ipt, region=hpac.REGION_BS_PRICE_GRAD, table_size=t, threshold=theta)
    yv, sv, _ = grad_region_reference(x)
    ora = oracle.iact(x, yv, sv, ipt, t, theta, out_init=np.full_like(yv, SENTINEL))
    gdec, f = trace_dec(tr)
    assert np.array_equal(gdec, ora["dec"])
    check_outputs(y, ora["out"], ora["scale"], what="iact grad " + name)
    say("  approx lanes %.4f" % (cnt[1] / x.shape[1]))


@pytest.mark.parametrize("block", [64, 192])
def test_iact_grad_block_sizes_match_oracle(block):
    """The price-and-Jacobian tables at other workgroup sizes (more or fewer
    20-float-entry tables per workgroup's LDS): same decisions and outputs."""
    x = inputs.periodic(65536, 2, jitter=1e-3)
    y, tr, cnt = run("iact", to_dev(x), 12, 16, block_size=block, region=hpac.REGION_BS_PRICE_GRAD, table_size=16,
                     threshold=0.05)
    yv, sv, _ = grad_region_reference(x)
    ora = oracle.iact(x, yv, sv, 16, 16, 0.05, out_init=np.full_like(yv, SENTINEL))
    gdec, f = trace_dec(tr)
    assert np.array_equal(gdec, ora["dec"])
    check_outputs(y, ora["out"], ora["scale"], what="iact grad block %d" % block)


@pytest.mark.parametrize("case", IACT_GRAD_CASES, ids=[c[0] for c in IACT_GRAD_CASES])
def test_memo_by_reference_equals_saved_jacobian(case):
    """iACT on the price-and-source region carries 4 bytes per item (the
    source item's index) instead of ten Jacobian columns: the same decisions
    and prices, bit for bit, as iACT on the price-and-Jacobian region; the
    source of every item equals the oracle's (its engine run with the item
    index as an output reuses entries exactly as it reuses prices); and the
    backward, recomputing the derivatives at each source item, equals the
    saved-Jacobian VJP bit for bit."""
    name, mk, ipt, t, theta = case
    say("memo by reference", name)
    x = mk()
    n = x.shape[1]
    xd = to_dev(x)
    y12, tr12, _ = run("iact", xd, 12, ipt, region=hpac.REGION_BS_PRICE_GRAD, table_size=t, threshold=theta)
    C, P = (torch.full((n,), SENTINEL, dtype=torch.float32, device=DEV) for _ in range(2))
    src = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    tr = torch.zeros(hpac.hpac_trace_entries(n, ipt), dtype=torch.int32, device=DEV)
    hpac.hpac_iact(xd, [C, P, src], t, theta, items_per_lane=ipt, region=hpac.REGION_BS_PRICE_REF, trace=tr)
    torch.cuda.synchronize()
    assert np.array_equal(tr.cpu().numpy().view(np.uint32), tr12)
    assert np.array_equal(C.cpu().numpy().astype(np.float64), y12[0])
    assert np.array_equal(P.cpu().numpy().astype(np.float64), y12[1])
    yv, sv = oracle.region_values_f32out(x)
    ora = oracle.iact(x, np.vstack([yv, np.arange(n, dtype=np.float64)]), None, ipt, t, theta)
    s = src.cpu().numpy()
    assert np.array_equal(s, ora["out"][2].astype(np.int64))
    approx = s != np.arange(n)
    say("  %.3f of the items reuse another item's prices and derivatives" % approx.mean())
    g = np.random.default_rng(9).standard_normal((2, n)).astype(np.float32)
    gC, gP = (torch.from_numpy(g[i]).to(DEV) for i in range(2))
    J = [torch.from_numpy(y12[2 + j].astype(np.float32)).to(DEV) for j in range(10)]
    a = [torch.empty(n, dtype=torch.float32, device=DEV) for _ in range(5)]
    b = [torch.empty(n, dtype=torch.float32, device=DEV) for _ in range(5)]
    hpac.hpac_bs_vjp(J, gC, gP, a)
    hpac.hpac_bs_vjp_ref(xd, src, gC, gP, b)
    torch.cuda.synchronize()
    for j in range(5):
        assert torch.equal(a[j], b[j]), j


def test_exact_source_column_and_bad_indices():
    """hpac_exact on the price-and-source region writes each item's own
    index; the by-reference backward turns an index outside [0, n) into NaN
    gradients for that item and reads nothing for it."""
    n = 10007
    x = inputs.portfolio(n, 1024)
    xd = to_dev(x)
    C, P = (torch.empty(n, dtype=torch.float32, device=DEV) for _ in range(2))
    src = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    hpac.hpac_exact(xd, [C, P, src], items_per_lane=3, region=hpac.REGION_BS_PRICE_REF)
    torch.cuda.synchronize()
    assert np.array_equal(src.cpu().numpy(), np.arange(n))
    bad = src.clone()
    bad[5], bad[6], bad[7] = -3, n, 2 ** 31 - 1
    ones = torch.ones(n, dtype=torch.float32, device=DEV)
    a = [torch.empty(n, dtype=torch.float32, device=DEV) for _ in range(5)]
    b = [torch.empty(n, dtype=torch.float32, device=DEV) for _ in range(5)]
    hpac.hpac_bs_adjoint(xd, ones, None, a)
    hpac.hpac_bs_vjp_ref(xd, bad, ones, None, b)
    torch.cuda.synchronize()
    for j in range(5):
        bj = b[j].cpu().numpy()
        assert np.all(np.isnan(bj[5:8]))
        keep = np.ones(n, bool)
        keep[5:8] = False
        assert np.array_equal(bj[keep], a[j].cpu().numpy()[keep])


def test_vjp_contracts_the_saved_jacobian():
    n = 100003
    x = inputs.portfolio(n, 1024)
    y, _, _ = run("exact", to_dev(x), 12, 1, region=hpac.REGION_BS_PRICE_GRAD)
    J = [torch.from_numpy(y[2 + j].astype(np.float32)).to(DEV) for j in range(10)]
    g = np.random.default_rng(5).standard_normal((2, n)).astype(np.float32)
    gC, gP = (torch.from_numpy(g[i]).to(DEV) for i in range(2))
    out = [torch.empty(n, dtype=torch.float32, device=DEV) for _ in range(5)]
    hpac.hpac_bs_vjp(J, gC, gP, out)
    torch.cuda.synchronize()
    Jn = y[2:].astype(np.float64)
    for j in range(5):
        ref = g[0] * Jn[j] + g[1] * Jn[5 + j]
        bound = 3 * 2.0 ** -24 * (np.abs(g[0] * Jn[j]) + np.abs(g[1] * Jn[5 + j])) + 1e-38
        assert np.all(np.abs(out[j].cpu().numpy() - ref) <= bound)
    # a missing upstream gradient counts as zero
    hpac.hpac_bs_vjp(J, gC, None, out)
    torch.cuda.synchronize()
    assert np.allclose(out[0].cpu().numpy(), g[0] * Jn[0], rtol=3e-7, atol=1e-38)


def test_recomputing_adjoint_equals_vjp_of_exact_jacobian():
    n = 65536
    x = inputs.portfolio(n, 1024)
    xd = to_dev(x)
    y, _, _ = run("exact", xd, 12, 1, region=hpac.REGION_BS_PRICE_GRAD)
    J = [torch.from_numpy(y[2 + j].astype(np.float32)).to(DEV) for j in range(10)]
    g = np.random.default_rng(6).standard_normal((2, n)).astype(np.float32)
    gC, gP = (torch.from_numpy(g[i]).to(DEV) for i in range(2))
    a = [torch.empty(n, dtype=torch.float32, device=DEV) for _ in range(5)]
    b = [torch.empty(n, dtype=torch.float32, device=DEV) for _ in range(5)]
    hpac.hpac_bs_vjp(J, gC, gP, a)
    hpac.hpac_bs_adjoint(xd, gC, gP, b)
    torch.cuda.synchronize()
    for j in range(5):
        assert torch.equal(a[j], b[j])


@pytest.mark.parametrize("technique", ["exact", "iact", "iact_jacobian"])
def test_autograd_greeks_against_closed_forms(technique):
    n = 65536
    x = inputs.portfolio(n, 1024) if technique == "exact" else inputs.periodic(n, 2, jitter=1e-3)
    xt = [torch.from_numpy(c).to(DEV).requires_grad_(True) for c in x]
    params = dict(table_size=16, threshold=0.05) if technique != "exact" else None
    C, P = bs_prices(*xt, technique=technique, params=params)
    gcall = torch.autograd.grad(C.sum(), xt, retain_graph=True)
    gput = torch.autograd.grad(P.sum(), xt)
    J, tolJ = jac_tolerance(x)
    if technique == "exact":
        for j in range(5):
            assert np.all(np.abs(gcall[j].cpu().numpy() - J[j]) <= tolJ[j] + 1e-30)
            assert np.all(np.abs(gput[j].cpu().numpy() - J[5 + j]) <= tolJ[5 + j] + 1e-30)
    else:
        # the gradients are the memoized Jacobian of the iACT forward
        yv, sv, _ = grad_region_reference(x)
        ora = oracle.iact(x, yv, sv, 16, 16, 0.05)
        assert (ora["dec"] == 1).mean() > 0.5
        for j in range(5):
            assert np.all(np.abs(gcall[j].cpu().numpy() - ora["out"][2 + j]) <= 1e-5 * ora["scale"][2 + j] + 1e-30)
            assert np.all(np.abs(gput[j].cpu().numpy() - ora["out"][7 + j]) <= 1e-5 * ora["scale"][7 + j] + 1e-30)

"""GPU parity of the Binomial Options region and its techniques
(hpac_bo_*) against the FP64 oracle.

Tolerance of a tree price computed in FP32: (N + 8) 2^-23 of the option's
scale S + K e^{-rT}.  Each of the N backward steps rounds every node value
(a product and a fused multiply-add, about 2^-23 relative) and the
positive, discount-weighted averages carry earlier errors forward
undamped, so the error is at most linear in N; the node prices' drift
between two exact recomputations (32 multiplications) stays below that.
Measured: about 2e-8 N.  Relative to each price (deep out-of-the-money
prices are far below that scale): (N + 8) 2^-23 of the price plus 64 u of
the expiry payoffs' absolute terms over the leaves in the money, down to
FP32's smallest normal number; measured at most 0.28 of that bound.

Decisions: each wavefront is one decision unit; the oracle's engines run
with one lane per unit at thread level (iACT with one table per lane).
iACT decides on FP32 input distances with the oracle's rounding sequence,
so its decisions must agree exactly; TAF decides on outputs, so a
disagreement must follow a vote within the band of its threshold.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, SENTINEL, compare_decisions, say, to_dev
from paper_2308_16877_amd import hpac, inputs

pytestmark = pytest.mark.gpu


def tol(steps):
    """Relative tolerance of an N-step FP32 tree (see the module doc)."""
    return (steps + 8) * 2.0 ** -23


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available()
    hpac.lib()


def run(fn, x, steps, ipt, trace=True, counters=True, **kw):
    n = x.shape[1]
    out = [torch.full((n,), SENTINEL, dtype=torch.float32, device=DEV) for _ in range(2)]
    units = hpac.hpac_bo_units(n, ipt)
    tr = torch.zeros(max(units * ipt, 1), dtype=torch.int32, device=DEV) if trace else None
    cnt = torch.zeros(hpac.NUM_COUNTERS, dtype=torch.int64, device=DEV) if counters else None
    fn(to_dev(x), out, steps, items_per_lane=ipt, trace=tr, counters=cnt, **kw)
    torch.cuda.synchronize()
    y = np.stack([o.cpu().numpy().astype(np.float64) for o in out])
    t = tr.cpu().numpy().view(np.uint32) if trace else None
    return y, t, (cnt.cpu().numpy() if counters else None)


def unit_records(t, units, ipt):
    """Per (unit, k) words -> approximated flags (units, ipt), visited mask."""
    w = t[:units * ipt].reshape(units, ipt)
    return ((w >> 24) & 1).astype(np.int16), (w >> 31).astype(bool)


def group_napprox(approx, visited, ipt):
    """(approximated units per (group of 64 units, k), whether the group had
    a visited unit) in the oracle's record layout."""
    units = approx.shape[0]
    a = approx.reshape(units // 64, 64, ipt).sum(axis=1)
    v = visited.reshape(units // 64, 64, ipt).any(axis=1)
    return a.astype(np.int16).ravel(), v.ravel()


def itm_leaf_scale(x, steps):
    """Per option and output, the discounted risk-neutral expectation on the
    tree of (X_N + K) over the leaves where the option ends in the money:
    the sum of the absolute terms of the expiry payoffs the price averages
    (a scale for its rounding error; the expectation of the plain tree
    definition, computed here in FP64 with log-space binomial weights)."""
    from scipy.special import gammaln
    S, K, T, r, v = (np.asarray(c, np.float64) for c in x)
    N = steps
    dt = T / N
    u = np.exp(v * np.sqrt(dt))
    a = np.exp(r * dt)
    p = (a - 1.0 / u) / (u - 1.0 / u)
    i = np.arange(N + 1)[:, None]
    lw = gammaln(N + 1) - gammaln(i + 1) - gammaln(N - i + 1) + i * np.log(p) + (N - i) * np.log1p(-p)
    w = np.exp(lw) / a ** N
    X = S * u ** (2.0 * i - N)
    call = np.sum(w * (X + K) * (X > K), axis=0)
    put = np.sum(w * (X + K) * (X < K), axis=0)
    return np.stack([call, put])


def oracle_values(x, steps, american=True):
    C, P, sc = oracle.binomial(*x, steps, american=american)
    return np.stack([C, P]), np.stack([sc, sc])


@pytest.mark.parametrize("n,steps,ipt,american", [
    (1, 1, 1, True), (5, 2, 1, False), (300, 63, 2, True), (4099, 64, 3, True), (2000, 127, 1, False),
    (1500, 512, 4, True), (513, 1023, 1, True),
])
def test_exact_tree_matches_oracle(n, steps, ipt, american):
    x = inputs.portfolio(n, 256)
    y, t, cnt = run(hpac.hpac_bo_exact, x, steps, ipt, american=american)
    ref, scale = oracle_values(x, steps, american)
    err = np.abs(y - ref) / scale
    say("N=%d n=%d: worst error/scale %.2e (%.2e N)" % (steps, n, err.max(), err.max() / steps))
    assert np.all(err <= tol(steps))
    # relative to each price: deep out-of-the-money options have prices far
    # below S + K e^{-rT}, and their error is bounded instead by the
    # rounding of the leaf payoffs that are in the money (their stock price
    # is rounded before K is subtracted) plus N roundings of the price
    # itself, down to FP32's smallest normal number (prices below it, down
    # to 1e-53 here, are held as subnormals or zero)
    bound = ((steps + 8) * 2.0 ** -23 * np.abs(ref) + 64 * 2.0 ** -24 * itm_leaf_scale(x, steps)
             + 2.0 ** -126)
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(np.abs(y - ref) > 0, np.abs(y - ref) / bound, 0.0)
    o, j = np.unravel_index(np.argmax(r), r.shape)
    say("  worst error / price-relative bound %.3f (output %d, x %s, gpu %.9g, oracle %.9g, itm scale %.3g)"
        % (r.max(), o, x[:, j], y[o, j], ref[o, j], itm_leaf_scale(x[:, j:j + 1], steps)[o, 0]))
    assert np.all(r <= 1.0)
    assert cnt[0] == n and cnt[1] == 0
    units = hpac.hpac_bo_units(n, ipt)
    _, visited = unit_records(t, units, ipt)
    assert visited.sum() == n


IACT_CASES = [
    ("pool1024", lambda: inputs.portfolio(16384, 1024), 8, 8, 0.05),
    ("periodic64", lambda: inputs.periodic(8192, 64, jitter=1e-3), 16, 4, 0.05),
    ("ragged", lambda: inputs.periodic(1001, 7, jitter=1e-4), 5, 2, 0.05),
    ("capacity", lambda: inputs.periodic(4096, 1024, jitter=1e-4), 8, 1, 0.05),
]


@pytest.mark.parametrize("case", IACT_CASES, ids=[c[0] for c in IACT_CASES])
def test_iact_matches_oracle(case):
    name, mk, ipt, tsize, theta = case
    x = mk()
    steps = 128
    y, t, cnt = run(hpac.hpac_bo_iact, x, steps, ipt, table_size=tsize, threshold=theta)
    yv, sv = oracle_values(x, steps)
    ora = oracle.iact(x, yv.astype(np.float32).astype(np.float64), sv, ipt, tsize, theta, tables_per_wave=64,
                      group=oracle.GROUP_THREAD, out_init=np.full_like(yv, SENTINEL))
    units = hpac.hpac_bo_units(x.shape[1], ipt)
    approx, visited = unit_records(t, units, ipt)
    g, v = group_napprox(approx, visited, ipt)
    assert np.array_equal(v, ora["dec"] != -1)
    assert np.array_equal(g, ora["napprox"])
    assert np.all(np.abs(y - ora["out"]) <= tol(steps) * ora["scale"] + 1e-30)
    say("iact %s: approximated %.3f of %d options" % (name, approx.sum() / x.shape[1], x.shape[1]))
    assert cnt[1] == approx.sum()


TAF_CASES = [
    # 512 units for 8192 options at 16 per unit: every unit sees one tuple
    ("unit_periodic", lambda: inputs.periodic(8192, 512, jitter=1e-3), 16, 4, 4, 0.01),
    ("pool1024", lambda: inputs.portfolio(8192, 1024), 8, 2, 2, 0.05),
    ("ragged", lambda: inputs.periodic(777, 3, jitter=1e-4), 7, 3, 1, 0.02),
]


@pytest.mark.parametrize("case", TAF_CASES, ids=[c[0] for c in TAF_CASES])
def test_taf_matches_oracle(case):
    name, mk, ipt, h, p, theta = case
    x = mk()
    steps = 128
    y, t, cnt = run(hpac.hpac_bo_taf, x, steps, ipt, history_size=h, prediction_size=p, rsd_threshold=theta)
    yv, sv = oracle_values(x, steps)
    band = 4 * tol(steps) * (1 + theta) / theta + 1e-5
    ora = oracle.taf(yv.astype(np.float32).astype(np.float64), sv, ipt, h, p, theta, band=band,
                     group=oracle.GROUP_THREAD, out_init=np.full_like(yv, SENTINEL))
    units = hpac.hpac_bo_units(x.shape[1], ipt)
    approx, visited = unit_records(t, units, ipt)
    g, v = group_napprox(approx, visited, ipt)
    assert np.array_equal(v, ora["dec"] != -1)
    agree, compared, explained, cascaded = compare_decisions(g, ora["napprox"], ipt, ora["fragile"], lag=1)
    say("taf %s: group-steps agree %d of %d (explained %d), approximated %.3f" % (
        name, agree, compared, explained, approx.sum() / x.shape[1]))
    assert agree >= 0.99 * compared
    if explained == 0:
        assert np.all(np.abs(y - ora["out"]) <= tol(steps) * ora["scale"] + 1e-30)


@pytest.mark.parametrize("kind,param,ipt", [("small", 4, 8), ("large", 3, 6), ("ini", 30, 2), ("fini", 25, 3)])
def test_perforation_matches_oracle(kind, param, ipt):
    x = inputs.portfolio(3001, 256)
    steps = 96
    y, t, cnt = run(hpac.hpac_bo_perfo, x, steps, ipt, kind=kind, param=param, offset=1)
    yv, sv = oracle_values(x, steps)
    ora = oracle.perfo(yv, sv, ipt, hpac.PERFO_KINDS[kind], param, 1, out_init=np.full_like(yv, SENTINEL))
    skipped = ora["out"][0] == SENTINEL
    assert np.all(y[:, skipped] == SENTINEL)
    assert np.all(np.abs(y[:, ~skipped] - ora["out"][:, ~skipped]) <= tol(steps) * sv[:, ~skipped])
    assert cnt[1] == skipped.sum()


@pytest.mark.parametrize("kind,param,ipt,offset", [
    ("small", 4, 8, 1), ("small", 10, 10, 0), ("small", 1, 4, 0), ("large", 3, 6, 2), ("ini", 30, 2, 0),
    ("fini", 25, 3, 0), ("fini", 100, 2, 0),
])
def test_dense_perforation_matches_traced(kind, param, ipt, offset):
    """Without trace or counters, small/large perforation prices only the
    kept steps' options, one per wavefront, and ini/fini the kept range:
    the same outputs, bit for bit, as the per-unit kernel."""
    x = inputs.portfolio(3001, 256)
    yt, _, _ = run(hpac.hpac_bo_perfo, x, 96, ipt, kind=kind, param=param, offset=offset)
    yd, _, _ = run(hpac.hpac_bo_perfo, x, 96, ipt, trace=False, counters=False, kind=kind, param=param,
                   offset=offset)
    assert np.array_equal(yd, yt)


@pytest.mark.parametrize("block", [64, 128, 192])
def test_block_size_changes_nothing(block):
    """Each wavefront prices and decides alone, so the units per workgroup
    change no output, trace word or counter (the 256-lane launch is checked
    against the oracle above)."""
    x = inputs.periodic(6000, 64, jitter=1e-3)
    for fn, kw in ((hpac.hpac_bo_exact, {}), (hpac.hpac_bo_iact, dict(table_size=4, threshold=0.05)),
                   (hpac.hpac_bo_taf, dict(history_size=2, prediction_size=2, rsd_threshold=0.02)),
                   (hpac.hpac_bo_perfo, dict(kind="small", param=3))):
        y0, t0, c0 = run(fn, x, 64, 4, **kw)
        y1, t1, c1 = run(fn, x, 64, 4, block_size=block, **kw)
        assert np.array_equal(y1, y0) and np.array_equal(t1, t0) and np.array_equal(c1, c0)


def test_thresholds_zero_collapse_to_exact():
    x = inputs.periodic(4096, 8, jitter=1e-4)
    ye, _, _ = run(hpac.hpac_bo_exact, x, 64, 8)
    yi, _, ci = run(hpac.hpac_bo_iact, x, 64, 8, table_size=4, threshold=0.0)
    yt, _, ct = run(hpac.hpac_bo_taf, x, 64, 8, history_size=2, prediction_size=2, rsd_threshold=0.0)
    yp, _, cp = run(hpac.hpac_bo_perfo, x, 64, 8, kind="small", param=0)
    for y, c in ((yi, ci), (yt, ct), (yp, cp)):
        assert np.array_equal(y, ye) and c[1] == 0


def test_empty_batch_is_a_no_op():
    out = [torch.zeros(0, dtype=torch.float32, device=DEV) for _ in range(2)]
    hpac.hpac_bo_exact([torch.zeros(0, device=DEV)] * 5, out, 64)
    torch.cuda.synchronize()

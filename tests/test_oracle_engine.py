"""Pins for the oracle's approximation engine (iACT, TAF, perforation, votes,
MAPE): hand-worked traces with closed-form counts, collapse to the exact
result at threshold or rate 0, and a brute-force re-statement on tiny
inputs (tests/brute.py) compared decision by decision."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import brute
import oracle

W = 64


def one_wave(ipt, fn):
    """Inputs/outputs for one full wave: item i = lane + 64 k."""
    n = W * ipt
    lane = np.arange(n) % W
    k = np.arange(n) // W
    return n, fn(lane, k)


# ---------------------------------------------------------------- TAF traces

def taf_closed_form(ipt, h, p):
    """Approximate steps for constant outputs: the window is full after h
    accurate steps, then each accurate step buys p approximate ones."""
    m = ipt - h
    return p * (m // (p + 1)) + min(m % (p + 1), p) if m > 0 else 0


@pytest.mark.parametrize("ipt,h,p", [(12, 4, 4), (20, 2, 2), (9, 1, 3), (33, 5, 7), (4, 4, 4), (3, 4, 2)])
def test_taf_constant_outputs_closed_form(ipt, h, p):
    n, y = one_wave(ipt, lambda lane, k: np.stack([np.full(lane.size, 3.5), np.full(lane.size, -1.25)]))
    r = oracle.taf(y, None, ipt, h, p, 0.01)
    approx_steps = int((r["dec"] == 1).sum())
    assert approx_steps == taf_closed_form(ipt, h, p)
    assert np.array_equal(r["out"], y)  # constant outputs: exact reuse
    if (ipt, h, p) == (12, 4, 4):
        assert list(np.nonzero(r["dec"] == 1)[0]) == [4, 5, 6, 7, 9, 10, 11]


def test_taf_ramp_crosses_threshold_without_window_reset():
    # y_k = 1 + 0.01 k, h = 2: RSD(y24, y25) = 0.004016 fails, RSD(y25, y26) = 0.003984 passes
    n, y = one_wave(40, lambda lane, k: (1.0 + 0.01 * k)[None, :])
    r = oracle.taf(y, None, 40, 2, 1, 0.004)
    dec = r["dec"]
    assert dec[:27].max() == 0 and dec[27] == 1
    # next accurate step 28 sees (y26, y28): RSD 0.0079 fails, no approximation at 29
    assert dec[28] == 0 and dec[29] == 0
    # step 29 sees (y28, y29): passes again, so step 30 approximates
    assert dec[30] == 1
    # the approximated step returns the last accurate output, y26
    assert np.all(r["out"][0, 27 * W:28 * W] == y[0, 26 * W])


def test_taf_rsd_special_cases():
    # zero mean with zero spread: RSD = 0 approximates whenever theta > 0
    n, y = one_wave(6, lambda lane, k: np.zeros((1, lane.size)))
    assert (oracle.taf(y, None, 6, 2, 1, 0.5)["dec"] == 1).sum() == 2
    assert (oracle.taf(y, None, 6, 2, 1, 0.0)["dec"] == 1).sum() == 0
    # zero mean with spread: RSD = inf never approximates
    n, y = one_wave(8, lambda lane, k: np.where(k % 2 == 0, 1.0, -1.0)[None, :])
    assert (oracle.taf(y, None, 8, 2, 1, 1e30)["dec"] == 1).sum() == 0
    # negative outputs use |mu|
    n, y = one_wave(6, lambda lane, k: np.full((1, lane.size), -2.0) + 0.001 * k)
    assert (oracle.taf(y, None, 6, 2, 1, 0.01)["dec"] == 1).sum() > 0


def test_taf_multi_output_uses_worst_output():
    # output 0 constant, output 1 wildly varying: never approximate
    n, y = one_wave(10, lambda lane, k: np.stack([np.ones(lane.size), 1.0 + (k % 2) * 5.0]))
    assert (oracle.taf(y, None, 10, 2, 2, 0.1)["dec"] == 1).sum() == 0


# --------------------------------------------------------------- iACT traces

def test_iact_constant_inputs():
    ipt = 5
    n, x = one_wave(ipt, lambda lane, k: np.tile(np.array([20.0, 25.0, 1.0, 0.02, 0.3])[:, None], (1, lane.size)))
    y = np.stack([np.arange(n) * 0.0 + 7.25, np.arange(n) * 0.0 + 0.5])
    r = oracle.iact(x, y, None, ipt, 2, 0.05)
    assert list(r["dec"]) == [0, 1, 1, 1, 1]
    assert r["writer"][0] == 0  # empty table: every distance infinite, lowest lane writes
    assert np.array_equal(r["out"], y)
    r0 = oracle.iact(x, y, None, ipt, 2, 0.0)
    assert list(r0["dec"]) == [0] * 5


@pytest.mark.parametrize("tsize,expect", [(2, 8), (1, 0), (4, 8)])
def test_iact_capacity_alternating_inputs(tsize, expect):
    ipt = 10
    xa = np.array([5.0, 10.0, 1.0, 0.02, 0.1])
    xb = np.array([30.0, 90.0, 9.0, 0.02, 0.5])
    n, x = one_wave(ipt, lambda lane, k: np.where((k % 2 == 0)[None, :], xa[:, None], xb[:, None]))
    y = np.stack([x[0] * 2, x[1] * 3])
    r = oracle.iact(x, y, None, ipt, tsize, 0.05)
    assert int((r["dec"] == 1).sum()) == expect


def test_iact_writer_is_farthest_lane():
    ipt = 2
    x0 = np.array([10.0, 20.0, 2.0, 0.02, 0.2])
    delta = 0.1  # > theta

    def gen(lane, k):
        x = np.tile(x0[:, None], (1, lane.size))
        x[0] = x[0] + np.where(k == 1, lane * delta, 0.0)
        return x
    n, x = one_wave(ipt, gen)
    y = np.stack([x[0], x[1]])
    r = oracle.iact(x, y, None, ipt, 4, 0.05)
    assert r["dec"][1] == 0 and r["votes"][1] == 1
    assert r["writer"][1] == 63


def test_iact_nearest_entry_ties_go_to_lowest_slot():
    ipt = 3
    xa = np.array([10.0, 20.0, 2.0, 0.0, 0.25])
    step = np.array([[0.0], [2.0], [1.0]])  # offsets of input 0 at steps 0, 1, 2

    def gen(lane, k):
        x = np.tile(xa[:, None], (1, lane.size))
        x[0] = x[0] + step[k, 0]
        return x
    n, x = one_wave(ipt, gen)
    y = np.stack([x[0] * 3.0, x[0] - 1.0])
    r = oracle.iact(x, y, None, ipt, 4, 1.5)
    # step 1 misses (distance 2 > 1.5) and stores the second entry; step 2 is
    # at distance 1 from both entries and must reuse slot 0's outputs
    assert list(r["dec"]) == [0, 0, 1]
    assert np.all(r["out"][:, 2 * W:] == y[:, :1])


@pytest.mark.parametrize("hits,expect", [(32, 0), (33, 1), (64, 1), (0, 0)])
def test_vote_majority_rule(hits, expect):
    ipt = 2
    x0 = np.array([10.0, 20.0, 2.0, 0.02, 0.2])

    def gen(lane, k):
        x = np.tile(x0[:, None], (1, lane.size))
        far = (k == 1) & (lane >= hits)
        x[1] = x[1] + np.where(far, 10.0 + lane, 0.0)
        return x
    n, x = one_wave(ipt, gen)
    y = np.stack([x[0], x[1]])
    r = oracle.iact(x, y, None, ipt, 4, 0.05)
    assert r["votes"][1] == hits and r["dec"][1] == expect


def test_vote_tail_wave_counts_active_lanes_only():
    # n = 69, ipt = 2: one wave; step 1 has 5 active lanes (items 64..68)
    n, ipt = 69, 2
    x = np.tile(np.array([10.0, 20.0, 2.0, 0.02, 0.2])[:, None], (1, n))
    x[1, 64 + 3:] += 50.0  # items 67, 68 far: 3 of 5 hit
    y = np.stack([x[0], x[1]])
    r = oracle.iact(x, y, None, ipt, 4, 0.05)
    assert oracle.num_lanes(n, ipt) == 64
    assert r["votes"][1] == 3 and r["dec"][1] == 1


# --------------------------------------------------------------- perforation

@pytest.mark.parametrize("kind,M,ipt,skipped", [
    (oracle.PERFO_SMALL, 10, 20, [9, 19]),
    (oracle.PERFO_SMALL, 10, 16, [9]),
    (oracle.PERFO_SMALL, 4, 8, [3, 7]),
    (oracle.PERFO_LARGE, 10, 20, [k for k in range(20) if k not in (0, 10)]),
])
def test_perforation_herded_steps(kind, M, ipt, skipped):
    n, y = one_wave(ipt, lambda lane, k: (1.0 + k)[None, :])
    init = np.full_like(y, -7.0)
    r = oracle.perfo(y, None, ipt, kind, M, 0, out_init=init)
    assert list(np.nonzero(r["dec"] == 1)[0]) == skipped
    for k in range(ipt):
        seg = r["out"][0, k * W:(k + 1) * W]
        assert np.all(seg == (-7.0 if k in skipped else 1.0 + k))
    assert r["evals"] == n - W * len(skipped)


def test_perforation_offset_rotates_pattern():
    n, y = one_wave(10, lambda lane, k: (1.0 + k)[None, :])
    r = oracle.perfo(y, None, 10, oracle.PERFO_SMALL, 5, 2)
    assert list(np.nonzero(r["dec"] == 1)[0]) == [2, 7]


@pytest.mark.parametrize("kind,p", [(oracle.PERFO_INI, 30), (oracle.PERFO_FINI, 25), (oracle.PERFO_INI, 100)])
def test_perforation_ini_fini_change_bounds(kind, p):
    n = 1000
    y = np.arange(n, dtype=np.float64)[None, :] + 1
    r = oracle.perfo(y, None, 4, kind, p, out_init=np.zeros_like(y))
    cut = p * n // 100
    done = r["out"][0] != 0
    if kind == oracle.PERFO_INI:
        assert not done[:cut].any() and done[cut:].all()
    else:
        assert done[:n - cut].all() and not done[n - cut:].any()


# ----------------------------------------------------------------- collapse

def test_collapse_at_zero_threshold_and_rate():
    from paper_2308_16877_amd import inputs
    x = inputs.periodic(5000, 8, jitter=1e-6)
    y, s = oracle.region_values_f32out(x)
    for ipt in (1, 3, 16):
        ri = oracle.iact(x, y, s, ipt, 8, 0.0)
        rt = oracle.taf(y, s, ipt, 2, 4, 0.0)
        rp = oracle.perfo(y, s, ipt, oracle.PERFO_SMALL, 0)
        for r in (ri, rt, rp):
            assert np.array_equal(r["out"], y)
            assert (r["dec"] == 1).sum() == 0
        # and with a positive threshold these inputs do approximate
        assert (oracle.taf(y, s, ipt, 2, 4, 0.01)["dec"] == 1).sum() > 0 or ipt < 3


# ------------------------------------------------------------- brute force

def _grid_case(data, max_n=300):
    n = data.draw(st.integers(1, max_n))
    ipt = data.draw(st.integers(1, 6))
    vals = data.draw(st.lists(st.integers(0, 3), min_size=n * 2, max_size=n * 2))
    x = np.array(vals, dtype=np.float64).reshape(2, n)
    return n, ipt, x


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(data=st.data())
def test_iact_matches_brute_force(data):
    n, ipt, x = _grid_case(data)
    tsize = data.draw(st.integers(1, 4))
    theta = data.draw(st.sampled_from([0.0, 0.5, 1.5, 2.5]))
    tpw = data.draw(st.sampled_from([1, 2, 4]))
    group = data.draw(st.sampled_from([1, 64, 128]))
    y = np.stack([x[0] * 10 + x[1], x[1] - x[0]])
    r = oracle.iact(x, y, None, ipt, tsize, theta, tables_per_wave=tpw, group=group)
    xs = [tuple(x[:, i]) for i in range(n)]
    ys = [tuple(y[:, i]) for i in range(n)]
    bout, bdec = brute.iact(xs, ys, ipt, tsize, float(np.float32(theta)), tpw, group)
    assert np.array_equal(r["out"].T, np.array(bout))
    for (w, k), d in bdec.items():
        assert r["dec"][w * ipt + k] == d, (w, k)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(data=st.data())
def test_taf_matches_brute_force(data):
    n, ipt, x = _grid_case(data)
    ipt = ipt + data.draw(st.integers(0, 6))
    h = data.draw(st.integers(1, 4))
    p = data.draw(st.integers(1, 5))
    theta = data.draw(st.sampled_from([0.0, 0.05, 0.3, 0.7, 2.0]))
    group = data.draw(st.sampled_from([1, 64, 128]))
    y = np.stack([x[0] + 5.0, x[1] * 0.5 + 1.0])
    r = oracle.taf(y, None, ipt, h, p, theta, group=group)
    ys = [tuple(y[:, i]) for i in range(n)]
    bout, bdec = brute.taf(ys, ipt, h, p, float(np.float32(theta)), group)
    assert np.array_equal(r["out"].T, np.array(bout))
    for (w, k), d in bdec.items():
        assert r["dec"][w * ipt + k] == d, (w, k)


def _taf_two_launches(y, L, a, b, h, p, theta, group):
    """Two launches with a carried state: the first a steps of every lane,
    then the next b (launch shapes n = a L and b L keep the L lanes)."""
    st = oracle.taf_state(a * L, a, h, y.shape[0])
    r1 = oracle.taf(y[:, :a * L], None, a, h, p, theta, group=group, state=st)
    st["shape"] = (b * L, b, h, y.shape[0])  # same lanes, the next steps
    r2 = oracle.taf(y[:, a * L:], None, b, h, p, theta, group=group, state=st)
    out = np.concatenate([r1["out"], r2["out"]], axis=1)
    dec = np.concatenate([r1["dec"].reshape(-1, a), r2["dec"].reshape(-1, b)], axis=1).ravel()
    return out, dec


def test_taf_state_constant_outputs_closed_form_across_launches():
    """C1 split over two launches (5 then 7 steps of one wave): the carried
    window and countdown give the 7 of 12 approximate steps of one launch."""
    y = np.full((2, 12 * W), 3.5)
    out, dec = _taf_two_launches(y, W, 5, 7, 4, 4, 0.01, 64)
    assert list(np.nonzero(dec == 1)[0]) == [4, 5, 6, 7, 9, 10, 11]
    assert np.array_equal(out, y)


@settings(max_examples=120, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(data=st.data())
def test_taf_state_continues_across_launches(data):
    """Two launches with a carried state equal one launch over both launches'
    steps (outputs and per-(wave, step) decisions), and both equal the brute
    force over the whole history of each lane."""
    waves = data.draw(st.integers(1, 3))
    L = waves * W
    a, b = data.draw(st.integers(1, 7)), data.draw(st.integers(1, 7))
    h = data.draw(st.integers(1, 4))
    p = data.draw(st.integers(1, 5))
    theta = data.draw(st.sampled_from([0.05, 0.3, 0.7]))
    group = data.draw(st.sampled_from([1, 64, 128]))
    n = (a + b) * L
    vals = data.draw(st.lists(st.integers(1, 4), min_size=n, max_size=n))
    y = np.stack([np.array(vals, np.float64), np.full(n, 2.0)])
    out, dec = _taf_two_launches(y, L, a, b, h, p, theta, group)
    one = oracle.taf(y, None, a + b, h, p, theta, group=group)
    assert np.array_equal(out, one["out"])
    assert np.array_equal(dec, one["dec"])
    bout, bdec = brute.taf([tuple(y[:, i]) for i in range(n)], a + b, h, p, float(np.float32(theta)), group)
    assert np.array_equal(out.T, np.array(bout))
    for (w, k), d in bdec.items():
        assert dec[w * (a + b) + k] == d, (w, k)


# ---------------------------------------------------------------------- MAPE

def test_mape_hand_example():
    m, nf, mr = oracle.mape([1.0, 2.0, 0.001], [1.1, 2.0, 0.0], tau=0.01)
    assert m == pytest.approx((0.1 + 0.0 + 0.1) / 3, rel=1e-14)
    assert nf == 1
    assert mr == pytest.approx(0.05, rel=1e-14)


def test_mape_of_exact_is_zero():
    x = np.linspace(-3, 3, 101)
    assert oracle.mape(x, x) == (0.0, int((np.abs(x) < oracle.MAPE_TAU).sum()), 0.0)


# ------------------------------------------------- iACT distance precision

def _real_case(data, max_n=300):
    """Real-valued inputs (not on a grid): FP32 and FP64 distances differ in
    their last bits, so the two readings can choose differently near ties."""
    n = data.draw(st.integers(1, max_n))
    ipt = data.draw(st.integers(1, 6))
    seed = data.draw(st.integers(0, 2**31 - 1))
    g = np.random.default_rng(seed)
    x = g.integers(0, 4, (2, n)).astype(np.float64) + g.normal(0, 0.3, (2, n))
    return n, ipt, x.astype(np.float32).astype(np.float64)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(data=st.data())
def test_iact_fp64_distances_match_brute_force(data):
    """The FP64 reading is the plain definition: on real-valued inputs it
    takes every decision the brute-force re-statement (distances in Python's
    double precision, summed in the same order) takes."""
    n, ipt, x = _real_case(data)
    tsize = data.draw(st.integers(1, 4))
    theta = data.draw(st.sampled_from([0.0, 0.5, 1.5, 2.5]))
    tpw = data.draw(st.sampled_from([1, 2, 4]))
    group = data.draw(st.sampled_from([1, 64, 128]))
    y = np.stack([x[0] * 10 + x[1], x[1] - x[0]])
    r = oracle.iact(x, y, None, ipt, tsize, theta, tables_per_wave=tpw, group=group, dist_fp64=True)
    xs = [tuple(float(np.float32(v)) for v in x[:, i]) for i in range(n)]
    ys = [tuple(y[:, i]) for i in range(n)]
    bout, bdec = brute.iact(xs, ys, ipt, tsize, float(np.float32(theta)), tpw, group)
    assert np.array_equal(r["out"].T, np.array(bout))
    for (w, k), d in bdec.items():
        assert r["dec"][w * ipt + k] == d, (w, k)


@settings(max_examples=100, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(data=st.data())
def test_iact_fp32_and_fp64_readings_agree_on_a_grid(data):
    """On integer-grid inputs every squared distance is exact in FP32, so
    the FP32 reading (the precision the kernels decide in) and the FP64
    definition take identical decisions, writers and outputs."""
    n, ipt, x = _grid_case(data)
    tsize = data.draw(st.integers(1, 4))
    theta = data.draw(st.sampled_from([0.5, 1.5, 2.5]))
    y = np.stack([x[0] * 10 + x[1], x[1] - x[0]])
    a = oracle.iact(x, y, None, ipt, tsize, theta)
    b = oracle.iact(x, y, None, ipt, tsize, theta, dist_fp64=True)
    for key in ("out", "dec", "votes", "writer", "napprox"):
        assert np.array_equal(a[key], b[key]), key


def test_iact_precision_mismatches_are_all_marked_fragile():
    """Real inputs whose distances cluster at the threshold: the FP32
    reading and the FP64 definition disagree somewhere, and the first
    disagreement of every wave (decision or writer) falls on a (wave, step)
    that the FP64 run marks fragile at a band of 1e-5; the band is what
    explains a GPU/oracle disagreement in the GPU parity tests."""
    from paper_2308_16877_amd import inputs
    x = inputs.periodic(65536, 8, jitter=1e-3)
    y, s = oracle.region_values_f32out(x)
    # a threshold at the median nearest-pool-tuple distance puts many lanes at it
    a = oracle.iact(x, y, s, 16, 8, 0.08)
    b = oracle.iact(x, y, s, 16, 8, 0.08, dist_fp64=True, band=1e-5)
    code_a = np.where(a["dec"] >= 0, a["dec"].astype(np.int32) * 128 + a["writer"] + 1, -1).reshape(-1, 16)
    code_b = np.where(b["dec"] >= 0, b["dec"].astype(np.int32) * 128 + b["writer"] + 1, -1).reshape(-1, 16)
    fr = b["fragile"].reshape(-1, 16)
    neq = code_a != code_b
    waves = np.nonzero(neq.any(axis=1))[0]
    for w in waves:
        k = int(np.argmax(neq[w]))
        assert fr[w, k], (w, k)
    assert fr.sum() >= len(waves)
    print("waves where the readings part: %d of %d; fragile steps %d" % (len(waves), fr.shape[0], int(fr.sum())))
    # and outside the waves where the readings part, the outputs agree
    # except at steps whose arg-min was a near tie
    L = oracle.num_lanes(65536, 16)
    i = np.arange(65536)
    wave, step = (i % L) // 64, i // L
    keep = ~neq.any(axis=1)[wave] & ~fr.astype(bool)[wave, step]
    assert np.array_equal(a["out"][:, keep], b["out"][:, keep])


def test_iact_precision_flip_is_marked_fragile():
    """A wave built so that the readings disagree: every lane stores (10, 10)
    at step 0 and meets (10.4447126, 10.7893143) at step 1, at a distance
    within 4e-7 of theta = 0.9059726 -- below it in FP64, not below it in
    FP32 (the FP32 sum rounds up).  The FP64 run approximates step 1, the
    FP32 run computes it, and the FP64 run marks that step fragile."""
    th = 0.9059725999832153
    x = np.zeros((2, 128), np.float32)
    x[:, :64] = 10.0
    x[0, 64:], x[1, 64:] = 10.44471263885498, 10.789314270019531
    x = x.astype(np.float64)
    y = np.stack([x[0] + 1.0, x[1] + 2.0])
    a = oracle.iact(x, y, None, 2, 2, th)
    b = oracle.iact(x, y, None, 2, 2, th, dist_fp64=True, band=1e-5)
    assert a["dec"][1] == 0 and b["dec"][1] == 1
    assert b["fragile"][1] == 1 and b["fragile"][0] == 0


def test_iact_fragile_band_marks_a_threshold_tie():
    """One wave of identical inputs at distance exactly theta from the
    stored entry: every lane's statistic is at the threshold, the vote is
    marked fragile at any positive band, and with band 0 nothing is."""
    x = np.zeros((2, 128))
    x[0, 64:] = 1.5  # step 1: distance 1.5 from step 0's inputs
    y = np.stack([x[0] + 1.0, x[1] + 2.0])
    r = oracle.iact(x, y, None, 2, 2, 1.5, dist_fp64=True, band=1e-5)
    assert r["fragile"][1] == 1 and r["fragile"][0] == 0
    assert r["dec"][1] == 0  # strict <: a distance equal to theta does not qualify
    r0 = oracle.iact(x, y, None, 2, 2, 1.5, dist_fp64=True)
    assert not r0["fragile"].any()


# ------------------------------------------------------------------- Adam

def test_adam_first_step_is_the_normalised_gradient():
    """From zero moments the bias corrections make m_hat = g and v_hat = g^2
    at step 1, so each parameter moves by -lr g / (|g| + eps): almost
    exactly lr against the sign of its gradient (eps = 0.5 makes a
    misplaced eps, e.g. under the square root, visible)."""
    g = np.random.default_rng(3).standard_normal((3, 50))
    w0 = np.random.default_rng(4).standard_normal(50)
    z = np.zeros(50)
    gs = g.sum(0)
    for eps in (1e-8, 0.5):
        w, m, v = oracle.adam(g, w0, z, z, 0.1, 0.9, 0.999, eps, 1)
        assert np.allclose(w, w0 - 0.1 * gs / (np.abs(gs) + eps), rtol=0, atol=1e-14)
        assert np.allclose(m, 0.1 * gs, rtol=1e-14) and np.allclose(v, 0.001 * gs * gs, rtol=1e-12)


def test_adam_constant_gradient_moves_a_fixed_amount_per_step():
    """With a constant gradient g from zero moments, m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so every step moves the parameter by exactly
    -lr g / (|g| + eps) whatever t (a wrong power in a bias correction
    breaks this from the second step on)."""
    g = np.array([[0.3, -2.0, 1e-3, 7.0]])
    w = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 9):
        w, m, v = oracle.adam(g, w, m, v, 0.01, 0.9, 0.99, 1e-3, t)
        assert np.allclose(w, -t * 0.01 * g[0] / (np.abs(g[0]) + 1e-3), rtol=1e-12, atol=0)


def test_adam_alternating_gradient_follows_the_geometric_series():
    """g_t = (-1)^(t+1) c: v_hat = c^2 at every t, while the first moment is
    a geometric series of ratio -b1, m_t = (1 - b1) g_t (1 - (-b1)^t) / (1 + b1)
    -- which tells b1 from b2, and m from v."""
    c = np.array([0.5, -1.5, 3.0])
    b1, b2, lr, eps = 0.8, 0.95, 0.05, 0.0
    w = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    for t in range(1, 7):
        g = c * (-1) ** (t + 1)
        w_prev = w
        w, m, v = oracle.adam(g[None, :], w, m, v, lr, b1, b2, eps, t)
        m_closed = (1 - b1) * g * (1 - (-b1) ** t) / (1 + b1)
        assert np.allclose(m, m_closed, rtol=1e-13)
        step = lr * (m_closed / (1 - b1 ** t)) / np.abs(c)
        assert np.allclose(w_prev - w, step, rtol=1e-12)


def test_adam_sums_the_partial_gradients():
    """The gradient is the sum of the partials: any split of it into blocks
    gives the one-block step (to rounding)."""
    rng = np.random.default_rng(5)
    total = rng.standard_normal(40)
    parts = rng.standard_normal((5, 40))
    parts[-1] = total - parts[:-1].sum(0)
    w0, m0, v0 = rng.standard_normal(40), rng.standard_normal(40) * 0.1, rng.random(40) * 0.1
    a = oracle.adam(parts, w0, m0, v0, 1e-2, 0.9, 0.999, 1e-8, 3)
    b = oracle.adam(total[None, :], w0, m0, v0, 1e-2, 0.9, 0.999, 1e-8, 3)
    for u, w in zip(a, b):
        assert np.allclose(u, w, rtol=1e-12, atol=1e-15)

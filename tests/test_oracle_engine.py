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


# ---------------------------------------------------------------------- MAPE

def test_mape_hand_example():
    m, nf, mr = oracle.mape([1.0, 2.0, 0.001], [1.1, 2.0, 0.0], tau=0.01)
    assert m == pytest.approx((0.1 + 0.0 + 0.1) / 3, rel=1e-14)
    assert nf == 1
    assert mr == pytest.approx(0.05, rel=1e-14)


def test_mape_of_exact_is_zero():
    x = np.linspace(-3, 3, 101)
    assert oracle.mape(x, x) == (0.0, int((np.abs(x) < oracle.MAPE_TAU).sum()), 0.0)

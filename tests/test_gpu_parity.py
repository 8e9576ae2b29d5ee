"""GPU parity: every entry point, called through the C ABI on seeded inputs,
against the CPU oracle.

Bars:
 - outputs within 1e-5 of the scale |S N(d1)| + |K e^{-rT} N(d2)| (and the
   put's analogue) of the item whose region evaluation produced them;
 - iACT decisions, votes and writers bit-exact (both sides evaluate the
   squared distance in FP32 with the same rounding sequence);
 - TAF decisions equal except at steps the oracle marks fragile (an RSD
   within the band of the threshold that could flip the majority), where
   the rest of that wave is excluded; at least 99.99% agree;
 - perforation decisions bit-exact, dropped items untouched;
 - MAPE against the FP64 exact prices within 1e-4 of the oracle's;
 - threshold or rate 0 reproduces hpac_exact bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import (DEV, SENTINEL, check_outputs, compare_decisions, mape_pair, run, say, to_dev, trace_dec)
from paper_2308_16877_amd import hpac, inputs

pytestmark = pytest.mark.gpu

LEVEL_GROUP = {"thread": 1, "wave": 64, "block": None}


def group_of(level, block_size):
    return block_size if level == "block" else LEVEL_GROUP[level]


def exact_ref(x):
    C, P, sC, sP = oracle.bs_price(*x)
    return np.stack([C, P]), np.stack([sC, sP])


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hpac.lib()  # fails loudly if the library is missing
    say("device:", torch.cuda.get_device_name(0))


# ------------------------------------------------------------------- exact

@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 4099, 65536])
@pytest.mark.parametrize("ipt", [1, 3, 16])
def test_exact_matches_oracle(n, ipt):
    say("exact n=%d ipt=%d" % (n, ipt))
    x = inputs.portfolio(n, 1024)
    y, t, cnt = run("exact", to_dev(x), 2, ipt)
    ref, scale = exact_ref(x)
    check_outputs(y, ref, scale, what="exact")
    assert cnt[0] == n


def test_exact_full_box_and_extremes():
    # uniform over the box plus its corners and deep in/out of the money
    x = inputs.uniform_box(200000, seed=31).astype(np.float32)
    corners = np.array([[5, 100, 0.25, 0.02, 0.1], [30, 1, 10, 0.02, 0.5], [5, 100, 10, 0.02, 0.5],
                        [30, 1, 0.25, 0.02, 0.1], [20, 20, 1, 0.02, 0.3]], np.float32).T
    x = np.concatenate([x, corners], axis=1)
    y, _, _ = run("exact", to_dev(x), 2, 4)
    ref, scale = exact_ref(x)
    check_outputs(y, ref, scale, what="exact box")


@pytest.mark.parametrize("block", [64, 128, 192, 256])
def test_exact_block_sizes(block):
    x = inputs.portfolio(10007, 1024)
    y, _, _ = run("exact", to_dev(x), 2, 5, block_size=block)
    ref, scale = exact_ref(x)
    check_outputs(y, ref, scale, what="exact block %d" % block)


# -------------------------------------------------------------------- iACT

IACT_CASES = [
    # name, input builder, ipt, table, theta, tables/wave, level
    ("config0", lambda: inputs.portfolio(65536, 1024), 16, 8, 0.05, 1, "wave"),
    ("periodic8", lambda: inputs.periodic(65536, 8, jitter=1e-4), 16, 8, 0.05, 1, "wave"),
    ("periodic2", lambda: inputs.periodic(65536, 2, jitter=1e-3), 16, 8, 0.05, 1, "wave"),
    ("periodic8_mixed", lambda: inputs.periodic(65536, 8, jitter=1e-3), 16, 8, 0.08, 1, "wave"),
    ("periodic16_t8", lambda: inputs.periodic(40000, 16, jitter=1e-4), 12, 8, 0.05, 1, "wave"),
    ("ragged", lambda: inputs.periodic(4099, 4, jitter=1e-4), 3, 4, 0.05, 1, "wave"),
    ("grouped", lambda: inputs.grouped(65536, 64, jitter=1e-4), 16, 4, 0.05, 1, "wave"),
    ("thread_tpw64", lambda: inputs.periodic(65536, 8, jitter=1e-4), 16, 2, 0.05, 64, "thread"),
    ("thread_tpw1", lambda: inputs.periodic(30000, 8, jitter=1e-3), 8, 8, 0.1, 1, "thread"),
    ("wave_tpw4", lambda: inputs.periodic(65536, 8, jitter=1e-4), 16, 4, 0.05, 4, "wave"),
    ("block_tpw2", lambda: inputs.periodic(65536, 8, jitter=1e-3), 16, 8, 0.08, 2, "block"),
    # padded tables would overflow 64 KiB of LDS: interleaved word by word
    ("thread_tpw64_t8", lambda: inputs.periodic(65536, 8, jitter=1e-4), 16, 8, 0.05, 64, "thread"),
    ("wave_tpw32_t16", lambda: inputs.periodic(65536, 16, jitter=1e-4), 16, 16, 0.05, 32, "wave"),
    ("block_tpw64_t8", lambda: inputs.periodic(65536, 8, jitter=1e-3), 16, 8, 0.08, 64, "block"),
    ("table32", lambda: inputs.periodic(65536, 32, jitter=1e-4), 64, 32, 0.05, 1, "wave"),
    ("table1", lambda: inputs.constant(5000), 7, 1, 0.05, 1, "wave"),
    # one table per wave in registers, sized to a power of two: table sizes
    # that fill it and that leave padded slots, at every level
    ("table16", lambda: inputs.periodic(65536, 16, jitter=1e-4), 32, 16, 0.05, 1, "wave"),
    ("table5", lambda: inputs.periodic(30000, 6, jitter=1e-4), 16, 5, 0.05, 1, "wave"),
    ("table12_block", lambda: inputs.periodic(65536, 16, jitter=1e-3), 24, 12, 0.08, 1, "block"),
    ("table20_thread", lambda: inputs.periodic(40000, 24, jitter=1e-4), 40, 20, 0.05, 1, "thread"),
    ("table3_ragged", lambda: inputs.periodic(5001, 4, jitter=1e-4), 9, 3, 0.05, 1, "wave"),
]


@pytest.mark.parametrize("case", IACT_CASES, ids=[c[0] for c in IACT_CASES])
def test_iact_matches_oracle(case):
    name, mk, ipt, t, theta, tpw, level = case
    say("iact", name)
    check_iact(name, mk(), ipt, t, theta, tpw, level, 256)


@pytest.mark.parametrize("tpw,t,level,block", [(64, 8, "wave", 64), (64, 8, "thread", 128), (32, 16, "wave", 64),
                                               (1, 8, "wave", 64), (16, 8, "thread", 192)])
def test_iact_block_sizes_match_oracle(tpw, t, level, block):
    """At thread and wave level the workgroup size changes only how many
    tables share its LDS (padded or interleaved layout) and the occupancy:
    decisions and outputs stay the oracle's."""
    say("iact tpw %d t %d %s block %d" % (tpw, t, level, block))
    x = inputs.periodic(65536, 16 if t == 16 else 8, jitter=1e-4)
    check_iact("block%d" % block, x, 16, t, 0.05, tpw, level, block)


def check_iact(name, x, ipt, t, theta, tpw, level, block):
    n = x.shape[1]
    y, tr, cnt = run("iact", to_dev(x), 2, ipt, block_size=block, table_size=t, threshold=theta, tables_per_wave=tpw,
                     level=level)
    yv, sv = oracle.region_values_f32out(x)
    ora = oracle.iact(x, yv, sv, ipt, t, theta, tables_per_wave=tpw, group=group_of(level, block),
                      out_init=np.full_like(yv, SENTINEL))
    gdec, f = trace_dec(tr)
    assert np.array_equal(gdec, ora["dec"]), "decision masks differ"
    act = f["active"]
    assert np.array_equal(f["votes"][act], ora["votes"][act])
    assert np.array_equal(f["napprox"][act], ora["napprox"][act])
    ow = ora["writer"]
    assert np.array_equal(f["writer_valid"] & act, (ow >= 0) & act)
    v = f["writer_valid"] & act
    assert np.array_equal(f["writer"][v], ow[v])
    check_outputs(y, ora["out"], ora["scale"], what="iact " + name)
    ref, _ = exact_ref(x)
    mg, mo = mape_pair(ref, y, ora["out"])
    assert abs(mg - mo) <= 1e-4
    assert cnt[0] == n and cnt[1] == int(ora["napprox"][act].sum())
    say("  approx lanes %.4f  mape gpu %.3g oracle %.3g" % (cnt[1] / n, mg, mo))


def flip_wave_inputs():
    """One wave that stores (S, K) = (10, 10) at step 0 and meets
    (10.4447126, 10.7893143) at step 1 (T, r, v unchanged): at a threshold
    of 0.9059726 the FP32 distance test fails and the FP64 one passes."""
    x = np.tile(np.array([[10.0], [10.0], [1.0], [0.02], [0.3]], np.float32), (1, 128))
    x[0, 64:], x[1, 64:] = 10.44471263885498, 10.789314270019531
    return x


IACT_FP64_CASES = [
    # name, input builder, ipt, table, theta, tables/wave, level
    ("config0", lambda: inputs.portfolio(65536, 1024), 16, 8, 0.05, 1, "wave"),
    ("periodic8_mixed", lambda: inputs.periodic(65536, 8, jitter=1e-3), 16, 8, 0.08, 1, "wave"),
    ("periodic2", lambda: inputs.periodic(65536, 2, jitter=1e-3), 16, 8, 0.05, 1, "wave"),
    ("thread_tpw1", lambda: inputs.periodic(30000, 8, jitter=1e-3), 8, 8, 0.1, 1, "thread"),
    ("block_tpw2", lambda: inputs.periodic(65536, 8, jitter=1e-3), 16, 8, 0.08, 2, "block"),
    ("flip", flip_wave_inputs, 2, 2, 0.9059725999832153, 1, "wave"),
]


@pytest.mark.parametrize("case", IACT_FP64_CASES, ids=[c[0] for c in IACT_FP64_CASES])
def test_iact_against_fp64_distances(case):
    """The kernels decide on the squared distance in FP32; the oracle here
    takes the plain FP64 definition instead.  Decisions and writers agree on
    at least 99.99% of (wave, step) records, and every first disagreement of
    a wave falls on a record where a distance lies within 1e-5 relative of
    the threshold (and could flip the vote), two writer candidates or two
    nearest entries lie within 1e-5 relative of each other: the FP32 reading
    hides no kernel defect.  Outputs away from such records match the
    oracle's to 1e-5 of scale, and the MAPE to 1e-4."""
    name, mk, ipt, t, theta, tpw, level = case
    say("iact fp64 distances", name)
    x = mk()
    n = x.shape[1]
    y, tr, cnt = run("iact", to_dev(x), 2, ipt, table_size=t, threshold=theta, tables_per_wave=tpw, level=level)
    yv, sv = oracle.region_values_f32out(x)
    ora = oracle.iact(x, yv, sv, ipt, t, theta, tables_per_wave=tpw, group=group_of(level, 256),
                      out_init=np.full_like(yv, SENTINEL), dist_fp64=True, band=GATE_BAND)
    gdec, f = trace_dec(tr)
    gw = np.where(f["writer_valid"], f["writer"], -1)
    gcode = np.where(gdec >= 0, gdec.astype(np.int32) * 128 + gw + 1, -1)
    ocode = np.where(ora["dec"] >= 0, ora["dec"].astype(np.int32) * 128 + ora["writer"] + 1, -1)
    agree, compared, explained, cascaded = compare_decisions(gcode, ocode, ipt, ora["fragile"], lag=0)
    if name == "flip":
        # one wave of two steps, built to part at its fragile second step
        assert explained == 1 and compared == 2 and agree == 1
    else:
        assert agree >= 0.9999 * compared
    say("  decisions agree %d/%d, explained %d, fragile records %d" % (agree, compared, explained,
                                                                       int(ora["fragile"].sum())))
    same_wave = np.all(gcode.reshape(-1, ipt) == ocode.reshape(-1, ipt), axis=1)
    L = oracle.num_lanes(n, ipt)
    i = np.arange(n)
    rec = ((i % L) // 64) * ipt + i // L
    mask = same_wave[(i % L) // 64] & ~ora["fragile"].astype(bool)[rec]
    check_outputs(y, ora["out"], ora["scale"], mask=mask, what="iact fp64 " + name)
    if mask.any():
        ref, _ = exact_ref(x)
        mg, mo = mape_pair(ref, y, ora["out"], mask=mask)
        assert abs(mg - mo) <= 1e-4


# --------------------------------------------------------------------- TAF

TAF_CASES = [
    # name, input builder, ipt, h, p, theta, level
    ("config0", lambda: inputs.portfolio(65536, 1024), 16, 4, 4, 0.01, "wave"),
    ("periodic8", lambda: inputs.periodic(65536, 8, jitter=1e-4), 16, 4, 4, 0.01, "wave"),
    ("periodic8_mixed", lambda: inputs.periodic(65536, 8, jitter=1e-3), 16, 4, 4, 0.007, "wave"),
    ("h2_p7", lambda: inputs.periodic(65536, 16, jitter=3e-4), 32, 2, 7, 0.005, "wave"),
    ("h8", lambda: inputs.periodic(65536, 16, jitter=1e-4), 32, 8, 3, 0.01, "wave"),
    ("ragged", lambda: inputs.periodic(4099, 4, jitter=1e-4), 5, 2, 2, 0.01, "wave"),
    ("thread", lambda: inputs.periodic(65536, 8, jitter=1e-3), 16, 3, 2, 0.003, "thread"),
    ("block", lambda: inputs.periodic(65536, 8, jitter=1e-3), 16, 3, 2, 0.006, "block"),
    ("h1", lambda: inputs.constant(6000), 9, 1, 2, 0.01, "wave"),
    ("mixed_h3", lambda: inputs.periodic(65536, 8, jitter=1e-3), 16, 3, 3, 0.006, "wave"),
]


# Decision gate: a mismatch is explained only by a statistic within 1e-5
# relative of its threshold (with the engine fed the GPU's own FP32 region
# values, both sides compute every statistic from identical numbers).
GATE_BAND = 1e-5


def taf_band(theta):
    """Relative band for the free-running comparison, where the oracle's
    region values are the FP64 prices rounded to FP32 and the GPU's are its
    own FP32 evaluations, a few ulp apart: such a difference moves a lane's
    RSD by up to about 2 eps (1 + RSD) with eps <= 2e-6.  Used only to
    decide which waves' outputs can be compared; decisions are gated by the
    replay at GATE_BAND."""
    return 1e-5 + 4e-6 * (1.0 + theta) / theta


def gpu_exact_values(x_dev):
    """The uncounted exact kernel's FP32 outputs, as float64 (the value
    source of the decision replay)."""
    y, _, _ = run("exact", x_dev, 2, 1, trace=False, counters=False)
    return y


@pytest.mark.parametrize("case", TAF_CASES, ids=[c[0] for c in TAF_CASES])
def test_taf_matches_oracle(case):
    name, mk, ipt, h, p, theta, level = case
    say("taf", name)
    check_taf(name, mk(), ipt, h, p, theta, level, 256)


@pytest.mark.parametrize("level,block", [("wave", 64), ("wave", 192), ("thread", 128), ("block", 128), ("block", 192)])
def test_taf_block_sizes_match_oracle(level, block):
    """The workgroup size is the decision group at block level (groups of
    128 or 192 lanes, the last one ragged) and only a launch shape at the
    other levels."""
    say("taf %s block %d" % (level, block))
    check_taf("%s_block%d" % (level, block), inputs.periodic(65536, 8, jitter=1e-3), 16, 3, 2, 0.006, level, block)


def check_taf(name, x, ipt, h, p, theta, level, block):
    n = x.shape[1]
    xd = to_dev(x)
    y, tr, cnt = run("taf", xd, 2, ipt, block_size=block, history_size=h, prediction_size=p,
                     rsd_threshold=theta, level=level)
    yv, sv = oracle.region_values_f32out(x)
    replay_taf(name, y, tr, gpu_exact_values(xd), sv, ipt, h, p, theta, level, block)
    ora = oracle.taf(yv, sv, ipt, h, p, theta, band=taf_band(theta), group=group_of(level, block),
                     out_init=np.full_like(yv, SENTINEL))
    gdec, f = trace_dec(tr)
    odec = ora["dec"]
    if level == "thread":
        # lanes decide alone: compare how many lanes of each wave approximated
        gdec = np.where(f["active"], f["napprox"], -1)
        odec = np.where(ora["dec"] >= 0, ora["napprox"], -1)
    agree, compared, explained, cascaded = compare_decisions(gdec, odec, ipt, ora["fragile"], lag=1)
    if level == "thread":
        # lanes decide alone: the mask is per lane; count lane-steps that
        # differ (at least |napprox_gpu - napprox_oracle| per wave-step)
        act_lanes = int(np.where(ora["dec"] >= 0, 1, 0).sum()) * 64
        diff = int(np.abs(np.where(gdec >= 0, gdec, 0) - np.where(odec >= 0, odec, 0)).sum())
        assert diff <= 1e-4 * act_lanes + cascaded * 64
    else:
        assert agree >= 0.9999 * compared
    say("  decisions agree %d/%d, explained %d, cascaded %d, fragile steps %d"
        % (agree, compared, explained, cascaded, int(ora["fragile"].sum())))
    # outputs on every wave whose history matched the oracle's
    g = gdec.reshape(-1, ipt)
    o = odec.reshape(-1, ipt)
    same_wave = np.all(g == o, axis=1)
    L = oracle.num_lanes(n, ipt)
    item_wave = ((np.arange(n) % L) // 64)
    mask = same_wave[item_wave]
    check_outputs(y, ora["out"], ora["scale"], mask=mask, what="taf " + name)
    ref, _ = exact_ref(x)
    mg, mo = mape_pair(ref, y, ora["out"])
    assert abs(mg - mo) <= 1e-4
    assert cnt[0] == n
    say("  approx lanes %.4f  mape gpu %.3g oracle %.3g" % (cnt[1] / n, mg, mo))


def replay_taf(name, y, tr, y_exact_gpu, sv, ipt, h, p, theta, level, block):
    """Decision replay: the oracle's TAF engine runs on the GPU exact
    kernel's FP32 outputs, so its RSD statistics come from the very numbers
    the kernel's windows hold.  Every (wave, step) decision must agree
    except where the oracle marks a statistic within GATE_BAND relative of
    the threshold that could flip the vote (the rest of that wave is then
    not compared); at least 99.99% agree; and on the agreeing waves the
    outputs are bit for bit the oracle's (both reuse identical values)."""
    ora = oracle.taf(y_exact_gpu, sv, ipt, h, p, theta, band=GATE_BAND, group=group_of(level, block),
                     out_init=np.full_like(y_exact_gpu, SENTINEL))
    gdec, f = trace_dec(tr)
    odec = ora["dec"]
    if level == "thread":
        gdec = np.where(f["active"], f["napprox"], -1)
        odec = np.where(ora["dec"] >= 0, ora["napprox"], -1)
    agree, compared, explained, cascaded = compare_decisions(gdec, odec, ipt, ora["fragile"], lag=1)
    assert agree >= 0.9999 * compared
    say("  replay: decisions agree %d/%d, explained %d" % (agree, compared, explained))
    n = y.shape[1]
    same_wave = np.all(gdec.reshape(-1, ipt) == odec.reshape(-1, ipt), axis=1)
    L = oracle.num_lanes(n, ipt)
    mask = same_wave[(np.arange(n) % L) // 64]
    assert np.array_equal(y[:, mask], ora["out"][:, mask]), "replayed outputs differ on agreeing waves"


@pytest.mark.parametrize("level,h,p,theta,block", [("wave", 4, 4, 0.01, 256), ("wave", 3, 2, 0.006, 192),
                                                    ("thread", 3, 2, 0.006, 256), ("block", 3, 2, 0.006, 128)])
def test_taf_persistent_state_continues_across_launches(level, h, p, theta, block):
    """With a persistent state, launches of 6 and then 10 steps per lane over
    consecutive parts of the inputs write exactly what one launch of 16
    steps writes, and their traces are that launch's (windows, fills and
    countdowns carried through the state, including approximate runs that
    straddle the two launches); the two launches also match the oracle's
    own two launches with a carried state, on the GPU exact kernel's values
    (decision replay)."""
    say("taf state %s h %d p %d" % (level, h, p))
    x = inputs.periodic(65536, 8, jitter=1e-3)
    n, a, b = x.shape[1], 6, 10
    L = oracle.num_lanes(n, a + b)
    n1 = a * L
    assert oracle.num_lanes(n1, a) == L and oracle.num_lanes(n - n1, b) == L
    kw = dict(block_size=block, history_size=h, prediction_size=p, rsd_threshold=theta, level=level)
    need = hpac.hpac_taf_state_bytes(hpac.REGION_BS_PRICE, n1, a, h)
    assert need == hpac.hpac_taf_state_bytes(hpac.REGION_BS_PRICE, n - n1, b, h) == L * (2 * h + 2) * 4
    state = torch.zeros(need, dtype=torch.uint8, device=DEV)
    xd = to_dev(x)
    y1, t1, _ = run("taf", to_dev(x[:, :n1]), 2, a, state=state, **kw)
    y2, t2, _ = run("taf", to_dev(x[:, n1:]), 2, b, state=state, **kw)
    y, t, _ = run("taf", xd, 2, a + b, **kw)
    assert np.array_equal(np.concatenate([y1, y2], axis=1), y)
    assert np.array_equal(np.concatenate([t1.reshape(-1, a), t2.reshape(-1, b)], axis=1).ravel(), t)
    gdec, _ = trace_dec(t)
    assert (gdec == 1).any() and (gdec == 0).any()  # mixed decisions
    # the oracle's two launches, state carried, on the GPU's exact values
    ye = gpu_exact_values(xd)
    _, sv = oracle.region_values_f32out(x)
    st = oracle.taf_state(n1, a, h)
    g = group_of(level, block)
    o1 = oracle.taf(ye[:, :n1], sv[:, :n1], a, h, p, theta, band=GATE_BAND, group=g, state=st)
    st["shape"] = (n - n1, b, h, 2)
    o2 = oracle.taf(ye[:, n1:], sv[:, n1:], b, h, p, theta, band=GATE_BAND, group=g, state=st)
    odec = np.concatenate([o1["dec"].reshape(-1, a), o2["dec"].reshape(-1, b)], axis=1).ravel()
    ofrag = np.concatenate([o1["fragile"].reshape(-1, a), o2["fragile"].reshape(-1, b)], axis=1).ravel()
    if level == "thread":
        f = hpac.trace_fields(t)
        gdec = np.where(f["active"], f["napprox"], -1)
        odec = np.concatenate([o1["napprox"].reshape(-1, a), o2["napprox"].reshape(-1, b)], axis=1).ravel()
        odec = np.where(np.concatenate([o1["dec"].reshape(-1, a), o2["dec"].reshape(-1, b)], axis=1).ravel() >= 0,
                        odec, -1)
    agree, compared, explained, _ = compare_decisions(gdec, odec, a + b, ofrag, lag=1)
    assert agree >= 0.9999 * compared
    oout = np.concatenate([o1["out"], o2["out"]], axis=1)
    same = np.all(gdec.reshape(-1, a + b) == odec.reshape(-1, a + b), axis=1)[(np.arange(n) % L) // 64]
    assert np.array_equal(y[:, same], oout[:, same])
    say("  decisions agree %d/%d, explained %d" % (agree, compared, explained))


# ------------------------------------------------------------- perforation

PERFO_CASES = [
    ("small10", "small", 10, 0, 20, 65536),
    ("small10_ipt16", "small", 10, 0, 16, 65536),
    ("small5", "small", 5, 0, 20, 65536),
    ("small2", "small", 2, 0, 20, 65536),
    ("small4_offset", "small", 4, 3, 9, 4099),
    ("large4", "large", 4, 0, 8, 65536),
    ("ini30", "ini", 30, 0, 4, 10007),
    ("fini25", "fini", 25, 0, 4, 10007),
]


@pytest.mark.parametrize("case", PERFO_CASES, ids=[c[0] for c in PERFO_CASES])
def test_perfo_matches_oracle(case):
    name, kind, param, offset, ipt, n = case
    say("perfo", name)
    x = inputs.portfolio(n, 1024)
    y, tr, cnt = run("perfo", to_dev(x), 2, ipt, kind=kind, param=param, offset=offset)
    yv, sv = oracle.region_values_f32out(x)
    k = {"small": 0, "large": 1, "ini": 2, "fini": 3}[kind]
    ora = oracle.perfo(yv, sv, ipt, k, param, offset, out_init=np.full_like(yv, SENTINEL))
    gdec, f = trace_dec(tr)
    assert np.array_equal(gdec, ora["dec"])
    skipped = ora["out"][0] == SENTINEL
    assert np.all(y[:, skipped] == SENTINEL), "dropped items must keep their previous contents"
    check_outputs(y, ora["out"], ora["scale"], mask=~skipped, what="perfo " + name)
    assert cnt[0] == n and cnt[1] == int(skipped.sum())


@pytest.mark.parametrize("block", [64, 128, 192])
@pytest.mark.parametrize("traced", [True, False])
def test_perfo_block_sizes_match_oracle(block, traced):
    """Herded perforation at other workgroup sizes, per-unit (traced) and
    dense kernels."""
    n, ipt = 40000, 20
    x = inputs.portfolio(n, 1024)
    y, tr, cnt = run("perfo", to_dev(x), 2, ipt, block_size=block, trace=traced, counters=traced, kind="small",
                     param=10, offset=0)
    yv, sv = oracle.region_values_f32out(x)
    ora = oracle.perfo(yv, sv, ipt, 0, 10, 0, out_init=np.full_like(yv, SENTINEL))
    skipped = ora["out"][0] == SENTINEL
    assert np.all(y[:, skipped] == SENTINEL)
    check_outputs(y, ora["out"], ora["scale"], mask=~skipped, what="perfo block %d" % block)
    if traced:
        gdec, _ = trace_dec(tr)
        assert np.array_equal(gdec, ora["dec"])
        assert cnt[0] == n and cnt[1] == int(skipped.sum())


DENSE_CASES = [
    ("small10", "small", 10, 0, 20, 65536),
    ("small2_off8", "small", 2, 8, 19, 551),
    ("small3_off1", "small", 3, 1, 7, 100003),
    ("large4_off3", "large", 4, 3, 9, 40000),
    ("large1", "large", 1, 0, 5, 3001),
    ("small1", "small", 1, 0, 5, 3001),
    ("ini30", "ini", 30, 0, 4, 10007),
    ("fini25", "fini", 25, 0, 4, 10007),
    ("fini100", "fini", 100, 0, 4, 999),
    # a period longer than the launch: most of the grid's positions fall past the last step
    ("small50_off7", "small", 50, 7, 20, 65536),
    # more periods than a grid dimension holds: the per-unit kernel runs instead
    ("large1_65536_steps", "large", 1, 0, 65536, 65536 * 64),
]


@pytest.mark.parametrize("case", DENSE_CASES, ids=[c[0] for c in DENSE_CASES])
def test_perfo_without_trace_matches_oracle(case):
    """Without trace or counters, perforation evaluates the kept items with
    one item per lane; the outputs must equal the herded pattern's."""
    name, kind, param, offset, ipt, n = case
    say("perfo dense", name)
    x = inputs.portfolio(n, 1024)
    y, _, _ = run("perfo", to_dev(x), 2, ipt, trace=False, counters=False, kind=kind, param=param, offset=offset)
    yv, sv = oracle.region_values_f32out(x)
    k = {"small": 0, "large": 1, "ini": 2, "fini": 3}[kind]
    ora = oracle.perfo(yv, sv, ipt, k, param, offset, out_init=np.full_like(yv, SENTINEL))
    skipped = ora["out"][0] == SENTINEL
    assert np.array_equal(y[:, skipped], ora["out"][:, skipped])
    check_outputs(y, ora["out"], ora["scale"], mask=~skipped, what="perfo dense " + name)
    # and bit for bit what the traced kernel writes
    yt, _, _ = run("perfo", to_dev(x), 2, ipt, kind=kind, param=param, offset=offset)
    assert np.array_equal(y, yt)


# --------------------------------------------------------------- collapse

@pytest.mark.parametrize("level", ["thread", "wave", "block"])
@pytest.mark.parametrize("ipt", [1, 7, 16])
def test_zero_threshold_reproduces_exact_bitwise(level, ipt):
    x = to_dev(inputs.periodic(20011, 8, jitter=1e-5))
    ye, _, _ = run("exact", x, 2, ipt)
    yi, ti, _ = run("iact", x, 2, ipt, table_size=8, threshold=0.0, level=level)
    yt, tt, _ = run("taf", x, 2, ipt, history_size=2, prediction_size=4, rsd_threshold=0.0, level=level)
    yp, tp, _ = run("perfo", x, 2, ipt, kind="small", param=0)
    for yy, tt_ in ((yi, ti), (yt, tt), (yp, tp)):
        assert np.array_equal(yy, ye)
        assert not hpac.trace_fields(tt_)["approx"].any()
    # the same inputs do approximate once the threshold is positive
    if ipt >= 7:
        _, t2, c2 = run("taf", x, 2, ipt, history_size=2, prediction_size=4, rsd_threshold=0.01, level=level)
        assert c2[1] > 0


def test_accurate_path_is_bitwise_exact_path():
    # where a technique computes, it writes exactly hpac_exact's value
    x = to_dev(inputs.periodic(65536, 8, jitter=1e-3))
    ye, _, _ = run("exact", x, 2, 16)
    yt, tr, _ = run("taf", x, 2, 16, history_size=4, prediction_size=4, rsd_threshold=0.007)
    f = hpac.trace_fields(tr)
    L = hpac.hpac_num_lanes(65536, 16)
    i = np.arange(65536)
    step = i // L
    wave = (i % L) // 64
    computed = ~f["approx"].reshape(-1, 16)[wave, step]
    assert computed.any() and (~computed).any()
    assert np.array_equal(yt[:, computed], ye[:, computed])


# ------------------------------------------------------------ determinism

def test_repeated_launches_are_bitwise_identical():
    x = to_dev(inputs.periodic(65536, 8, jitter=1e-3))
    runs = [run("iact", x, 2, 16, table_size=8, threshold=0.08) for _ in range(5)]
    runs += [run("taf", x, 2, 16, history_size=4, prediction_size=4, rsd_threshold=0.007) for _ in range(5)]
    for a, b in zip(runs[:4], runs[1:5]):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for a, b in zip(runs[5:9], runs[6:10]):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("technique,level,tpw", [("iact", "wave", 1), ("iact", "block", 1), ("iact", "wave", 4),
                                                  ("iact", "thread", 64), ("taf", "block", 1)])
def test_stale_lds_of_a_previous_launch_is_never_read(technique, level, tpw):
    """Tables and block tallies live in LDS, which a launch does not clear
    for the next.  A first launch on one repeated option fills every wave's
    tables with entries that would be hits for it (and leaves block tallies
    at a passing majority); a second launch on the same option must still
    start from empty tables and fresh windows: its first step computes
    everywhere, and its decisions and outputs are the oracle's."""
    x = inputs.constant(65536)
    xd = to_dev(x)
    kw = (dict(table_size=4, threshold=0.05, tables_per_wave=tpw, level=level) if technique == "iact"
          else dict(history_size=2, prediction_size=2, rsd_threshold=0.01, level=level))
    run(technique, xd, 2, 8, **kw)
    y, t, cnt = run(technique, xd, 2, 8, **kw)
    gdec, f = trace_dec(t)
    assert np.all(gdec.reshape(-1, 8)[:, 0] == 0), "a first step approximated"
    yv, sv = oracle.region_values_f32out(x)
    if technique == "iact":
        ora = oracle.iact(x, yv, sv, 8, 4, 0.05, tables_per_wave=tpw, group=group_of(level, 256))
    else:
        ora = oracle.taf(yv, sv, 8, 2, 2, 0.01, group=group_of(level, 256))
    odec = ora["dec"]
    if level == "thread":
        gdec = np.where(f["active"], f["napprox"], -1)
        odec = np.where(ora["dec"] >= 0, ora["napprox"], -1)
    assert np.array_equal(gdec, odec)
    check_outputs(y, ora["out"], ora["scale"], what="second launch")


# --------------------------------------------------- full size (2^24 items)

def test_full_size_config_against_oracle():
    """2^24 options sorted by spot (pool 65,536): exact and each technique
    at the launch configuration the benchmark times, against the oracle; the
    uncounted launches the benchmark times (dense perforation among them)
    write the counted launches' outputs bit for bit."""
    n = 1 << 24
    say("full-size inputs")
    x = inputs.portfolio(n, 65536, sort_by_spot=True)
    xd = to_dev(x)
    ref, scale = exact_ref(x)
    ye, _, c = run("exact", xd, 2, 1, trace=False)
    check_outputs(ye, ref, scale, what="exact 2^24")
    # the uncounted launch the benchmark times (one item per lane), every element
    yu, _, _ = run("exact", xd, 2, 1, trace=False, counters=False)
    check_outputs(yu, ref, scale, what="uncounted exact 2^24")
    assert np.array_equal(yu, ye)
    del ye, yu
    yv, sv = oracle.region_values_f32out(x)
    say("full-size iact")
    yi, ti, _ = run("iact", xd, 2, 16, table_size=8, threshold=0.05)
    ora = oracle.iact(x, yv, sv, 16, 8, 0.05)
    assert np.array_equal(trace_dec(ti)[0], ora["dec"])
    check_outputs(yi, ora["out"], ora["scale"], what="iact 2^24")
    # the uncounted launch the benchmark times writes the same outputs
    yu, _, _ = run("iact", xd, 2, 16, trace=False, counters=False, table_size=8, threshold=0.05)
    assert np.array_equal(yu, yi)
    del yi, yu, ora
    say("full-size taf")
    yt, tt, _ = run("taf", xd, 2, 16, history_size=4, prediction_size=4, rsd_threshold=0.01)
    replay_taf("2^24", yt, tt, gpu_exact_values(xd), sv, 16, 4, 4, 0.01, "wave", 256)
    ora = oracle.taf(yv, sv, 16, 4, 4, 0.01, band=taf_band(0.01))
    compare_decisions(trace_dec(tt)[0], ora["dec"], 16, ora["fragile"], lag=1)
    mg, mo = mape_pair(ref, yt, ora["out"])
    assert abs(mg - mo) <= 1e-4
    yu, _, _ = run("taf", xd, 2, 16, trace=False, counters=False, history_size=4, prediction_size=4,
                   rsd_threshold=0.01)
    assert np.array_equal(yu, yt)
    del yt, yu, ora
    say("full-size perfo")
    yp, tp, _ = run("perfo", xd, 2, 20, kind="small", param=10)
    ora = oracle.perfo(yv, sv, 20, 0, 10, 0, out_init=np.full_like(yv, SENTINEL))
    skipped = ora["out"][0] == SENTINEL
    assert abs(skipped.mean() - 0.1) < 1e-3
    check_outputs(yp, ora["out"], ora["scale"], mask=~skipped, what="perfo 2^24")
    assert np.all(yp[:, skipped] == SENTINEL)
    # the dense kernel the benchmark times: the same outputs, dropped items untouched
    yu, _, _ = run("perfo", xd, 2, 20, trace=False, counters=False, kind="small", param=10)
    assert np.array_equal(yu, yp)

"""GPU checks of the reduced-precision variants: half-precision columns with
the FP32 body, and the FP16 / BF16 bodies, against the FP64 oracle, with the
per-result error reported.

Bars:
 - FP32 body on half columns: the result equals the exact price at the
   half-rounded inputs, rounded to the column type: within 1e-5 of the scale
   plus one rounding of the output (2^-11 relative for FP16, 2^-8 for BF16);
 - FP16 / BF16 bodies: error relative to the scale |S N(d1)| + |K e^{-rT} N(d2)|
   (floored at 1e-4) of the rounded inputs below 5e-2 (FP16) and 1e-1 (BF16) for every result,
   the median below 2e-3 and 2e-2 (d1 divides ln(S/K) by v sqrt(T) >= 0.05, so one
   rounding of the logarithm moves d1 by up to 5e-4 * 4.6 / 0.05 = 0.05); the
   distribution is printed;
 - iACT on half columns: decisions bit-exact with the oracle on the
   half-rounded inputs.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, say, trace_dec
from paper_2308_16877_amd import hpac, inputs

pytestmark = pytest.mark.gpu

TYPES = {hpac.F32: torch.float32, hpac.F16: torch.float16, hpac.BF16: torch.bfloat16}
OUT_ULP = {hpac.F32: 0.0, hpac.F16: 2.0 ** -11, hpac.BF16: 2.0 ** -8}


def to_dev_typed(x, dtype):
    return [torch.from_numpy(c.astype(np.float32)).to(DEV).to(TYPES[dtype]) for c in x]


def rounded_inputs(x, dtype):
    return np.stack([torch.from_numpy(c.astype(np.float32)).to(TYPES[dtype]).to(torch.float64).numpy() for c in x])


def run_typed(fn, x, region, dtype, ipt=1, trace=False, **kw):
    xd = to_dev_typed(x, dtype)
    n = x.shape[1]
    outs = [torch.zeros(n, dtype=TYPES[dtype], device=DEV) for _ in range(2)]
    tr = torch.zeros(max(hpac.hpac_trace_entries(n, ipt), 1), dtype=torch.int32, device=DEV) if trace else None
    fn(xd, outs, region=region, items_per_lane=ipt, trace=tr, **kw)
    torch.cuda.synchronize()
    y = np.stack([o.to(torch.float64).cpu().numpy() for o in outs])
    return y, (tr.cpu().numpy().view(np.uint32) if trace else None)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available()
    hpac.lib()


@pytest.mark.parametrize("dtype", [hpac.F16, hpac.BF16])
def test_fp32_body_on_half_columns(dtype):
    x = inputs.portfolio(100003, 1024)
    y, _ = run_typed(hpac.hpac_exact, x, hpac.REGION_BS_PRICE, dtype, ipt=4)
    xr = rounded_inputs(x, dtype)
    C, P, sC, sP = oracle.bs_price(*xr)
    ref, scale = np.stack([C, P]), np.stack([sC, sP])
    tol = 1e-5 * scale + OUT_ULP[dtype] * np.abs(ref) + 1e-30
    if dtype == hpac.F16:
        tol += 2.0 ** -24  # FP16 subnormal spacing
    assert np.all(np.abs(y - ref) <= tol), float(np.max(np.abs(y - ref) / tol))


@pytest.mark.parametrize("region,dtype,bound,median", [
    (hpac.REGION_BS_PRICE_F16, hpac.F32, 5e-2, 2e-3),
    (hpac.REGION_BS_PRICE_F16, hpac.F16, 5e-2, 2e-3),
    (hpac.REGION_BS_PRICE_BF16, hpac.F32, 1e-1, 2e-2),
    (hpac.REGION_BS_PRICE_BF16, hpac.BF16, 1e-1, 2e-2),
])
def test_reduced_precision_bodies_error(region, dtype, bound, median):
    x = inputs.uniform_box(200000, seed=47).astype(np.float32)
    y, _ = run_typed(hpac.hpac_exact, x, region, dtype, ipt=2)
    # the body rounds its inputs to its own precision first
    body_t = hpac.F16 if region == hpac.REGION_BS_PRICE_F16 else hpac.BF16
    xr = rounded_inputs(x, body_t)
    C, P, sC, sP = oracle.bs_price(*xr)
    # relative to the scale, floored at 1e-4 price units (FP16's normal range
    # starts at 6.1e-5; below the floor both sides are zero or nearly so)
    err = np.abs(y - np.stack([C, P])) / np.maximum(np.stack([sC, sP]), 1e-4)
    q = np.quantile(err, [0.5, 0.99, 0.999, 1.0])
    say("region %d dtype %d: error/scale median %.2e p99 %.2e p99.9 %.2e max %.2e" % (region, dtype, *q))
    assert q[3] <= bound and q[0] <= median


@pytest.mark.parametrize("dtype", [hpac.F16, hpac.BF16])
def test_iact_on_half_columns(dtype):
    x = inputs.periodic(65536, 2, jitter=1e-3)
    ipt, t, theta = 16, 8, 0.05
    y, tr = run_typed(hpac.hpac_iact, x, hpac.REGION_BS_PRICE, dtype, ipt=ipt, trace=True, table_size=t,
                      threshold=theta)
    xr = rounded_inputs(x, dtype)
    C, P, sC, sP = oracle.bs_price(*xr)
    yv = np.stack([C, P]).astype(np.float32).astype(np.float64)
    ora = oracle.iact(xr.astype(np.float32), yv, np.stack([sC, sP]), ipt, t, theta)
    assert np.array_equal(trace_dec(tr)[0], ora["dec"])
    tol = 1e-5 * ora["scale"] + OUT_ULP[dtype] * np.abs(ora["out"]) + 1e-30 + (2.0 ** -24 if dtype == hpac.F16 else 0)
    assert np.all(np.abs(y - ora["out"]) <= tol)


@pytest.mark.parametrize("dtype", [hpac.F16, hpac.BF16])
def test_taf_and_perforation_on_half_columns(dtype):
    x = inputs.periodic(65536, 8, jitter=1e-4)
    xr = rounded_inputs(x, dtype)
    C, P, sC, sP = oracle.bs_price(*xr)
    yv = np.stack([C, P]).astype(np.float32).astype(np.float64)
    y, tr = run_typed(hpac.hpac_taf, x, hpac.REGION_BS_PRICE, dtype, ipt=16, trace=True, history_size=4,
                      prediction_size=4, rsd_threshold=0.01)
    ora = oracle.taf(yv, np.stack([sC, sP]), 16, 4, 4, 0.01)
    g, o = trace_dec(tr)[0], ora["dec"]
    assert (g == o).mean() >= 0.999  # decisions from outputs rounded to the column type
    yp, _ = run_typed(hpac.hpac_perfo, x, hpac.REGION_BS_PRICE, dtype, ipt=20, kind="small", param=5)
    orp = oracle.perfo(yv, np.stack([sC, sP]), 20, 0, 5, out_init=np.zeros_like(yv))
    kept = ~((np.arange(x.shape[1]) // oracle.num_lanes(x.shape[1], 20)) % 5 == 4)
    tol = 1e-5 * np.stack([sC, sP]) + OUT_ULP[dtype] * np.abs(yv) + 1e-30 + (2.0 ** -24 if dtype == hpac.F16 else 0)
    assert np.all(np.abs(yp - orp["out"])[:, kept] <= tol[:, kept])
    assert np.all(yp[:, ~kept] == 0)


@pytest.mark.parametrize("region,dtype", [(hpac.REGION_BS_PRICE_F16, hpac.F16), (hpac.REGION_BS_PRICE_BF16, hpac.BF16),
                                          (hpac.REGION_BS_PRICE, hpac.F16)])
@pytest.mark.parametrize("block", [64, 192])
def test_half_paths_do_not_depend_on_block_size(region, dtype, block):
    """The half-precision bodies and columns give the same bits at any
    workgroup size (checked against the oracle at 256 lanes above)."""
    x = inputs.portfolio(30001, 1024)
    y0, _ = run_typed(hpac.hpac_exact, x, region, dtype, ipt=2)
    y1, _ = run_typed(hpac.hpac_exact, x, region, dtype, ipt=2, block_size=block)
    assert np.array_equal(y1, y0)


def test_prepared_launch_keeps_its_columns_alive():
    """A prepared launch built from temporary tensors (here half-precision
    copies) must keep them alive: replaying it after the temporaries went out
    of scope and the allocator reused memory gives the same outputs."""
    n = 1 << 18
    x = inputs.portfolio(n, 1024)
    xd = [torch.from_numpy(c).to(DEV) for c in x]
    out = [torch.zeros(n, dtype=torch.float16, device=DEV) for _ in range(2)]
    prep = hpac.prepare("exact", [c.to(torch.float16) for c in xd], out, items_per_lane=1)
    prep()
    torch.cuda.synchronize()
    first = [o.clone() for o in out]
    junk = [torch.full((n,), float("nan"), dtype=torch.float16, device=DEV) for _ in range(16)]
    for o in out:
        o.zero_()
    prep()
    torch.cuda.synchronize()
    del junk
    assert all(torch.equal(a, b) for a, b in zip(first, out))


@pytest.mark.parametrize("dtype", [hpac.F32, hpac.F16])
def test_packed_fp16_pairs_equal_single_items(dtype):
    """With two or more items per lane and no trace or counters, the FP16
    body evaluates a lane's steps in pairs with packed FP16 arithmetic (an
    odd last step paired with itself); every element is rounded as in the
    single-item body, so the outputs are the same bit for bit (ragged n)."""
    x = inputs.portfolio(50001, 1024)
    xd = to_dev_typed(x, dtype)
    ys = {}
    for ipt in (1, 2, 3, 16):
        out = [torch.zeros(x.shape[1], dtype=TYPES[dtype], device=DEV) for _ in range(2)]
        hpac.hpac_exact(xd, out, items_per_lane=ipt, region=hpac.REGION_BS_PRICE_F16)
        torch.cuda.synchronize()
        ys[ipt] = np.stack([o.float().cpu().numpy() for o in out])
    for ipt in (2, 3, 16):
        assert np.array_equal(ys[ipt], ys[1]), ipt

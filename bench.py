#!/usr/bin/env python3
"""Benchmark of the approximated Black-Scholes region on one MI355X.

Workload: 2^24 European options (FP32 SoA columns S, K, T, r, v) drawn from a
pool of 65,536 tuples with 1e-3 relative jitter, sorted by spot.  One step
runs the whole hot path once over the batch: the exact region, iACT
(table 8, threshold 0.05), TAF (window 4, prediction 4, RSD 0.01) and small
perforation (M = 10, i.e. 10%), each one launch through the C ABI.  Inputs
rotate over three resident copies so the 256 MB last-level cache cannot
serve them between launches.

The last line printed is one JSON object of under 4 KB: the step's region
items/s (counting the items of the launches whose MAPE against the exact
kernel meets the 0.5% bar), per-technique time, speedup and MAPE, the
roofline of the dominant kernel (HIP-event durations on the launch stream,
beside the committed rocprofv3 average of the same kernel code), the CPU
oracle timed on a bounded sample, and one or two figures from each further
leg.  The legs themselves are written to --legs-out: the 65,536-option
configuration, the technique-parameter grid and TAF prediction sizes on the
2^24 options, the structured-locality variants, the Greeks adjoint, the
reduced-precision variants, the decision hierarchy and items-per-lane
study, the Binomial Options workload, the MLP surrogate and the Sedov hydro
under TAF and perforation.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MAPE_TAU = 1e-2
MAPE_BAR = 0.005

TECHS = {
    # name: (entry point, items per lane, parameters)
    "exact": ("exact", 1, {}),
    "iact": ("iact", 16, dict(table_size=8, threshold=0.05, tables_per_wave=1, level="wave")),
    "taf": ("taf", 16, dict(history_size=4, prediction_size=4, rsd_threshold=0.01, level="wave")),
    "perfo": ("perfo", 20, dict(kind="small", param=10, offset=0)),
}
KERNEL_NAMES = {"exact": "k_exact", "iact": "k_iact", "taf": "k_taf_wave", "perfo": "k_perfo_dense"}
# the timed region records each launch's events on one step in EVENT_EVERY
EVENT_EVERY = 4
# VALU issue peak: 256 CUs x 4 SIMDs x 32 FP32 lanes per clock x 2.4 GHz = 78.6
# tera lane-instructions per second (157.3 TFLOP/s in FMAs).  A wave64 FP32
# instruction whose operands are all vector registers or constants issues in
# two clocks; one with a scalar-register operand takes four (the probe
# measures both).  Packed FP32 is disabled at build time.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    # the part runs below its working clocks for the first tens of ms of work
    # after idling: 100 warm-up steps are about 40 ms, 200 timed ones 75 ms
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--n", type=int, default=1 << 24)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-structured", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=1 << 24)
    p.add_argument("--legs-out", default=os.path.join("results", "bench_legs.json"),
                   help="file for the full results of every leg (the printed line summarises them)")
    p.add_argument("--pmc-probe", action="store_true",
                   help="only launch each kernel of the step three times plus a 256 MiB copy probe, untimed, "
                        "for hardware-counter runs")
    return p.parse_args()


COPY_PROBE_BYTES = 256 << 20
# the structured-locality variants: (name, pool period)
STRUCTURED = (("lane_periodic_1024", 1024), ("wave_periodic_2", 2))


def pmc_probe(torch, hpac, x_copies, n):
    """Launches for a counter run: each technique 3 times on rotating inputs,
    then the plain copy kernel 3 times over COPY_PROBE_BYTES (its counter
    readings calibrate the byte counters)."""
    dev = x_copies[0][0].device
    outs = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
    for r in range(3):
        for t in TECHS:
            launch(hpac, t, x_copies[r % len(x_copies)], outs)
    # the same launches on the two structured-locality variants, in turn
    # (dispatches 3..5 and 6..8 of each technique kernel)
    from paper_2308_16877_amd import inputs
    for _, period in STRUCTURED:
        xs = [torch.from_numpy(c).to(dev) for c in inputs.periodic(n, period, jitter=1e-3)]
        for r in range(3):
            for t in TECHS:
                launch(hpac, t, xs, outs)
        del xs
    src = torch.zeros(COPY_PROBE_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for r in range(3):
        hpac.hpac_probe_copy(src, dst, COPY_PROBE_BYTES)
    torch.cuda.synchronize()
    # the surrogate's inference (initial weights: the work does not depend on them)
    from paper_2308_16877_amd import surrogate
    from paper_2308_16877_amd.hydro import Hydro
    s = surrogate.Surrogate(surrogate.init_params(), surrogate.box_norm([torch.tensor([0.0, 1.0])] * 2))
    for r in range(3):
        s(x_copies[r % len(x_copies)], outs)
    # three exact steps of the 90^3 blast
    h = Hydro(90)
    h.run(3)
    del h
    # the Binomial Options techniques on the structured variant of their leg
    n_bo = 65536
    xb = [torch.from_numpy(c).to(dev) for c in inputs.periodic(n_bo, hpac.hpac_bo_units(n_bo, 16), jitter=1e-3)]
    ob = [torch.zeros(n_bo, dtype=torch.float32, device=dev) for _ in range(2)]
    for r in range(3):
        for fn, ipt, params in BO_TECHS.values():
            f = {"exact": hpac.hpac_bo_exact, "iact": hpac.hpac_bo_iact, "taf": hpac.hpac_bo_taf,
                 "perfo": hpac.hpac_bo_perfo}[fn]
            f(xb, ob, 512, items_per_lane=ipt, **params)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": "done", "n": n, "copy_bytes": COPY_PROBE_BYTES}), flush=True)


def launch(hpac, name, x, outs, block=256, **extra):
    fn, ipt, params = TECHS[name]
    f = {"exact": hpac.hpac_exact, "iact": hpac.hpac_iact, "taf": hpac.hpac_taf, "perfo": hpac.hpac_perfo}[fn]
    f(x, outs, items_per_lane=ipt, block_size=block, **params, **extra)


def mape_torch(torch, exact, approx):
    e = torch.stack(exact).double()
    a = torch.stack(approx).double()
    return float(((e - a).abs() / e.abs().clamp_min(MAPE_TAU)).mean())


def committed_profile(kind, kernel, workload):
    """A committed rocprofv3 counter summary (profiles/<kind>_<kernel>_<workload>.json)
    or None when absent or taken on other kernel code."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s.json" % (kind, kernel, workload))
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    from paper_2308_16877_amd.profiling import kernel_source_sha
    if d.get("kernel_source_sha") != kernel_source_sha(kernel):
        return None
    return d


def valu_ceiling(torch, hpac, workgroups=2048, iters=1024):
    """Measured FP32 FMA issue rate (tera lane-instructions/s) of the probe
    kernel with vector-register and with scalar-register operands."""
    out = torch.empty(workgroups * 256, dtype=torch.float32, device="cuda:0")
    res = {}
    for name, scalar in (("vector_operands", 0), ("scalar_operand", 1)):
        ms = time_pairs(torch, {"p": [lambda s=scalar: hpac.hpac_probe_valu(out, workgroups, iters, s)]}, 3, 1)["p"]
        res[name] = workgroups * 256 * iters * 64 / (ms * 1e-3) / 1e12
    return res


def skipped_work_counters():
    """Work each technique kernel skips, from the committed counter summaries
    of the counter probe (rocprofv3 --pmc on the same 2^24 options): per
    workload, 1 - issued VALU / the exact kernel's and 1 - HBM bytes / the
    exact kernel's, per launch.  None where a summary is missing or stale."""
    out = {}
    for workload in ["bs2p24_sorted"] + ["bs2p24_" + v for v, _ in STRUCTURED]:
        base_v = committed_profile("valu", KERNEL_NAMES["exact"], workload)
        base_t = committed_profile("traffic", KERNEL_NAMES["exact"], workload)
        row = {}
        for t, kernel in KERNEL_NAMES.items():
            if t == "exact":
                continue
            v = committed_profile("valu", kernel, workload)
            tr = committed_profile("traffic", kernel, workload)
            row[t] = {
                "valu_skipped_frac": (1 - v["lane_instructions_per_dispatch"] / base_v["lane_instructions_per_dispatch"])
                if v and base_v else None,
                "hbm_bytes_saved_frac": (1 - tr["hbm_bytes_per_launch"] / base_t["hbm_bytes_per_launch"])
                if tr and base_t else None}
        out[workload] = row
    return out


def measured_traffic(kernel, workload, launches_bytes):
    """HBM bytes per launch from the committed counter summary, or None."""
    d = committed_profile("traffic", kernel, workload)
    return d.get("hbm_bytes_per_launch") if d else None


def run_workload(torch, hpac, x_copies, n, steps, warmup, with_stats=True, min_warm_s=0.0):
    """Time `steps` steps after at least `warmup` untimed ones, and after at
    least min_warm_s seconds of warm-up work (the part runs below its
    working clocks for the first tens of ms of work after idling)."""
    dev = x_copies[0][0].device
    outs = {t: [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)] for t in TECHS}
    stream = torch.cuda.current_stream()
    names = list(TECHS)
    # argument marshalling done once per (technique, input copy)
    prep = {t: [hpac.prepare(TECHS[t][0], xs, outs[t], items_per_lane=TECHS[t][1], block_size=256,
                             stream=stream, **TECHS[t][2]) for xs in x_copies] for t in names}
    # launch j of step s reads copy (s + j) mod 3: consecutive launches never
    # read the same copy, and a copy was last read three launches earlier
    nc = len(x_copies)
    w, tw = 0, time.perf_counter()
    while w < warmup or time.perf_counter() - tw < min_warm_s:
        for j, t in enumerate(names):
            prep[t][(w + j) % nc]()
        w += 1
        if w >= warmup:
            torch.cuda.synchronize()  # host time then follows the GPU's
    torch.cuda.synchronize()
    # per-kernel events on every EVENT_EVERY-th step of the timed region only:
    # an event between two launches costs the step a few microseconds
    timed = [s for s in range(steps) if s % EVENT_EVERY == 0]
    ev = {s: [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for s in timed}
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for s in range(steps):
        e = ev.get(s)
        if e:
            e[0].record(stream)
        for j, t in enumerate(names):
            prep[t][(s + j) % nc]()
            if e:
                e[j + 1].record(stream)
    stop.record(stream)
    host_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(stop)
    per = {t: [ev[s][j].elapsed_time(ev[s][j + 1]) for s in timed] for j, t in enumerate(names)}
    res = {"total_ms": total_ms, "wall_s": wall, "host_enqueue_s": host_s, "warmup_steps_run": w,
           "per_kernel_ms": {t: sum(v) / len(v) for t, v in per.items()},
           "per_kernel_median_ms": {t: sorted(v)[len(v) // 2] for t, v in per.items()},
           "per_kernel_min_ms": {t: min(v) for t, v in per.items()}}
    if with_stats:
        # one untimed launch per technique with counters on the same inputs
        stats = {}
        xs = x_copies[0]
        exact_out = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
        launch(hpac, "exact", xs, exact_out)
        for t in names:
            o = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
            cnt = torch.zeros(hpac.NUM_COUNTERS, dtype=torch.int64, device=dev)
            launch(hpac, t, xs, o, counters=cnt)
            torch.cuda.synchronize()
            c = cnt.cpu().tolist()
            stats[t] = {"approx_frac": c[1] / max(c[0], 1), "mape": mape_torch(torch, exact_out, o),
                        "approx_wave_step_frac": c[2] / max(c[3], 1)}
        res["stats"] = stats
    return res


def algorithmic_bytes(tech, n, approx_frac):
    """Compulsory HBM bytes of one launch: 20 B of inputs per evaluated item,
    8 B of outputs per written item."""
    if tech in ("exact", "iact"):
        return 28.0 * n
    if tech == "taf":
        return 8.0 * n + 20.0 * n * (1.0 - approx_frac)
    if tech == "perfo":
        return 28.0 * n * (1.0 - approx_frac)
    raise KeyError(tech)


def summarize(res, n):
    ex = res["per_kernel_ms"]["exact"]
    out = {}
    for t, ms in res["per_kernel_ms"].items():
        st = res["stats"][t]
        out[t] = {"ms": round(ms, 5), "ms_median": round(res["per_kernel_median_ms"][t], 5),
                  "items_per_s": n / (ms * 1e-3), "speedup_vs_exact": ex / ms,
                  "mape": st["mape"], "approx_frac": st["approx_frac"],
                  "items_per_lane": TECHS[t][1], "params": TECHS[t][2]}
    return out


def time_pairs(torch, legs, steps, warmup):
    """Average HIP-event time (ms) of each named sequence of launches."""
    stream = torch.cuda.current_stream()
    out = {}
    for name, fns in legs.items():
        for _ in range(warmup):
            for f in fns:
                f()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            for f in fns:
                f()
        b.record(stream)
        torch.cuda.synchronize()
        out[name] = a.elapsed_time(b) / steps
    return out


def greeks_leg(torch, hpac, x_dev, n, steps):
    """Call Greeks (upstream (1, 0)) for 2^24 options: exact forward + the
    recomputing adjoint, against iACT (table 16, threshold 0.05) memoizing
    (price, gradient) by reference (the price-and-source region + the
    backward recomputing at each source item) and by value (the
    price-and-Jacobian region + the saved-Jacobian VJP); on the benchmark's
    options and on the wave-periodic variant, where iACT finds reuse."""
    from paper_2308_16877_amd import inputs
    res = greeks_point(torch, hpac, x_dev, n, steps)
    xs = [torch.from_numpy(c).to(x_dev[0].device) for c in inputs.periodic(n, 2, jitter=1e-3)]
    res["wave_periodic_2"] = greeks_point(torch, hpac, xs, n, steps)
    res["wave_periodic_2"]["workload"] = "the same on item i = pool tuple i mod 2, 1e-3 jitter (structured-locality variant)"
    return res


def greeks_point(torch, hpac, x_dev, n, steps):
    dev = x_dev[0].device
    f32 = dict(dtype=torch.float32, device=dev)
    ones = torch.ones(n, **f32)
    price = [torch.zeros(n, **f32) for _ in range(2)]
    grads_exact = [torch.zeros(n, **f32) for _ in range(5)]
    grads_ref = [torch.zeros(n, **f32) for _ in range(5)]
    grads_jac = [torch.zeros(n, **f32) for _ in range(5)]
    full = [torch.zeros(n, **f32) for _ in range(12)]
    ref_out = [torch.zeros(n, **f32) for _ in range(2)] + [torch.zeros(n, dtype=torch.int32, device=dev)]
    stream = torch.cuda.current_stream()
    fwd_exact = hpac.prepare("exact", x_dev, price, items_per_lane=1, block_size=256, stream=stream)
    fwd_ref = hpac.prepare("iact", x_dev, ref_out, items_per_lane=16, block_size=256, stream=stream,
                           region=hpac.REGION_BS_PRICE_REF, table_size=16, threshold=0.05)
    fwd_jac = hpac.prepare("iact", x_dev, full, items_per_lane=16, block_size=256, stream=stream,
                           region=hpac.REGION_BS_PRICE_GRAD, table_size=16, threshold=0.05)
    legs = {
        "exact_fwd_adjoint": [fwd_exact, lambda: hpac.hpac_bs_adjoint(x_dev, ones, None, grads_exact)],
        "iact_ref_fwd_vjp": [fwd_ref, lambda: hpac.hpac_bs_vjp_ref(x_dev, ref_out[2], ones, None, grads_ref)],
        "iact_jacobian_fwd_vjp": [fwd_jac, lambda: hpac.hpac_bs_vjp(full[2:], ones, None, grads_jac)],
    }
    t = time_pairs(torch, legs, steps, 2)
    cnt = torch.zeros(hpac.NUM_COUNTERS, dtype=torch.int64, device=dev)
    hpac.hpac_iact(x_dev, ref_out, 16, 0.05, items_per_lane=16, region=hpac.REGION_BS_PRICE_REF, counters=cnt)
    hpac.hpac_bs_vjp_ref(x_dev, ref_out[2], ones, None, grads_ref)
    torch.cuda.synchronize()
    c = cnt.cpu().tolist()
    return {"workload": "call Greeks (delta, dC/dK, theta, rho, vega) of the benchmark's 2^24 options",
            "exact_fwd_adjoint_ms": t["exact_fwd_adjoint"], "iact_fwd_vjp_ms": t["iact_ref_fwd_vjp"],
            "iact_jacobian_fwd_vjp_ms": t["iact_jacobian_fwd_vjp"],
            "exact_items_per_s": n / (t["exact_fwd_adjoint"] * 1e-3),
            "iact_items_per_s": n / (t["iact_ref_fwd_vjp"] * 1e-3),
            "iact_speedup_vs_exact": t["exact_fwd_adjoint"] / t["iact_ref_fwd_vjp"],
            "iact_jacobian_speedup_vs_exact": t["exact_fwd_adjoint"] / t["iact_jacobian_fwd_vjp"],
            "iact_approx_frac": c[1] / max(c[0], 1),
            "iact_gradient_mape_vs_exact": mape_torch(torch, grads_exact, grads_ref),
            "memo_forms_bitwise_equal": all(bool(torch.equal(a, b)) for a, b in zip(grads_ref, grads_jac))}


def precision_leg(torch, hpac, x_dev, n, steps):
    """The exact region on the benchmark's 2^24 options with half-precision
    columns (10 B in + 4 B out per item) and with the FP16 / BF16 bodies:
    items/s and the error of each result against the FP32 exact kernel,
    relative to max(|price|, tau)."""
    stream = torch.cuda.current_stream()
    ref = [torch.zeros(n, dtype=torch.float32, device=x_dev[0].device) for _ in range(2)]
    hpac.hpac_exact(x_dev, ref, items_per_lane=1)
    variants = {
        # name: (region, column type, items per lane; 2 pairs the FP16 body's items in packed FP16)
        "fp32_body_fp32_columns": (hpac.REGION_BS_PRICE, torch.float32, 1),
        "fp32_body_fp16_columns": (hpac.REGION_BS_PRICE, torch.float16, 1),
        "fp32_body_bf16_columns": (hpac.REGION_BS_PRICE, torch.bfloat16, 1),
        "fp16_body_fp16_columns": (hpac.REGION_BS_PRICE_F16, torch.float16, 1),
        "fp16_body_fp16_columns_packed": (hpac.REGION_BS_PRICE_F16, torch.float16, 2),
        "bf16_body_bf16_columns": (hpac.REGION_BS_PRICE_BF16, torch.bfloat16, 1),
        "fp16_body_fp32_columns": (hpac.REGION_BS_PRICE_F16, torch.float32, 1),
        "fp16_body_fp32_columns_packed": (hpac.REGION_BS_PRICE_F16, torch.float32, 2),
    }
    legs, outs = {}, {}
    for name, (region, dt, ipt) in variants.items():
        xs = [c.to(dt) for c in x_dev]
        o = [torch.zeros(n, dtype=dt, device=x_dev[0].device) for _ in range(2)]
        outs[name] = o
        legs[name] = [hpac.prepare("exact", xs, o, items_per_lane=ipt, block_size=256, stream=stream, region=region)]
    t = time_pairs(torch, legs, steps, 2)
    res = {}
    for name in variants:
        e = torch.stack(ref).double()
        a = torch.stack([c.double() for c in outs[name]])
        rel = (e - a).abs() / e.abs().clamp_min(MAPE_TAU)
        res[name] = {"ms": t[name], "items_per_s": n / (t[name] * 1e-3),
                     "speedup_vs_fp32": t["fp32_body_fp32_columns"] / t[name],
                     "mape_vs_fp32": float(rel.mean()), "max_rel_err_vs_fp32": float(rel.max())}
    return res


def surrogate_leg(torch, hpac, n):
    """The MLP surrogate: trained on 2^20 exact-labelled samples of the box
    by the library's gradient and Adam kernels, then BF16-MFMA inference on
    2^24 uniform box options with 5% moved outside the box (exact fallback).
    Error and speed against the exact kernel on the same inputs."""
    import numpy as np
    from paper_2308_16877_amd import inputs, surrogate
    dev = "cuda:0"
    t0 = time.perf_counter()
    xs, ys = surrogate.make_training_set(1 << 20)
    s, hist = surrogate.train(xs, ys)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    x0 = inputs.uniform_box(n, seed=inputs.SEED_DRAW).astype(np.float32)
    x, moved = inputs.with_out_of_box(x0, 0.05)
    xd = [torch.from_numpy(np.ascontiguousarray(c)).to(dev) for c in x]
    out = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
    ref = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
    stream = torch.cuda.current_stream()
    exact = hpac.prepare("exact", xd, ref, items_per_lane=1, block_size=256, stream=stream)
    t = time_pairs(torch, {"exact": [exact], "surrogate": [lambda: s(xd, out)]}, 10, 2)
    e = torch.stack(ref).double()
    a = torch.stack(out).double()
    return {"workload": "2^24 uniform options of the training box, 5%% moved outside it (%d to the exact "
                        "fallback)" % len(moved),
            "train_samples": 1 << 20, "train_s": round(train_s, 2), "final_loss": hist[-1],
            "surrogate_ms": t["surrogate"], "exact_ms": t["exact"],
            "items_per_s": n / (t["surrogate"] * 1e-3), "speedup_vs_exact": t["exact"] / t["surrogate"],
            "rel_l2_vs_exact": float((a - e).norm() / e.norm()), "mape_vs_exact": mape_torch(torch, ref, out),
            "fallback_count": int(s.count.item())}


def technique_point(torch, hpac, x_copies, n, fn, ipt, params, exact_out, steps=6):
    """Time one technique configuration (HIP events, rotating input copies)
    and measure its approximated fraction and MAPE against exact_out."""
    dev = x_copies[0][0].device
    out = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
    stream = torch.cuda.current_stream()
    params = dict(params)
    block = params.pop("block_size", 256)
    preps = [hpac.prepare(fn, xs, out, items_per_lane=ipt, block_size=block, stream=stream, **params)
             for xs in x_copies]
    t = time_pairs(torch, {"p": preps}, steps, 1)["p"] / len(preps)
    cnt = torch.zeros(hpac.NUM_COUNTERS, dtype=torch.int64, device=dev)
    {"exact": hpac.hpac_exact, "iact": hpac.hpac_iact, "taf": hpac.hpac_taf, "perfo": hpac.hpac_perfo}[fn](
        x_copies[0], out, items_per_lane=ipt, block_size=block, counters=cnt, **params)
    torch.cuda.synchronize()
    c = cnt.cpu().tolist()
    return {"ms": t, "approx_frac": c[1] / max(c[0], 1), "mape": mape_torch(torch, exact_out, out)}


SWEEP = {
    # technique: (items per lane, parameter grid)
    "iact": (16, [dict(table_size=t, threshold=th, tables_per_wave=1, level="wave")
                  for t in (4, 8, 16, 32) for th in (0.01, 0.05, 0.1)]),
    "taf": (16, [dict(history_size=h, prediction_size=h, rsd_threshold=th, level="wave")
                 for h in (2, 4, 8) for th in (0.001, 0.01, 0.1)]),
    "perfo": (20, [dict(kind="small", param=m, offset=0) for m in (10, 5, 2)]),
}


def sweep_leg(torch, hpac, x_copies, n):
    """The parameter grid of the 2^24-option workload: iACT tables
    {4, 8, 16, 32} x thresholds {0.01, 0.05, 0.1}, TAF windows {2, 4, 8} x RSD
    {0.001, 0.01, 0.1} (prediction size = window), small perforation at 10,
    20 and 50% (M = 10, 5, 2).  Per point: ms per launch, speedup over the
    exact kernel, approximated fraction and MAPE; and the fastest point within
    the 0.5% MAPE bar."""
    dev = x_copies[0][0].device
    ex = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
    hpac.hpac_exact(x_copies[0], ex, items_per_lane=1)
    # the exact kernel's launch shapes; speedups are against the fastest
    exact = {}
    for ipt in (1, 2, 4, 8, 16):
        for block in (128, 256):
            exact["ipt%d_block%d" % (ipt, block)] = technique_point(torch, hpac, x_copies, n, "exact", ipt,
                                                                    dict(block_size=block), ex)["ms"]
    best_exact = min(exact, key=exact.get)
    exact_ms = exact[best_exact]
    points = []
    grid = [(tech, ipt, params) for tech, (ipt, g) in SWEEP.items() for params in g]
    # items per lane of the memoization techniques at their headline parameters
    grid += [(tech, ipt, dict(TECHS[tech][2])) for tech in ("iact", "taf") for ipt in (4, 64, 256)]
    for tech, ipt, params in grid:
        r = technique_point(torch, hpac, x_copies, n, tech, ipt, params, ex)
        r.update(technique=tech, items_per_lane=ipt, params=params, speedup_vs_exact=exact_ms / r["ms"])
        points.append(r)
    ok = [p for p in points if p["mape"] <= MAPE_BAR]
    best = max(ok, key=lambda p: p["speedup_vs_exact"]) if ok else None
    return {"exact_ms_by_shape": exact, "best_exact": best_exact, "exact_ms": exact_ms, "points": points,
            "best_at_mape_0.005": best}


def hierarchy_and_ipt_leg(torch, hpac, n):
    """The decision hierarchy (thread, wave, block) and the items-per-lane
    trade-off of the paper's insights, on the structured variants where the
    techniques find reuse: TAF on the lane-periodic inputs, iACT on the
    wave-periodic ones.  Times are per launch over 2^24 items; speedups are
    against the exact kernel on the same inputs."""
    import numpy as np  # noqa: F401
    from paper_2308_16877_amd import inputs
    dev = "cuda:0"
    res = {}
    for vname, period, tech, params in (
            ("lane_periodic_1024", 1024, "taf", dict(history_size=4, prediction_size=4, rsd_threshold=0.01)),
            ("wave_periodic_2", 2, "iact", dict(table_size=8, threshold=0.05, tables_per_wave=1))):
        xs = inputs.periodic(n, period, jitter=1e-3)
        copies = [[torch.from_numpy(c).to(dev) for c in xs] for _ in range(3)]
        ex = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
        hpac.hpac_exact(copies[0], ex, items_per_lane=1)
        exact_ms = technique_point(torch, hpac, copies, n, "exact", 1, {}, ex)["ms"]
        levels = {}
        for level in ("thread", "wave", "block"):
            r = technique_point(torch, hpac, copies, n, tech, 16, dict(params, level=level), ex)
            r["speedup_vs_exact"] = exact_ms / r["ms"]
            levels[level] = r
        ipts = {}
        for ipt in (1, 2, 4, 8, 16, 32, 64):
            r = technique_point(torch, hpac, copies, n, tech, ipt, dict(params, level="wave"), ex)
            r["speedup_vs_exact"] = exact_ms / r["ms"]
            ipts[str(ipt)] = r
        res[tech] = {"variant": vname, "params": params, "exact_ms": exact_ms, "levels_at_ipt16": levels,
                     "items_per_lane_at_wave_level": ipts}
        del copies
    # tables per wave (the paper's tables per warp): lane l sees pool tuple
    # l mod 64 at every step, so a wave meets 64 tuples -- more than one
    # 8-entry table holds -- while each lane alone meets one
    xs = inputs.periodic(n, 64, jitter=1e-3)
    copies = [[torch.from_numpy(c).to(dev) for c in xs] for _ in range(3)]
    ex = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
    hpac.hpac_exact(copies[0], ex, items_per_lane=1)
    exact_ms = technique_point(torch, hpac, copies, n, "exact", 1, {}, ex)["ms"]
    tables = {}
    for tpw in (1, 2, 4, 8, 16, 32, 64):
        r = technique_point(torch, hpac, copies, n, "iact", 16,
                            dict(table_size=8, threshold=0.05, tables_per_wave=tpw, level="wave"), ex)
        r["speedup_vs_exact"] = exact_ms / r["ms"]
        tables[str(tpw)] = r
    # one table per lane fills a 256-lane workgroup's 64 KiB of LDS (two per
    # CU, 8 waves); 64-lane workgroups take 16 KiB (ten per CU, 10 waves)
    r = technique_point(torch, hpac, copies, n, "iact", 16,
                        dict(table_size=8, threshold=0.05, tables_per_wave=64, level="wave", block_size=64), ex)
    r["speedup_vs_exact"] = exact_ms / r["ms"]
    tables["64_block64"] = r
    res["iact_tables_per_wave"] = {"variant": "lane_periodic_64", "params": dict(table_size=8, threshold=0.05),
                                   "items_per_lane": 16, "exact_ms": exact_ms, "tables_per_wave": tables}
    del copies
    return res


BO_TECHS = {
    # name: (entry point, options per unit, parameters)
    "exact": ("exact", 1, {}),
    "iact": ("iact", 16, dict(table_size=8, threshold=0.05)),
    "taf": ("taf", 8, dict(history_size=4, prediction_size=4, rsd_threshold=0.01)),
    "perfo": ("perfo", 10, dict(kind="small", param=10)),
}


def binomial_leg(torch, hpac, n=65536, steps=512):
    """American call and put on a 512-step tree for 65,536 options, one
    wavefront per option: the portfolio workload (pool of 1,024 tuples, 1e-3
    jitter) and a structured variant in which every unit (wavefront) of the
    16-options-per-unit techniques sees one tuple at every option.  Per technique: ms, options/s, speedup over the
    exact tree, approximated fraction and MAPE against the exact tree."""
    from paper_2308_16877_amd import inputs
    dev = "cuda:0"
    res = {}
    units = hpac.hpac_bo_units(n, 16)
    for vname, x in (("portfolio_pool1024", inputs.portfolio(n, 1024)),
                     ("unit_periodic", inputs.periodic(n, units, jitter=1e-3))):
        xd = [torch.from_numpy(c).to(dev) for c in x]
        ex = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
        hpac.hpac_bo_exact(xd, ex, steps, items_per_lane=1)
        out = {}
        for name, (fn, ipt, params) in BO_TECHS.items():
            f = {"exact": hpac.hpac_bo_exact, "iact": hpac.hpac_bo_iact, "taf": hpac.hpac_bo_taf,
                 "perfo": hpac.hpac_bo_perfo}[fn]
            o = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
            call = (lambda f=f, o=o, ipt=ipt, params=params: f(xd, o, steps, items_per_lane=ipt, **params))
            ms = time_pairs(torch, {"t": [call]}, 3, 1)["t"]
            cnt = torch.zeros(hpac.NUM_COUNTERS, dtype=torch.int64, device=dev)
            f(xd, o, steps, items_per_lane=ipt, counters=cnt, **params)
            torch.cuda.synchronize()
            c = cnt.cpu().tolist()
            out[name] = {"ms": ms, "options_per_s": n / (ms * 1e-3), "approx_frac": c[1] / max(c[0], 1),
                         "mape_vs_exact": mape_torch(torch, ex, o), "items_per_lane": ipt, "params": params}
        for name in out:
            out[name]["speedup_vs_exact"] = out["exact"]["ms"] / out[name]["ms"]
        res[vname] = out
    # options per unit: more options give the memo more reuse but fewer
    # wavefronts (65,536 / IPT) to fill 1,024 SIMDs; each IPT on inputs in
    # which every unit sees one tuple
    study = {}
    for ipt in (4, 8, 16, 32):
        x = inputs.periodic(n, hpac.hpac_bo_units(n, ipt), jitter=1e-3)
        xd = [torch.from_numpy(c).to(dev) for c in x]
        ex = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
        e_ms = time_pairs(torch, {"t": [lambda: hpac.hpac_bo_exact(xd, ex, steps, items_per_lane=1)]}, 3, 1)["t"]
        row = {"exact_ms": e_ms}
        for name in ("iact", "taf"):
            fn, _, params = BO_TECHS[name]
            f = {"iact": hpac.hpac_bo_iact, "taf": hpac.hpac_bo_taf}[fn]
            o = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
            ms = time_pairs(torch, {"t": [lambda f=f, o=o: f(xd, o, steps, items_per_lane=ipt, **params)]}, 3, 1)["t"]
            cnt = torch.zeros(hpac.NUM_COUNTERS, dtype=torch.int64, device=dev)
            f(xd, o, steps, items_per_lane=ipt, counters=cnt, **params)
            torch.cuda.synchronize()
            c = cnt.cpu().tolist()
            row[name] = {"ms": ms, "speedup_vs_exact": e_ms / ms, "approx_frac": c[1] / max(c[0], 1),
                         "mape_vs_exact": mape_torch(torch, ex, o)}
        study[str(ipt)] = row
    return {"workload": "American call+put, %d-step CRR tree, %d options, one wavefront per option" % (steps, n),
            "variants": res, "unit_periodic_items_per_unit": study}


HYDRO_TECHS = {
    # name: hydro technique arguments (the TAF grid is in HYDRO_SWEEP); the
    # FP64 oracle's run of each is stored under the same name
    "exact": {},
    "eos_taf_thread_h4_p2_0.001": dict(eos=(4, 2, 0.001, "thread")),
    "eos_taf_wave_h4_p4_0.01": dict(eos=(4, 4, 0.01, "wave")),
    "hg_perfo_small_M2_ipt2": dict(perfo=("small", 2, 2)),
    "hg_perfo_small_M10": dict(perfo=("small", 10, 1)),
    "hg_perfo_fini_20": dict(perfo=("fini", 20, 1)),
    "hg_perfo_ini_20": dict(perfo=("ini", 20, 1)),
}


def hydro_leg(torch, n=90, steps=500):
    """The Sedov blast on n^3 elements for `steps` timesteps, exact and under
    each hydro technique: ms per step, speedup, and the error of the origin
    energy (the quantity of interest) against the exact GPU run and against
    the FP64 oracle's stored run of the same configuration."""
    from paper_2308_16877_amd.hydro import Hydro, Tech
    golden = os.path.join(ROOT, "tests", "golden", "hydro_sedov90_qoi.json")
    ref64, tech64 = None, {}
    if n == 90 and steps == 500 and os.path.exists(golden):
        with open(golden) as f:
            g = json.load(f)
        ref64 = g["records"][-1]["origin_energy"]
        tech64 = {k: v["records"][-1]["origin_energy"] for k, v in g.get("techniques", {}).items()}
    res = {}
    base = None
    for name, kw in HYDRO_TECHS.items():
        h = Hydro(n, tech=Tech(**kw))
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        h.run(steps)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        q = h.origin_energy()
        if base is None:
            base = (ms, q)
        ie, ke = h.energy()
        q64 = tech64.get(name)
        res[name] = {"ms_per_step": ms / steps, "element_steps_per_s": n ** 3 * steps / (ms * 1e-3),
                     "speedup_vs_exact": base[0] / ms, "origin_energy": q,
                     "qoi_err_vs_exact_gpu": abs(q / base[1] - 1),
                     "qoi_err_vs_fp64_oracle": abs(q / ref64 - 1) if ref64 else None,
                     # the technique's own QoI error in the FP64 oracle (its run against the oracle's exact run)
                     "oracle_qoi_err_vs_oracle_exact": abs(q64 / ref64 - 1) if q64 is not None and ref64 else None,
                     "total_energy": ie + ke, "time": h.time()}
        del h
    sweep = hydro_sweep(torch, res["exact"]["ms_per_step"], res["exact"]["origin_energy"], ref64, n, steps)
    return {"workload": "Sedov blast, %d^3 elements, %d steps, FP32 state, FP64 dt" % (n, steps),
            "fp64_oracle_origin_energy": ref64, "techniques": res, "sweep": sweep}


HYDRO_SWEEP = (
    # TAF on each region at thread, wave and block level over the grid of the
    # 2^24-option workload (prediction = window), and hourglass perforation
    # at 10, 20 and 50%
    [("%s_taf_%s_h%d_%g" % (region, level, h, th), {region: (h, h, th, level)})
     for region in ("eos", "hg") for level in ("thread", "wave", "block") for h in (2, 4, 8)
     for th in (0.001, 0.01, 0.1)]
    + [("hg_perfo_small_M%d" % m, dict(perfo=("small", m, 1))) for m in (10, 5, 2)])


def hydro_sweep(torch, exact_ms_per_step, exact_q, ref64, n=90, steps=500):
    """Each point of HYDRO_SWEEP over the whole run: ms per step, speedup,
    QoI error against the exact GPU run and the FP64 oracle's run, and the
    fraction of (wave, step) decisions that approximated each region (a
    second, recorded run of the same deterministic trajectory)."""
    from paper_2308_16877_amd.hydro import Hydro, Tech
    pts = {}
    for name, kw in HYDRO_SWEEP:
        h = Hydro(n, tech=Tech(**kw))
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        h.run(steps)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        q = h.origin_energy()
        del h
        frac = {}
        if "eos" in kw or "hg" in kw:
            region = "eos" if "eos" in kw else "hg"
            h = Hydro(n, tech=Tech(**kw))
            groups = {"thread": h.E, "wave": h.W, "block": -(-h.E // 256)}[kw[region][3]]
            acc = torch.zeros((), dtype=torch.int64, device="cuda:0")
            for _ in range(steps):
                h.step(record=True)
                acc += getattr(h, "dec_" + region)[:groups].sum()
            frac = {region: int(acc) / (groups * steps)}
            del h
        else:
            frac = {"hg": 1.0 / kw["perfo"][1]}
        pts[name] = {"ms_per_step": ms, "speedup_vs_exact": exact_ms_per_step / ms,
                     "qoi_err_vs_exact_gpu": abs(q / exact_q - 1),
                     "qoi_err_vs_fp64_oracle": abs(q / ref64 - 1) if ref64 else None,
                     "approx_frac": frac}
    ok = {k: v for k, v in pts.items() if v["qoi_err_vs_exact_gpu"] <= MAPE_BAR}
    best = max(ok, key=lambda k: ok[k]["speedup_vs_exact"]) if ok else None
    return {"points": pts, "best_at_qoi_err_0.005": {"technique": best, **ok[best]} if best else None}


def hydro_cpu_baseline(steps=16, n=90):
    """The oracle hydro (FP64, exact regions) for a few steps of the same mesh."""
    import oracle
    s = oracle.hydro_init(n, (1.0 / 8.0) * n ** 3)
    t0 = time.perf_counter()
    for k in range(steps):
        oracle.hydro_step(s, k)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n ** 3 * steps / dt, "unit": "element-steps/s", "cores": cores, "kind": "oracle",
            "sample": "first %d steps of the %d^3 blast, %.1f s wall" % (steps, n, dt)}


def cpu_baseline(x, sample):
    """The oracle, untuned, on the first `sample` items of the workload: the
    same four legs as one GPU step (exact prices; iACT, TAF and perforation
    on the oracle's FP64 region values)."""
    import oracle
    xs = x[:, :sample]
    t0 = time.perf_counter()
    oracle.bs_price(*xs)
    yv, sv = oracle.region_values_f32out(xs)
    oracle.iact(xs, yv, sv, 16, 8, 0.05)
    yv, sv = oracle.region_values_f32out(xs)
    oracle.taf(yv, sv, 16, 4, 4, 0.01)
    yv, sv = oracle.region_values_f32out(xs)
    oracle.perfo(yv, sv, 20, 0, 10)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 4 * sample / dt, "unit": "region items/s", "cores": cores, "kind": "oracle",
            "sample": "first %d of the %d items, all four legs of one step (exact, iACT, TAF, perforation), "
                      "%.1f s wall" % (sample, x.shape[1], dt)}


def config0_leg(torch, hpac, steps=200):
    """The 65,536-option configuration (pool of 1,024 tuples, 1e-3 jitter,
    random order): each launch of the step on it, timed over many launches
    (1.75 MiB of columns stay in the last-level cache, so the launches are
    latency- and launch-bound, not HBM-bound), with its approximated
    fraction and MAPE against the exact kernel."""
    from paper_2308_16877_amd import inputs
    dev = "cuda:0"
    n = 65536
    x = inputs.portfolio(n, 1024)
    xd = [torch.from_numpy(c).to(dev) for c in x]
    ex = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
    hpac.hpac_exact(xd, ex, items_per_lane=1)
    out = {}
    for t, (fn, ipt, params) in TECHS.items():
        r = technique_point(torch, hpac, [xd], n, fn, ipt, params, ex, steps=steps)
        r["items_per_s"] = n / (r["ms"] * 1e-3)
        r["items_per_lane"] = ipt
        out[t] = r
    for t in out:
        out[t]["speedup_vs_exact"] = out["exact"]["ms"] / out[t]["ms"]
    return {"workload": "65,536 options, pool of 1,024 tuples, 1e-3 relative jitter, random order (cache-resident)",
            "techniques": out}


PSIZE = (2, 4, 8, 16, 32, 64, 128, 256, 512)


def psize_leg(torch, hpac, n):
    """TAF's prediction size over the paper's range (2 .. 512), window 4,
    RSD 0.01, wave level: on the benchmark's sorted options at 16 items per
    lane, and on the lane-periodic variant (the temporal locality TAF
    exploits) at 64 and 512 items per lane, where long predictions fit."""
    from paper_2308_16877_amd import inputs
    dev = "cuda:0"
    res = {}
    for vname, mk, ipts in (("sorted", lambda: inputs.portfolio(n, 65536, sort_by_spot=True), (16,)),
                            ("lane_periodic_1024", lambda: inputs.periodic(n, 1024, jitter=1e-3), (64, 512))):
        xs = mk()
        copies = [[torch.from_numpy(c).to(dev) for c in xs] for _ in range(3)]
        del xs
        ex = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
        hpac.hpac_exact(copies[0], ex, items_per_lane=1)
        exact_ms = technique_point(torch, hpac, copies, n, "exact", 1, {}, ex)["ms"]
        rows = {}
        for ipt in ipts:
            for p in PSIZE:
                if ipt == 16 and p > 16:
                    continue  # beyond the steps a lane has
                r = technique_point(torch, hpac, copies, n, "taf", ipt,
                                    dict(history_size=4, prediction_size=p, rsd_threshold=0.01, level="wave"), ex)
                r["speedup_vs_exact"] = exact_ms / r["ms"]
                rows["ipt%d_p%d" % (ipt, p)] = r
        ok = {k: v for k, v in rows.items() if v["mape"] <= MAPE_BAR}
        best = max(ok, key=lambda k: ok[k]["speedup_vs_exact"]) if ok else None
        res[vname] = {"exact_ms": exact_ms, "points": rows,
                      "best_at_mape_0.005": dict(point=best, **ok[best]) if best else None}
        del copies
    return res


def committed_trace_average(kernel, workload):
    """rocprofv3's average duration (us) of `kernel` over the timed region of
    the step, from the committed kernel-trace summary, while that summary was
    taken on the current kernel code; else None."""
    path = os.path.join(ROOT, "profiles", "kernel_trace_%s.json" % workload)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    from paper_2308_16877_amd.profiling import kernel_source_sha
    k = d.get("timed_region", {}).get(kernel)
    if not k or k.get("kernel_source_sha") != kernel_source_sha(kernel):
        return None
    return k.get("avg_us")


def _round(v, digits=4):
    """Floats to `digits` significant digits, recursively (the headline line
    stays short)."""
    if isinstance(v, float):
        return float("%.*g" % (digits, v)) if v == v and abs(v) != float("inf") else None
    if isinstance(v, dict):
        return {k: _round(x, digits) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_round(x, digits) for x in v]
    return v


def _pick(d, *keys):
    return None if d is None else {k: d.get(k) for k in keys if k in d}


def leg_summary(legs):
    """One or two figures per further leg for the headline line (the legs
    themselves go to the legs file)."""
    s = {}
    st = legs.get("structured_locality")
    if st:
        s["structured_best_at_mape_0.005"] = st.get("best_at_mape_0.005")
    sw = legs.get("parameter_sweep")
    if sw:
        b = sw.get("best_at_mape_0.005") or {}
        s["sweep_best_at_mape_0.005"] = {"technique": b.get("technique"), "items_per_lane": b.get("items_per_lane"),
                                         "speedup_vs_exact": b.get("speedup_vs_exact"), "mape": b.get("mape"),
                                         "exact_best_shape": sw.get("best_exact")}
    c0 = legs.get("config0_65536")
    if c0:
        s["config0_items_per_s"] = {t: v["items_per_s"] for t, v in c0["techniques"].items()}
    ps = legs.get("psize_sweep")
    if ps:
        s["psize_best_at_mape_0.005"] = {v: _pick(d.get("best_at_mape_0.005"), "point", "speedup_vs_exact", "mape")
                                         for v, d in ps.items()}
    g = legs.get("greeks")
    if g:
        s["greeks"] = {"memo_speedup_vs_recompute": g.get("iact_speedup_vs_exact"),
                       "memo_speedup_wave_periodic_2": g.get("wave_periodic_2", {}).get("iact_speedup_vs_exact"),
                       "gradient_mape_wave_periodic_2": g.get("wave_periodic_2", {}).get("iact_gradient_mape_vs_exact")}
    pr = legs.get("precision")
    if pr:
        ok = {k: v for k, v in pr.items() if v["mape_vs_fp32"] <= MAPE_BAR and k != "fp32_body_fp32_columns"}
        b = max(ok, key=lambda k: ok[k]["speedup_vs_fp32"]) if ok else None
        s["precision_best_at_mape_0.005"] = {"variant": b, "speedup_vs_fp32": ok[b]["speedup_vs_fp32"],
                                             "mape": ok[b]["mape_vs_fp32"]} if b else None
    h = legs.get("hierarchy_and_items_per_lane")
    if h:
        s["taf_level_speedups"] = {lv: r["speedup_vs_exact"] for lv, r in h["taf"]["levels_at_ipt16"].items()}
        s["iact_level_speedups"] = {lv: r["speedup_vs_exact"] for lv, r in h["iact"]["levels_at_ipt16"].items()}
        # the parallelism-against-approximation study: speedup and approximated
        # fraction per items per lane, wave level
        s["items_per_lane_study"] = {t: {ipt: [r["speedup_vs_exact"], r["approx_frac"]]
                                         for ipt, r in h[t]["items_per_lane_at_wave_level"].items()}
                                     for t in ("taf", "iact")}
    bo = legs.get("binomial_options")
    if bo:
        u = bo["variants"]["unit_periodic"]
        s["binomial_unit_periodic"] = {t: {"speedup_vs_exact": u[t]["speedup_vs_exact"], "mape": u[t]["mape_vs_exact"]}
                                       for t in ("iact", "taf", "perfo")}
    su = legs.get("surrogate")
    if su:
        s["surrogate"] = _pick(su, "speedup_vs_exact", "mape_vs_exact", "rel_l2_vs_exact", "items_per_s")
    hy = legs.get("hydro")
    if hy:
        b = hy["sweep"].get("best_at_qoi_err_0.005") or {}
        ex = hy["techniques"]["exact"]
        s["hydro"] = {"exact_ms_per_step": ex["ms_per_step"], "exact_element_steps_per_s": ex["element_steps_per_s"],
                      "best_at_qoi_err_0.005": _pick(b, "technique", "speedup_vs_exact", "qoi_err_vs_exact_gpu"),
                      "cpu_baseline_element_steps_per_s": (hy.get("cpu_baseline") or {}).get("value")}
    return s


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2308_16877_amd import hpac, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    hpac.lib()
    dev = "cuda:0"
    n = args.n
    print("[bench] generating %d items" % n, file=sys.stderr, flush=True)
    x = inputs.portfolio(n, 65536, sort_by_spot=True)
    x_copies = []
    for c in range(3):
        xd = [torch.from_numpy(col).to(dev) for col in x]
        if c:
            # distinct buffers with the same values (rotated order of columns would change the workload)
            xd = [col.clone() for col in xd]
        x_copies.append(xd)
    torch.cuda.synchronize()
    if args.pmc_probe:
        pmc_probe(torch, hpac, x_copies, n)
        return
    print("[bench] timing %d steps after %d warmup" % (args.steps, args.warmup), file=sys.stderr, flush=True)
    res = run_workload(torch, hpac, x_copies, n, args.steps, args.warmup, min_warm_s=0.05)
    tech = summarize(res, n)
    ms_per_step = res["total_ms"] / args.steps
    leg_steps = max(min(args.steps // 2, 10), 3)  # timed steps of the further legs
    # the headline counts the items of the launches whose MAPE meets the bar
    # (perforation's dropped outputs keep their previous contents, so its
    # MAPE is about its rate); every launch's time is in the step
    ok = {t: v for t, v in tech.items() if v["mape"] <= MAPE_BAR}
    value = n * len(ok) / (ms_per_step * 1e-3)
    best = max((t for t in ok if t != "exact"), key=lambda t: ok[t]["speedup_vs_exact"], default="exact")

    # dominant kernel and its roofline: HBM (algorithmic bytes) and, when a
    # counter summary of this kernel code exists, VALU issue (instructions the
    # kernel issues per launch, SQ_INSTS_VALU x 64 lanes); the larger
    # fraction is the bound
    dom = max(res["per_kernel_ms"], key=lambda t: res["per_kernel_ms"][t])
    dom_ms = res["per_kernel_ms"][dom]
    ab = algorithmic_bytes(dom, n, res["stats"][dom]["approx_frac"])
    achieved = ab / (dom_ms * 1e-3) / 1e9
    workload = "bs2p24_sorted"
    kname = KERNEL_NAMES[dom]
    traffic = measured_traffic(kname, workload, ab)
    rp_us = committed_trace_average(kname, workload)
    hbm = {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes_per_launch": ab,
           "avg_launch_ms": dom_ms,
           "rocprof_avg_us": rp_us, "frac_rocprof": (ab / (rp_us * 1e-6) / 1e9 / HBM_PEAK_GBS) if rp_us else None}
    roofline = hbm
    valu = committed_profile("valu", kname, workload)
    if valu:
        ops = valu["lane_instructions_per_dispatch"]
        tops = ops / (dom_ms * 1e-3) / 1e12
        ceil = valu_ceiling(torch, hpac)
        alu = {"kernel": kname, "bound": "alu", "achieved": tops, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
               "frac": tops / VALU_PEAK_TOPS, "traffic": traffic, "valu_lane_instructions_per_launch": ops,
               "avg_launch_ms": dom_ms, "hbm_frac": hbm["frac"], "hbm_frac_rocprof": hbm["frac_rocprof"],
               "measured_fma_issue_tops": ceil["vector_operands"]}
        if alu["frac"] > hbm["frac"]:
            roofline = alu
        else:
            roofline = dict(hbm, alu_frac=alu["frac"])
    for t in tech:
        abt = algorithmic_bytes(t, n, res["stats"][t]["approx_frac"])
        tech[t]["algorithmic_GBps"] = abt / (tech[t]["ms"] * 1e-3) / 1e9

    legs = {"techniques": tech, "skipped_work_counters": skipped_work_counters()}
    if not args.no_structured:
        structured = {}
        variants = {
            # wave-level input reuse: every wave sees the same two tuples (iACT's case)
            "wave_periodic_2": (2, "item i uses pool tuple i mod 2, 1e-3 jitter"),
            # per-lane output reuse across steps: lane l sees tuple l mod 1024 at every
            # step (TAF's case: temporal locality of one thread's invocations)
            "lane_periodic_1024": (1024, "item i uses pool tuple i mod 1024, 1e-3 jitter; every lane sees one "
                                         "tuple at every step"),
        }
        for vname, (period, desc) in variants.items():
            print("[bench] structured-locality variant %s" % vname, file=sys.stderr, flush=True)
            xs = inputs.periodic(n, period, jitter=1e-3)
            xs_copies = [[torch.from_numpy(col).to(dev) for col in xs] for _ in range(3)]
            rs = run_workload(torch, hpac, xs_copies, n, leg_steps, 2)
            ts = summarize(rs, n)
            structured[vname] = {
                "workload": desc + " (structured-locality variant, not a paper workload)",
                "techniques": {t: {k: v[k] for k in ("ms", "items_per_s", "speedup_vs_exact", "mape",
                                                      "approx_frac")} for t, v in ts.items()}}
            del xs_copies
        cands = [(v, t, r) for v, d in structured.items() for t, r in d["techniques"].items()
                 if r["mape"] <= MAPE_BAR and t != "exact"]
        if cands:
            v, t, r = max(cands, key=lambda c: c[2]["speedup_vs_exact"])
            structured["best_at_mape_0.005"] = {"variant": v, "technique": t,
                                                "speedup_vs_exact": r["speedup_vs_exact"], "mape": r["mape"]}
        legs["structured_locality"] = structured
        steps_of = (
            ("config0_65536", "configuration of 65,536 options", lambda: config0_leg(torch, hpac)),
            ("parameter_sweep", "parameter sweep", lambda: sweep_leg(torch, hpac, x_copies, n)),
            ("psize_sweep", "TAF prediction sizes", lambda: psize_leg(torch, hpac, n)),
            ("greeks", "greeks", lambda: greeks_leg(torch, hpac, x_copies[0], n, leg_steps)),
            ("precision", "precision variants", lambda: precision_leg(torch, hpac, x_copies[0], n, leg_steps)),
            ("hierarchy_and_items_per_lane", "hierarchy and items-per-lane study",
             lambda: hierarchy_and_ipt_leg(torch, hpac, n)),
            ("binomial_options", "binomial options", lambda: binomial_leg(torch, hpac)),
            ("surrogate", "surrogate", lambda: surrogate_leg(torch, hpac, n)),
            ("hydro", "hydro", lambda: hydro_leg(torch)),
        )
        for key, what, fn in steps_of:
            print("[bench] %s" % what, file=sys.stderr, flush=True)
            legs[key] = fn()

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(x, min(args.cpu_sample, n))
        if "hydro" in legs:
            legs["hydro"]["cpu_baseline"] = hydro_cpu_baseline()

    legs_path = args.legs_out
    if legs_path:
        os.makedirs(os.path.dirname(os.path.abspath(legs_path)), exist_ok=True)
        with open(legs_path, "w") as f:
            json.dump(legs, f, indent=1)
    line = headline(args, res, tech, value, ms_per_step, best, roofline, cpu, leg_summary(legs), legs_path)
    print(json.dumps(line), flush=True)


def headline(args, res, tech, value, ms_per_step, best, roofline, cpu, summary, legs_path):
    """The one JSON line the benchmark prints last (kept under 4 KB: every
    leg is summarised by a figure or two, the legs themselves are in the
    legs file)."""
    n = args.n
    ok = [t for t in TECHS if tech[t]["mape"] <= MAPE_BAR]
    line = {
        "metric": "region items/s + speedup over exact kernel at <=0.5% MAPE, same MI355X",
        "value": value,
        "unit": "region items/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_steps_run": res["warmup_steps_run"],
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "black_scholes_2^24_options_pool65536_sorted_by_spot", "n": n,
                   "step": "exact + iACT(t8, 0.05) + TAF(h4, p4, 0.01) + small perforation (M10) launches",
                   "value_counts": "items of the launches within 0.5% MAPE: " + ", ".join(ok),
                   "parallelism": "single GPU"},
        "all_launch_items_per_s": n * len(TECHS) / (ms_per_step * 1e-3),
        "techniques": {t: {"ms": v["ms"], "speedup_vs_exact": v["speedup_vs_exact"], "mape": v["mape"],
                           "approx_frac": v["approx_frac"]} for t, v in tech.items()},
        "best_at_mape_0.005": {"technique": best, "speedup_vs_exact": tech[best]["speedup_vs_exact"],
                               "mape": tech[best]["mape"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "legs": summary,
        "legs_file": legs_path,
    }
    return _round(line)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the approximated Black-Scholes region on one MI355X.

Workload: 2^24 European options (FP32 SoA columns S, K, T, r, v) drawn from a
pool of 65,536 tuples with 1e-3 relative jitter, sorted by spot.  One step
runs the whole hot path once over the batch: the exact region, iACT
(table 8, threshold 0.05), TAF (window 4, prediction 4, RSD 0.01) and small
perforation (M = 10, i.e. 10%), each one launch through the C ABI.  Inputs
rotate over three resident copies so the 256 MB last-level cache cannot
serve them between launches.

Prints one JSON line: whole-step region items/s, per-technique items/s,
speedup over the exact kernel and MAPE against the exact kernel's outputs,
the roofline of the dominant kernel (HIP-event durations on the launch
stream), and the CPU oracle timed on a bounded sample.
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
KERNEL_NAMES = {"exact": "k_exact", "iact": "k_iact", "taf": "k_taf", "perfo": "k_perfo_dense"}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--n", type=int, default=1 << 24)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-structured", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=1 << 24)
    p.add_argument("--pmc-probe", action="store_true",
                   help="only launch each kernel of the step three times plus a 256 MiB copy probe, untimed, "
                        "for hardware-counter runs")
    return p.parse_args()


COPY_PROBE_BYTES = 256 << 20


def pmc_probe(torch, hpac, x_copies, n):
    """Launches for a counter run: each technique 3 times on rotating inputs,
    then the plain copy kernel 3 times over COPY_PROBE_BYTES (its counter
    readings calibrate the byte counters)."""
    dev = x_copies[0][0].device
    outs = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)]
    for r in range(3):
        for t in TECHS:
            launch(hpac, t, x_copies[r % len(x_copies)], outs)
    src = torch.zeros(COPY_PROBE_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for r in range(3):
        hpac.hpac_probe_copy(src, dst, COPY_PROBE_BYTES)
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


def measured_traffic(kernel, workload, launches_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary for
    this kernel and workload, or None when absent or taken on other code."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    from paper_2308_16877_amd.profiling import kernel_source_sha
    if d.get("kernel_source_sha") != kernel_source_sha():
        return None
    return d.get("hbm_bytes_per_launch")


def run_workload(torch, hpac, x_copies, n, steps, warmup, with_stats=True):
    dev = x_copies[0][0].device
    outs = {t: [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(2)] for t in TECHS}
    stream = torch.cuda.current_stream()
    names = list(TECHS)
    # argument marshalling done once per (technique, input copy)
    prep = {t: [hpac.prepare(TECHS[t][0], xs, outs[t], items_per_lane=TECHS[t][1], block_size=256,
                             stream=stream, **TECHS[t][2]) for xs in x_copies] for t in names}
    for s in range(warmup):
        for t in names:
            prep[t][s % len(x_copies)]()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(steps)]
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for s in range(steps):
        c = s % len(x_copies)
        ev[s][0].record(stream)
        for j, t in enumerate(names):
            prep[t][c]()
            ev[s][j + 1].record(stream)
    stop.record(stream)
    host_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(stop)
    per = {t: [ev[s][j].elapsed_time(ev[s][j + 1]) for s in range(steps)] for j, t in enumerate(names)}
    res = {"total_ms": total_ms, "wall_s": wall, "host_enqueue_s": host_s,
           "per_kernel_ms": {t: sum(v) / len(v) for t, v in per.items()},
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
        out[t] = {"ms": round(ms, 5), "items_per_s": n / (ms * 1e-3), "speedup_vs_exact": ex / ms,
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
    recomputing adjoint, against iACT (table 16, threshold 0.05) on the
    price-and-Jacobian region + the saved-Jacobian VJP."""
    dev = x_dev[0].device
    f32 = dict(dtype=torch.float32, device=dev)
    ones = torch.ones(n, **f32)
    price = [torch.zeros(n, **f32) for _ in range(2)]
    grads_exact = [torch.zeros(n, **f32) for _ in range(5)]
    grads_iact = [torch.zeros(n, **f32) for _ in range(5)]
    full = [torch.zeros(n, **f32) for _ in range(12)]
    stream = torch.cuda.current_stream()
    fwd_exact = hpac.prepare("exact", x_dev, price, items_per_lane=1, block_size=256, stream=stream)
    fwd_iact = hpac.prepare("iact", x_dev, full, items_per_lane=16, block_size=256, stream=stream,
                            region=hpac.REGION_BS_PRICE_GRAD, table_size=16, threshold=0.05)
    legs = {
        "exact_fwd_adjoint": [fwd_exact, lambda: hpac.hpac_bs_adjoint(x_dev, ones, None, grads_exact)],
        "iact_fwd_vjp": [fwd_iact, lambda: hpac.hpac_bs_vjp(full[2:], ones, None, grads_iact)],
    }
    t = time_pairs(torch, legs, steps, 2)
    cnt = torch.zeros(hpac.NUM_COUNTERS, dtype=torch.int64, device=dev)
    hpac.hpac_iact(x_dev, full, 16, 0.05, items_per_lane=16, region=hpac.REGION_BS_PRICE_GRAD, counters=cnt)
    hpac.hpac_bs_vjp(full[2:], ones, None, grads_iact)
    torch.cuda.synchronize()
    c = cnt.cpu().tolist()
    return {"workload": "call Greeks (delta, dC/dK, theta, rho, vega) of the benchmark's 2^24 options",
            "exact_fwd_adjoint_ms": t["exact_fwd_adjoint"], "iact_fwd_vjp_ms": t["iact_fwd_vjp"],
            "exact_items_per_s": n / (t["exact_fwd_adjoint"] * 1e-3),
            "iact_items_per_s": n / (t["iact_fwd_vjp"] * 1e-3),
            "iact_speedup_vs_exact": t["exact_fwd_adjoint"] / t["iact_fwd_vjp"],
            "iact_approx_frac": c[1] / max(c[0], 1),
            "iact_gradient_mape_vs_exact": mape_torch(torch, grads_exact, grads_iact)}


def precision_leg(torch, hpac, x_dev, n, steps):
    """The exact region on the benchmark's 2^24 options with half-precision
    columns (10 B in + 4 B out per item) and with the FP16 / BF16 bodies:
    items/s and the error of each result against the FP32 exact kernel,
    relative to max(|price|, tau)."""
    stream = torch.cuda.current_stream()
    ref = [torch.zeros(n, dtype=torch.float32, device=x_dev[0].device) for _ in range(2)]
    hpac.hpac_exact(x_dev, ref, items_per_lane=1)
    variants = {
        "fp32_body_fp32_columns": (hpac.REGION_BS_PRICE, torch.float32),
        "fp32_body_fp16_columns": (hpac.REGION_BS_PRICE, torch.float16),
        "fp32_body_bf16_columns": (hpac.REGION_BS_PRICE, torch.bfloat16),
        "fp16_body_fp16_columns": (hpac.REGION_BS_PRICE_F16, torch.float16),
        "bf16_body_bf16_columns": (hpac.REGION_BS_PRICE_BF16, torch.bfloat16),
        "fp16_body_fp32_columns": (hpac.REGION_BS_PRICE_F16, torch.float32),
    }
    legs, outs = {}, {}
    for name, (region, dt) in variants.items():
        xs = [c.to(dt) for c in x_dev]
        o = [torch.zeros(n, dtype=dt, device=x_dev[0].device) for _ in range(2)]
        outs[name] = o
        legs[name] = [hpac.prepare("exact", xs, o, items_per_lane=1, block_size=256, stream=stream, region=region)]
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


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
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
    res = run_workload(torch, hpac, x_copies, n, args.steps, args.warmup)
    tech = summarize(res, n)
    ms_per_step = res["total_ms"] / args.steps
    items_per_step = n * len(TECHS)
    value = items_per_step / (ms_per_step * 1e-3)

    # dominant kernel and its roofline
    dom = max(res["per_kernel_ms"], key=lambda t: res["per_kernel_ms"][t])
    dom_ms = res["per_kernel_ms"][dom]
    ab = algorithmic_bytes(dom, n, res["stats"][dom]["approx_frac"])
    achieved = ab / (dom_ms * 1e-3) / 1e9
    workload = "bs2p24_sorted"
    traffic = measured_traffic(KERNEL_NAMES[dom], workload, ab)
    roofline = {"kernel": KERNEL_NAMES[dom], "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": ab, "avg_launch_ms": round(dom_ms, 5)}
    for t in tech:
        abt = algorithmic_bytes(t, n, res["stats"][t]["approx_frac"])
        tech[t]["algorithmic_GBps"] = abt / (tech[t]["ms"] * 1e-3) / 1e9
    ok = {t: v for t, v in tech.items() if v["mape"] <= MAPE_BAR}
    best = max(ok, key=lambda t: ok[t]["speedup_vs_exact"])

    structured = None
    if not args.no_structured:
        print("[bench] structured-locality variant", file=sys.stderr, flush=True)
        xs = inputs.periodic(n, 2, jitter=1e-3)
        xs_copies = [[torch.from_numpy(col).to(dev) for col in xs] for _ in range(3)]
        rs = run_workload(torch, hpac, xs_copies, n, max(args.steps // 2, 3), 2)
        ts = summarize(rs, n)
        structured = {"workload": "item i uses pool tuple i mod 2, 1e-3 jitter (structured-locality variant, "
                                  "not a paper workload)",
                      "techniques": {t: {k: v[k] for k in ("ms", "items_per_s", "speedup_vs_exact", "mape",
                                                            "approx_frac")} for t, v in ts.items()}}
        del xs_copies

    greeks = None
    if not args.no_structured:
        print("[bench] greeks", file=sys.stderr, flush=True)
        greeks = greeks_leg(torch, hpac, x_copies[0], n, max(args.steps // 2, 3))

    precision = None
    if not args.no_structured:
        print("[bench] precision variants", file=sys.stderr, flush=True)
        precision = precision_leg(torch, hpac, x_copies[0], n, max(args.steps // 2, 3))

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(x, min(args.cpu_sample, n))

    line = {
        "metric": "region items/s + speedup over exact kernel at <=0.5% MAPE, same MI355X",
        "value": value,
        "unit": "region items/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "black_scholes_2^24_options_pool65536_sorted_by_spot", "n": n,
                   "step": "exact + iACT(t8, 0.05) + TAF(h4, p4, 0.01) + small perforation (M10) launches",
                   "parallelism": "single GPU"},
        "techniques": tech,
        "best_at_mape_0.005": {"technique": best, "speedup_vs_exact": ok[best]["speedup_vs_exact"],
                               "mape": ok[best]["mape"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "structured_locality": structured,
        "greeks": greeks,
        "precision": precision,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

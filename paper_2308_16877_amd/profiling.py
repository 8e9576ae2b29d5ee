"""Turns rocprofv3 CSV output into the short text/JSON summaries kept under
profiles/.

  python -m paper_2308_16877_amd.profiling trace <kernel_stats.csv> <kernel_trace.csv> <bench.json> <out.txt> "<command>"
  python -m paper_2308_16877_amd.profiling traffic <fetch counter_collection.csv> <write counter_collection.csv> \
        <kernel-name-substring> <workload> <out.json> "<fetch command>" "<write command>" [a:b]
  python -m paper_2308_16877_amd.profiling valu <sq counter_collection.csv> <kernel-name-substring> <workload> \
        <items per dispatch> <out.json> "<command>" [a:b]

The optional a:b keeps dispatches a..b-1 of the kernel, in dispatch order
(the counter probe launches each workload's kernels three times in turn).
  python -m paper_2308_16877_amd.profiling kernels <kernel_stats.csv> <name-substring> <out.txt> "<title>" "<command>"
  python -m paper_2308_16877_amd.profiling stall <sq counter_collection.csv> <kernel-name-substring> <workload> \
        <out.json> "<command>" [a:b]

The traffic summary scales each kernel's FETCH_SIZE and WRITE_SIZE (KiB per
dispatch) by what the same counter reports for the plain copy probe of a
known size (bench.py --pmc-probe), and records the hash of the kernel's sources
(its translation unit and the headers it includes) it was measured on, so
that the benchmark reports it only while that code is unchanged.
"""
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2308_16877_amd", "csrc")
COPY_KERNEL = "k_copy"
COPY_BYTES = 256 << 20
# translation unit of each kernel family (by kernel-name prefix)
KERNEL_UNITS = (("k_hydro", "hydro_kernels.hip"), ("k_mlp", "mlp_kernels.hip"), ("k_bs_", "greeks_kernels.hip"),
                ("k_binomial", "binomial_kernels.hip"), ("k_", "approx_kernels.hip"))


def _unit_files(unit):
    """The translation unit and every csrc header it includes, transitively."""
    seen, todo = [], [unit]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.append(f)
        for line in open(os.path.join(CSRC, f)):
            line = line.strip()
            if line.startswith('#include "'):
                inc = line.split('"')[1]
                if os.path.exists(os.path.join(CSRC, inc)):
                    todo.append(inc)
    return sorted(seen)


def kernel_source_sha(kernel="k_exact"):
    """Hash of the sources a kernel is compiled from; a counter summary is
    only used while it matches."""
    unit = next(u for prefix, u in KERNEL_UNITS if kernel.startswith(prefix))
    h = hashlib.sha256()
    for f in _unit_files(unit):
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def short_name(name):
    """The kernel's name without its parameter list, nested template
    closers written ">>" whichever demangler printed the name."""
    base = name.split("(")[0].replace("void ", "")
    return re.sub(r">\s+(?=>)", ">", base)


BS_KERNELS = ("k_exact", "k_iact", "k_taf", "k_taf_wave", "k_perfo", "k_perfo_dense")
# the kernel each technique of the benchmark step launches (trace names)
STEP_KERNELS = {"exact": "hpac::k_exact<hpac::RegionBSPrice, false>",
                "iact": "hpac::k_iact<hpac::Streamed<hpac::RegionBSPrice>, 1, false, true>",
                "taf": "hpac::k_taf_wave<hpac::Streamed<hpac::RegionBSPrice>, 4, false>",
                "perfo": "hpac::k_perfo_dense<hpac::RegionBSPrice>"}


def _is_bs(name):
    return any(_kernel_match(name, k) for k in BS_KERNELS)


def trace_summary(stats_csv, trace_csv, bench_json, out_txt, command):
    """Kernel statistics and per-dispatch durations of the Black-Scholes
    technique kernels in a benchmark run, beside the HIP-event averages that
    run printed."""
    stats = [r for r in csv.DictReader(open(stats_csv)) if _is_bs(r["Name"])]
    trace = [r for r in csv.DictReader(open(trace_csv)) if _is_bs(r.get("Kernel_Name", ""))]
    bench = json.loads([l for l in open(bench_json) if l.startswith("{")][-1])
    lines = ["# rocprofv3 kernel-trace summary", "", "command (run from the repository root on one MI355X):", "",
             "    " + command, "", "kernel | calls | avg us | min us | max us | share %", "--- | --- | --- | --- | --- | ---"]
    for r in stats:
        if "hpac" not in r["Name"]:
            continue
        lines.append("%s | %s | %.1f | %.1f | %.1f | %.2f" % (
            short_name(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    # per-dispatch durations in launch order, and the bench's HIP-event averages of the same run
    per = {}
    for r in trace:
        n = r.get("Kernel_Name", "")
        if "hpac" in n:
            per.setdefault(short_name(n), []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines += ["", "HIP-event averages printed by the same run (timed region only), us:", ""]
    for t, v in bench["techniques"].items():
        lines.append("    %s: %.1f" % (t, v["ms"] * 1e3))
    lines += ["", "per-dispatch durations (us), launch order:", ""]
    for k, v in per.items():
        lines.append("    %s: %s" % (k, " ".join("%.0f" % d for d in v)))
    # the step runs first: dispatches W .. W+K-1 of each step kernel are its timed region
    w, k = int(bench.get("warmup_steps_run", bench.get("warmup", 0))), int(bench.get("steps", 0))
    lines += ["", "timed region of the step (dispatches %d..%d of each kernel), rocprofv3 average beside the "
              "HIP-event average of the same launches, us:" % (w, w + k - 1), ""]
    timed = {}
    for t, name in STEP_KERNELS.items():
        d = per.get(name, [])[w:w + k]
        if d and t in bench["techniques"]:
            lines.append("    %s (%s): %.1f (HIP events %.1f)" % (t, name, sum(d) / len(d),
                                                                bench["techniques"][t]["ms"] * 1e3))
            kernel = name.split("<")[0].replace("hpac::", "")
            timed[kernel] = {"technique": t, "trace_name": name, "avg_us": sum(d) / len(d), "dispatches": len(d),
                             "hip_event_avg_us": bench["techniques"][t]["ms"] * 1e3,
                             "kernel_source_sha": kernel_source_sha(kernel)}
    rf = bench.get("roofline", {})
    lines += ["", "roofline reported by that run: %s" % json.dumps(rf)]
    open(out_txt, "w").write("\n".join(lines) + "\n")
    # the timed-region averages, for the benchmark's rocprofv3-based fraction
    json.dump({"command": command, "timed_region": timed}, open(os.path.splitext(out_txt)[0] + ".json", "w"),
              indent=1)


def _pmc(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    return rows


def _dispatch_slice(rows, dispatches):
    """The rows of dispatches a..b-1 (in dispatch order) for "a:b", else all."""
    if not dispatches:
        return rows
    a, b = (int(v) for v in dispatches.split(":"))
    ids = sorted({int(r["Dispatch_Id"]) for r in rows})[a:b]
    keep = set(ids)
    return [r for r in rows if int(r["Dispatch_Id"]) in keep]


def traffic_summary(fetch_csv, write_csv, kernel_sub, workload, out_json, fetch_cmd, write_cmd, dispatches=None):
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _pmc(path, counter)
        copy = [float(r["Counter_Value"]) for r in rows if _kernel_match(r["Kernel_Name"], COPY_KERNEL)]
        kern = [float(r["Counter_Value"])
                for r in _dispatch_slice([r for r in rows if _kernel_match(r["Kernel_Name"], kernel_sub)], dispatches)]
        if not copy or not kern:
            raise SystemExit("no %s rows for %s or the copy probe in %s" % (counter, kernel_sub, path))
        copy_kib = sum(copy) / len(copy)
        kib = sum(kern) / len(kern)
        # the copy probe reads and writes COPY_BYTES once each
        scale = (COPY_BYTES / 1024.0) / copy_kib
        res[counter] = {"kib_per_dispatch": kib, "copy_probe_kib_per_dispatch": copy_kib, "scale": scale,
                        "bytes_per_dispatch": kib * 1024.0 * scale, "dispatches": len(kern)}
    out = {"kernel": kernel_sub, "workload": workload, "kernel_source_sha": kernel_source_sha(kernel_sub),
           "hbm_bytes_per_launch": res["FETCH_SIZE"]["bytes_per_dispatch"] + res["WRITE_SIZE"]["bytes_per_dispatch"],
           "fetch": res["FETCH_SIZE"], "write": res["WRITE_SIZE"],
           "commands": [fetch_cmd, write_cmd], "dispatches": dispatches or "all",
           "copy_probe_bytes": COPY_BYTES}
    json.dump(out, open(out_json, "w"), indent=1)
    return out


def _kernel_match(name, sub):
    """sub names a kernel (every instantiation of it) or, ending in a
    template-argument prefix such as "k_binomial<9, 1", some of them."""
    base = short_name(name)
    if "<" in sub:
        return base.startswith("hpac::" + sub)
    return base.startswith("hpac::" + sub + "<") or base == "hpac::" + sub


def valu_summary(sq_csv, kernel_sub, workload, items, out_json, command, dispatches=None):
    """Vector instructions issued per dispatch (SQ_INSTS_VALU, wave
    instructions, summed over the chip) and the other SQ counters of the same
    run, for the kernel whose name is hpac::<kernel_sub><...>."""
    rows = _dispatch_slice([r for r in csv.DictReader(open(sq_csv)) if _kernel_match(r["Kernel_Name"], kernel_sub)],
                           dispatches)
    if not rows:
        raise SystemExit("no rows for %s in %s" % (kernel_sub, sq_csv))
    per = {}
    for r in rows:
        per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    avg = {c: sum(v) / len(v) for c, v in per.items()}
    items = int(items)
    out = {"kernel": kernel_sub, "workload": workload, "kernel_source_sha": kernel_source_sha(kernel_sub),
           "dispatches": len(per.get("SQ_INSTS_VALU", [])), "counters_per_dispatch": avg,
           "lane_instructions_per_dispatch": avg["SQ_INSTS_VALU"] * 64.0,
           "items_per_dispatch": items, "valu_instructions_per_item": avg["SQ_INSTS_VALU"] * 64.0 / items,
           "command": command, "dispatches": dispatches or "all"}
    json.dump(out, open(out_json, "w"), indent=1)
    return out


def stall_summary(sq_csv, kernel_sub, workload, out_json, command, dispatches=None):
    """Where a kernel's waves spend their time, from one SQ counter pass:
    SQ_WAVE_CYCLES (wave-cycles resident) split into SQ_ACTIVE_INST_ANY
    (working on an instruction), SQ_WAIT_INST_ANY (an instruction ready but
    not issued: the issue ports or the execution units are busy with other
    waves' work) and SQ_WAIT_ANY (waiting on a counter: memory, LDS or
    scalar loads in flight); SQ_ACTIVE_INST_VALU against SQ_BUSY_CYCLES
    gives the vector units' share."""
    rows = _dispatch_slice([r for r in csv.DictReader(open(sq_csv)) if _kernel_match(r["Kernel_Name"], kernel_sub)],
                           dispatches)
    if not rows:
        raise SystemExit("no rows for %s in %s" % (kernel_sub, sq_csv))
    per = {}
    for r in rows:
        per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    avg = {c: sum(v) / len(v) for c, v in per.items()}
    wc = avg["SQ_WAVE_CYCLES"]
    out = {"kernel": kernel_sub, "workload": workload, "kernel_source_sha": kernel_source_sha(kernel_sub),
           "counters_per_dispatch": avg,
           "frac_of_wave_cycles": {"active_inst_any": avg["SQ_ACTIVE_INST_ANY"] / wc,
                                   "wait_inst_any (ready, not issued)": avg["SQ_WAIT_INST_ANY"] / wc,
                                   "wait_any (waiting on a counter)": avg["SQ_WAIT_ANY"] / wc},
           "command": command, "dispatches": dispatches or "all"}
    json.dump(out, open(out_json, "w"), indent=1)
    return out


def kernels_summary(stats_csv, sub, out_txt, title, command):
    """Per-kernel rocprofv3 statistics of the hpac kernels whose name contains sub."""
    stats = list(csv.DictReader(open(stats_csv)))
    lines = ["# " + title, "", "command (run from the repository root on one MI355X):", "", "    " + command, "",
             "kernel | calls | avg us | min us | max us | total us", "--- | --- | --- | --- | --- | ---"]
    for r in stats:
        if "hpac" not in r["Name"] or sub not in r["Name"]:
            continue
        lines.append("%s | %s | %.2f | %.2f | %.2f | %.1f" % (
            short_name(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e3))
    open(out_txt, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace_summary(*sys.argv[2:7])
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic_summary(*sys.argv[2:10]), indent=1))
    elif sys.argv[1] == "valu":
        print(json.dumps(valu_summary(*sys.argv[2:9]), indent=1))
    elif sys.argv[1] == "stall":
        print(json.dumps(stall_summary(*sys.argv[2:8]), indent=1))
    elif sys.argv[1] == "kernels":
        kernels_summary(*sys.argv[2:7])
    else:
        raise SystemExit(__doc__)

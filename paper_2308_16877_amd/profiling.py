"""Turns rocprofv3 CSV output into the short text/JSON summaries kept under
profiles/.

  python -m paper_2308_16877_amd.profiling trace <kernel_stats.csv> <kernel_trace.csv> <bench.json> <out.txt> "<command>"
  python -m paper_2308_16877_amd.profiling traffic <fetch counter_collection.csv> <write counter_collection.csv> \
        <kernel-name-substring> <workload> <out.json> "<fetch command>" "<write command>"

The traffic summary scales each kernel's FETCH_SIZE and WRITE_SIZE (KiB per
dispatch) by what the same counter reports for the plain copy probe of a
known size (bench.py --pmc-probe), and records the hash of the kernel sources
it was measured on, so that the benchmark reports it only while the kernels
are unchanged.
"""
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ("approx_kernels.hip", "region_bs.hpp", "wave.hpp", "launch.hpp")
COPY_KERNEL = "k_copy"
COPY_BYTES = 256 << 20


def kernel_source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2308_16877_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def short_name(name):
    base = name.split("(")[0].replace("void ", "")
    return base


def trace_summary(stats_csv, trace_csv, bench_json, out_txt, command):
    stats = list(csv.DictReader(open(stats_csv)))
    trace = list(csv.DictReader(open(trace_csv)))
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
    rf = bench.get("roofline", {})
    lines += ["", "roofline reported by that run: %s" % json.dumps(rf)]
    open(out_txt, "w").write("\n".join(lines) + "\n")


def _pmc(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    return rows


def traffic_summary(fetch_csv, write_csv, kernel_sub, workload, out_json, fetch_cmd, write_cmd):
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _pmc(path, counter)
        copy = [float(r["Counter_Value"]) for r in rows if COPY_KERNEL in r["Kernel_Name"]]
        kern = [float(r["Counter_Value"]) for r in rows if kernel_sub in r["Kernel_Name"] and COPY_KERNEL not in r["Kernel_Name"]]
        if not copy or not kern:
            raise SystemExit("no %s rows for %s or the copy probe in %s" % (counter, kernel_sub, path))
        copy_kib = sum(copy) / len(copy)
        kib = sum(kern) / len(kern)
        # the copy probe reads and writes COPY_BYTES once each
        scale = (COPY_BYTES / 1024.0) / copy_kib
        res[counter] = {"kib_per_dispatch": kib, "copy_probe_kib_per_dispatch": copy_kib, "scale": scale,
                        "bytes_per_dispatch": kib * 1024.0 * scale, "dispatches": len(kern)}
    out = {"kernel": kernel_sub, "workload": workload, "kernel_source_sha": kernel_source_sha(),
           "hbm_bytes_per_launch": res["FETCH_SIZE"]["bytes_per_dispatch"] + res["WRITE_SIZE"]["bytes_per_dispatch"],
           "fetch": res["FETCH_SIZE"], "write": res["WRITE_SIZE"],
           "commands": [fetch_cmd, write_cmd],
           "copy_probe_bytes": COPY_BYTES}
    json.dump(out, open(out_json, "w"), indent=1)
    return out


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace_summary(*sys.argv[2:7])
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic_summary(*sys.argv[2:9]), indent=1))
    else:
        raise SystemExit(__doc__)

"""Writes hydro_sedov90_qoi.json: the FP64 oracle's Sedov blast on the
benchmark mesh (90^3 elements, 500 steps), its origin energy (the quantity
of interest), time and energies every 50 steps, for the exact regions and
for each hydro technique the benchmark reports (TAF on the EOS region at
thread and wave level, perforation of the hourglass loop).  Calls only
oracle/.

    python tests/golden/make_hydro_qoi.py        (about 5 minutes per run on 8 cores)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

N, STEPS = 90, 500
# name: keyword arguments of oracle.hydro_step (TAF: (history, prediction,
# threshold, group of 1 = thread or 64 = wave elements); perforation:
# (kind, parameter, items per lane))
TECHS = {
    "exact": {},
    "eos_taf_thread_h4_p2_0.001": dict(eos=(4, 2, 0.001, 1)),
    "eos_taf_wave_h4_p4_0.01": dict(eos=(4, 4, 0.01, 64)),
    "hg_perfo_small_M2_ipt2": dict(perfo=(oracle.PERFO_SMALL, 2, 2)),
    "hg_perfo_small_M10": dict(perfo=(oracle.PERFO_SMALL, 10, 1)),
    "hg_perfo_fini_20": dict(perfo=(oracle.PERFO_FINI, 20, 1)),
    "hg_perfo_ini_20": dict(perfo=(oracle.PERFO_INI, 20, 1)),
}


def run(kw):
    e_origin = (1.0 / 8.0) / (1.0 / N) ** 3  # an eighth of unit energy, unit side, unit density
    s = oracle.hydro_init(N, e_origin, eos_h=kw["eos"][0] if "eos" in kw else 0)
    rec = []
    t0 = time.time()
    for k in range(STEPS):
        oracle.hydro_step(s, k, **kw)
        if (k + 1) % 50 == 0:
            ie, ke = oracle.hydro_energy(s)
            rec.append({"steps": k + 1, "origin_energy": float(s.e[0]), "time": s.time,
                        "internal": ie, "kinetic": ke, "flags": int(s.flags)})
            print(rec[-1], "%.0f s" % (time.time() - t0), flush=True)
    return e_origin, rec


def main():
    out = {"mesh": N, "steps": STEPS, "params": oracle.HYDRO_DEFAULTS,
           "generator": "tests/golden/make_hydro_qoi.py (FP64 oracle)", "techniques": {}}
    for name, kw in TECHS.items():
        print(name, flush=True)
        e_origin, rec = run(kw)
        out["e_origin"] = e_origin
        out["techniques"][name] = {"step_kwargs": {k: list(v) for k, v in kw.items()}, "records": rec}
    out["records"] = out["techniques"]["exact"]["records"]  # the exact run, as before
    with open(os.path.join(HERE, "hydro_sedov90_qoi.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()

"""Writes hydro_sedov90_qoi.json: the FP64 oracle's Sedov blast on the
benchmark mesh (90^3 elements, 500 steps, exact regions), its origin energy
(the quantity of interest) and time, every 50 steps.  Calls only oracle/.

    python tests/golden/make_hydro_qoi.py        (about 5 minutes on 8 cores)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

N, STEPS = 90, 500


def main():
    e_origin = (1.0 / 8.0) / (1.0 / N) ** 3  # an eighth of unit energy, unit side, unit density
    s = oracle.hydro_init(N, e_origin)
    rec = []
    t0 = time.time()
    for k in range(STEPS):
        oracle.hydro_step(s, k)
        if (k + 1) % 50 == 0:
            ie, ke = oracle.hydro_energy(s)
            rec.append({"steps": k + 1, "origin_energy": float(s.e[0]), "time": s.time,
                        "internal": ie, "kinetic": ke})
            print(rec[-1], "%.0f s" % (time.time() - t0), flush=True)
    out = {"mesh": N, "steps": STEPS, "e_origin": e_origin, "params": oracle.HYDRO_DEFAULTS,
           "generator": "tests/golden/make_hydro_qoi.py (FP64 oracle, exact regions)", "records": rec}
    with open(os.path.join(HERE, "hydro_sedov90_qoi.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()

"""Helpers for the GPU parity tests: move seeded inputs to the device, run an
entry point through the C ABI, and compare its outputs and per-(wave, step)
decisions with the oracle's."""
import sys

import numpy as np
import torch

import oracle
from paper_2308_16877_amd import hpac

DEV = "cuda:0"
SENTINEL = -12345.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x):
    return [torch.from_numpy(np.ascontiguousarray(c, dtype=np.float32)).to(DEV) for c in x]


def outputs(n_out, n, fill=SENTINEL):
    return [torch.full((n,), fill, dtype=torch.float32, device=DEV) for _ in range(n_out)]


def run(technique, x_dev, n_out, ipt, *, block_size=0, trace=True, counters=True, fill=SENTINEL, **params):
    """Run one entry point; returns (outputs (n_out, n) float64 numpy,
    trace words or None, counters or None)."""
    n = x_dev[0].numel()
    outs = outputs(n_out, n, fill)
    tr = None
    if trace:
        tr = torch.zeros(max(hpac.hpac_trace_entries(n, ipt), 1), dtype=torch.int32, device=DEV)
    cnt = torch.zeros(hpac.NUM_COUNTERS, dtype=torch.int64, device=DEV) if counters else None
    fn = {"exact": hpac.hpac_exact, "iact": hpac.hpac_iact, "taf": hpac.hpac_taf, "perfo": hpac.hpac_perfo}[technique]
    fn(x_dev, outs, items_per_lane=ipt, block_size=block_size, trace=tr, counters=cnt, **params)
    torch.cuda.synchronize()
    y = np.stack([o.cpu().numpy().astype(np.float64) for o in outs])
    t = tr.cpu().numpy().view(np.uint32) if tr is not None else None
    return y, t, (cnt.cpu().numpy() if cnt is not None else None)


def check_outputs(y_gpu, y_ref, scale, rel=1e-5, mask=None, what=""):
    """|gpu - ref| <= rel * scale elementwise (scale = the oracle's sum of
    absolute terms of each price); returns the worst ratio."""
    err = np.abs(y_gpu - y_ref)
    tol = rel * scale + 1e-30
    if mask is not None:
        err, tol = err[:, mask], tol[:, mask]
    ratio = err / tol
    worst = float(ratio.max()) if ratio.size else 0.0
    assert worst <= 1.0, "%s: worst |err|/tol = %.3g at %s" % (what, worst, np.unravel_index(ratio.argmax(), ratio.shape))
    return worst


def trace_dec(t):
    """GPU trace words -> decision codes like the oracle's (-1 inactive)."""
    f = hpac.trace_fields(t)
    d = np.where(f["active"], f["approx"].astype(np.int8), -1).astype(np.int8)
    return d, f


def compare_decisions(gpu_dec, ora_dec, ipt, fragile=None, lag=0):
    """Walk each wave's steps in order.  Returns (agree, compared, explained,
    cascaded).  A disagreement first seen at step k is explained only where
    the oracle marked step k - lag fragile (a statistic within the band of
    its threshold could flip the vote there; for TAF the vote at step k-1
    decides step k, so lag = 1).  The rest of that wave then follows a
    different history and is not compared.  Any unexplained disagreement
    fails."""
    g = gpu_dec.reshape(-1, ipt)
    o = ora_dec.reshape(-1, ipt)
    fr = fragile.reshape(-1, ipt) if fragile is not None else np.zeros_like(o, dtype=np.uint8)
    neq = g != o
    explained = cascaded = 0
    bad = []
    for w in np.nonzero(neq.any(axis=1))[0]:
        k = int(np.argmax(neq[w]))
        if k - lag >= 0 and fr[w, k - lag]:
            explained += 1
            cascaded += ipt - k - 1
        else:
            bad.append((int(w), k, int(g[w, k]), int(o[w, k])))
    compared = g.size - cascaded
    agree = compared - explained - len(bad)
    assert not bad, "unexplained decision mismatches (wave, step, gpu, oracle): %s" % bad[:10]
    return agree, compared, explained, cascaded


def mape_pair(y_exact, y_gpu, y_ora, mask=None):
    if mask is not None:
        y_exact, y_gpu, y_ora = y_exact[:, mask], y_gpu[:, mask], y_ora[:, mask]
    mg = oracle.mape(y_exact, y_gpu)[0]
    mo = oracle.mape(y_exact, y_ora)[0]
    return mg, mo

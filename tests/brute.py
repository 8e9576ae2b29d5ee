"""Brute-force re-statement of the approximation semantics for tiny inputs.

Written independently of the oracle's engine and structured differently:
every iACT table is rebuilt at each step from the complete list of writes
made to it so far, and every TAF window from the complete list of a lane's
accurate outputs.  Meant for inputs on an integer grid, where FP32 squared
distances are exact, so no rounding order matters.
"""
import math
import statistics


def lanes(n, ipt):
    per = -(-n // ipt)
    return 64 * (-(-per // 64))


def _majority(yes, act):
    return 2 * yes > act


def iact(x, y, ipt, tsize, theta, tables_per_wave=1, group=64):
    """x: list of input tuples, y: list of output tuples, one per item.
    Returns (out, dec) with dec[(w, k)] in {0, 1}, the per-wave record."""
    n = len(x)
    L = lanes(n, ipt)
    lpt = 64 // tables_per_wave
    out = [None] * n
    dec = {}
    writes = {}  # table id -> list of (x, y)
    thr = theta * theta

    def table(tid):
        ws = writes.get(tid, [])
        slots = {}
        for idx, e in enumerate(ws):
            slots[idx % tsize] = e
        return [slots[s] for s in sorted(slots)]  # valid slots in slot order

    unit = max(group, 64)
    for u0 in range(0, L, unit):
        for k in range(ipt):
            lanes_u = [l for l in range(u0, min(u0 + unit, L))]
            info = {}
            for l in lanes_u:
                i = l + k * L
                if i >= n:
                    continue
                tid = l // lpt
                tab = table(tid)
                best, arg = math.inf, None
                for s, (tx, ty) in enumerate(tab):
                    d2 = sum((a - b) ** 2 for a, b in zip(x[i], tx))
                    if d2 < best:
                        best, arg = d2, s
                info[l] = dict(i=i, tid=tid, d2=best, arg=arg, tab=tab,
                               hit=len(tab) > 0 and best < thr)
            computing = []
            for g0 in range(u0, min(u0 + unit, L), group):
                members = [l for l in range(g0, g0 + group) if l in info]
                if not members:
                    continue
                yes = sum(info[l]["hit"] for l in members)
                approx = _majority(yes, len(members))
                for l in members:
                    lane_approx = info[l]["hit"] if group == 1 else approx
                    if lane_approx and info[l]["arg"] is not None:
                        out[info[l]["i"]] = info[l]["tab"][info[l]["arg"]][1]
                    else:
                        out[info[l]["i"]] = y[info[l]["i"]]
                        computing.append(l)
                if group >= 64:
                    for w in range(g0 // 64, (g0 + group) // 64):
                        if any(w * 64 <= l < w * 64 + 64 for l in members):
                            dec[(w, k)] = int(approx)
            if group == 1:
                for l in info:
                    w = l // 64
                    dec[(w, k)] = max(dec.get((w, k), 0), int(l not in computing))
            # one writer per table: farthest computing lane, lowest on ties
            by_table = {}
            for l in computing:
                by_table.setdefault(info[l]["tid"], []).append(l)
            for tid, ls in by_table.items():
                w_l = max(ls, key=lambda l: (info[l]["d2"], -l))
                i = info[w_l]["i"]
                writes.setdefault(tid, []).append((x[i], y[i]))
    return out, dec


def taf(y, ipt, hsize, psize, theta, group=64):
    """y: list of output tuples per item.  Returns (out, dec)."""
    n = len(y)
    L = lanes(n, ipt)
    out = [None] * n
    dec = {}
    history = {}  # lane -> list of accurate outputs
    countdown = {}  # group id -> remaining stable steps

    def rsd(vals):
        mu = statistics.fmean(vals)
        sd = statistics.pstdev(vals)
        if sd == 0:
            return 0.0
        if mu == 0:
            return math.inf
        return sd / abs(mu)

    for k in range(ipt):
        for g0 in range(0, L, group):
            members = [l for l in range(g0, min(g0 + group, L)) if l + k * L < n]
            if not members:
                continue
            gid = g0 // group
            if countdown.get(gid, 0) > 0:
                for l in members:
                    out[l + k * L] = history[l][-1]
                countdown[gid] -= 1
                for l in members:
                    dec[(l // 64, k)] = 1
                continue
            yes, full = 0, True
            for l in members:
                i = l + k * L
                out[i] = y[i]
                history.setdefault(l, []).append(y[i])
                h = history[l]
                if len(h) < hsize:
                    full = False
                    continue
                win = h[-hsize:]
                r = max(rsd([v[o] for v in win]) for o in range(len(y[i])))
                yes += r < theta
            for l in members:
                dec[(l // 64, k)] = max(dec.get((l // 64, k), 0), 0)
            if full and _majority(yes, len(members)):
                countdown[gid] = psize
    return out, dec

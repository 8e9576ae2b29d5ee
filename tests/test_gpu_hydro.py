"""GPU parity of the hydro path (hpac_hydro_init / hpac_hydro_step) against
the FP64 oracle.

Per-step replay: the GPU state after k steps (FP32) is copied into the
oracle, which takes step k in FP64; the GPU takes the same step in FP32 and
the two states are compared field by field.  One FP32 step differs from the
FP64 step by rounding only, so each field is held to 1e-5 of its scale
(largest magnitude over the mesh); the kernels form element geometry from
edge differences and corner-relative sums so that FP32 coordinates of
magnitude 1 still resolve elements of size 1/n (measured worst: 1e-6 for q,
below 4e-7 for the other fields).
TAF decisions must agree on every wave whose vote is not fragile (the
statistic within a relative band of its threshold on either side); the
fraction of agreeing waves is reported.

Whole runs: the GPU's FP32 run and the oracle's FP64 run of the blast agree
on the quantity of interest (origin energy) within 1e-3 relative after 100
steps, and the GPU conserves total energy to FP32 rounding accumulated over
the run.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import say
from paper_2308_16877_amd import hpac
from paper_2308_16877_amd.hydro import Hydro, Tech, sedov_origin_energy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available()
    hpac.lib()


def _group(t):
    level = t[3] if len(t) > 3 else "wave"
    if level in ("thread", hpac.LEVEL_THREAD):
        return 1
    return 256 if level in ("block", hpac.LEVEL_BLOCK) else 64


def oracle_tech(tech):
    kw = {}
    if tech.eos:
        kw["eos"] = tuple(tech.eos[:3]) + (_group(tech.eos),)
    if tech.hg:
        kw["hg"] = tuple(tech.hg[:3]) + (_group(tech.hg),)
    if tech.perfo:
        kind = hpac.PERFO_KINDS[tech.perfo[0]] if isinstance(tech.perfo[0], str) else tech.perfo[0]
        kw["perfo"] = (kind, tech.perfo[1], tech.perfo[2])
    return kw


def to_oracle(h):
    """The GPU state as an oracle state (FP32 values, exact in FP64)."""
    g = h.numpy_state()
    t = h.tech
    s = oracle.HydroState(h.n, eos_h=t.eos[0] if t.eos else 0, hg_h=t.hg[0] if t.hg else 0)
    for f in ("x", "u", "mnode", "e", "p", "q", "c", "vol", "mass", "clock"):
        getattr(s, f)[...] = g[f]
    if t.eos:
        s.weos[...] = g["weos"]
        s.rho_eos[...] = g["rho_eos"]
        s.z_eos[...] = g["z_eos"]
    if t.hg:
        s.whg[...] = g["whg"]
        s.rho_hg[...] = g["rho_hg"]
        s.z_hg[...] = g["z_hg"]
        # the GPU keeps the last accurate forces only as the newest window
        # slot of each decision group; the oracle keeps them apart
        hs, E = t.hg[0], h.n ** 3
        pushes = g["z_hg"][np.arange(E) // _group(t.hg)]
        newest = g["whg"].reshape(hs, 24, E)[(pushes - 1) % hs, :, np.arange(E)].T
        s.fhg[...] = np.where(pushes > 0, newest, 0.0)
    return s


def rel_err(gpu, ref):
    scale = np.abs(ref).max()
    return float(np.abs(gpu - ref).max() / scale) if scale > 0 else float(np.abs(gpu).max())


# Unit roundoff of FP32, and the rounding steps allowed for one of the EOS
# region's cancelling sums (21 to 24 products, each input rounded once or
# twice before the product, with a factor-two margin).
U32 = 2.0 ** -24
K_ROUND = 64


def _corner_nodes(n, zs):
    i, j, k = zs % n, (zs // n) % n, zs // (n * n)
    return np.stack([(i + (c & 1)) + (n + 1) * ((j + ((c >> 1) & 1)) + (n + 1) * (k + ((c >> 2) & 1)))
                     for c in range(8)], axis=1)


def rounding_bounds(h, s, before, zs):
    """First-order FP32 rounding bounds of the EOS region's outputs e, p, q at
    elements zs, from the oracle's FP64 step.  e' = e - dt sum F.u/m, the
    volume rate sum B.(u_c - u_0) and the volume V = sum B.(x_c - x_0) / 3
    all cancel: the rounding error of each is at most K_ROUND u times the sum
    of the magnitudes of what it adds (for the volume rate, |B| (|u_c| +
    |u_0|): the corner velocities are rounded before they are differenced).
    p = (gamma - 1) e' m / V and q = rho (cq du^2 + cl c |du|), du = vdot /
    V^(2/3), carry those errors at their first-order sensitivities."""
    par, n, E = h.par, h.n, h.E
    nodes = _corner_nodes(n, zs)
    dt = float(s.clock[1])
    out = {f: np.zeros(len(zs)) for f in ("e", "p", "q")}
    for r, z in enumerate(zs):
        nd = nodes[r]
        xc = s.x[:, nd].T
        ub = 0.5 * (before["u"][:, nd] + s.u[:, nd]).T
        V1, B1 = oracle.hex_volume(xc)
        F = s.force[:, z].reshape(8, 3)
        m = float(s.mass[z])
        rho1 = m / V1
        eabs = abs(before["e"][z]) + dt * float(np.sum(np.abs(F) * np.abs(ub))) / m
        vdot = float(np.sum(B1 * ub))
        vabs = float(np.sum(np.abs(B1[1:]) * (np.abs(ub[1:]) + np.abs(ub[0]))))
        # relative rounding bound of V (the corner differences are exact)
        rv = K_ROUND * U32 * float(np.sum(np.abs(B1[1:]) * np.abs(xc[1:] - xc[0]))) / (3.0 * V1)
        v23 = V1 ** (2.0 / 3.0)
        du = vdot / v23
        dq = rho1 * (2.0 * par["cq"] * abs(du) + par["cl"] * before["c"][z]) / v23 if du < 0 else 0.0
        out["e"][r] = K_ROUND * U32 * eabs
        out["p"][r] = K_ROUND * U32 * ((par["gamma"] - 1.0) * rho1 * eabs + abs(s.p[z])) + abs(s.p[z]) * rv
        out["q"][r] = K_ROUND * U32 * (dq * vabs + abs(s.q[z])) + abs(s.q[z]) * (5.0 / 3.0) * rv
    return out


def replay_step(h, band=1e-3):
    """One GPU step and the oracle's step from the same state; returns
    (field errors, decision agreement or None).  A field's error is its
    largest deviation over its scale; for e, p and q an element may exceed
    1e-5 of scale by no more than its rounding bound (rounding_bounds), and
    the error reported is the largest excess over that bound (raw errors
    under raw_*)."""
    s = to_oracle(h)
    before = {f: getattr(s, f).copy() for f in ("u", "e", "c")}
    rec = oracle.hydro_step(s, h.steps, record=True, band=band, **oracle_tech(h.tech))
    h.step(record=True)
    torch.cuda.synchronize()
    g = h.numpy_state()
    errs = {f: rel_err(g[f], getattr(s, f)) for f in ("x", "u", "e", "p", "q", "c", "vol", "force")}
    errs["dt"] = abs(g["clock"][1] - s.clock[1]) / s.clock[1]
    for f in ("e", "p", "q"):
        errs["raw_" + f] = errs[f]
        ref = getattr(s, f)
        scale = np.abs(ref).max()
        dev = np.abs(g[f] - ref)
        zs = np.nonzero(dev > TOL[f] * scale)[0]
        if scale == 0 or zs.size == 0:
            continue
        assert zs.size <= max(64, h.E // 100), "%s: %d elements past 1e-5 of scale" % (f, zs.size)
        excess = dev.copy()
        excess[zs] = np.maximum(dev[zs] - rounding_bounds(h, s, before, zs)[f], TOL[f] * scale)
        errs[f] = float(excess.max() / scale)
        errs["bounded_" + f] = int(zs.size)
    dec = {}
    for region, on in (("eos", h.tech.eos), ("hg", h.tech.hg)):
        if not on:
            continue
        od = rec["dec_" + region]
        gd = getattr(h, "dec_" + region).cpu().numpy()[:od.size]
        frag = rec["frag_" + region].astype(bool)
        dec[region] = (gd, od, frag)
    return errs, dec, s


TOL = dict(x=1e-5, u=1e-5, vol=1e-5, force=1e-5, e=1e-5, p=1e-5, q=1e-5, c=1e-5, dt=1e-5)


def check_errs(errs, what):
    bad = {f: errs[f] for f in TOL if errs[f] > TOL[f]}
    assert not bad, "%s: %s" % (what, bad)


def test_init_matches_oracle():
    n = 12
    h = Hydro(n)
    torch.cuda.synchronize()
    s = oracle.hydro_init(n, sedov_origin_energy(n))
    g = h.numpy_state()
    for f in ("x", "e", "p", "c"):
        assert rel_err(g[f], getattr(s, f)) <= 2e-7, f
    # the volume from FP32 corner coordinates: edge differences of about
    # 2^-24 relative, a few roundings in the Gauss sum
    for f in ("mnode", "vol", "mass"):
        assert rel_err(g[f], getattr(s, f)) <= 1e-6, f
    assert g["clock"][0] == 0 and g["clock"][1] == s.clock[1]
    assert not g["u"].any() and not g["q"].any()


@pytest.mark.parametrize("n,steps", [(13, 80), (24, 40)])
def test_exact_step_replay(n, steps):
    h = Hydro(n)
    worst = {}
    for k in range(steps):
        if k % 10 == 9 or k == steps - 1:
            errs, _, _ = replay_step(h)
            check_errs(errs, "n=%d step %d" % (n, k))
            worst = {f: max(worst.get(f, 0), e) for f, e in errs.items()}
        else:
            h.step()
    say("n=%d worst relative errors %s" % (n, {f: "%.1e" % e for f, e in worst.items()}))


def test_exact_run_quantity_of_interest_and_energy():
    n, steps = 16, 100
    h = Hydro(n)
    ie0, ke0 = h.energy()
    h.run(steps)
    torch.cuda.synchronize()
    s = oracle.hydro_init(n, sedov_origin_energy(n))
    for k in range(steps):
        oracle.hydro_step(s, k)
    q_gpu, q_ref = h.origin_energy(), float(s.e[0])
    ie, ke = h.energy()
    say("origin energy GPU %.6e oracle %.6e (rel %.2e); time %.4e vs %.4e; energy drift %.2e"
        % (q_gpu, q_ref, abs(q_gpu / q_ref - 1), h.time(), s.time, (ie + ke) / (ie0 + ke0) - 1))
    assert abs(q_gpu / q_ref - 1) < 1e-3
    assert abs(h.time() / s.time - 1) < 1e-3
    assert abs((ie + ke) / (ie0 + ke0) - 1) < 1e-4
    assert ke > 0.1 * (ie0 + ke0)


TAF_CASES = [
    ("eos", Tech(eos=(4, 4, 0.01))),
    ("hourglass", Tech(hg=(4, 4, 0.05))),
    ("both", Tech(eos=(2, 8, 0.05), hg=(3, 2, 0.1))),
    ("eos_thread", Tech(eos=(4, 4, 0.01, "thread"))),
    ("both_thread", Tech(eos=(3, 2, 0.02, "thread"), hg=(2, 3, 0.05, "thread"))),
    ("both_block", Tech(eos=(3, 2, 0.02, "block"), hg=(2, 3, 0.05, "block"))),
    ("mixed_levels", Tech(eos=(2, 2, 0.01, "block"), hg=(4, 2, 0.05, "thread"))),
]


@pytest.mark.parametrize("name,tech", TAF_CASES, ids=[c[0] for c in TAF_CASES])
def test_taf_step_replay(name, tech):
    n, steps = 16, 90
    h = Hydro(n, tech=tech)
    agree = total = napprox = 0
    for k in range(steps):
        errs, dec, _ = replay_step(h)
        check_errs(errs, "%s step %d" % (name, k))
        for region, (gd, od, frag) in dec.items():
            mism = gd != od
            assert not np.any(mism & ~frag), (region, k, np.flatnonzero(mism & ~frag)[:8])
            agree += int((~mism).sum())
            total += gd.size
            napprox += int((gd == 1).sum())
    say("%s: decisions agree on %d of %d wave-steps, %d approximate" % (name, agree, total, napprox))
    assert napprox > 0
    assert agree >= 0.9999 * total


@pytest.mark.parametrize("perfo", [("small", 4, 8), ("large", 3, 6), ("ini", 20, 1), ("fini", 20, 1)])
def test_perforation_step_replay(perfo):
    n, steps = 14, 40
    h = Hydro(n, tech=Tech(perfo=perfo))
    for k in range(steps):
        errs, _, _ = replay_step(h)
        check_errs(errs, "%s step %d" % (perfo, k))


def test_taf_at_threshold_zero_equals_exact():
    n, steps = 12, 60
    a = Hydro(n)
    b = Hydro(n, tech=Tech(eos=(4, 4, 0.0), hg=(4, 4, 0.0)))
    a.run(steps)
    b.run(steps)
    torch.cuda.synchronize()
    for f in ("x", "u", "e", "p", "q", "c"):
        assert torch.equal(getattr(a, f), getattr(b, f)), f


def test_full_mesh_steps():
    """90^3 elements: steps 8..10 replayed against the oracle (the windows
    fill in steps 0..3, steps 4..7 approximate, step 8 computes, 9..12
    approximate again wherever the vote passed)."""
    h = Hydro(90, tech=Tech(eos=(4, 4, 0.01)))
    for k in range(8):
        h.step()
    approx = []
    for k in range(8, 11):
        errs, dec, _ = replay_step(h)
        check_errs(errs, "90^3 step %d" % k)
        gd, od, frag = dec["eos"]
        assert np.all((gd == od) | frag)
        approx.append((gd == 1).mean())
    say("90^3 approximate wave fraction at steps 8..10: %s" % approx)
    assert approx[0] == 0 and approx[1] > 0.9  # the quiet mesh is approximated


@pytest.mark.parametrize("n,tech", [
    (1, Tech()), (2, Tech(eos=(2, 2, 0.05))), (5, Tech(eos=(2, 3, 0.05), hg=(2, 2, 0.1))),
    (5, Tech(eos=(2, 3, 0.05, "thread"), hg=(3, 1, 0.1, "thread"))), (7, Tech(perfo=("small", 3, 4))),
    (9, Tech(perfo=("large", 2, 64))), (7, Tech(eos=(2, 2, 0.05, "block"), hg=(2, 2, 0.1, "block"))),
], ids=["n1", "n2_eos", "n5_both_wave", "n5_both_thread", "n7_small", "n9_large_ipt64", "n7_both_block"])
def test_small_and_ragged_meshes(n, tech):
    """Meshes of one element, of fewer elements than a wave, and with a
    ragged last wave (125 = 64 + 61 elements), stepped and replayed."""
    h = Hydro(n, tech=tech)
    for k in range(30):
        errs, dec, _ = replay_step(h)
        check_errs(errs, "n=%d step %d" % (n, k))
        for region, (gd, od, frag) in dec.items():
            assert np.all((gd == od) | frag), (region, k)


@pytest.mark.parametrize("tech", [
    Tech(), Tech(eos=(2, 2, 0.01, "thread"), hg=(2, 2, 0.05)), Tech(perfo=("small", 3, 1)),
    Tech(perfo=("fini", 30, 1)),
], ids=["exact", "taf_both", "perfo_small", "perfo_fini"])
@pytest.mark.parametrize("k", [5, 6])
def test_library_loop_equals_single_steps(tech, k):
    """hpac_hydro_run issues the launches of k hpac_hydro_step calls (odd
    and even k: the latest velocities end in unew or u): the states are
    identical, bit for bit, and stepping can continue from either."""
    a, b = Hydro(12, tech=tech), Hydro(12, tech=tech)
    a.run(3)
    for _ in range(3):
        b.step()
    a.run(k)
    for _ in range(k):
        b.step()
    a.step()
    b.step()
    torch.cuda.synchronize()
    ga, gb = a.numpy_state(), b.numpy_state()
    for f, va in ga.items():
        if va is not None:
            assert np.array_equal(va, gb[f]), f
    assert a.steps == b.steps == k + 4


def test_numeric_failure_is_reported():
    """The failure path: the tangling configuration of the oracle's test
    (Courant factor 3, volume-change limit lifted, time step allowed to
    double) sets the device's numeric-failure flag, which hpac_hydro_check
    turns into HPAC_ENUMERIC, within a few steps of where the FP64 oracle
    first reports a non-positive volume on the same run; the workload's own
    constants raise nothing over 150 steps.  Nothing faults: no index
    depends on a value."""
    n, par = 10, dict(cfl=3.0, dvmax=10.0, growth=2.0)
    s = oracle.hydro_init(n, sedov_origin_energy(n), **par)
    first_oracle = None
    for k in range(60):
        oracle.hydro_step(s, k)
        if s.flags and first_oracle is None:
            first_oracle = k
    h = Hydro(n, **par)
    first = None
    for k in range(60):
        h.step()
        try:
            h.check()
        except hpac.HpacError as e:
            assert e.status == hpac.HPAC_ENUMERIC and "volume" in str(e), str(e)
            first = k
            break
    say("first flagged step: GPU %s, oracle %s" % (first, first_oracle))
    assert first is not None and first_oracle is not None and abs(first - first_oracle) <= 5
    assert int(h.status.item()) & hpac.HYDRO_BAD_VOLUME
    ok = Hydro(n)
    ok.run(150)
    ok.check()
    assert int(ok.status.item()) == 0


CONFIG_TECHS = [
    # the bench-reported techniques at the configuration's mesh (90^3, 500 steps)
    ("exact", Tech()),
    ("eos_taf_thread_h4_p2_0.001", Tech(eos=(4, 2, 0.001, "thread"))),
    ("eos_taf_wave_h4_0.01", Tech(eos=(4, 4, 0.01))),
    ("hg_perfo_small_M10", Tech(perfo=("small", 10, 1))),
]


@pytest.mark.parametrize("name,tech", CONFIG_TECHS, ids=[c[0] for c in CONFIG_TECHS])
def test_config_mesh_late_step_replay(name, tech):
    """The 90^3 blast run on the GPU to steps 100, 250 and 499 of its 500,
    each of those steps replayed by the FP64 oracle from the GPU's state:
    every field within 1e-5 of its scale (e, p and q: or within the FP32
    rounding bound of their cancelling sums, which the weakening blast's
    small velocity differences make exceed 1e-5 of scale for q, at 1.1e-5,
    from step 250 on) and TAF decisions equal wherever
    the vote is not fragile (the statistic within a relative 1e-3 of the
    threshold, for the oracle's FP64 region values against the GPU's FP32
    ones).  Wave-level EOS TAF is unstable on this blast (its free run
    leaves the exact trajectory by orders of magnitude, in the FP64 oracle
    as on the GPU); the replay shows that each of its steps is still the
    method's step, not a kernel error."""
    h = Hydro(90, tech=tech)
    for target in (100, 250, 499):
        h.run(target - h.steps)
        errs, dec, _ = replay_step(h)
        say("90^3 %s step %d: %s" % (name, target, {f: "%.1e" % e for f, e in errs.items()}))
        check_errs(errs, "90^3 %s step %d" % (name, target))
        for region, (gd, od, frag) in dec.items():
            assert np.all((gd == od) | frag), (region, target, int(((gd != od) & ~frag).sum()))
            say("  %s decisions: %d of %d groups approximate, %d fragile" % (
                region, int((gd == 1).sum()), gd.size, int(frag.sum())))


QOI_TECHS = [
    ("eos_taf_thread_h4_p2_0.001", Tech(eos=(4, 2, 0.001, "thread"))),
    ("eos_taf_thread_h2_p2_0.001", Tech(eos=(2, 2, 0.001, "thread"))),
    ("hg_taf_thread_h4_p4_0.01", Tech(hg=(4, 4, 0.01, "thread"))),
    ("hg_perfo_small_M10", Tech(perfo=("small", 10, 1))),
    ("hg_perfo_fini_20", Tech(perfo=("fini", 20, 1))),
]


@pytest.mark.parametrize("name,tech", QOI_TECHS, ids=[c[0] for c in QOI_TECHS])
def test_whole_run_qoi_error_matches_oracle(name, tech):
    """Well-conditioned whole runs (16^3 x 100 steps and 24^3 x 150): the
    quantity-of-interest error each technique causes (origin energy against
    the exact run of the same precision) on the GPU equals the oracle's own
    free run's within 1e-4 absolute."""
    for n, steps in ((16, 100), (24, 150)):
        qg, qo = {}, {}
        for key, t in (("exact", Tech()), (name, tech)):
            h = Hydro(n, tech=t)
            h.run(steps)
            torch.cuda.synchronize()
            qg[key] = h.origin_energy()
            kw = oracle_tech(t)
            s = oracle.hydro_init(n, sedov_origin_energy(n), eos_h=t.eos[0] if t.eos else 0,
                                  hg_h=t.hg[0] if t.hg else 0)
            for k in range(steps):
                oracle.hydro_step(s, k, **kw)
            qo[key] = float(s.e[0])
        eg, eo = abs(qg[name] / qg["exact"] - 1), abs(qo[name] / qo["exact"] - 1)
        say("%s n=%d: QoI error GPU %.3e oracle %.3e" % (name, n, eg, eo))
        assert abs(eg - eo) <= 1e-4

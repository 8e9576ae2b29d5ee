"""Pins of the FP64 oracle hydro (oracle/hydro.c) against facts that do not
come from the oracle itself: exact volumes of affine images of a cube,
finite differences of the volume, the Euler identities of a volume
gradient, the closed-form hourglass force of a cube, the vanishing of
hourglass forces on linear velocity fields, a quiescent mesh at rest,
conservation of total energy, the octant symmetry of the blast, and the
Sedov-Taylor shock radius from the similarity solution.  Then the
approximation semantics across timesteps: TAF at threshold 0 and no
perforation reproduce the exact run bit for bit, TAF countdowns follow the
paper's prediction-size rule, approximated and perforated elements keep
their outputs.
"""
import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

import oracle

CUBE = np.array([[(c >> d) & 1 for d in range(3)] for c in range(8)], np.float64)  # corner a + 2b + 4c
SGN = 2 * CUBE - 1


def rnd_hex(seed, amp=0.15):
    g = np.random.default_rng(seed)
    A = np.eye(3) + 0.2 * g.standard_normal((3, 3))
    return CUBE @ A.T + amp * g.standard_normal((8, 3)) + g.standard_normal(3)


def test_volume_of_affine_images_of_the_cube():
    g = np.random.default_rng(1)
    for _ in range(20):
        A = np.eye(3) + 0.3 * g.standard_normal((3, 3))
        b = g.standard_normal(3)
        V, _ = oracle.hex_volume(CUBE @ A.T + b)
        assert abs(V - np.linalg.det(A)) <= 1e-13 * abs(np.linalg.det(A))


def test_volume_gradient_matches_central_differences():
    for seed in range(5):
        xc = rnd_hex(seed)
        V, B = oracle.hex_volume(xc)
        fd = np.zeros((8, 3))
        for c in range(8):
            for d in range(3):
                h = 1e-6
                xp, xm = xc.copy(), xc.copy()
                xp[c, d] += h
                xm[c, d] -= h
                fd[c, d] = (oracle.hex_volume(xp)[0] - oracle.hex_volume(xm)[0]) / (2 * h)
        assert np.max(np.abs(fd - B)) <= 1e-8 * np.max(np.abs(B))


def test_volume_gradient_euler_identities():
    """V is invariant under translation (sum_c B_c = 0), scales by lambda when
    one coordinate scales by lambda, and is invariant under a shear of one
    coordinate by another: sum_c x_cj B_ci = delta_ij V."""
    for seed in range(5):
        xc = rnd_hex(seed, amp=0.25)
        V, B = oracle.hex_volume(xc)
        assert np.max(np.abs(B.sum(axis=0))) <= 1e-13 * np.abs(B).max()
        assert np.max(np.abs(xc.T @ B - V * np.eye(3))) <= 1e-12 * abs(V)


def test_hourglass_force_on_a_cube_closed_form():
    """On an undistorted cube the hourglass vectors are the base vectors
    themselves, so a pure mode u_x = U Gamma_1 (Gamma_1 = s_y s_z) gives
    f_x = -khg rho c V^(2/3) U Gamma_1 and no other component."""
    h = 0.7
    xc = CUBE * h + 3.0
    U, rho, c, khg = 0.3, 1.7, 2.5, 0.1
    G1 = SGN[:, 1] * SGN[:, 2]
    uc = np.zeros((8, 3))
    uc[:, 0] = U * G1
    f = oracle.hex_hourglass(xc, uc, rho, c, khg)
    ref = -khg * rho * c * (h ** 3) ** (2 / 3) * U * G1
    assert np.allclose(f[:, 0], ref, rtol=1e-13, atol=1e-15)
    assert np.all(f[:, 1:] == 0)


def test_hourglass_force_vanishes_on_linear_fields_and_dissipates():
    g = np.random.default_rng(7)
    for seed in range(5):
        xc = rnd_hex(seed, amp=0.2)
        Gm = g.standard_normal((3, 3))
        a = g.standard_normal(3)
        f = oracle.hex_hourglass(xc, xc @ Gm.T + a, 1.0, 1.0, 0.1)
        assert np.max(np.abs(f)) <= 1e-13 * (np.abs(xc @ Gm.T).max() + 1)
        u = g.standard_normal((8, 3))
        f = oracle.hex_hourglass(xc, u, 1.0, 1.0, 0.1)
        assert np.sum(f * u) < 0
        # linear in the velocity and in khg, rho, c
        f2 = oracle.hex_hourglass(xc, 2 * u, 1.5, 2.0, 0.3)
        assert np.allclose(f2, 2 * 1.5 * 2.0 * 3 * f, rtol=1e-12, atol=1e-15)


def test_quiescent_mesh_stays_at_rest():
    s = oracle.hydro_init(6, 0.0)
    x0 = s.x.copy()
    for k in range(20):
        oracle.hydro_step(s, k)
    assert np.array_equal(s.x, x0)
    assert not s.u.any() and not s.e.any() and not s.p.any() and not s.q.any()


def sedov(n, steps, **kw):
    s = oracle.hydro_init(n, (1.0 / 8) * n ** 3, **kw)  # full-space energy 1, density 1, side 1
    for k in range(steps):
        oracle.hydro_step(s, k)
    return s


def test_total_energy_is_conserved():
    s = oracle.hydro_init(10, (1.0 / 8) * 1000)
    e0 = sum(oracle.hydro_energy(s))
    for k in range(150):
        oracle.hydro_step(s, k)
    ie, ke = oracle.hydro_energy(s)
    assert ke > 0.1 * e0  # the blast has moved material
    assert abs(ie + ke - e0) <= 1e-12 * e0


def test_octant_symmetry():
    n = 10
    s = sedov(n, 120)
    e = s.e.reshape(n, n, n)  # [k, j, i]
    scale = np.abs(e).max()
    for perm in [(0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0)]:
        assert np.max(np.abs(e - e.transpose(perm))) <= 1e-10 * scale
    x = [s.x[d].reshape(n + 1, n + 1, n + 1) for d in range(3)]
    # swapping the x and y axes maps x to y
    assert np.max(np.abs(x[0] - x[1].transpose(0, 2, 1))) <= 1e-12


def sedov_xi0(gamma):
    """Constant of the Sedov-Taylor radius R = xi0 (E t^2 / rho0)^(1/5) of a
    spherical blast: integrate the similarity equations of mass, momentum and
    entropy from the strong-shock state at xi = 1 inwards and normalise by the
    energy integral."""
    def rhs(xi, y):
        U, G, P = y
        a = U - xi
        A = np.array([[a, 0.0, 1.0 / G], [G, a, 0.0], [0.0, -a * gamma / G, a / P]])
        b = np.array([1.5 * U, -2.0 * G * U / xi, 3.0])
        return np.linalg.solve(A, b)
    y0 = [2 / (gamma + 1), (gamma + 1) / (gamma - 1), 2 / (gamma + 1)]
    sol = solve_ivp(rhs, [1.0, 1e-6], y0, rtol=1e-10, atol=1e-12, dense_output=True)

    def integrand(xi):
        U, G, P = sol.sol(xi)
        return (0.5 * G * U * U + P / (gamma - 1)) * xi * xi
    I = quad(integrand, 1e-6, 1.0, limit=200)[0]
    return ((16 * np.pi / 25) * I) ** -0.2


def test_sedov_constant():
    # the energy constant alpha = xi0^-5 of gamma = 1.4 is 0.851 in the literature
    assert abs(sedov_xi0(1.4) ** -5 - 0.851) < 1e-3


def element_centres(s):
    n = s.n
    xs = [s.x[d].reshape(n + 1, n + 1, n + 1) for d in range(3)]
    return [0.125 * sum(a[k:k + n, j:j + n, i:i + n] for k in (0, 1) for j in (0, 1) for i in (0, 1)).ravel()
            for a in xs]


def test_shock_radius_follows_sedov_taylor():
    n = 30
    s = sedov(n, 250)
    cx, cy, cz = element_centres(s)
    r = np.sqrt(cx ** 2 + cy ** 2 + cz ** 2)
    R = r[np.argmax(s.mass / s.vol)]
    R_th = sedov_xi0(1.4) * (s.time ** 2) ** 0.2
    assert R * n >= 10
    assert abs(R / R_th - 1) < 0.10, (R, R_th)


# ------------------------------------------------------- approximation semantics

def run(n, steps, **tech):
    s = oracle.hydro_init(n, (1.0 / 8) * n ** 3, eos_h=(tech.get("eos") or (0,))[0],
                         hg_h=(tech.get("hg") or (0,))[0])
    recs = [oracle.hydro_step(s, k, record=True, **tech) for k in range(steps)]
    return s, recs


def same_state(a, b):
    return all(np.array_equal(getattr(a, f), getattr(b, f)) for f in ("x", "u", "e", "p", "q", "c", "vol"))


def test_techniques_collapse_to_exact():
    ref, _ = run(8, 60)
    for tech in (dict(eos=(4, 4, 0.0)), dict(hg=(4, 4, 0.0)), dict(eos=(2, 8, 0.0), hg=(8, 2, 0.0)),
                 dict(perfo=(0, 0, 4))):
        s, recs = run(8, 60, **tech)
        assert same_state(s, ref), tech
        assert all((r["dec_eos"] != 1).all() and (r["dec_hg"] != 1).all() for r in recs)


def test_taf_countdown_follows_prediction_size():
    """With a threshold no finite RSD reaches, every wave votes to
    approximate as soon as its window is full: h accurate steps, then p
    approximate steps after every accurate one."""
    h, p = 3, 2
    s, recs = run(8, 20, eos=(h, p, 1e300))
    dec = np.stack([r["dec_eos"] for r in recs])  # (steps, waves)
    expect = [0] * h + ([1] * p + [0]) * 10
    for w in range(dec.shape[1]):
        assert list(dec[:, w]) == expect[:20]


def test_approximated_elements_keep_their_outputs():
    n, h, p = 8, 2, 3
    s = oracle.hydro_init(n, (1.0 / 8) * n ** 3, eos_h=h, hg_h=h)
    for k in range(40):
        before = s.copy()
        rec = oracle.hydro_step(s, k, eos=(h, p, 0.05), hg=(h, p, 0.05), record=True)
        for w in np.flatnonzero(rec["dec_eos"] == 1):
            sl = slice(64 * w, 64 * (w + 1))
            for f in ("e", "p", "q", "c"):
                assert np.array_equal(getattr(s, f)[sl], getattr(before, f)[sl])
        for w in np.flatnonzero(rec["dec_hg"] == 1):
            sl = slice(64 * w, 64 * (w + 1))
            assert np.array_equal(s.fhg[:, sl], before.fhg[:, sl])
        for w in np.flatnonzero(rec["dec_hg"] == 0):
            sl = slice(64 * w, 64 * (w + 1))
            assert np.array_equal(s.whg[(before.z_hg[w] % h) * 24:(before.z_hg[w] % h + 1) * 24, sl], s.fhg[:, sl])


@pytest.mark.parametrize("kind,param,ipt", [(0, 4, 8), (1, 3, 6), (2, 20, 1), (3, 20, 1)])
def test_perforated_elements_add_no_hourglass_force(kind, param, ipt):
    """A skipped iteration of the hourglass loop computes and adds nothing:
    the element's corner forces are its pressure forces (p + q) B alone; a
    computed one adds the hourglass force of its corners."""
    n = 8
    E = n ** 3
    s = oracle.hydro_init(n, (1.0 / 8) * n ** 3)
    L = oracle.num_lanes(E, ipt)
    z = np.arange(E)
    k_of = z // L
    checked_hg = 0
    for step in range(30):
        before = s.copy()
        oracle.hydro_step(s, step, perfo=(kind, param, ipt))
        if kind == 0:
            skipped = (k_of + step) % param == param - 1
        elif kind == 1:
            skipped = (k_of + step) % param != 0
        elif kind == 2:
            skipped = z < param * E // 100
        else:
            skipped = z >= E - param * E // 100
        if step % 6:
            continue
        for e in range(0, E, 7):
            i, j, k = e % n, (e // n) % n, e // (n * n)
            nodes = [(i + (c & 1)) + (n + 1) * ((j + ((c >> 1) & 1)) + (n + 1) * (k + ((c >> 2) & 1)))
                     for c in range(8)]
            xc = before.x[:, nodes].T
            uc = before.u[:, nodes].T
            V, B = oracle.hex_volume(xc)
            f = s.force[:, e].reshape(8, 3)
            fp = (before.p[e] + before.q[e]) * B
            if skipped[e]:
                assert np.array_equal(f, fp)
            else:
                fh = oracle.hex_hourglass(xc, uc, before.mass[e] / V, before.c[e], s.par["khg"])
                assert np.array_equal(f, fp + fh)
                checked_hg += int(np.any(fh != 0))
    assert checked_hg > 0


def test_thread_level_taf_decides_per_element():
    """Thread level (section 3.1.2): each element keeps its own countdown, so
    within one wave some elements compute while others reuse; with a
    threshold no finite RSD reaches every element follows the h, then
    (p approximate + 1 accurate) pattern; threshold 0 is exact."""
    h, p = 3, 2
    s, recs = run(8, 20, eos=(h, p, 1e300, 1))
    dec = np.stack([r["dec_eos"] for r in recs])  # (steps, elements)
    assert dec.shape[1] == 8 ** 3
    expect = [0] * h + ([1] * p + [0]) * 10
    assert all(list(dec[:, z]) == expect[:20] for z in range(dec.shape[1]))
    s, recs = run(10, 60, eos=(4, 4, 0.01, 1), hg=(4, 4, 0.05, 1))
    mixed = 0
    for r in recs:
        d = r["dec_eos"][:(len(r["dec_eos"]) // 64) * 64].reshape(-1, 64)
        mixed += int(np.sum((d == 1).any(axis=1) & (d == 0).any(axis=1)))
    assert mixed > 0
    ref, _ = run(8, 40)
    s, _ = run(8, 40, eos=(4, 4, 0.0, 1), hg=(2, 3, 0.0, 1))
    assert same_state(s, ref)


def test_block_level_taf_decides_per_256_elements():
    """Block level (section 3.1.2's team): 256 consecutive elements share one
    countdown and vote by majority, so a ragged last block is a group of its
    own; with a threshold no finite RSD reaches every block follows the h,
    then (p approximate + 1 accurate) pattern; threshold 0 is exact; and a
    block decides for elements that, deciding alone, disagree."""
    h, p = 3, 2
    s, recs = run(9, 20, eos=(h, p, 1e300, 256), hg=(h, p, 1e300, 256))
    for region in ("dec_eos", "dec_hg"):
        dec = np.stack([r[region] for r in recs])  # (steps, blocks)
        assert dec.shape[1] == -(-9 ** 3 // 256)
        expect = [0] * h + ([1] * p + [0]) * 10
        assert all(list(dec[:, b]) == expect[:20] for b in range(dec.shape[1]))
    ref, _ = run(8, 40)
    s, _ = run(8, 40, eos=(4, 4, 0.0, 256), hg=(2, 3, 0.0, 256))
    assert same_state(s, ref)
    _, rt = run(10, 60, eos=(4, 4, 0.01, 1))
    split = 0  # blocks whose elements, deciding alone, disagree at some step
    for r in rt:
        t = r["dec_eos"][:(len(r["dec_eos"]) // 256) * 256].reshape(-1, 256)
        split += int(np.sum((t == 1).any(axis=1) & (t == 0).any(axis=1)))
    assert split > 0


def test_numeric_failure_flags_of_a_tangling_run():
    """The failure path: with the volume-change limit lifted (dvmax 10), a
    Courant factor of 3 and a time step allowed to double every step, the
    blast tangles the mesh within a few tens of steps and the oracle
    reports a non-positive element volume; with the workload's own
    constants (Courant factor 0.3, dvmax 0.1) no step is flagged."""
    n = 10
    s = oracle.hydro_init(n, (1.0 / 8) * n ** 3, cfl=3.0, dvmax=10.0, growth=2.0)
    first = None
    for k in range(60):
        oracle.hydro_step(s, k)
        if s.flags and first is None:
            first = k
    assert s.flags & 1 and first is not None and first < 40
    ok = oracle.hydro_init(n, (1.0 / 8) * n ** 3)
    for k in range(150):
        oracle.hydro_step(ok, k)
    assert ok.flags == 0

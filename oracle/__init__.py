"""CPU oracle for the approximated-region hot path of HPAC-Offload
(arXiv 2308.16877) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never calls it and shares no code
with it.  The arithmetic lives in ``oracle.c``, ``hydro.c`` and ``binomial.c`` (plain
C, FP64, built with gcc); this module only marshals numpy arrays into them.

Conventions: inputs are float32 columns (the region's declared input type),
region values are float64.  ``region_values_f32out`` rounds the exact FP64
region outputs to float32, the region's declared output type, because the
approximation engine stores and reuses what the region writes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "hydro.c"), os.path.join(_HERE, "binomial.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# perforation kinds (section 2.3: small, large, ini, fini)
PERFO_SMALL, PERFO_LARGE, PERFO_INI, PERFO_FINI = 0, 1, 2, 3
# decision groups (section 3.1.2): thread = 1 lane, wave = 64 lanes
GROUP_THREAD, GROUP_WAVE = 1, 64


def build(force=True):
    """Compile liboracle.so with gcc (FP64, no FP contraction, OpenMP)."""
    if not force and not _stale():
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp] + _SRCS + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _stale():
    return not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _stale():
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, f32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_double
    lib.or_num_lanes.restype = i64
    lib.or_num_lanes.argtypes = [i64, i32]
    lib.or_bs_price.restype = None
    lib.or_bs_price.argtypes = [i64] + [P] * 9
    lib.or_bs_jacobian.restype = None
    lib.or_bs_jacobian.argtypes = [i64] + [P] * 6
    lib.or_iact.restype = ctypes.c_int
    lib.or_iact.argtypes = [i64, i32, i32, i32, P, i32, P, P, i32, f32, i32, P, P, P, P, P, P, P, i32, f64, P]
    lib.or_adam.restype = None
    lib.or_adam.argtypes = [i64, i64, P, P, P, P, f64, f64, f64, f64, i32]
    lib.or_taf.restype = ctypes.c_int
    lib.or_taf.argtypes = [i64, i32, i32, i32, P, P, i32, i32, f32, f64, P, P, P, P, P, P, P, P]
    lib.or_perfo.restype = ctypes.c_int
    lib.or_perfo.argtypes = [i64, i32, i32, P, P, i32, i32, i32, P, P, P, P]
    lib.or_mape.restype = None
    lib.or_mape.argtypes = [i64, P, P, f64, P, P, P]
    lib.or_mlp_num_params.restype = i32
    lib.or_mlp_num_params.argtypes = []
    lib.or_bf16.restype = f64
    lib.or_bf16.argtypes = [f64]
    lib.or_mlp_gelu.restype = f64
    lib.or_mlp_gelu.argtypes = [f64]
    lib.or_mlp_forward.restype = None
    lib.or_mlp_forward.argtypes = [i64, P, P, P, P, P, P, P, i32, i32, P]
    lib.or_mlp_loss_grad.restype = f64
    lib.or_mlp_loss_grad.argtypes = [i64, P, P, P, P, P, P, P, P, i32, P]
    lib.or_binomial.restype = None
    lib.or_binomial.argtypes = [i64, P, P, P, P, P, i32, i32, P, P, P]
    lib.hy_init.restype = ctypes.c_int
    lib.hy_init.argtypes = [P, f64, P]
    lib.hy_step.restype = ctypes.c_int
    lib.hy_step.argtypes = [P, P, i32, P, P]
    lib.hy_energy.restype = None
    lib.hy_energy.argtypes = [P, P, P, P]
    lib.hy_hex_volume.restype = f64
    lib.hy_hex_volume.argtypes = [P, P]
    lib.hy_hex_hourglass.restype = None
    lib.hy_hex_hourglass.argtypes = [P, P, f64, f64, f64, P]
    _lib = lib
    return lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _cols(arrs):
    arr = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    return arr


def _as_f32_cols(x):
    return [np.ascontiguousarray(c, dtype=np.float32) for c in x]


def _as_f64_cols(y):
    return [np.ascontiguousarray(np.atleast_1d(c), dtype=np.float64) for c in y]


def num_lanes(n, ipt):
    """Number of logical lanes L of the grid-stride mapping."""
    return int(_load().or_num_lanes(int(n), int(ipt)))


def num_waves(n, ipt):
    return num_lanes(n, ipt) // 64


def bs_price(S, K, T, r, v):
    """Exact European call and put prices in FP64 and their tolerance scales.
    Inputs of any float type are taken at their exact value (float32 inputs
    upcast exactly)."""
    S, K, T, r, v = _as_f64_cols([S, K, T, r, v])
    n = S.size
    C, P, sC, sP = (np.empty(n, np.float64) for _ in range(4))
    _load().or_bs_price(n, *map(_ptr, (S, K, T, r, v, C, P, sC, sP)))
    return C, P, sC, sP


def bs_jacobian(S, K, T, r, v):
    """Closed-form Jacobian d(C, P)/d(S, K, T, r, v): array (10, n)."""
    S, K, T, r, v = _as_f64_cols([S, K, T, r, v])
    n = S.size
    J = np.empty((10, n), np.float64)
    rows = [J[j] for j in range(10)]
    _load().or_bs_jacobian(n, *map(_ptr, (S, K, T, r, v)), _cols(rows))
    return J


def region_values_f32out(x):
    """Black-Scholes region values as the FP32 output array holds them:
    (y, scale) with y = exact FP64 prices rounded to float32."""
    C, P, sC, sP = bs_price(*x)
    y = np.stack([C.astype(np.float32).astype(np.float64), P.astype(np.float32).astype(np.float64)])
    return y, np.stack([sC, sP])


def _out_arrays(n_out, n, out_init):
    if out_init is None:
        out = np.zeros((n_out, n), np.float64)
    else:
        out = np.array(out_init, dtype=np.float64, copy=True).reshape(n_out, n)
    return out, np.zeros((n_out, n), np.float64)


def iact(x, y, s, ipt, table_size, threshold, tables_per_wave=1, group=GROUP_WAVE, out_init=None,
         dist_fp64=False, band=0.0):
    """iACT engine over region values y (n_out, n) for inputs x (n_in, n).
    dist_fp64 takes the squared distance and its threshold test in FP64 (the
    plain definition) instead of FP32 with the fixed rounding order; band > 0
    marks the (wave, step) records where the other precision could choose
    differently (`fragile`)."""
    x = _as_f32_cols(x)
    y = _as_f64_cols(y)
    s = _as_f64_cols(s) if s is not None else [np.zeros_like(c) for c in y]
    n = x[0].size
    out, osc = _out_arrays(len(y), n, out_init)
    W = num_waves(n, ipt)
    dec = np.empty(W * ipt, np.int8)
    votes = np.empty(W * ipt, np.int16)
    writer = np.empty(W * ipt, np.int16)
    napprox = np.empty(W * ipt, np.int16)
    fragile = np.empty(W * ipt, np.uint8)
    evals = ctypes.c_int64(0)
    rc = _load().or_iact(n, ipt, group, len(x), _cols(x), len(y), _cols(y), _cols(s),
                         table_size, np.float32(threshold), tables_per_wave,
                         _cols(list(out)), _cols(list(osc)), _ptr(dec), _ptr(votes),
                         _ptr(writer), _ptr(napprox), ctypes.byref(evals), int(bool(dist_fp64)), float(band),
                         _ptr(fragile) if band > 0 else None)
    if rc != 0:
        raise ValueError("or_iact rejected its arguments")
    if band <= 0:
        fragile[:] = 0
    return dict(out=out, scale=osc, dec=dec, votes=votes, writer=writer,
                napprox=napprox, evals=evals.value, ipt=ipt, fragile=fragile)


def adam(partials, w, m, v, lr, beta1, beta2, eps, step):
    """One Adam step in FP64 on copies of w, m, v (arrays of p); partials is
    (blocks, p), summed to the gradient.  Returns (w, m, v)."""
    partials = np.ascontiguousarray(np.atleast_2d(partials), dtype=np.float64)
    w, m, v = (np.array(a, dtype=np.float64, copy=True) for a in (w, m, v))
    blocks, p = partials.shape
    _load().or_adam(p, blocks, _ptr(partials), _ptr(w), _ptr(m), _ptr(v), float(lr), float(beta1), float(beta2),
                    float(eps), int(step))
    return w, m, v


class _TafState(ctypes.Structure):
    _fields_ = [("win", ctypes.c_void_p), ("last", ctypes.c_void_p), ("lasts", ctypes.c_void_p),
                ("fill", ctypes.c_void_p), ("rho", ctypes.c_void_p)]


def taf_state(n, ipt, history_size, n_out=2):
    """A fresh state for TAF launches of this shape carrying windows and
    countdowns across launches (numpy arrays, updated in place by taf())."""
    L = num_lanes(n, ipt)
    return dict(win=np.zeros(L * n_out * history_size), last=np.zeros(L * n_out), lasts=np.zeros(L * n_out),
                fill=np.zeros(L, np.int32), rho=np.zeros(L, np.int32), shape=(n, ipt, history_size, n_out))


def taf(y, s, ipt, history_size, prediction_size, threshold, band=0.0, group=GROUP_WAVE, out_init=None,
        state=None):
    """TAF engine over region values y (n_out, n); with state (taf_state),
    the launch starts from it and leaves its end state in it."""
    y = _as_f64_cols(y)
    s = _as_f64_cols(s) if s is not None else [np.zeros_like(c) for c in y]
    n = y[0].size
    out, osc = _out_arrays(len(y), n, out_init)
    W = num_waves(n, ipt)
    dec = np.empty(W * ipt, np.int8)
    votes = np.empty(W * ipt, np.int16)
    fragile = np.empty(W * ipt, np.uint8)
    napprox = np.empty(W * ipt, np.int16)
    evals = ctypes.c_int64(0)
    st = None
    if state is not None:
        assert state["shape"] == (n, ipt, history_size, len(y)), "state of another launch shape"
        st = _TafState(*[_ptr(state[k]) for k in ("win", "last", "lasts", "fill", "rho")])
    rc = _load().or_taf(n, ipt, group, len(y), _cols(y), _cols(s), history_size, prediction_size,
                        np.float32(threshold), float(band), _cols(list(out)), _cols(list(osc)),
                        _ptr(dec), _ptr(votes), _ptr(fragile), _ptr(napprox), ctypes.byref(evals),
                        ctypes.byref(st) if st is not None else None)
    if rc != 0:
        raise ValueError("or_taf rejected its arguments")
    return dict(out=out, scale=osc, dec=dec, votes=votes, fragile=fragile,
                napprox=napprox, evals=evals.value, ipt=ipt)


def perfo(y, s, ipt, kind, param, offset=0, out_init=None):
    """Herded perforation over region values y (n_out, n)."""
    y = _as_f64_cols(y)
    s = _as_f64_cols(s) if s is not None else [np.zeros_like(c) for c in y]
    n = y[0].size
    out, osc = _out_arrays(len(y), n, out_init)
    W = num_waves(n, ipt)
    dec = np.empty(W * ipt, np.int8)
    evals = ctypes.c_int64(0)
    rc = _load().or_perfo(n, ipt, len(y), _cols(y), _cols(s), kind, param, offset,
                          _cols(list(out)), _cols(list(osc)), _ptr(dec), ctypes.byref(evals))
    if rc != 0:
        raise ValueError("or_perfo rejected its arguments")
    return dict(out=out, scale=osc, dec=dec, evals=evals.value, ipt=ipt)


MAPE_TAU = 1e-2  # price-unit floor of the MAPE denominator


def mape(exact, approx, tau=MAPE_TAU):
    """MAPE as a fraction with floored denominator; returns
    (mape, number of floored entries, MAPE over the unfloored entries)."""
    e = np.ascontiguousarray(np.ravel(exact), np.float64)
    a = np.ascontiguousarray(np.ravel(approx), np.float64)
    assert e.size == a.size
    m = ctypes.c_double(0)
    nf = ctypes.c_int64(0)
    mr = ctypes.c_double(0)
    _load().or_mape(e.size, _ptr(e), _ptr(a), float(tau), ctypes.byref(m), ctypes.byref(nf), ctypes.byref(mr))
    return m.value, nf.value, mr.value


# ---------------------------------------------------------------- surrogate

def mlp_num_params():
    return int(_load().or_mlp_num_params())


def bf16(v):
    """Nearest BF16 value (ties to even) of each element, as float64."""
    f = _load().or_bf16
    return np.vectorize(lambda a: f(float(a)))(np.asarray(v, np.float64))


def _norm_arrays(norm):
    """in_center, in_scale, out_mean, out_scale and out_shift (zeros when absent)."""
    arrs = [np.ascontiguousarray(norm[k], np.float64) for k in ("in_center", "in_scale", "out_mean", "out_scale")]
    return arrs + [np.ascontiguousarray(norm.get("out_shift", np.zeros(2)), np.float64)]


def mlp_forward(x, params, norm, round_act=True, act=True):
    """Surrogate outputs (2, n) in FP64 on BF16-rounded weights; with
    round_act the layer inputs are rounded to BF16 as the GPU's MFMA path does."""
    x = _as_f64_cols(x)
    n = x[0].size
    w = np.ascontiguousarray(params, np.float64)
    assert w.size == mlp_num_params()
    c, s, mu, sc, sh = _norm_arrays(norm)
    y = np.empty((2, n), np.float64)
    _load().or_mlp_forward(n, _cols(x), _ptr(w), _ptr(c), _ptr(s), _ptr(mu), _ptr(sc), _ptr(sh), int(round_act),
                           int(act), _cols([y[0], y[1]]))
    return y


def mlp_loss_grad(x, targets, params, norm, act=True):
    """(loss, gradient) of the mean squared error in normalised output space."""
    x = _as_f64_cols(x)
    t = _as_f64_cols(targets)
    n = x[0].size
    w = np.ascontiguousarray(params, np.float64)
    c, s, mu, sc, sh = _norm_arrays(norm)
    g = np.empty(mlp_num_params(), np.float64)
    loss = _load().or_mlp_loss_grad(n, _cols(x), _cols(t), _ptr(w), _ptr(c), _ptr(s), _ptr(mu), _ptr(sc), _ptr(sh),
                                    int(act), _ptr(g))
    return loss, g


def gelu(v):
    f = _load().or_mlp_gelu
    return np.vectorize(lambda a: f(float(a)))(np.asarray(v, np.float64))


# ---------------------------------------------------------------- hydro

class _HyPar(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("side", ctypes.c_double), ("gamma", ctypes.c_double),
                ("cq", ctypes.c_double), ("cl", ctypes.c_double), ("khg", ctypes.c_double),
                ("cfl", ctypes.c_double), ("growth", ctypes.c_double), ("dvmax", ctypes.c_double),
                ("dt0", ctypes.c_double)]


class _HyState(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p * 3), ("u", ctypes.c_void_p * 3), ("unew", ctypes.c_void_p * 3)] + \
               [(f, ctypes.c_void_p) for f in ("mnode", "e", "p", "q", "c", "vol", "mass", "force", "fhg",
                                                "weos", "rho_eos", "z_eos", "whg", "rho_hg", "z_hg", "clock")]


class _HyTech(ctypes.Structure):
    _fields_ = [("eos_h", ctypes.c_int32), ("eos_p", ctypes.c_int32), ("eos_theta", ctypes.c_double),
                ("eos_group", ctypes.c_int32),
                ("hg_h", ctypes.c_int32), ("hg_p", ctypes.c_int32), ("hg_theta", ctypes.c_double),
                ("hg_group", ctypes.c_int32),
                ("perfo_kind", ctypes.c_int32), ("perfo_param", ctypes.c_int32), ("perfo_ipt", ctypes.c_int32),
                ("band", ctypes.c_double)]


class _HyRec(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in ("dec_eos", "dec_hg", "frag_eos", "frag_hg")]


HYDRO_DEFAULTS = dict(side=1.0, gamma=1.4, cq=1.5, cl=0.25, khg=0.1, cfl=0.3, growth=1.1, dvmax=0.1, dt0=1e-7)


class HydroState:
    """FP64 state of the oracle hydro on an n^3 mesh (numpy arrays, the C
    layout): x, u (3, nodes); e, p, q, c, vol, mass (elements); force, fhg
    (24, elements); TAF windows weos (h*4, E), whg (h*24, E) and per-wave
    counters; clock = [time, last dt]."""

    def __init__(self, n, eos_h=0, hg_h=0, **par):
        self.par = dict(HYDRO_DEFAULTS, **par)
        self.n = int(n)
        E, Nn = self.n ** 3, (self.n + 1) ** 3
        W = (E + 63) // 64
        self.E, self.Nn, self.W = E, Nn, W
        z = lambda *sh: np.zeros(sh, np.float64)
        self.x, self.u, self.unew = z(3, Nn), z(3, Nn), z(3, Nn)
        self.mnode = z(Nn)
        self.e, self.p, self.q, self.c, self.vol, self.mass = (z(E) for _ in range(6))
        self.force, self.fhg = z(24, E), z(24, E)
        self.weos = z(max(eos_h, 1) * 4, E)
        self.whg = z(max(hg_h, 1) * 24, E)
        # decision-group state, sized for one group per element (thread level)
        self.rho_eos, self.z_eos, self.rho_hg, self.z_hg = (np.zeros(E, np.int32) for _ in range(4))
        self.clock = z(2)
        self.eos_h, self.hg_h = eos_h, hg_h
        self.flags = 0  # numeric-failure flags of the steps taken (see hydro_step)

    def _cpar(self):
        return _HyPar(n=self.n, **self.par)

    def _cstate(self):
        for a in ("x", "u", "unew", "mnode", "e", "p", "q", "c", "vol", "mass", "force", "fhg", "weos", "whg",
                  "clock"):
            arr = getattr(self, a)
            assert arr.dtype == np.float64 and arr.flags.c_contiguous, a
        for a in ("rho_eos", "z_eos", "rho_hg", "z_hg"):
            arr = getattr(self, a)
            assert arr.dtype == np.int32 and arr.flags.c_contiguous, a
        st = _HyState()
        for d in range(3):
            st.x[d] = self.x[d].ctypes.data
            st.u[d] = self.u[d].ctypes.data
            st.unew[d] = self.unew[d].ctypes.data
        for f in ("mnode", "e", "p", "q", "c", "vol", "mass", "force", "fhg", "weos", "rho_eos", "z_eos", "whg",
                  "rho_hg", "z_hg", "clock"):
            setattr(st, f, getattr(self, f).ctypes.data)
        return st

    @property
    def time(self):
        return float(self.clock[0])

    def copy(self):
        c = HydroState.__new__(HydroState)
        for k, v in self.__dict__.items():
            c.__dict__[k] = v.copy() if isinstance(v, np.ndarray) else (dict(v) if isinstance(v, dict) else v)
        return c


def hydro_init(n, e_origin, eos_h=0, hg_h=0, **par):
    """Initial Sedov state: unit density at rest, specific energy e_origin in
    the element at the origin."""
    s = HydroState(n, eos_h=eos_h, hg_h=hg_h, **par)
    cp, cs = s._cpar(), s._cstate()
    if _load().hy_init(ctypes.byref(cp), float(e_origin), ctypes.byref(cs)) != 0:
        raise ValueError("hy_init rejected its arguments")
    return s


def hydro_step(s, step, eos=None, hg=None, perfo=None, band=0.0, record=False):
    """One timestep in place.  eos / hg = (h, p, theta[, group]) for TAF on
    the EOS / hourglass region, group = 64 (wave level, the default), 1
    (thread level) or 256 (block level, four waves); perfo = (kind, param, items_per_lane) for the hourglass
    region.  With record, returns per-group decisions and fragile flags
    {dec_eos, dec_hg, frag_eos, frag_hg}."""
    t = _HyTech(band=float(band), eos_group=GROUP_WAVE, hg_group=GROUP_WAVE)
    if eos:
        assert eos[0] <= s.eos_h
        t.eos_h, t.eos_p, t.eos_theta = int(eos[0]), int(eos[1]), float(eos[2])
        t.eos_group = int(eos[3]) if len(eos) > 3 else GROUP_WAVE
    if hg:
        assert hg[0] <= s.hg_h
        t.hg_h, t.hg_p, t.hg_theta = int(hg[0]), int(hg[1]), float(hg[2])
        t.hg_group = int(hg[3]) if len(hg) > 3 else GROUP_WAVE
    if perfo:
        t.perfo_kind, t.perfo_param, t.perfo_ipt = int(perfo[0]), int(perfo[1]), int(perfo[2])
    rec, out = None, None
    if record:
        ne, nh = -(-s.E // t.eos_group), -(-s.E // t.hg_group)
        out = dict(dec_eos=np.full(ne, -1, np.int8), dec_hg=np.full(nh, -1, np.int8),
                   frag_eos=np.zeros(ne, np.uint8), frag_hg=np.zeros(nh, np.uint8))
        rec = _HyRec(**{k: v.ctypes.data for k, v in out.items()})
    cp, cs = s._cpar(), s._cstate()
    rc = _load().hy_step(ctypes.byref(cp), ctypes.byref(t), int(step), ctypes.byref(cs),
                         ctypes.byref(rec) if rec is not None else None)
    if rc < 0:
        raise ValueError("hy_step rejected its arguments")
    # numeric-failure flags (1: a non-positive element volume, 2: a time step
    # that is not finite and positive), accumulated over the steps taken
    s.flags |= rc
    return out


def hydro_energy(s):
    """(internal, kinetic) energy of the state."""
    ie, ke = ctypes.c_double(), ctypes.c_double()
    _load().hy_energy(ctypes.byref(s._cpar()), ctypes.byref(s._cstate()), ctypes.byref(ie), ctypes.byref(ke))
    return ie.value, ke.value


def hex_volume(xc):
    """Volume and its gradient (8, 3) of a hexahedron with corners xc (8, 3)
    in the local order a + 2b + 4c."""
    xc = np.ascontiguousarray(xc, np.float64).reshape(8, 3)
    B = np.zeros((8, 3))
    V = _load().hy_hex_volume(_ptr(xc), _ptr(B))
    return V, B


def hex_hourglass(xc, uc, rho, c, khg):
    """Hourglass corner forces (8, 3) of one hexahedron."""
    xc = np.ascontiguousarray(xc, np.float64).reshape(8, 3)
    uc = np.ascontiguousarray(uc, np.float64).reshape(8, 3)
    f = np.zeros((8, 3))
    _load().hy_hex_hourglass(_ptr(xc), _ptr(uc), float(rho), float(c), float(khg), _ptr(f))
    return f


# ------------------------------------------------------------ binomial

def binomial(S, K, T, r, v, steps, american=True):
    """(call, put, scale) of the Cox-Ross-Rubinstein tree with `steps` time
    steps, American or European exercise; scale = S + K e^{-rT}."""
    cols = _as_f64_cols([S, K, T, r, v])
    n = cols[0].size
    C, P, sc = np.zeros(n), np.zeros(n), np.zeros(n)
    _load().or_binomial(n, *[_ptr(c) for c in cols], int(steps), int(bool(american)), _ptr(C), _ptr(P), _ptr(sc))
    return C, P, sc

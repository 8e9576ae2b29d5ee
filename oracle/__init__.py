"""CPU oracle for the approximated-region hot path of HPAC-Offload
(arXiv 2308.16877) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never calls it and shares no code
with it.  The arithmetic lives in ``oracle.c`` (plain C, FP64, built with
gcc); this module only marshals numpy arrays into it.

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
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# perforation kinds (section 2.3: small, large, ini, fini)
PERFO_SMALL, PERFO_LARGE, PERFO_INI, PERFO_FINI = 0, 1, 2, 3
# decision groups (section 3.1.2): thread = 1 lane, wave = 64 lanes
GROUP_THREAD, GROUP_WAVE = 1, 64


def build(force=True):
    """Compile liboracle.so with gcc (FP64, no FP contraction, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
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
    lib.or_iact.argtypes = [i64, i32, i32, i32, P, i32, P, P, i32, f32, i32, P, P, P, P, P, P, P]
    lib.or_taf.restype = ctypes.c_int
    lib.or_taf.argtypes = [i64, i32, i32, i32, P, P, i32, i32, f32, f64, P, P, P, P, P, P, P]
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
    lib.or_mlp_forward.argtypes = [i64, P, P, P, P, P, P, i32, i32, P]
    lib.or_mlp_loss_grad.restype = f64
    lib.or_mlp_loss_grad.argtypes = [i64, P, P, P, P, P, P, P, i32, P]
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


def iact(x, y, s, ipt, table_size, threshold, tables_per_wave=1, group=GROUP_WAVE, out_init=None):
    """iACT engine over region values y (n_out, n) for inputs x (n_in, n)."""
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
    evals = ctypes.c_int64(0)
    rc = _load().or_iact(n, ipt, group, len(x), _cols(x), len(y), _cols(y), _cols(s),
                         table_size, np.float32(threshold), tables_per_wave,
                         _cols(list(out)), _cols(list(osc)), _ptr(dec), _ptr(votes),
                         _ptr(writer), _ptr(napprox), ctypes.byref(evals))
    if rc != 0:
        raise ValueError("or_iact rejected its arguments")
    return dict(out=out, scale=osc, dec=dec, votes=votes, writer=writer,
                napprox=napprox, evals=evals.value, ipt=ipt)


def taf(y, s, ipt, history_size, prediction_size, threshold, band=0.0, group=GROUP_WAVE, out_init=None):
    """TAF engine over region values y (n_out, n)."""
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
    rc = _load().or_taf(n, ipt, group, len(y), _cols(y), _cols(s), history_size, prediction_size,
                        np.float32(threshold), float(band), _cols(list(out)), _cols(list(osc)),
                        _ptr(dec), _ptr(votes), _ptr(fragile), _ptr(napprox), ctypes.byref(evals))
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
    return [np.ascontiguousarray(norm[k], np.float64) for k in ("in_center", "in_scale", "out_mean", "out_scale")]


def mlp_forward(x, params, norm, round_act=True, act=True):
    """Surrogate outputs (2, n) in FP64 on BF16-rounded weights; with
    round_act the layer inputs are rounded to BF16 as the GPU's MFMA path does."""
    x = _as_f64_cols(x)
    n = x[0].size
    w = np.ascontiguousarray(params, np.float64)
    assert w.size == mlp_num_params()
    c, s, mu, sc = _norm_arrays(norm)
    y = np.empty((2, n), np.float64)
    _load().or_mlp_forward(n, _cols(x), _ptr(w), _ptr(c), _ptr(s), _ptr(mu), _ptr(sc), int(round_act), int(act),
                           _cols([y[0], y[1]]))
    return y


def mlp_loss_grad(x, targets, params, norm, act=True):
    """(loss, gradient) of the mean squared error in normalised output space."""
    x = _as_f64_cols(x)
    t = _as_f64_cols(targets)
    n = x[0].size
    w = np.ascontiguousarray(params, np.float64)
    c, s, mu, sc = _norm_arrays(norm)
    g = np.empty(mlp_num_params(), np.float64)
    loss = _load().or_mlp_loss_grad(n, _cols(x), _cols(t), _ptr(w), _ptr(c), _ptr(s), _ptr(mu), _ptr(sc),
                                    int(act), _ptr(g))
    return loss, g


def gelu(v):
    f = _load().or_mlp_gelu
    return np.vectorize(lambda a: f(float(a)))(np.asarray(v, np.float64))

"""Python binding of libhpac.so: argument marshalling only.

Every function here has the name of the C entry point it calls (include/
hpac.h) and forwards device pointers and sizes; all work runs in the HIP
kernels.  Columns may be torch tensors on the GPU (float32, contiguous, one
dimension) or raw device addresses (ints).  The stream defaults to torch's
current stream.  A missing library raises; there is no fallback path.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhpac.so")

HPAC_OK, HPAC_EINVAL, HPAC_EUNSUPPORTED, HPAC_EHIP, HPAC_ENUMERIC = 0, -1, -2, -3, -4
HYDRO_BAD_VOLUME, HYDRO_BAD_DT = 1, 2
HYDRO_NOALLOC_MAX_N = 256
REGION_BS_PRICE, REGION_BS_PRICE_GRAD, REGION_BS_PRICE_F16, REGION_BS_PRICE_BF16 = 0, 1, 2, 3
REGION_BINOMIAL = 4
REGION_BS_PRICE_REF = 5
REGION_SHAPE = {REGION_BS_PRICE: (5, 2), REGION_BS_PRICE_GRAD: (5, 12), REGION_BS_PRICE_F16: (5, 2),
                REGION_BS_PRICE_BF16: (5, 2), REGION_BINOMIAL: (5, 2), REGION_BS_PRICE_REF: (5, 3)}
F32, F16, BF16 = 0, 1, 2
LEVEL_THREAD, LEVEL_WAVE, LEVEL_BLOCK = 0, 1, 2
LEVELS = {"thread": LEVEL_THREAD, "wave": LEVEL_WAVE, "warp": LEVEL_WAVE, "block": LEVEL_BLOCK, "team": LEVEL_BLOCK}
PERFO_SMALL, PERFO_LARGE, PERFO_INI, PERFO_FINI = 0, 1, 2, 3
PERFO_KINDS = {"small": PERFO_SMALL, "large": PERFO_LARGE, "ini": PERFO_INI, "fini": PERFO_FINI}
NUM_COUNTERS = 4


class hpac_region_io(ctypes.Structure):
    _fields_ = [
        ("region", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("in_", ctypes.POINTER(ctypes.c_void_p)),
        ("n_in", ctypes.c_int32),
        ("out", ctypes.POINTER(ctypes.c_void_p)),
        ("n_out", ctypes.c_int32),
        ("items_per_lane", ctypes.c_int32),
        ("block_size", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("trace", ctypes.c_void_p),
        ("counters", ctypes.c_void_p),
    ]


class hpac_mlp_norm(ctypes.Structure):
    _fields_ = [("in_center", ctypes.c_float * 5), ("in_scale", ctypes.c_float * 5),
                ("out_mean", ctypes.c_float * 2), ("out_scale", ctypes.c_float * 2),
                ("out_shift", ctypes.c_float * 2)]


MLP_NUM_PARAMS = 4674


def make_norm(in_center, in_scale, out_mean, out_scale, out_shift=(0.0, 0.0)):
    return hpac_mlp_norm((ctypes.c_float * 5)(*map(float, in_center)), (ctypes.c_float * 5)(*map(float, in_scale)),
                         (ctypes.c_float * 2)(*map(float, out_mean)), (ctypes.c_float * 2)(*map(float, out_scale)),
                         (ctypes.c_float * 2)(*map(float, out_shift)))


class HpacError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (status %d)" % (message, status))
        self.status = status


class hpac_hydro_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32)] + [(f, ctypes.c_double) for f in
                                          ("side", "gamma", "cq", "cl", "khg", "cfl", "growth", "dvmax", "dt0")]


class hpac_hydro_state(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p * 3), ("u", ctypes.c_void_p * 3), ("unew", ctypes.c_void_p * 3)] + \
               [(f, ctypes.c_void_p) for f in ("mnode", "e", "p", "q", "c", "vol", "mass", "force", "weos",
                                                "rho_eos", "z_eos", "whg", "rho_hg", "z_hg", "clock",
                                                "dt_partials", "status")]


class hpac_hydro_tech(ctypes.Structure):
    _fields_ = [("eos_history", ctypes.c_int32), ("eos_prediction", ctypes.c_int32),
                ("eos_threshold", ctypes.c_float), ("eos_level", ctypes.c_int32), ("hg_history", ctypes.c_int32),
                ("hg_prediction", ctypes.c_int32), ("hg_threshold", ctypes.c_float), ("hg_level", ctypes.c_int32),
                ("perfo_kind", ctypes.c_int32), ("perfo_param", ctypes.c_int32),
                ("perfo_items_per_lane", ctypes.c_int32)]


_lib = None


def lib():
    """Load libhpac.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhpac.so is not built; run `python -m paper_2308_16877_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    IO = ctypes.POINTER(hpac_region_io)
    i32, i64, f32, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p
    L.hpac_exact.argtypes = [IO]
    L.hpac_iact.argtypes = [IO, i32, f32, i32, i32]
    L.hpac_taf.argtypes = [IO, i32, i32, f32, i32, vp]
    L.hpac_taf_state_bytes.argtypes = [i32, i64, i32, i32]
    L.hpac_taf_state_bytes.restype = i64
    L.hpac_perfo.argtypes = [IO, i32, i32, i32]
    L.hpac_probe_copy.argtypes = [vp, vp, i64, vp]
    L.hpac_probe_valu.argtypes = [vp, i32, i32, i32, vp]
    L.hpac_probe_valu.restype = i32
    PP = ctypes.POINTER(ctypes.c_void_p)
    NP = ctypes.POINTER(hpac_mlp_norm)
    FP = ctypes.POINTER(ctypes.c_float)
    L.hpac_surrogate.argtypes = [IO, vp, NP, FP, FP, vp, vp]
    L.hpac_mlp_grad_blocks.argtypes = [i64]
    L.hpac_mlp_grad_blocks.restype = i64
    L.hpac_mlp_grad.argtypes = [i64, PP, PP, vp, NP, i64, vp, vp, vp]
    L.hpac_mlp_adam.argtypes = [vp, i64, vp, vp, vp, f32, f32, f32, f32, i32, vp]
    for f in (L.hpac_surrogate, L.hpac_mlp_grad, L.hpac_mlp_adam):
        f.restype = i32
    L.hpac_bs_vjp.argtypes = [i64, PP, vp, vp, PP, vp]
    L.hpac_bs_adjoint.argtypes = [i64, PP, vp, vp, PP, vp]
    L.hpac_bs_vjp_ref.argtypes = [i64, PP, vp, vp, vp, PP, vp]
    L.hpac_bs_vjp_ref.restype = i32
    for f in (L.hpac_exact, L.hpac_iact, L.hpac_taf, L.hpac_perfo, L.hpac_probe_copy, L.hpac_bs_vjp,
              L.hpac_bs_adjoint):
        f.restype = i32
    HP, HS, HT = (ctypes.POINTER(t) for t in (hpac_hydro_params, hpac_hydro_state, hpac_hydro_tech))
    L.hpac_hydro_waves.argtypes = [i32]
    L.hpac_hydro_waves.restype = i64
    L.hpac_hydro_groups.argtypes = [i32, i32]
    L.hpac_hydro_groups.restype = i64
    L.hpac_hydro_partials.argtypes = [i32]
    L.hpac_hydro_partials.restype = i64
    L.hpac_hydro_init.argtypes = [HP, ctypes.c_double, HS, vp]
    L.hpac_hydro_init.restype = i32
    L.hpac_hydro_step.argtypes = [HP, HT, i32, HS, vp, vp, vp]
    L.hpac_hydro_step.restype = i32
    L.hpac_hydro_step_noalloc.argtypes = [HP, HT, i32, HS, vp, vp, vp]
    L.hpac_hydro_step_noalloc.restype = i32
    L.hpac_hydro_run.argtypes = [HP, HT, i32, i32, HS, vp]
    L.hpac_hydro_run.restype = i32
    L.hpac_hydro_check.argtypes = [HS, vp]
    L.hpac_hydro_check.restype = i32
    L.hpac_bo_units.argtypes = [i64, i32]
    L.hpac_bo_units.restype = i64
    L.hpac_bo_exact.argtypes = [IO, i32, i32]
    L.hpac_bo_iact.argtypes = [IO, i32, i32, i32, f32]
    L.hpac_bo_taf.argtypes = [IO, i32, i32, i32, i32, f32]
    L.hpac_bo_perfo.argtypes = [IO, i32, i32, i32, i32, i32]
    for f in (L.hpac_bo_exact, L.hpac_bo_iact, L.hpac_bo_taf, L.hpac_bo_perfo):
        f.restype = i32
    L.hpac_num_lanes.argtypes = [i64, i32]
    L.hpac_num_lanes.restype = i64
    L.hpac_trace_entries.argtypes = [i64, i32]
    L.hpac_trace_entries.restype = i64
    L.hpac_last_error.argtypes = []
    L.hpac_last_error.restype = ctypes.c_char_p
    L.hpac_abi_version.argtypes = []
    L.hpac_abi_version.restype = i32
    _lib = L
    return L


def _addr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("columns must be GPU tensors")
    return t.data_ptr()


# element types a device buffer argument may have, by kind
_KINDS = {"u32": ("int32", "uint32"), "u64": ("int64", "uint64"), "i32": ("int32",), "i8": ("int8", "uint8"),
          "f32": ("float32",), "f64": ("float64",), "bytes": None}


def _check_buf(t, need, kind, what):
    """A device buffer the kernels write or read beyond the columns: a torch
    tensor must be contiguous, of the element type `kind` and hold at least
    `need` elements (bytes for kind "bytes"), since a short buffer would be
    written out of bounds on the device.  Raw addresses (ints) are the
    caller's responsibility; None passes (optional buffers)."""
    if t is None or isinstance(t, int):
        return
    allowed = _KINDS[kind]
    dt = str(t.dtype).replace("torch.", "")
    if allowed is not None and dt not in allowed:
        raise ValueError("%s must have element type %s, got %s" % (what, " or ".join(allowed), dt))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    have = t.numel() * (t.element_size() if allowed is None else 1)
    if have < need:
        raise ValueError("%s holds %d %s, the call needs at least %d" % (
            what, have, "bytes" if allowed is None else "elements", need))


def _dtype_code(t):
    import torch
    return {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}.get(t.dtype)


def _check_column(t, n, dtype=F32):
    if isinstance(t, int):
        return
    if _dtype_code(t) != dtype or t.dim() != 1 or not t.is_contiguous() or t.numel() != n:
        raise ValueError("each column must be a contiguous 1-D tensor of n elements of the call's dtype")


def _stream(stream, cols):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    if any(not isinstance(c, int) for c in cols):
        import torch
        return torch.cuda.current_stream().cuda_stream
    return None


def make_io(inputs, outputs, n=None, region=None, items_per_lane=1, block_size=0,
            stream=None, trace=None, counters=None, dtype=None):
    """Build the hpac_region_io descriptor (the arrays it points to are kept
    alive on the returned object).  dtype defaults to the columns' type."""
    inputs, outputs = list(inputs), list(outputs)
    if region is None:
        region = REGION_BS_PRICE if len(outputs) == 2 else REGION_BS_PRICE_GRAD
    if n is None:
        n = outputs[0].numel()
    if dtype is None:
        first = next((c for c in inputs + outputs if not isinstance(c, int)), None)
        dtype = F32 if first is None else _dtype_code(first)
    cols = inputs + outputs
    if region == REGION_BS_PRICE_REF and len(outputs) == 3:
        # the source-item column holds int32 indices
        _check_buf(outputs[2], n, "i32", "source column")
        if not isinstance(outputs[2], int) and outputs[2].numel() != n:
            raise ValueError("the source column must hold n elements")
        cols = inputs + outputs[:2]
    for c in cols:
        _check_column(c, n, dtype)
    if trace is not None and not isinstance(trace, int):
        if region == REGION_BINOMIAL:
            need = hpac_bo_units(n, items_per_lane) * items_per_lane
        else:
            need = hpac_trace_entries(n, items_per_lane)
        if need < 0:
            raise ValueError("n = %d or items_per_lane = %d out of range" % (n, items_per_lane))
        _check_buf(trace, need, "u32", "trace")
    _check_buf(counters, NUM_COUNTERS, "u64", "counters")
    ins = (ctypes.c_void_p * max(len(inputs), 1))(*[_addr(c) for c in inputs])
    outs = (ctypes.c_void_p * max(len(outputs), 1))(*[_addr(c) for c in outputs])
    io = hpac_region_io(region, dtype, n, ctypes.cast(ins, ctypes.POINTER(ctypes.c_void_p)), len(inputs),
                        ctypes.cast(outs, ctypes.POINTER(ctypes.c_void_p)), len(outputs),
                        items_per_lane, block_size, _stream(stream, inputs + outputs),
                        _addr(trace), _addr(counters))
    # keep the pointer arrays and the tensors they point into alive as long
    # as the descriptor (a prepared launch may be replayed much later)
    io._keep = (ins, outs, inputs, outputs, trace, counters)
    return io


def _call(name, status):
    if status != HPAC_OK:
        raise HpacError(status, "%s: %s" % (name, lib().hpac_last_error().decode()))


def _level(level):
    return LEVELS[level] if isinstance(level, str) else int(level)


def hpac_exact(inputs, outputs, **kw):
    io = make_io(inputs, outputs, **kw)
    _call("hpac_exact", lib().hpac_exact(ctypes.byref(io)))


def hpac_iact(inputs, outputs, table_size, threshold, tables_per_wave=1, level="wave", **kw):
    io = make_io(inputs, outputs, **kw)
    _call("hpac_iact", lib().hpac_iact(ctypes.byref(io), table_size, threshold, tables_per_wave, _level(level)))


def hpac_taf_state_bytes(region, n, items_per_lane, history_size):
    return int(lib().hpac_taf_state_bytes(int(region), int(n), int(items_per_lane), int(history_size)))


def hpac_taf(inputs, outputs, history_size, prediction_size, rsd_threshold, level="wave", state=None, **kw):
    """state: None (state within the launch) or a device buffer of
    hpac_taf_state_bytes(...) bytes, zeroed before the first launch of a
    sequence, carrying each lane's window and countdown across launches."""
    io = make_io(inputs, outputs, **kw)
    if state is not None:
        need = hpac_taf_state_bytes(io.region, io.n, io.items_per_lane, history_size)
        if need < 0:
            raise ValueError("hpac_taf: no persistent state for these arguments")
        _check_buf(state, need, "bytes", "state")
    _call("hpac_taf", lib().hpac_taf(ctypes.byref(io), history_size, prediction_size, rsd_threshold, _level(level),
                                     _addr(state)))


def hpac_perfo(inputs, outputs, kind, param, offset=0, **kw):
    io = make_io(inputs, outputs, **kw)
    k = PERFO_KINDS[kind] if isinstance(kind, str) else int(kind)
    _call("hpac_perfo", lib().hpac_perfo(ctypes.byref(io), k, param, offset))


class Prepared:
    """A launch whose argument marshalling is done once: calling it issues
    the same entry point with the same columns and parameters again on the
    given stream (default: the stream chosen at preparation).  For timing
    loops and serving loops where per-call Python work would dominate."""

    _ENTRY = {"exact": "hpac_exact", "iact": "hpac_iact", "taf": "hpac_taf", "perfo": "hpac_perfo"}

    def __init__(self, technique, inputs, outputs, params=(), **io_kw):
        self.name = self._ENTRY[technique]
        self.io = make_io(inputs, outputs, **io_kw)
        self.fn = getattr(lib(), self.name)
        self.args = (ctypes.byref(self.io),) + tuple(params)

    def __call__(self, stream=None):
        if stream is not None:
            self.io.stream = stream if isinstance(stream, int) else stream.cuda_stream
        st = self.fn(*self.args)
        if st != HPAC_OK:
            _call(self.name, st)


def prepare(technique, inputs, outputs, **kw):
    """Prepared launch of hpac_<technique>; keyword arguments as for the
    function of that name."""
    io_keys = ("n", "region", "items_per_lane", "block_size", "stream", "trace", "counters", "dtype")
    io_kw = {k: kw.pop(k) for k in list(kw) if k in io_keys}
    if technique == "iact":
        params = (kw.pop("table_size"), ctypes.c_float(kw.pop("threshold")), kw.pop("tables_per_wave", 1),
                  _level(kw.pop("level", "wave")))
    elif technique == "taf":
        params = (kw.pop("history_size"), kw.pop("prediction_size"), ctypes.c_float(kw.pop("rsd_threshold")),
                  _level(kw.pop("level", "wave")), None)
    elif technique == "perfo":
        k = kw.pop("kind")
        params = (PERFO_KINDS[k] if isinstance(k, str) else int(k), kw.pop("param"), kw.pop("offset", 0))
    else:
        params = ()
    if kw:
        raise TypeError("unexpected arguments: %s" % sorted(kw))
    return Prepared(technique, inputs, outputs, params, **io_kw)


def _ptr_array(cols):
    arr = (ctypes.c_void_p * len(cols))(*[_addr(c) for c in cols])
    return ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), arr


def hpac_bs_vjp(jacobian, grad_call, grad_put, grad_in, n=None, stream=None):
    """grad_in[j] = grad_call * dC/dx_j + grad_put * dP/dx_j from the 10
    saved Jacobian columns; grad_call / grad_put may be None."""
    n = grad_in[0].numel() if n is None else n
    for c in list(jacobian) + list(grad_in) + [g for g in (grad_call, grad_put) if g is not None]:
        _check_column(c, n)
    jp, keep1 = _ptr_array(jacobian)
    gp, keep2 = _ptr_array(grad_in)
    st = _stream(stream, list(grad_in))
    _call("hpac_bs_vjp", lib().hpac_bs_vjp(n, jp, _addr(grad_call), _addr(grad_put), gp, st))


def hpac_bs_adjoint(inputs, grad_call, grad_put, grad_in, n=None, stream=None):
    """The same contraction with the derivatives recomputed from the inputs."""
    n = grad_in[0].numel() if n is None else n
    for c in list(inputs) + list(grad_in) + [g for g in (grad_call, grad_put) if g is not None]:
        _check_column(c, n)
    ip, keep1 = _ptr_array(inputs)
    gp, keep2 = _ptr_array(grad_in)
    st = _stream(stream, list(grad_in))
    _call("hpac_bs_adjoint", lib().hpac_bs_adjoint(n, ip, _addr(grad_call), _addr(grad_put), gp, st))


def hpac_bs_vjp_ref(inputs, source, grad_call, grad_put, grad_in, n=None, stream=None):
    """The contraction with the derivatives recomputed at each item's source
    item (the int32 column a forward on REGION_BS_PRICE_REF wrote)."""
    n = grad_in[0].numel() if n is None else n
    for c in list(inputs) + list(grad_in) + [g for g in (grad_call, grad_put) if g is not None]:
        _check_column(c, n)
    _check_buf(source, n, "i32", "source")
    ip, keep1 = _ptr_array(inputs)
    gp, keep2 = _ptr_array(grad_in)
    st = _stream(stream, list(grad_in))
    _call("hpac_bs_vjp_ref", lib().hpac_bs_vjp_ref(n, ip, _addr(source), _addr(grad_call), _addr(grad_put), gp, st))


def hpac_surrogate(inputs, outputs, params, norm, box_lo, box_hi, queue, queue_count, stream=None, n=None):
    """Surrogate inference with the exact region as fallback outside the box."""
    io = make_io(inputs, outputs, n=n, region=REGION_BS_PRICE, stream=stream)
    _check_buf(params, MLP_NUM_PARAMS, "f32", "params")
    _check_buf(queue, io.n, "i32", "queue")
    _check_buf(queue_count, 1, "i32", "queue_count")
    lo = (ctypes.c_float * 5)(*map(float, box_lo))
    hi = (ctypes.c_float * 5)(*map(float, box_hi))
    _call("hpac_surrogate", lib().hpac_surrogate(ctypes.byref(io), _addr(params), ctypes.byref(norm), lo, hi,
                                                 _addr(queue), _addr(queue_count)))


def hpac_mlp_grad_blocks(batch):
    return lib().hpac_mlp_grad_blocks(batch)


def hpac_mlp_grad(x, t, params, norm, loss_count, grad_partials, loss_partials, n=None, stream=None):
    n = x[0].numel() if n is None else n
    for c in list(x) + list(t):
        _check_column(c, n)
    blocks = hpac_mlp_grad_blocks(n)
    _check_buf(params, MLP_NUM_PARAMS, "f32", "params")
    _check_buf(grad_partials, blocks * MLP_NUM_PARAMS, "f32", "grad_partials")
    _check_buf(loss_partials, blocks, "f32", "loss_partials")
    xp, k1 = _ptr_array(x)
    tp, k2 = _ptr_array(t)
    st = _stream(stream, list(x))
    _call("hpac_mlp_grad", lib().hpac_mlp_grad(n, xp, tp, _addr(params), ctypes.byref(norm), loss_count,
                                               _addr(grad_partials), _addr(loss_partials), st))


def hpac_mlp_adam(grad_partials, blocks, params, m, v, lr, beta1, beta2, eps, step, stream=None):
    _check_buf(grad_partials, blocks * MLP_NUM_PARAMS, "f32", "grad_partials")
    for t, what in ((params, "params"), (m, "m"), (v, "v")):
        _check_buf(t, MLP_NUM_PARAMS, "f32", what)
    st = _stream(stream, [params])
    _call("hpac_mlp_adam", lib().hpac_mlp_adam(_addr(grad_partials), blocks, _addr(params), _addr(m), _addr(v),
                                               lr, beta1, beta2, eps, step, st))


def hpac_probe_copy(src, dst, nbytes, stream=None):
    _check_buf(src, nbytes, "bytes", "src")
    _check_buf(dst, nbytes, "bytes", "dst")
    _call("hpac_probe_copy", lib().hpac_probe_copy(_addr(src), _addr(dst), nbytes, _stream(stream, [src, dst])))


def hpac_probe_valu(out, workgroups, iters, scalar_operand, stream=None):
    _check_buf(out, int(workgroups) * 256, "f32", "out")
    _call("hpac_probe_valu", lib().hpac_probe_valu(_addr(out), int(workgroups), int(iters), int(bool(scalar_operand)),
                                                   _stream(stream, [out])))


def hpac_num_lanes(n, items_per_lane):
    return lib().hpac_num_lanes(n, items_per_lane)


def hpac_trace_entries(n, items_per_lane):
    return lib().hpac_trace_entries(n, items_per_lane)


def hpac_last_error():
    return lib().hpac_last_error().decode()


def hpac_abi_version():
    return lib().hpac_abi_version()


# trace word fields (hpac.h)
def trace_fields(t):
    """Decode a numpy/torch int array of trace words into a dict of arrays."""
    import numpy as np
    t = np.asarray(t).astype(np.uint64)
    return dict(votes=(t & 0x7F).astype(np.int64), napprox=((t >> 8) & 0x7F).astype(np.int64),
                writer=((t >> 16) & 0x3F).astype(np.int64), writer_valid=((t >> 22) & 1).astype(bool),
                approx=((t >> 24) & 1).astype(bool), voted=((t >> 25) & 1).astype(bool),
                active=((t >> 31) & 1).astype(bool))


def hpac_hydro_waves(n):
    return lib().hpac_hydro_waves(n)


def hpac_hydro_groups(n, level):
    return lib().hpac_hydro_groups(n, _level(level))


def hpac_hydro_partials(n):
    return lib().hpac_hydro_partials(n)


def _torch_stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def hpac_hydro_init(params, e_origin, state, stream=None):
    _call("hpac_hydro_init", lib().hpac_hydro_init(ctypes.byref(params), float(e_origin), ctypes.byref(state),
                                                   _torch_stream(stream)))


def hpac_hydro_step(params, tech, step, state, dec_eos=None, dec_hg=None, stream=None):
    if tech.eos_history:
        _check_buf(dec_eos, hpac_hydro_groups(params.n, tech.eos_level), "i8", "dec_eos")
    if tech.hg_history:
        _check_buf(dec_hg, hpac_hydro_groups(params.n, tech.hg_level), "i8", "dec_hg")
    _call("hpac_hydro_step", lib().hpac_hydro_step(ctypes.byref(params), ctypes.byref(tech), int(step),
                                                   ctypes.byref(state), _addr(dec_eos), _addr(dec_hg),
                                                   _torch_stream(stream)))


def hpac_hydro_step_noalloc(params, tech, step, state, dec_eos=None, dec_hg=None, stream=None):
    if tech.eos_history:
        _check_buf(dec_eos, hpac_hydro_groups(params.n, tech.eos_level), "i8", "dec_eos")
    if tech.hg_history:
        _check_buf(dec_hg, hpac_hydro_groups(params.n, tech.hg_level), "i8", "dec_hg")
    _call("hpac_hydro_step_noalloc",
          lib().hpac_hydro_step_noalloc(ctypes.byref(params), ctypes.byref(tech), int(step), ctypes.byref(state),
                                        _addr(dec_eos), _addr(dec_hg), _torch_stream(stream)))


def hpac_hydro_run(params, tech, first_step, steps, state, stream=None):
    _call("hpac_hydro_run", lib().hpac_hydro_run(ctypes.byref(params), ctypes.byref(tech), int(first_step),
                                                 int(steps), ctypes.byref(state), _torch_stream(stream)))


def hpac_hydro_check(state, stream=None):
    """Raises HpacError(HPAC_ENUMERIC) if a hydro step left the numeric
    domain (waits for the stream)."""
    _call("hpac_hydro_check", lib().hpac_hydro_check(ctypes.byref(state), _torch_stream(stream)))


# ------------------------------------------------------------ binomial

def hpac_bo_units(n, items_per_lane):
    return lib().hpac_bo_units(n, items_per_lane)


def _bo_io(inputs, outputs, kw):
    kw = dict(kw)
    kw["region"] = REGION_BINOMIAL
    return make_io(inputs, outputs, **kw)


def hpac_bo_exact(inputs, outputs, steps, american=True, **kw):
    io = _bo_io(inputs, outputs, kw)
    _call("hpac_bo_exact", lib().hpac_bo_exact(ctypes.byref(io), steps, int(american)))


def hpac_bo_iact(inputs, outputs, steps, table_size, threshold, american=True, **kw):
    io = _bo_io(inputs, outputs, kw)
    _call("hpac_bo_iact", lib().hpac_bo_iact(ctypes.byref(io), steps, int(american), table_size, threshold))


def hpac_bo_taf(inputs, outputs, steps, history_size, prediction_size, rsd_threshold, american=True, **kw):
    io = _bo_io(inputs, outputs, kw)
    _call("hpac_bo_taf", lib().hpac_bo_taf(ctypes.byref(io), steps, int(american), history_size, prediction_size,
                                           rsd_threshold))


def hpac_bo_perfo(inputs, outputs, steps, kind, param, offset=0, american=True, **kw):
    io = _bo_io(inputs, outputs, kw)
    k = PERFO_KINDS[kind] if isinstance(kind, str) else int(kind)
    _call("hpac_bo_perfo", lib().hpac_bo_perfo(ctypes.byref(io), steps, int(american), k, param, offset))

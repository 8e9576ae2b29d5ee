"""Host-side checks of the C ABI: the library loads, exports every entry
point include/hpac.h declares, and rejects invalid arguments with
HPAC_EINVAL before touching the GPU (so these run without one)."""
import ctypes
import os
import re

import pytest

from paper_2308_16877_amd import hpac

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hpac.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpac_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert {"hpac_exact", "hpac_iact", "hpac_taf", "hpac_perfo"} <= set(names)
    lib = hpac.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert lib.hpac_abi_version() == 3


def test_lane_mapping():
    assert hpac.hpac_num_lanes(65536, 16) == 4096
    assert hpac.hpac_num_lanes(69, 2) == 64
    assert hpac.hpac_num_lanes(0, 4) == 0
    assert hpac.hpac_num_lanes(1, 1) == 64
    assert hpac.hpac_num_lanes(2**24, 16) == 2**20
    assert hpac.hpac_trace_entries(65536, 16) == 4096 // 64 * 16
    assert hpac.hpac_num_lanes(-1, 1) == -1 and hpac.hpac_num_lanes(10, 0) == -1


FAKE = 0x7F0000000000  # never dereferenced: every call below fails validation first


def io(**kw):
    args = dict(inputs=[FAKE] * 5, outputs=[FAKE] * 2, n=1000, items_per_lane=4)
    args.update(kw)
    return args


def expect(status, fn, *a, **kw):
    with pytest.raises(hpac.HpacError) as e:
        fn(*a, **kw)
    assert e.value.status == status, str(e.value)
    return str(e.value)


def test_invalid_io_is_rejected_before_any_hip_call():
    E = hpac.HPAC_EINVAL
    expect(E, hpac.hpac_exact, **io(items_per_lane=0))
    expect(E, hpac.hpac_exact, **io(items_per_lane=65537))
    expect(E, hpac.hpac_exact, **io(block_size=96))
    expect(E, hpac.hpac_exact, **io(block_size=512))
    expect(E, hpac.hpac_exact, **io(n=-5))
    expect(E, hpac.hpac_exact, **io(n=2**40 + 1))
    expect(E, hpac.hpac_exact, **io(n=2**40, items_per_lane=1))  # 2^32 workgroups
    expect(E, hpac.hpac_exact, **io(inputs=[FAKE] * 4))
    expect(E, hpac.hpac_exact, **io(outputs=[FAKE] * 3, region=0))
    expect(E, hpac.hpac_exact, **io(inputs=[FAKE, 0, FAKE, FAKE, FAKE]))
    expect(E, hpac.hpac_exact, **io(outputs=[FAKE + 2, FAKE]))
    expect(E, hpac.hpac_exact, **io(region=7))
    expect(E, hpac.hpac_exact, **io(trace=FAKE + 1))
    msg = expect(E, hpac.hpac_exact, **io(counters=FAKE + 4))
    assert "aligned" in msg


def test_invalid_technique_parameters_are_rejected():
    E = hpac.HPAC_EINVAL
    for t in (0, 33):
        expect(E, hpac.hpac_iact, table_size=t, threshold=0.1, **io())
    for thr in (-0.1, float("nan"), float("inf")):
        expect(E, hpac.hpac_iact, table_size=8, threshold=thr, **io())
        expect(E, hpac.hpac_taf, history_size=4, prediction_size=4, rsd_threshold=thr, **io())
    for g in (0, 3, 128):
        expect(E, hpac.hpac_iact, table_size=8, threshold=0.1, tables_per_wave=g, **io())
    expect(E, hpac.hpac_iact, table_size=8, threshold=0.1, level=5, **io())
    for h in (0, 9):
        expect(E, hpac.hpac_taf, history_size=h, prediction_size=4, rsd_threshold=0.1, **io())
    expect(E, hpac.hpac_taf, history_size=4, prediction_size=0, rsd_threshold=0.1, **io())
    expect(E, hpac.hpac_taf, history_size=4, prediction_size=4, rsd_threshold=0.1, level=-1, **io())
    expect(E, hpac.hpac_perfo, kind=4, param=2, **io())
    expect(E, hpac.hpac_perfo, kind="small", param=-1, **io())
    expect(E, hpac.hpac_perfo, kind="ini", param=101, **io())
    expect(E, hpac.hpac_perfo, kind="small", param=2, offset=-1, **io())
    expect(E, hpac.hpac_probe_copy, FAKE, FAKE, 15)
    for wg, it in ((0, 1), (65537, 1), (1, 0), (1, 65537)):
        expect(E, hpac.hpac_probe_valu, FAKE, wg, it, 0, stream=0)
    expect(E, hpac.hpac_probe_valu, 0, 1, 1, 0, stream=0)
    expect(E, hpac.hpac_probe_valu, FAKE + 2, 1, 1, 0, stream=0)


def test_unsupported_requests():
    # 64 tables of 32 entries for 12 outputs per wave exceed the LDS budget
    expect(hpac.HPAC_EUNSUPPORTED, hpac.hpac_iact, table_size=32, threshold=0.1, tables_per_wave=64,
           **io(outputs=[FAKE] * 12))
    # price tables interleaved at 64 per wave: 8 entries fill 64 KiB exactly, 9 do not
    expect(hpac.HPAC_EUNSUPPORTED, hpac.hpac_iact, table_size=9, threshold=0.1, tables_per_wave=64, **io())
    # the Jacobian region takes FP32 columns only; the FP16 body does not take BF16 columns
    args = io()
    d = hpac.make_io(args["inputs"], [FAKE] * 12, n=args["n"], items_per_lane=4, region=hpac.REGION_BS_PRICE_GRAD)
    d.dtype = hpac.F16
    assert hpac.lib().hpac_exact(ctypes.byref(d)) == hpac.HPAC_EUNSUPPORTED
    d = hpac.make_io(args["inputs"], args["outputs"], n=args["n"], items_per_lane=4, region=hpac.REGION_BS_PRICE_F16)
    d.dtype = hpac.BF16
    assert hpac.lib().hpac_exact(ctypes.byref(d)) == hpac.HPAC_EUNSUPPORTED
    d.dtype = 7
    assert hpac.lib().hpac_exact(ctypes.byref(d)) == hpac.HPAC_EINVAL
    # half-precision columns need 2-byte alignment only
    d = hpac.make_io([FAKE + 2] * 5, [FAKE + 2] * 2, n=0, region=hpac.REGION_BS_PRICE, dtype=hpac.F16)
    assert hpac.lib().hpac_exact(ctypes.byref(d)) == hpac.HPAC_OK


def test_zero_items_is_a_no_op():
    # n == 0 passes validation and launches nothing (no device needed)
    hpac.hpac_exact([FAKE] * 5, [FAKE] * 2, n=0)
    hpac.hpac_taf([FAKE] * 5, [FAKE] * 2, 4, 4, 0.01, n=0)
    hpac.hpac_iact([FAKE] * 5, [FAKE] * 2, 8, 0.05, n=0)
    hpac.hpac_perfo([FAKE] * 5, [FAKE] * 2, "small", 10, n=0)


def hydro_state(**over):
    s = hpac.hpac_hydro_state()
    for d in range(3):
        s.x[d] = FAKE
        s.u[d] = FAKE
        s.unew[d] = FAKE
    for f in ("mnode", "e", "p", "q", "c", "vol", "mass", "force", "weos", "rho_eos", "z_eos", "whg",
              "rho_hg", "z_hg"):
        setattr(s, f, FAKE)
    s.clock = FAKE
    s.dt_partials = FAKE
    s.status = FAKE
    for k, v in over.items():
        setattr(s, k, v)
    return s


def hydro_params(**over):
    p = dict(n=10, side=1.0, gamma=1.4, cq=1.5, cl=0.25, khg=0.1, cfl=0.3, growth=1.1, dvmax=0.1, dt0=1e-7)
    p.update(over)
    return hpac.hpac_hydro_params(**p)


def hydro_tech(**over):
    t = hpac.hpac_hydro_tech(eos_level=hpac.LEVEL_WAVE, hg_level=hpac.LEVEL_WAVE)
    for k, v in over.items():
        setattr(t, k, v)
    return t


def test_hydro_sizes():
    assert hpac.hpac_hydro_waves(90) == (90 ** 3 + 63) // 64
    assert hpac.hpac_hydro_groups(90, hpac.LEVEL_THREAD) == 90 ** 3
    assert hpac.hpac_hydro_groups(90, hpac.LEVEL_WAVE) == (90 ** 3 + 63) // 64
    assert hpac.hpac_hydro_groups(90, hpac.LEVEL_BLOCK) == (90 ** 3 + 255) // 256
    assert hpac.hpac_hydro_groups(90, 3) == -1
    assert hpac.hpac_hydro_partials(90) == ((90 ** 3 + 63) // 64 * 64 + 255) // 256
    assert hpac.hpac_hydro_waves(0) == -1 and hpac.hpac_hydro_waves(1001) == -1


def hstep(*a):
    return hpac.hpac_hydro_step(*a, stream=0)  # a stream handle that is never used: validation fails first


def hinit(*a):
    return hpac.hpac_hydro_init(*a, stream=0)


def test_invalid_hydro_arguments_are_rejected():
    E = hpac.HPAC_EINVAL
    S, P, T = hydro_state(), hydro_params(), hydro_tech()
    for bad in (dict(n=0), dict(n=1001), dict(gamma=1.0), dict(cfl=0.0), dict(growth=0.5), dict(dt0=0.0),
                dict(side=float("nan")), dict(khg=-1.0)):
        expect(E, hstep, hydro_params(**bad), T, 0, S)
        expect(E, hinit, hydro_params(**bad), 1.0, S)
    expect(E, hinit, P, -1.0, S)
    expect(E, hinit, P, float("inf"), S)
    expect(E, hstep, P, T, -1, S)
    expect(E, hstep, P, T, 0, hydro_state(e=0))
    expect(E, hstep, P, T, 0, hydro_state(force=FAKE + 2))
    expect(E, hstep, P, T, 0, hydro_state(clock=FAKE + 4))
    # the numeric-failure flags are required, by the steps and by the check
    msg = expect(E, hstep, P, T, 0, hydro_state(status=0))
    assert "status" in msg
    expect(E, hstep, P, T, 0, hydro_state(status=FAKE + 2))
    expect(E, hinit, P, 1.0, hydro_state(status=0))
    expect(E, hpac.hpac_hydro_check, hydro_state(status=0), 0)
    for bad in (dict(eos_history=9, eos_prediction=1), dict(eos_history=2, eos_prediction=0),
                dict(hg_history=-1), dict(eos_history=2, eos_prediction=2, eos_threshold=-0.1),
                dict(eos_history=2, eos_prediction=2, eos_level=3),
                dict(hg_history=2, hg_prediction=2, perfo_param=2, perfo_items_per_lane=2),
                dict(perfo_kind=4, perfo_param=2, perfo_items_per_lane=2),
                dict(perfo_kind=hpac.PERFO_INI, perfo_param=101, perfo_items_per_lane=1),
                dict(perfo_param=2, perfo_items_per_lane=0), dict(perfo_param=2, perfo_items_per_lane=65)):
        expect(E, hstep, P, hydro_tech(**bad), 0, S)
    expect(E, hstep, P, hydro_tech(eos_history=2, eos_prediction=2), 0, hydro_state(weos=0))
    expect(E, hstep, P, hydro_tech(hg_history=2, hg_prediction=2), 0, hydro_state(whg=0))
    expect(E, hstep, P, hydro_tech(hg_history=2, hg_prediction=2), 0, hydro_state(z_hg=0))
    # the multi-step entry point checks the same arguments, and its own
    hrun = lambda *a: hpac.hpac_hydro_run(*a, stream=0)
    expect(E, hrun, P, T, 0, -1, S)
    expect(E, hrun, P, T, 2 ** 31 - 10, 11, S)
    expect(E, hrun, P, T, -1, 1, S)
    expect(E, hrun, hydro_params(n=0), T, 0, 1, S)
    expect(E, hrun, P, hydro_tech(hg_history=2, hg_prediction=2), 0, 1, hydro_state(whg=0))
    # the allocation-free step: its own mesh limit, the same checks otherwise
    hna = lambda *a: hpac.hpac_hydro_step_noalloc(*a, stream=0)
    msg = expect(E, hna, hydro_params(n=hpac.HYDRO_NOALLOC_MAX_N + 1), T, 0, hydro_state(dt_partials=0))
    assert "scratch" in msg
    expect(E, hna, hydro_params(n=0), T, 0, hydro_state(dt_partials=0))
    expect(E, hna, P, T, 0, hydro_state(e=0, dt_partials=0))
    expect(E, hna, P, T, -1, hydro_state(dt_partials=0))
    expect(E, hna, P, hydro_tech(eos_history=2, eos_prediction=2), 0, hydro_state(weos=0, dt_partials=0))


def bo_io(**kw):
    args = dict(inputs=[FAKE] * 5, outputs=[FAKE] * 2, n=1000, items_per_lane=4, stream=0)
    args.update(kw)
    return args


def test_invalid_binomial_arguments_are_rejected():
    E = hpac.HPAC_EINVAL
    assert hpac.hpac_bo_units(1000, 4) == 256 and hpac.hpac_bo_units(-1, 4) == -1
    for steps in (0, 1024, -5):
        expect(E, hpac.hpac_bo_exact, steps=steps, **bo_io())
    expect(E, hpac.hpac_bo_exact, steps=64, american=2, **bo_io())
    expect(E, hpac.hpac_bo_exact, steps=64, **bo_io(n=2 ** 31 + 1))
    expect(E, hpac.hpac_bo_exact, steps=64, **bo_io(items_per_lane=0))
    expect(E, hpac.hpac_bo_exact, steps=64, **bo_io(block_size=96))
    expect(E, hpac.hpac_bo_exact, steps=64, **bo_io(inputs=[FAKE, FAKE, 0, FAKE, FAKE]))
    expect(E, hpac.hpac_bo_exact, steps=64, **bo_io(outputs=[FAKE, FAKE + 2]))
    expect(hpac.HPAC_EUNSUPPORTED, hpac.hpac_bo_exact, steps=64, **bo_io(dtype=hpac.F16))
    for t in (0, 33):
        expect(E, hpac.hpac_bo_iact, steps=64, table_size=t, threshold=0.1, **bo_io())
    expect(E, hpac.hpac_bo_iact, steps=64, table_size=4, threshold=-1.0, **bo_io())
    for h in (0, 9):
        expect(E, hpac.hpac_bo_taf, steps=64, history_size=h, prediction_size=2, rsd_threshold=0.1, **bo_io())
    expect(E, hpac.hpac_bo_taf, steps=64, history_size=2, prediction_size=0, rsd_threshold=0.1, **bo_io())
    expect(E, hpac.hpac_bo_perfo, steps=64, kind=7, param=2, **bo_io())
    expect(E, hpac.hpac_bo_perfo, steps=64, kind="ini", param=101, **bo_io())
    expect(E, hpac.hpac_bo_perfo, steps=64, kind="small", param=2, offset=-1, **bo_io())
    # the Black-Scholes entry points do not take the binomial region, nor the reverse
    expect(E, hpac.hpac_exact, **io(region=hpac.REGION_BINOMIAL))
    with pytest.raises(hpac.HpacError):
        lib = hpac.lib()
        desc = hpac.make_io([FAKE] * 5, [FAKE] * 2, n=10, region=hpac.REGION_BS_PRICE, stream=0)
        hpac._call("hpac_bo_exact", lib.hpac_bo_exact(ctypes.byref(desc), 64, 1))


def test_grids_beyond_32_bit_lane_counts_are_rejected():
    """A dispatch counts its lanes in 32 bits: a grid-stride mapping whose
    grid would exceed 2^32-1 lanes is refused at validation (with a hint to
    raise items_per_lane), and one just inside is accepted."""
    E = hpac.HPAC_EINVAL
    msg = expect(E, hpac.hpac_exact, **io(n=2**32 + 1, items_per_lane=1))
    assert "items_per_lane" in msg
    expect(E, hpac.hpac_iact, table_size=8, threshold=0.1, **io(n=2**33, items_per_lane=1))
    expect(E, hpac.hpac_taf, history_size=4, prediction_size=4, rsd_threshold=0.1, **io(n=2**33, items_per_lane=1))
    expect(E, hpac.hpac_perfo, kind="small", param=10, **io(n=2**33, items_per_lane=1))
    # 2^40 items at 256 per lane need 2^32 lanes: one too many
    expect(E, hpac.hpac_exact, **io(n=2**40, items_per_lane=256))
    # binomial: 64 lanes per unit
    expect(E, hpac.hpac_bo_exact, [FAKE] * 5, [FAKE] * 2, 64, n=2**26, items_per_lane=1)
    # training batches: one lane per sample
    nm = hpac.make_norm([0] * 5, [1] * 5, [0, 0], [1, 1])
    expect(E, hpac.hpac_mlp_grad, [FAKE] * 5, [FAKE] * 2, FAKE, nm, 1, FAKE, FAKE, n=2**32)
    # output shifts (log outputs) must be finite and >= 0
    for bad in ((-0.01, 0.0), (0.0, float("nan")), (float("inf"), 0.0)):
        nm = hpac.make_norm([0] * 5, [1] * 5, [0, 0], [1, 1], bad)
        msg = expect(E, hpac.hpac_mlp_grad, [FAKE] * 5, [FAKE] * 2, FAKE, nm, 1, FAKE, FAKE, n=64)
        assert "shift" in msg


def test_persistent_taf_state_sizes_and_checks():
    L = hpac.hpac_num_lanes(1000, 4)
    assert hpac.hpac_taf_state_bytes(hpac.REGION_BS_PRICE, 1000, 4, 4) == L * (4 * 2 + 2) * 4
    assert hpac.hpac_taf_state_bytes(hpac.REGION_BS_PRICE_GRAD, 1000, 4, 2) == L * (2 * 12 + 2) * 4
    assert hpac.hpac_taf_state_bytes(hpac.REGION_BS_PRICE_REF, 1000, 4, 2) == -1
    assert hpac.hpac_taf_state_bytes(hpac.REGION_BS_PRICE, 1000, 4, 9) == -1
    assert hpac.hpac_taf_state_bytes(hpac.REGION_BS_PRICE, 1000, 0, 2) == -1
    msg = expect(hpac.HPAC_EINVAL, hpac.hpac_taf, [FAKE] * 5, [FAKE] * 2, 4, 4, 0.01, n=1000, items_per_lane=4,
                 stream=0, state=FAKE + 2)
    assert "persistent_state" in msg
    import torch
    with pytest.raises(ValueError, match="state holds"):
        hpac.hpac_taf([FAKE] * 5, [FAKE] * 2, 4, 4, 0.01, n=1000, items_per_lane=4, stream=0,
                      state=torch.zeros(L * 10 * 4 - 1, dtype=torch.uint8))


def test_short_or_mistyped_buffers_are_rejected_by_the_binding():
    """The binding checks every device buffer a kernel writes beyond the
    columns (trace, counters, the surrogate's queue, training partials):
    a short one would be written out of bounds on the device."""
    import torch
    n, ipt = 1000, 4
    need = hpac.hpac_trace_entries(n, ipt)
    with pytest.raises(ValueError, match="trace holds"):
        hpac.hpac_exact(**io(trace=torch.zeros(need - 1, dtype=torch.int32)))
    with pytest.raises(ValueError, match="element type"):
        hpac.hpac_exact(**io(trace=torch.zeros(need, dtype=torch.float32)))
    with pytest.raises(ValueError, match="counters holds"):
        hpac.hpac_exact(**io(counters=torch.zeros(3, dtype=torch.int64)))
    with pytest.raises(ValueError, match="element type"):
        hpac.hpac_exact(**io(counters=torch.zeros(4, dtype=torch.int32)))
    # binomial traces have one word per (unit, option of the unit)
    units = hpac.hpac_bo_units(n, ipt)
    with pytest.raises(ValueError, match="trace holds"):
        hpac.hpac_bo_exact([FAKE] * 5, [FAKE] * 2, 64, n=n, items_per_lane=ipt,
                           trace=torch.zeros(units * ipt - 1, dtype=torch.int32))
    nm = hpac.make_norm([0] * 5, [1] * 5, [0, 0], [1, 1])
    lo, hi = [0.0] * 5, [1.0] * 5
    x, y = [FAKE] * 5, [FAKE] * 2
    with pytest.raises(ValueError, match="queue holds"):
        hpac.hpac_surrogate(x, y, FAKE, nm, lo, hi, torch.zeros(n - 1, dtype=torch.int32), FAKE, n=n)
    with pytest.raises(ValueError, match="params holds"):
        hpac.hpac_surrogate(x, y, torch.zeros(10), nm, lo, hi, FAKE, FAKE, n=n)
    with pytest.raises(ValueError, match="queue_count"):
        hpac.hpac_surrogate(x, y, FAKE, nm, lo, hi, FAKE, torch.zeros(1, dtype=torch.int64), n=n)
    blocks = hpac.hpac_mlp_grad_blocks(n)
    with pytest.raises(ValueError, match="grad_partials holds"):
        hpac.hpac_mlp_grad([FAKE] * 5, [FAKE] * 2, FAKE, nm, n,
                           torch.zeros(blocks * hpac.MLP_NUM_PARAMS - 1), FAKE, n=n)
    with pytest.raises(ValueError, match="loss_partials holds"):
        hpac.hpac_mlp_grad([FAKE] * 5, [FAKE] * 2, FAKE, nm, n, FAKE, torch.zeros(blocks - 1), n=n)
    with pytest.raises(ValueError, match="m holds"):
        hpac.hpac_mlp_adam(FAKE, 1, FAKE, torch.zeros(100), FAKE, 1e-3, 0.9, 0.999, 1e-8, 1)
    with pytest.raises(ValueError, match="dst holds"):
        hpac.hpac_probe_copy(FAKE, torch.zeros(3, dtype=torch.float32), 16)


def test_source_item_region_arguments():
    """The price-and-source region: 3 outputs, exact and iACT only, int32
    indices (n <= 2^31 - 1); its backward checks its source column."""
    E, U = hpac.HPAC_EINVAL, hpac.HPAC_EUNSUPPORTED
    ref = dict(region=hpac.REGION_BS_PRICE_REF, outputs=[FAKE] * 3)
    expect(E, hpac.hpac_exact, **io(region=hpac.REGION_BS_PRICE_REF))  # 2 outputs for a 3-output region
    expect(U, hpac.hpac_taf, history_size=4, prediction_size=4, rsd_threshold=0.1, **io(**ref))
    expect(U, hpac.hpac_perfo, kind="small", param=10, **io(**ref))
    expect(E, hpac.hpac_iact, table_size=8, threshold=0.1, **io(n=2**31, items_per_lane=64, **ref))
    expect(E, hpac.hpac_bs_vjp_ref, [FAKE] * 5, 0, FAKE, FAKE, [FAKE] * 5, n=10)
    expect(E, hpac.hpac_bs_vjp_ref, [FAKE] * 5, FAKE + 2, FAKE, FAKE, [FAKE] * 5, n=10)
    expect(E, hpac.hpac_bs_vjp_ref, [FAKE] * 5, FAKE, FAKE, FAKE, [FAKE] * 5, n=2**31)
    import torch
    with pytest.raises(ValueError, match="source"):
        hpac.hpac_exact([FAKE] * 5, [FAKE, FAKE, torch.zeros(999, dtype=torch.int32)], n=1000,
                        region=hpac.REGION_BS_PRICE_REF)

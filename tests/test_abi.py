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
    assert lib.hpac_abi_version() == 1


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


def test_unsupported_requests():
    # 64 tables of 32 entries for 12 outputs per wave exceed the LDS budget
    expect(hpac.HPAC_EUNSUPPORTED, hpac.hpac_iact, table_size=32, threshold=0.1, tables_per_wave=64,
           **io(outputs=[FAKE] * 12))
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

"""Host logic of bench.py that runs without a GPU: the one-GPU guard and the
algorithmic byte counts behind the roofline figure."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_algorithmic_bytes_per_technique():
    n = 1000
    # 5 FP32 inputs read and 2 FP32 outputs written per evaluated item
    assert bench.algorithmic_bytes("exact", n, 0.0) == 28 * n
    assert bench.algorithmic_bytes("iact", n, 0.7) == 28 * n  # iACT reads every input to decide
    # TAF's approximated items read nothing and store the last output
    assert bench.algorithmic_bytes("taf", n, 0.25) == 8 * n + 20 * n * 0.75
    # perforated items are neither read nor written
    assert bench.algorithmic_bytes("perfo", n, 0.1) == pytest.approx(28 * n * 0.9)
    with pytest.raises(KeyError):
        bench.algorithmic_bytes("other", n, 0.0)


def test_every_step_technique_names_its_kernel():
    assert set(bench.TECHS) == set(bench.KERNEL_NAMES)
    assert bench.VALU_PEAK_TOPS == pytest.approx(78.6432)


def _fake_legs():
    """Legs shaped like a full run's (every key leg_summary reads)."""
    techs = {t: {"ms": 0.1, "items_per_s": 1.6e11, "speedup_vs_exact": 1.0, "mape": 0.001, "approx_frac": 0.5,
                 "items_per_lane": 16} for t in bench.TECHS}
    pt = {"ms": 0.1, "approx_frac": 0.2, "mape": 0.003, "speedup_vs_exact": 1.2, "technique": "taf",
          "items_per_lane": 16, "params": {"history_size": 4}}
    lvl = {lv: dict(pt) for lv in ("thread", "wave", "block")}
    bo = {t: {"ms": 3.0, "speedup_vs_exact": 2.0, "mape_vs_exact": 0.002} for t in ("exact", "iact", "taf", "perfo")}
    return {
        "structured_locality": {"best_at_mape_0.005": {"variant": "lane_periodic_1024", "technique": "taf",
                                                       "speedup_vs_exact": 1.8, "mape": 0.002}},
        "parameter_sweep": {"best_at_mape_0.005": pt, "best_exact": "ipt1_block256", "points": [pt] * 60},
        "config0_65536": {"techniques": techs},
        "psize_sweep": {"sorted": {"best_at_mape_0.005": dict(pt, point="ipt16_p4")},
                        "lane_periodic_1024": {"best_at_mape_0.005": dict(pt, point="ipt512_p512")}},
        "greeks": {"iact_speedup_vs_exact": 0.9, "wave_periodic_2": {"iact_speedup_vs_exact": 1.1,
                                                                     "iact_gradient_mape_vs_exact": 0.001}},
        "precision": {"fp32_body_fp32_columns": {"speedup_vs_fp32": 1.0, "mape_vs_fp32": 0.0},
                      "fp32_body_fp16_columns": {"speedup_vs_fp32": 1.4, "mape_vs_fp32": 0.0006}},
        "hierarchy_and_items_per_lane": {t: {"levels_at_ipt16": lvl, "items_per_lane_at_wave_level": {
            str(2 ** k): {"speedup_vs_exact": 1.0123456, "approx_frac": 0.7483123, "mape": 0.002} for k in range(7)}}
            for t in ("taf", "iact")},
        "binomial_options": {"variants": {"unit_periodic": bo}},
        "surrogate": {"speedup_vs_exact": 0.2, "mape_vs_exact": 0.004, "rel_l2_vs_exact": 0.001,
                      "items_per_s": 3e10},
        "hydro": {"techniques": {"exact": {"ms_per_step": 0.07, "element_steps_per_s": 1e10}},
                  "sweep": {"best_at_qoi_err_0.005": {"technique": "eos_taf_thread_h2_0.001",
                                                      "speedup_vs_exact": 1.07, "qoi_err_vs_exact_gpu": 1e-6}},
                  "cpu_baseline": {"value": 8.7e6}},
    }


def test_headline_line_is_short_and_complete():
    """The driver keeps a few KB of the benchmark's output: the last line
    must be a complete JSON object of under 4 KB with the contract's keys,
    whatever the legs hold."""
    import json
    import types
    args = types.SimpleNamespace(n=1 << 24, steps=200, warmup=100)
    tech = {t: {"ms": 0.09, "speedup_vs_exact": 0.9, "mape": 0.09 if t == "perfo" else 0.0, "approx_frac": 0.1}
            for t in bench.TECHS}
    res = {"warmup_steps_run": 137}
    roofline = {"kernel": "k_iact", "bound": "hbm", "achieved": 4800.123456, "peak": 8000.0, "unit": "GB/s",
                "frac": 0.6000001, "traffic": 469878710.2464, "algorithmic_bytes_per_launch": 469762048.0,
                "avg_launch_ms": 0.0978, "rocprof_avg_us": 97.5, "frac_rocprof": 0.602, "alu_frac": 0.51}
    cpu = {"value": 8.8e7, "unit": "region items/s", "cores": 16, "kind": "oracle",
           "sample": "first 16777216 of the 16777216 items, all four legs of one step (exact, iACT, TAF, "
                     "perforation), 0.8 s wall"}
    summary = bench.leg_summary(_fake_legs())
    line = bench.headline(args, res, tech, 1.3e11, 0.36, "iact", roofline, cpu, summary, "results/bench_legs.json")
    text = json.dumps(line)
    assert len(text.encode()) < 4096, len(text)
    back = json.loads(text)
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in back
    assert back["config"]["workload"]
    assert set(back["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert set(back["cpu_baseline"]) >= {"value", "unit", "cores", "kind", "sample"}
    # perforation (9% MAPE) is left out of the items the value counts
    assert "perfo" not in back["config"]["value_counts"]
    assert set(back["legs"]) >= {"config0_items_per_s", "psize_best_at_mape_0.005", "hydro", "surrogate", "greeks"}


def test_round_keeps_structure():
    assert bench._round({"a": [1.23456789, float("nan")], "b": 3}) == {"a": [1.235, None], "b": 3}

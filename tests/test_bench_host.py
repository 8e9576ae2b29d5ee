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

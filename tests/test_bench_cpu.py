"""Host-side checks of bench.py (no GPU): the one-GPU contract, the
mirror-symmetry test the roofline work model relies on, and the lookup of
the recorded HBM traffic."""
import copy
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from synthetic import configs, models  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")  # no JSON line


def test_fc3_mirror_symmetry_detection():
    m = models.diamond()
    assert bench.fc3_mirror_symmetric(m)
    assert bench.fc3_mirror_symmetric(configs.model_for(configs.CONFIGS["C3"]))
    # break the symmetry of one (i, j, k) / (i, k, j) pair
    bad = copy.deepcopy(m)
    t = int(np.flatnonzero(bad.fc3_j != bad.fc3_k)[0])
    bad.fc3_val = bad.fc3_val.copy()
    bad.fc3_val[t] += 1e-3 * np.abs(bad.fc3_val).max()
    assert not bench.fc3_mirror_symmetric(bad)


def test_recorded_traffic_lookup():
    # a workload or kernel without a record reports nothing
    assert bench.measured_traffic("lw_fused", "C3") is None
    assert bench.measured_traffic("gm_gemm", "C2") is None
    # the recorded C2 figure is returned only while the hashed sources are
    # the ones it was measured on
    v = bench.measured_traffic("lw_fused", "C2")
    assert v is None or (isinstance(v, int) and v > 0)

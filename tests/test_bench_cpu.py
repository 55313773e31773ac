"""The benchmark's contract pieces that need no GPU: one GPU only (any other --gpus exits
with a message, before touching a device), the generator's operation counts it reports,
and the committed counter summary it attaches while the kernel source is unchanged."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_opcount_and_counter_summary():
    import bench

    if not os.path.exists(bench.OPCOUNT_FILE):
        pytest.skip("kernels not generated")
    oc = bench.opcount(6)
    assert oc["with_traces"] > oc["no_traces"] > 0 and oc["N"] == 84
    ctr = bench.measured_counters()
    if ctr is not None:  # taken on the current p = 6 kernel source
        assert ctr["bytes_per_launch"] == ctr["bytes_read"] + ctr["bytes_written"]
        assert ctr["bytes_per_launch"] > 196608 * (36 * 84 + 40)  # at least the algorithmic bytes
        assert ctr["kernel"].startswith("dgm_phase_p6<float, true, false")

"""bench.py contract checks that need no GPU."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "error" in json.loads(r.stdout.strip().splitlines()[-1])


def test_traffic_table_matches_the_kernel_source():
    """roofline.traffic is reported only for the kernel source its counters were
    taken on: a change to the kernels needs the FETCH_SIZE / WRITE_SIZE runs again."""
    src = os.path.join(ROOT, "paper_2310_16668_amd", "csrc", "device", "kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    tr = bench.NEAR_TRAFFIC["f32"]
    assert tr["kernel"] == "k_near_sym"
    assert tr["kernels_sha256"] == digest
    assert sorted(tr["bytes_by_tpl"]) == [1, 2, 3, 4]
    assert all(v > 0 for v in tr["bytes_by_tpl"].values())


def test_alu_peaks_are_the_published_vector_figures():
    assert bench.PEAK_TFLOPS == {"f64": 78.6, "f32": 157.3}
    assert bench.MIX_CYCLES_PER_64_SYM_PAIRS["f32"] == 40

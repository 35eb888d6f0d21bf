"""bench.py contract checks that need no GPU."""
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


def test_traffic_is_reported_only_for_the_measured_kernel_source(monkeypatch):
    """roofline.traffic comes from FETCH_SIZE / WRITE_SIZE runs of one source of the
    pair kernel: it is reported for that source only, and null after any change."""
    tr = bench.NEAR_TRAFFIC["f32"]
    assert tr["kernel"] == "k_near_sym"
    assert sorted(tr["bytes_by_tpl"]) == [1, 2, 3, 4]
    assert all(v > 0 for v in tr["bytes_by_tpl"].values())
    digest = bench.pair_kernel_digest()
    assert len(digest) == 16
    monkeypatch.setitem(tr, "kernels_sha256", digest)
    assert bench.near_traffic("f32", "k_near_sym", 3) == tr["bytes_by_tpl"][3]
    assert bench.near_traffic("f32", "k_near", 3) is None
    assert bench.near_traffic("c128", "k_near_sym", 3) is None   # a path never measured
    for path in ("f32_fused", "f64"):
        assert sorted(bench.NEAR_TRAFFIC[path]["bytes_by_tpl"]) == [1, 2, 3, 4]
    monkeypatch.setitem(tr, "kernels_sha256", "0" * 16)
    assert bench.near_traffic("f32", "k_near_sym", 3) is None


def test_alu_peaks_are_the_published_vector_figures():
    assert bench.PEAK_TFLOPS == {"f64": 78.6, "f32": 157.3}
    assert bench.MIX_CYCLES_PER_64_SYM_PAIRS["f32"] == 32
    assert bench.MIX_CYCLES_PER_64_SYM_PAIRS["f32_fused"] == 36

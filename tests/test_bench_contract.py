"""bench.py's contract pieces that need no GPU: the refusal of more than one
GPU, the roofline object's fields and arithmetic, the algorithmic byte
model of each pass."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


class W:
    def __init__(self, n, nf):
        self.n = n
        self.cells = 1
        for v in n:
            self.cells *= v
        self.fields = [None] * nf


def test_algorithmic_bytes():
    w = W((2048, 2048), 1)
    n = 2048 * 2048 * 8
    assert bench.algorithmic_bytes("xpass", w, 8) == 2 * n
    assert bench.algorithmic_bytes("kpass", w, 8) == 4 * n
    w2 = W((512, 512), 2)
    assert bench.algorithmic_bytes("kpass", w2, 4) == 4 * 2 * 512 * 512 * 4
    w3 = W((256, 256, 256), 1)
    assert bench.algorithmic_bytes("ypass_inv", w3, 8) == 2 * 256 ** 3 * 8


def test_roofline_object():
    w = W((2048, 2048), 1)
    # per-launch event totals (ms, launches) for 200 steps, back-to-back means
    prof = {"xpass": (200 * 0.0214, 200), "kpass": (200 * 0.0245, 200),
            "mean_b2b": {"xpass": 0.0212, "kpass": 0.0246}, "tiles": [4, 1, 0, 4, 0, 8]}
    rec = {"bytes_per_launch": {"kpass": 134480000.0}}
    r = bench.roofline(w, "f64", dict(prof), rec)
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["kernel"] == "kpass"
    want = 4 * 2048 * 2048 * 8 / (0.0245e-3) / 1e9
    assert r["achieved"] == pytest.approx(want, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-3)
    assert r["traffic"] == 134480000.0
    assert r["mean_launch_us_back_to_back"]["kpass"] == pytest.approx(24.6)


def test_whole_step_fraction():
    w = W((2048, 2048), 1)
    prof = {"xpass": (200 * 0.0214, 200), "kpass": (200 * 0.0245, 200),
            "mean_b2b": {"xpass": 0.0212, "kpass": 0.0246}, "tiles": None}
    r = bench.roofline(w, "f32", dict(prof), None, 0.050)
    ws = r["whole_step"]
    assert ws["bytes_per_step"] == 6 * 2048 * 2048 * 4
    assert ws["achieved"] == pytest.approx(6 * 2048 * 2048 * 4 / 50e-6 / 1e9, rel=1e-3)
    assert ws["frac"] == pytest.approx(ws["achieved"] / 8000.0, rel=1e-3)
    assert bench.step_bytes(W((256, 256, 256), 1), 8) == 10 * 256 ** 3 * 8
    assert bench.step_bytes(W((512, 512), 2), 4) == 12 * 512 * 512 * 4


def test_cpu_baseline_uses_the_host_cores():
    """The oracle leg on a tiny workload: the threaded and the one-thread
    figures, the core count and the CPU model are reported."""
    from paper_2109_02598_amd import inputs
    w = inputs.allen_cahn_2d(n=32, seed=1, steps=2)
    r = bench.cpu_baseline(w, budget_s=0.2)
    assert r["kind"] == "oracle" and r["value"] > 0
    assert r["cores"] == max(1, min(16, r["host"]["usable_cpus"]))
    assert r["single_thread"]["cores"] == 1 and r["single_thread"]["value"] > 0
    assert r["host"]["cpu_model"] and r["host"]["nproc"] >= 1

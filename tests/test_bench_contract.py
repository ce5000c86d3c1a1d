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


def write_counters(d, rows):
    """A rocprofv3 counter_collection.csv with the given (kernel, counter,
    value) rows, in dispatch order."""
    import csv
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (k, c, v) in enumerate(rows):
            w.writerow([i + 1, i + 1, k, c, float(v)])


def test_traffic_record_from_counter_runs(tmp_path):
    """Counters per dispatch (KiB) scaled by the copy calibration; only the
    timed configuration's dispatches (after each precision's refresh of the
    carried spectrum) count, and the tuner's trials before it do not."""
    kp64 = "void ss::kpass_kernel<double, 2048, true, 0>(ss::KArgs)"
    xp64 = "void ss::xpass_kernel<double, 2048, 1, 2, 0>(ss::XArgs)"
    sf64 = "void ss::xpass_kernel<double, 2048, 1, 2, 3>(ss::XArgs)"
    kf64 = "void ss::kfwd_kernel<double, 2048>(ss::KArgs)"
    kp32 = "void ss::kpass_kernel<float, 2048, true, 0>(ss::KArgs)"
    xp32 = "void ss::xpass_kernel<float, 2048, 1, 2, 0>(ss::XArgs)"
    kf32 = "void ss::kfwd_kernel<float, 2048>(ss::KArgs)"
    for c, v64, v32 in (("FETCH_SIZE", (65000.0, 33000.0), (33000.0, 16500.0)),
                        ("WRITE_SIZE", (65536.0, 32768.0), (32768.0, 16384.0))):
        rows = [(kp64, c, 1.0), (xp64, c, 1.0), (kf64, c, 1.0),          # trials, then the refresh
                (xp64, c, v64[1]), (kp64, c, v64[0]), (sf64, c, 5.0), (xp64, c, v64[1]), (kp64, c, v64[0]),
                (kp32, c, 1.0), (kf32, c, 1.0), (xp32, c, v32[1]), (kp32, c, v32[0])]
        write_counters(str(tmp_path / c), rows)
    copy = "__amd_rocclr_copyBuffer"
    write_counters(str(tmp_path / "cf"), [(copy, "FETCH_SIZE", 32768.0)] * 3)
    write_counters(str(tmp_path / "cw"), [(copy, "WRITE_SIZE", 65536.0)] * 3)
    out = bench.traffic_record("ch2048", str(tmp_path / "FETCH_SIZE"), str(tmp_path / "WRITE_SIZE"),
                               str(tmp_path / "cf"), str(tmp_path / "cw"), out_dir=str(tmp_path))
    assert out["f64"]["kpass"] == pytest.approx((65000.0 * 2 + 65536.0) * 1024)
    assert out["f64"]["xpass"] == pytest.approx((33000.0 * 2 + 32768.0) * 1024)
    assert out["f32"]["kpass"] == pytest.approx((33000.0 * 2 + 32768.0) * 1024)
    rec = bench.json.load(open(tmp_path / "traffic_ch2048_f64.json"))
    assert rec["source_hash"] == bench.kernel_source_hash()
    assert rec["copy_factor_fetch"] == pytest.approx(2.0) and rec["copy_factor_write"] == pytest.approx(1.0)


def test_trace_summary_counts_the_timed_configuration(tmp_path):
    import csv
    rows = [("void ss::kpass_kernel<double, 2048, true, 0>(ss::KArgs)", 0, 50000),   # a trial
            ("void ss::kfwd_kernel<double, 2048>(ss::KArgs)", 100000, 118000),
            ("void ss::kpass_kernel<double, 2048, true, 0>(ss::KArgs)", 200000, 224000),
            ("void ss::kpass_kernel<double, 2048, true, 0>(ss::KArgs)", 300000, 326000),
            ("void ss::kpass_kernel<float, 2048, true, 0>(ss::KArgs)", 400000, 414000)]   # before its refresh
    os.makedirs(tmp_path / "kt")
    with open(tmp_path / "kt" / "x_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for i, (k, a, b) in enumerate(rows):
            w.writerow([i + 1, k, a, b])
    table = bench.trace_summary(str(tmp_path / "kt"))
    assert "| `void ss::kpass_kernel<double, 2048, true, 0>(ss::KArgs)` | 2 | 25.00 | 24.00 |" in table
    assert "float" not in table


def test_trace_per_load_takes_the_dispatches_after_each_load(tmp_path):
    import csv
    K = "void ss::kpass_kernel<double, 2048, true, 0>(ss::KArgs)"
    X = "void ss::xpass_kernel<double, 2048, 1, 2, 0>(ss::XArgs)"
    F = "void ss::kfwd_kernel<double, 2048>(ss::KArgs)"
    seq = [(X, 90), (K, 90),                      # trials before the first load
           (F, 5), (X, 20), (K, 30), (X, 22), (K, 32), (X, 90),
           (F, 5), (X, 10), (K, 12)]
    os.makedirs(tmp_path / "kt")
    with open(tmp_path / "kt" / "x_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for i, (k, us) in enumerate(seq):
            w.writerow([i + 1, k, 1000 * i, 1000 * i + 1000 * us])
    out = bench.trace_per_load(str(tmp_path / "kt"), 4)
    first, second = out.split("load 2")
    assert "load 1 (dispatch 3)" in first and "(dispatch 9)" in second
    assert "| `%s` | 2 | 21.00 | 20.00 |" % X in first and "| `%s` | 2 | 31.00 | 30.00 |" % K in first
    assert "| `%s` | 1 | 10.00 | 10.00 |" % X in second and "| `%s` | 1 | 12.00 | 12.00 |" % K in second
    assert "90.00" not in out


def test_sq_table_per_wave_after_the_refresh(tmp_path):
    import csv
    X = "void ss::xpass_kernel<double, 2048, 1, 2, 0, false>(ss::XArgs)"
    F = "void ss::kfwd_kernel<double, 2048>(ss::KArgs)"
    runs = {"a": {"SQ_WAVES": 2048, "SQ_INSTS_VALU": 2048 * 100, "SQ_INSTS_LDS": 2048 * 10},
            "b": {"SQ_ACTIVE_INST_LDS": 400, "SQ_LDS_BANK_CONFLICT": 100}}
    dirs = []
    for name, counters in runs.items():
        os.makedirs(tmp_path / name)
        with open(tmp_path / name / "x_counter_collection.csv", "w", newline="") as f:
            w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
            w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            for c, v in counters.items():
                w.writerow([1, X, c, 7 * v])        # a trial before the refresh
                w.writerow([2, F, c, 1])
                w.writerow([3, X, c, v])
        dirs.append(str(tmp_path / name))
    row = [l for l in bench.sq_table(dirs).splitlines() if l.startswith("| x pass FP64")][0].split("|")
    assert row[2].strip() == "2048" and row[3].strip() == "100" and row[6].strip() == "10"
    assert row[-2].strip() == "0.25"

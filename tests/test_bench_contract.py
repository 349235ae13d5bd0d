"""Host-side parts of the benchmark's contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_priming_ends_right_after_a_residual_check():
    """The timed region starts at a multiple of the residual interval, after at least
    one whole interval of untimed steps (so the graph used after every check exists)."""
    K = bench.RESIDUAL_INTERVAL
    for w in range(0, 3 * K + 7):
        p = bench.priming_steps(w)
        assert (w + p) % K == 0
        assert K < p <= 2 * K


def test_kernel_hash_covers_the_step_kernel_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0


def test_cpu_baseline_reports_the_contract_fields():
    """The oracle baseline: a positive rate in MLUPS, the thread count it used, its
    kind and the sample it was measured on, and the one-thread rate beside it."""
    r = bench.cpu_baseline(target_s=0.2, single_s=0.1)
    assert r["unit"] == "MLUPS" and r["kind"] == "oracle"
    assert r["value"] > 0 and r["single_thread_value"] > 0 and r["cores"] >= 1
    assert "256x256x16" in r["sample"] and "1 thread" in r["single_thread_sample"]
    assert r["nproc"] >= 1 and isinstance(r["cpu_model"], str)


def test_measured_traffic_reads_the_committed_counter_summary():
    value, path = bench.measured_traffic("step_d3q27_f32dev_duct256")
    assert path is not None and os.path.exists(path)
    assert value is None or value > 3.0e9    # HBM bytes per launch, near the 3.62e9 algorithmic ones
    assert bench.measured_traffic("no_such_kernel") == (None, None)

"""Host-side pieces of bench.py (CPU): the one-GPU guard and the oracle CPU
baseline (one thread and all host cores) on a small workload."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    # imported by name, so that the spawned oracle processes can import it too
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    return bench


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU only" in (r.stdout + r.stderr)


def test_cpu_baseline_reports_one_thread_and_all_cores():
    from paper_2405_10505_amd.inputs import workloads
    b = _bench()
    w = workloads.small_cvt()
    out = b.cpu_baseline(w, 3)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["value"] > 0
    assert "3 FB-LTS coarse steps" in out["sample"]
    ncpu = min(16, len(os.sched_getaffinity(0)))
    if ncpu > 1:
        a = out["all_cores"]
        assert a["cores"] == ncpu and a["value"] > 0
    else:
        pytest.skip("one host core")

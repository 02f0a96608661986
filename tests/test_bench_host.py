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


def test_paper_time_step_order():
    """Largest fine step first (within 2%), then the largest M; the fastest
    row is reported separately."""
    b = _bench()
    rows = [dict(M=4, margin=1.0, dt_fine=10.4, sim_seconds_per_wall_second=194.0),
            dict(M=3, margin=0.8, dt_fine=13.2, sim_seconds_per_wall_second=265.0),
            dict(M=2, margin=0.65, dt_fine=14.55, sim_seconds_per_wall_second=258.0),
            dict(M=4, margin=0.65, dt_fine=14.49, sim_seconds_per_wall_second=230.0),
            dict(M=6, margin=0.65, dt_fine=14.43, sim_seconds_per_wall_second=241.0),
            dict(M=8, margin=0.8, dt_fine=12.7, sim_seconds_per_wall_second=200.0)]
    paper, fastest = b.paper_choice(rows)
    assert (paper["M"], paper["margin"]) == (6, 0.65)
    assert (fastest["M"], fastest["margin"]) == (3, 0.8)
    # a fine step 3% below the best is not "equal": M = 8 at 12.7 s never wins
    paper, _ = b.paper_choice(rows[:3] + [dict(M=8, margin=1.0, dt_fine=14.1, sim_seconds_per_wall_second=1.0)])
    assert (paper["M"], paper["margin"]) == (2, 0.65)

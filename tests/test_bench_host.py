"""Host-side logic of bench.py on the CPU: the one-GPU rule, the counter
summary's validity check, and the workload constants."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_counter_summary_matches_the_measured_kernel_source():
    """The committed counters were taken on the current filter kernel: its
    source hash matches, so the bench reports the traffic; any other text
    would not match."""
    import hashlib
    src = bench.filter_kernel_source()
    assert "k_cheb_blk_lds" in src and "template void cheb_blk<double>" in src
    assert bench.measured_traffic() is not None
    assert bench.measured_traffic(bench.COUNTERS_C3) is not None
    # the 512-column summary holds a row per autotuner candidate; its chosen
    # schedule's row gives the headline bytes, and an unmeasured one gives None
    whole = bench.measured_traffic(bench.COUNTERS_C3)
    rows = [bench.measured_traffic(bench.COUNTERS_C3, (m, cw, g, v, 0, 1))
            for m, cw, g, v in [(1, 0, 1, 0), (2, 64, 64, 0), (2, 32, 64, 4)]]
    assert all(r is not None and 0.9 * whole < r < 1.5 * whole for r in rows)
    assert bench.measured_traffic(bench.COUNTERS_C3, (2, 48, 64, 0, 0, 1)) is None
    assert hashlib.sha256((src + " ").encode()).hexdigest() != \
        hashlib.sha256(src.encode()).hexdigest()


def test_paper_rows_are_the_printed_table():
    assert len(bench.PAPER_ROWS) == 12
    grids = {(r[0], r[1]) for r in bench.PAPER_ROWS}
    assert grids == {(2, 343), (2, 729), (2, 1000), (3, 49), (3, 81), (3, 100)}
    # nmv is about deg * niter (niter printed to the nearest ten) plus the Ritz
    # checks, in every printed row
    for r in bench.PAPER_ROWS:
        deg, niter, nmv = r[5], r[6], r[7]
        assert deg * niter <= nmv <= deg * (niter + 10) + 2 * r[4] + 100


def test_precision_leg_reports_a_failure_instead_of_raising():
    """Without a device the leg's first GPU call fails: the leg returns the
    error, so the rest of the bench line stands."""
    import argparse
    args = argparse.Namespace(prec="f64", tol=1e-8)
    r = bench.precision_leg(None, None, None, args, {"nev": 980}, 38.7, lambda m: None)
    assert set(r) == {"error"} and r["error"]

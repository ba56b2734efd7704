"""Host-side checks of bench.py's command line (no GPU): the one-GPU guard,
the profiling script it prints, and that summarizing an empty output folder
leaves the committed summaries alone."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_script_runs_every_case_under_a_time_limit():
    r = run_bench("--profile-script", "gpurun_out/prof")
    assert r.returncode == 0, r.stderr
    lines = [ln for ln in r.stdout.splitlines() if "rocprofv3" in ln]
    traces = [c for c, (k, _) in bench.PROFILE_CASES.items() if k == "trace"]
    pmcs = [c for c, (k, _) in bench.PROFILE_CASES.items() if k == "pmc"]
    for case in traces:
        assert sum(f"/{case} " in ln for ln in lines) == 1, case
    for case in pmcs:
        for counter in bench.PMC_COUNTERS:
            assert sum(f"/{case}_{counter} " in ln for ln in lines) == 1, (case, counter)
    for ln in lines:
        assert ln.startswith("timeout "), ln
        # counters are never combined with a trace in one run
        assert not ("--pmc" in ln and "--kernel-trace" in ln), ln


def test_summarizing_an_empty_folder_changes_nothing(tmp_path):
    pdir = os.path.join(ROOT, "profiles")
    before = {f: os.stat(os.path.join(pdir, f)).st_mtime_ns for f in os.listdir(pdir)}
    r = run_bench("--summarize-profiles", str(tmp_path))
    assert r.returncode == 0, r.stderr
    after = {f: os.stat(os.path.join(pdir, f)).st_mtime_ns for f in os.listdir(pdir)}
    assert before == after

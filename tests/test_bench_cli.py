"""The benchmark's command line on the CPU: the parts that need no GPU.

* More than one GPU is refused with a message and exit status 2, before any device call.
* The counter summary sums rocprofv3's per-dispatch counter rows over the kernels that match,
  per kernel and in total, and counts the dispatches.
* The algorithmic operation count the roofline uses comes from the committed event counts and
  instruction costs.
"""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, cwd=ROOT):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          cwd=cwd, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "single MI355X" in r.stderr and r.stdout == ""


def test_counter_summary(tmp_path):
    rows = [("1", "void eq::k_sweep<0, false, false>(eq::SweepArgs)", "SQ_WAVES", "10"),
            ("1", "void eq::k_sweep<0, false, false>(eq::SweepArgs)", "SQ_INSTS_VALU", "100"),
            ("2", "void eq::k_sweep<1, false, false>(eq::SweepArgs)", "SQ_WAVES", "12"),
            ("3", "eq::k_stats(long long const*)", "SQ_WAVES", "1000")]
    d = tmp_path / "pmc"
    d.mkdir()
    with open(d / "run_counter_collection.csv", "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for did, name, counter, value in rows:
            fh.write(f'{did},"{name}",{counter},{value}\n')
    r = run_bench("--summarize-counters", str(d), "k_sweep")
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout)
    assert out["dispatches"] == 2
    assert out["sums"] == {"SQ_WAVES": 22.0, "SQ_INSTS_VALU": 100.0}
    per = {k.split("(")[0]: v for k, v in out["per_kernel"].items()}
    assert per["void eq::k_sweep<0, false, false>"] == {"dispatches": 1, "sums": {"SQ_WAVES": 10.0,
                                                                                  "SQ_INSTS_VALU": 100.0}}


def test_algorithmic_operation_count():
    sys.path.insert(0, ROOT)
    import bench
    ops = bench.algorithmic_ops()
    counts = json.load(open(bench.OP_COUNTS_JSON))
    assert counts["workload"] == "dag1000" and counts["K"] == 20000
    assert 700.0 < ops < 1000.0
    # the same events at the fixed prices of the first priced build: no build since is dearer
    fixed = bench.algorithmic_ops(bench.OP_COSTS_FIXED_JSON)
    assert ops <= fixed < 1000.0

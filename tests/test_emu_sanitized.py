"""The library's own sources (C-ABI host code and every kernel) built for the host with a CPU
emulation of HIP, run under AddressSanitizer and UndefinedBehaviorSanitizer (float-to-int
overflow included), and compared with the oracle bit for bit; and the oracle itself under the
same sanitizers.  No GPU is needed.

Each case runs in a child process with the ASan runtime preloaded (tests/emu/cases.py); a
sanitizer finding, a wavefront operation reached by part of a wavefront, a workgroup barrier
that never completes, a readfirstlane of a value that is not uniform across the wavefront, or
a result that differs from the oracle fails the case.  Every device buffer is a separate heap
block, so an access past any buffer of the run (state, inflow slots, tile sums, records,
routed counts, sample tables, tables of the network) is reported where it happens.

The record-and-sojourn cases use the inputs of the GPU case that once ended in a device fault
(100-station layered network, 400 steps, 70 replications, record of steps 40..400, walks
started anywhere including the last two recorded intervals), for both schemes, with and
without a staffing schedule.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emu"))

import build as emu_build  # noqa: E402


@pytest.fixture(scope="module")
def emu_env():
    emu_build.build()
    return emu_build.asan_env()


def run_case(env, *args, timeout=600):
    r = subprocess.run([sys.executable, os.path.join(HERE, "emu", "cases.py"), *map(str, args)], env=env,
                       capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0 and "case ok" in r.stdout, \
        f"case {args} exited {r.returncode}\n--- stdout ---\n{r.stdout[-3000:]}\n--- stderr ---\n{r.stderr[-6000:]}"


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("staff", [0, 1])
def test_record_and_sojourn_sanitized(emu_env, scheme, staff):
    run_case(emu_env, "record_sojourn", scheme, staff)


@pytest.mark.parametrize("scheme", [0, 1])
def test_both_kernels_sanitized(emu_env, scheme):
    run_case(emu_env, "kernels", scheme)


def test_scores_and_reductions_sanitized(emu_env):
    run_case(emu_env, "scores")


def test_batch_graph_and_replay_sanitized(emu_env):
    run_case(emu_env, "batch")


def test_oracle_sanitized(emu_env, tmp_path):
    import oracle
    lib = oracle.build_variant([], str(tmp_path), "liboracle_asan.so",
                               extra_flags=["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                                            "-fno-sanitize-recover=all"])
    run_case(emu_env, "oracle", lib)


def test_allocation_free_entry_point_sanitized(emu_env):
    run_case(emu_env, "noalloc")


def test_stalled_inversion_sums_sanitized(emu_env):
    run_case(emu_env, "stalls")

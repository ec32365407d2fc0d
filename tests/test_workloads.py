"""The synthetic workloads regenerate to the arrays they had when their results were recorded:
every network's SHA-256 (and the batch's combined hash) equals tests/golden/workload_fingerprints.json,
written by tests/golden/make_fingerprints.py."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_fingerprints  # noqa: E402


def test_workload_fingerprints_are_stable():
    want = json.load(open(os.path.join(HERE, "golden", "workload_fingerprints.json")))
    assert make_fingerprints.workload_fingerprints() == want

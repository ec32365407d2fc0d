"""The benchmark's operation count per station-step is built from two committed tables; both
must describe the current sources.

* tests/isa/op_costs_gfx950.json: the VALU instructions of each sampler building block in the
  gfx950 build (probes compiled from eq_device.h) and the event costs made from them.
* tests/golden/op_counts_dag1000.json: the oracle's event counts per station-step on the
  benchmark workload (tests/golden/make_op_counts.py), made with the current oracle source on
  the current network; and they are the counts of a fresh oracle run over a shorter horizon to
  within the difference between horizons (the queues' build-up changes the mix only mildly).
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, os.path.join(HERE, "isa"))

import netgen  # noqa: E402
import oracle  # noqa: E402
import op_costs  # noqa: E402


def test_op_cost_table_is_current():
    table = json.load(open(op_costs.COSTS_JSON))
    p = op_costs.probe_counts()
    assert p == table["probes"]
    assert op_costs.event_costs(p) == table["events"]
    assert p["philox"] >= 40 and p["div"] >= 5          # sanity: real instruction counts


def test_op_counts_are_current():
    rec = json.load(open(os.path.join(HERE, "golden", "op_counts_dag1000.json")))
    src = open(os.path.join(ROOT, "oracle", "euler_oracle.c"), "rb").read()
    assert rec["oracle_sha256"] == hashlib.sha256(src).hexdigest(), "regenerate with tests/golden/make_op_counts.py"
    w = netgen.config3()
    assert rec["network_sha256"] == w.net.fingerprint()
    costs = json.load(open(op_costs.COSTS_JSON))["events"]
    assert set(rec["backward"]) | {"station_step", "binomial_call"} == set(costs)
    # a fresh count over the first quarter of the horizon, four replications
    oracle.op_counts(reset=True)
    oracle.run(w.net, oracle.BACKWARD, w.dt, w.K // 4, 0, np.arange(4))
    c = oracle.op_counts(reset=True)
    ss = c.pop("station_step")
    fresh = {k: v / ss for k, v in c.items()}
    a = op_costs.algorithmic_ops(fresh, costs)
    b = op_costs.algorithmic_ops(rec["backward"], costs)
    assert abs(a - b) < 0.15 * b, (a, b)

"""Write tests/golden/op_counts_dag1000.json: the oracle's event counts (Philox blocks, uniforms,
sampler set-ups, search steps, rejection attempts and their logarithmic tests, routed edges,
pushes) per station-step on the 1000-station workload of the benchmark, over its full horizon
(20000 steps), replications 0..15, each scheme.  Calls only the oracle (and netgen for the
input).  The benchmark prices these events with the instruction counts of tests/isa/op_costs.py
to state the algorithm's operations per station-step."""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import netgen  # noqa: E402
import oracle  # noqa: E402


def op_counts(reps: int = 16) -> dict:
    w = netgen.config3()
    out = {"workload": "dag1000", "network_sha256": w.net.fingerprint(), "K": w.K, "replications": reps,
           "oracle_sha256": hashlib.sha256(open(os.path.join(ROOT, "oracle", "euler_oracle.c"), "rb").read()).hexdigest()}
    for scheme, name in ((oracle.BACKWARD, "backward"), (oracle.FORWARD, "forward")):
        oracle.op_counts(reset=True)
        oracle.run(w.net, scheme, w.dt, w.K, 0, np.arange(reps))
        c = oracle.op_counts(reset=True)
        ss = c["station_step"]
        assert ss == w.net.n * w.K * reps
        out[name] = {k: v / ss for k, v in c.items() if k != "station_step"}
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "op_counts_dag1000.json"), "w") as fh:
        json.dump(op_counts(), fh, indent=1, sort_keys=True)
        fh.write("\n")

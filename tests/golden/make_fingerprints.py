"""Write tests/golden/workload_fingerprints.json: the SHA-256 of every synthetic workload's
network arrays (netgen.Network.fingerprint) and of the run parameters that go with it.  numpy's
Generator streams are not promised stable across numpy versions, so a test regenerates the
workloads and compares with these values.  Calls only netgen (input generation)."""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import netgen  # noqa: E402


def workload_fingerprints() -> dict:
    out = {}
    for name, make in (("tandem4", netgen.config1), ("layered100", netgen.config2), ("dag1000", netgen.config3),
                       ("grad1000", netgen.config5)):
        w = make()
        out[name] = {"network": w.net.fingerprint(), "n": int(w.net.n), "nnz": int(w.net.nnz), "dt": w.dt, "T": w.T,
                     "reps": w.reps}
    hold, staff = netgen.config5_costs(netgen.config5().net.n)
    out["grad1000"]["costs"] = hashlib.sha256(np.ascontiguousarray(hold).tobytes() +
                                              np.ascontiguousarray(staff).tobytes()).hexdigest()
    h = hashlib.sha256()
    ws = netgen.config4()
    for w in ws:
        h.update(w.net.fingerprint().encode())
        h.update(repr((w.T, w.dt, w.reps, w.net_id)).encode())
    out["batch512"] = {"networks": h.hexdigest(), "count": len(ws),
                       "station_steps": int(sum(w.net.n * w.K for w in ws) * ws[0].reps)}
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "workload_fingerprints.json"), "w") as fh:
        json.dump(workload_fingerprints(), fh, indent=1, sort_keys=True)
        fh.write("\n")

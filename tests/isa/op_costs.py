"""VALU instructions per building block of the samplers in the gfx950 build, and from them the
algorithmic operation cost of every event the oracle counts (oracle.op_counts); run as a script
it writes tests/isa/op_costs_gfx950.json, which the benchmark reads.

`probe_counts()` compiles tests/isa/probes.hip to gfx950 assembly with the library's own flags
and counts the vector-ALU instructions (v_*) between the markers of each probe.  `event_costs()`
prices each counted event as the sum of the building blocks and plain arithmetic operations the
samplers' source performs for it (the formulas below, read off eq_device.h and eq_sweep.h):
compiler bookkeeping (register moves, loop control, address arithmetic, the wavefront
reductions' shuffles) is not algorithmic work and is left out.
"""
import json
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2402_13259_amd import build as libbuild  # noqa: E402

PROBES = ["philox", "unit", "ln", "ln1p_small", "ln_corr", "ex", "expm1_small", "div", "sqrt", "floor",
          "stirling_series", "fma64"]


def assembly() -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in libbuild.FLAGS if f not in ("-shared", "-fPIC")]
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "probes.s")
        subprocess.run([hipcc, *flags, "-S", "--offload-device-only", "-I", libbuild.CSRC, "-I", libbuild.INCLUDE,
                        os.path.join(HERE, "probes.hip"), "-o", out], check=True, capture_output=True)
        return open(out).read()


def probe_counts(asm: str = None) -> dict:
    """{probe: VALU instructions between its markers}."""
    asm = assembly() if asm is None else asm
    out = {}
    for name in PROBES:
        m = re.search(r"_Z\d+probe_%s\w*:(.*?)\.Lfunc_end" % name, asm, re.S)
        assert m, f"probe_{name} not found in the assembly"
        body = m.group(1)
        i, j = body.index("; probe begin"), body.index("; probe end")
        assert body.count("; probe begin") == 1 and body.count("; probe end") == 1
        region = body[i:j]
        out[name] = sum(1 for line in region.splitlines() if re.match(r"\s+v_\w+", line))
    return out


def event_costs(p: dict) -> dict:
    """Algorithmic operations per counted event (plain operations as 1 each, building blocks as
    counted in the build).  ln1p and exm1 take their general branches, stirling_tail its series."""
    # ln1p, |x| >= 1/4: |x| test, u = 1 + x, the rounding error (two subtractions, a select), c / u
    L1P = 5 + p["div"] + p["ln_corr"]
    ST = p["stirling_series"]
    # exm1, |x| >= ln2 / 2: range tests, k = rint(x / ln2), two reduction fmas, 2^k, the final fma
    EXM1 = 8 + p["expm1_small"]
    return {
        # Philox4x32-10 block; one uniform: the conversion
        "philox": p["philox"],
        "uniform": p["unit"],
        # every binomial draw: n <= 0, n p < 80 (cvt, mul, cmp), the flip n - k
        "binomial_call": 5,
        # inversion: g = r (n + 1), f0 = e^{n lq} (the exponential's steps, with the exponent scale:
        # its test, the offset, the uniform's factor), kmax, go;  step: f fma(g, 1/k, -r), F + f, k,
        # two tests
        "bin_inv": 3 + 1 + p["ex"] + 4 + 1 + 2,
        "bin_inv_step": 6,
        # BTRS set-up (spq, b, a, c, alpha, vr, mode, nm, the mode's log-ratio and Stirling terms)
        "btrs": 30 + p["sqrt"] + 3 * p["div"] + p["floor"] + p["fma64"] + L1P + 2 * ST,
        # attempt: us, candidate k = floor((2a / us + b) u + c), the squeeze test
        "btrs_try": 8 + p["div"] + p["floor"],
        # the logarithmic test: lhs = ln(v alpha / (a / us^2 + b)), rhs by Stirling's series
        "btrs_slow": 18 + 4 * p["div"] + p["ln"] + 2 * L1P + p["fma64"] + 2 * ST,
        # PTRS set-up, attempt, logarithmic test (the same pattern)
        "ptrs": 10 + p["sqrt"] + p["ln"] + 2 * p["div"],
        "ptrs_try": 8 + p["div"] + p["floor"],
        "ptrs_slow": 14 + 3 * p["div"] + p["ln"] + L1P + ST,
        # Poisson inversion: e^{-lam};  step: k + 1, p lam / k, F + p, three tests
        "pois_inv": 2 + p["ex"],
        "pois_inv_step": 8,
        # Erlang: d, c = 1 / sqrt(9 d), T = G / (m mu);  polar try: x1, x2, s, test;
        # attempt: z = x1 sqrt(-2 ln s / s), t, t^3, squeeze;  logarithmic test: ln u, ln v
        "gamma": 3 + p["sqrt"] + 2 * p["div"],
        "gamma_polar": 8,
        "gamma_try": 12 + p["ln"] + p["div"] + p["sqrt"],
        "gamma_slow": 6 + 2 * p["ln"],
        # x > m: the split probability (dt / T, or the T <= h branch's expm1) and its constants
        "bin_prep": 7 + 2 * p["div"] + L1P,
        "expm1": 2 + EXM1,
        # a departure draw's branch; a routed edge (rem > 0, rem - R); a push (address, add)
        "depart": 2,
        "edge": 2,
        "push": 3,
        # per station-step: x = N + inflow, N = x - D + A, q = (N - m)^+, three statistic sums
        "station_step": 8,
    }


COSTS_JSON = os.path.join(HERE, "op_costs_gfx950.json")


def algorithmic_ops(counts: dict, costs: dict) -> float:
    """Operations per station-step: every counted event per station-step times its cost, plus
    the per-station-step work and one binomial dispatch per inversion or BTRS draw."""
    total = costs["station_step"] + costs["binomial_call"] * (counts["bin_inv"] + counts["btrs"])
    for name, per_ss in counts.items():
        total += per_ss * costs[name]
    return total


if __name__ == "__main__":
    p = probe_counts()
    table = {"probes": p, "events": event_costs(p)}
    with open(COSTS_JSON, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(table, indent=1))

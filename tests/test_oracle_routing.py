"""Pins of the oracle's multinomial routing split on rows with several edges (Section 2.2:
the routed counts of a station's departures are Multinomial(D, p_i1, ..., p_in, p_exit);
Algorithm 1 routes every station's departures this way).

* Conditional on the departure count D = d, the joint counts (R_1, R_2, R_3, exit) that the
  oracle records for station 0 of the branching network follow Multinomial(d, .5, .25, .15, .1)
  (G-test over every composition of d), and each edge's total is p_e times the total departures.
* Every recorded interval balances exactly against the network's own targets.
* Against the exact DES on the same network (constant rates, a feed-forward Jackson network):
  the DES matches each station's M/M/c mean (Erlang C) with the total rates of the traffic
  equations; the two schemes bracket the DES (Theorem 2) with the steady per-station gap
  lambda~_i h; their average is within its second-order error of Erlang C.
* Planted mistakes in the oracle's split (edges taken in reverse order, a swapped target, the
  next edge's conditional probability, the unconditional probability, the remainder given to
  the last edge) each fail at least one of these pins: a mutated copy of the oracle is built on
  the CPU and run through them.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.stats as st

import netgen
import oracle
from test_oracle_des import erlang_c

P0 = np.array([0.5, 0.25, 0.15, 0.1])   # station 0: edges to 1, 2, 3 and the exit


def record_branching(K=400, R=800, dt=0.1, seed=3):
    net = netgen.branching()
    return net, oracle.run_record(net, oracle.BACKWARD, dt, K, seed, np.arange(R), rec_t0=1, rec_len=K)


def joint_multinomial_pvalues(rec, dmax=6, min_expected=5.0):
    """For each d in 1..dmax: G-test p-value of station 0's recorded (R_1, R_2, R_3, exit) given
    D_0 = d against Multinomial(d, P0), cells of low expectation merged."""
    D = rec["D"][:, :, 0].ravel()
    R = rec["R"][:, :, 0:3].reshape(-1, 3)
    out = {}
    for d in range(1, dmax + 1):
        sel = D == d
        if sel.sum() < 200:
            continue
        rows = np.concatenate([R[sel], (d - R[sel].sum(1))[:, None]], axis=1)
        assert (rows >= 0).all()
        comps = [c for c in itertools.product(range(d + 1), repeat=3) if sum(c) <= d]
        comps = [c + (d - sum(c),) for c in comps]
        index = {c: k for k, c in enumerate(comps)}
        obs = np.zeros(len(comps))
        for r in map(tuple, rows):
            obs[index[r]] += 1
        pmf = np.array([st.multinomial.pmf(c, d, P0) for c in comps])
        order = np.argsort(-pmf)
        obs, exp = obs[order], pmf[order] * sel.sum()
        # merge the rarest cells until every cell expects at least min_expected
        while len(exp) > 1 and exp[-1] < min_expected:
            exp[-2] += exp[-1]
            obs[-2] += obs[-1]
            exp, obs = exp[:-1], obs[:-1]
        nz = obs > 0
        G = 2.0 * float((obs[nz] * np.log(obs[nz] / exp[nz])).sum())
        out[d] = float(st.chi2.sf(G, len(exp) - 1))
    return out


def check_joint_multinomial(rec):
    p = joint_multinomial_pvalues(rec)
    assert len(p) >= 4, p
    assert min(p.values()) > 1e-4 / len(p), p


def check_edge_totals(rec):
    """Sum over intervals of R_e against p_e times the summed departures (z-scores)."""
    D = rec["D"][:, :, 0].astype(np.float64).ravel()
    R = rec["R"][:, :, 0:3].reshape(-1, 3).astype(np.float64)
    n = D.sum()
    for e in range(3):
        z = (R[:, e].sum() - P0[e] * n) / math.sqrt(n * P0[e] * (1 - P0[e]))
        assert abs(z) < 5, (e, z)
    zx = ((D - R.sum(1)).sum() - P0[3] * n) / math.sqrt(n * P0[3] * (1 - P0[3]))
    assert abs(zx) < 5, zx


def check_balance(net, rec):
    """N_tau - N_{tau-1} + D_tau equals the routed inflow by the network's own targets (plus
    external arrivals at the source)."""
    Rn, K, n = rec["N"].shape
    inflow = np.zeros(rec["N"].shape, np.int64)
    for i in range(n):
        for e in range(net.row_ptr[i], net.row_ptr[i + 1]):
            inflow[:, :, net.col[e]] += rec["R"][:, :, e]
    prev = np.concatenate([np.zeros((Rn, 1, n), np.int64), rec["N"][:, :-1, :]], axis=1)
    ext = rec["N"] - prev + rec["D"] - inflow
    assert (ext[:, :, 1:] == 0).all()
    assert (ext[:, :, 0] >= 0).all()


def erlang_c_means(net):
    lt = net.total_rates()
    out = []
    for i in range(net.n):
        c, mu = int(net.servers[i]), float(net.mu[i])
        rho = lt[i] / (c * mu)
        out.append(c * rho + rho / (1 - rho) * erlang_c(c, rho))
    return np.array(out), lt


def long_runs(h=0.02, K=3000, R=2000, seed=0):
    """Both schemes (common random numbers) and the DES on the branching network; second-half
    time averages from the counter-based streams (a run of K/2 steps is the first half)."""
    net = netgen.branching()
    reps = np.arange(R)
    out = {"net": net, "h": h, "R": R}
    for s in (oracle.BACKWARD, oracle.FORWARD):
        full = oracle.run(net, s, h, K, seed, reps)
        half = oracle.run(net, s, h, K // 2, seed, reps)
        out[s] = {"final": full["final"], "avg2": (full["sumN"] - half["sumN"]) / (K - K // 2)}
    d = oracle.des(net, h, K, seed + 101, reps)
    dh = oracle.des(net, h, K // 2, seed + 101, reps)
    out["des"] = {"final": d["final"], "avg2": (d["sumN"] - dh["sumN"]) / (K - K // 2)}
    return out


def check_average_scheme_vs_erlang_c(t):
    """The average of the two schemes' second-half means is within 4.5 SE (plus a second-order
    allowance of 5 % of the per-station gap lambda~ h) of the Erlang C mean of each station."""
    EN, lt = erlang_c_means(t["net"])
    R = t["R"]
    avg = 0.5 * (t[oracle.BACKWARD]["avg2"] + t[oracle.FORWARD]["avg2"])
    for i in range(t["net"].n):
        se = avg[:, i].std() / math.sqrt(R)
        assert abs(avg[:, i].mean() - EN[i]) < 4.5 * se + 0.05 * lt[i] * t["h"] + 0.01, (i, avg[:, i].mean(), EN[i])


# ---------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def branch_record():
    return record_branching()


def test_branching_total_rates():
    net = netgen.branching()
    assert np.allclose(net.total_rates(), [20, 10, 5, 7, 9.5])
    assert net.is_index_dag() and all(np.diff(net.row_ptr)[:4] >= 1) and np.diff(net.row_ptr)[0] == 3


def test_split_given_departures_is_multinomial(branch_record):
    check_joint_multinomial(branch_record[1])


def test_split_edge_totals(branch_record):
    check_edge_totals(branch_record[1])


def test_split_balances_with_the_networks_targets(branch_record):
    check_balance(*branch_record)


@pytest.fixture(scope="module")
def branch_long():
    return long_runs()


def test_des_matches_erlang_c_per_station(branch_long):
    """The DES routes by its own categorical draw: each station's second-half mean is the
    M/M/c mean at the total rate lambda~_i of the traffic equations (Jackson network)."""
    t = branch_long
    EN, _ = erlang_c_means(t["net"])
    for i in range(t["net"].n):
        d = t["des"]["avg2"][:, i]
        assert abs(d.mean() - EN[i]) < 4.5 * d.std() / math.sqrt(t["R"]) + 0.02, (i, d.mean(), EN[i])


def test_steady_gap_per_station(branch_long):
    """Theorem 2 (i) on a branching network: E[N^b(i)] - E[N^f(i)] = lambda~_i h."""
    t = branch_long
    lt = t["net"].total_rates()
    diff = t[oracle.BACKWARD]["avg2"] - t[oracle.FORWARD]["avg2"]
    for i in range(t["net"].n):
        se = diff[:, i].std() / math.sqrt(t["R"])
        assert abs(diff[:, i].mean() - lt[i] * t["h"]) < 4.5 * se + 0.01 * lt[i] * t["h"], (i, diff[:, i].mean())


def test_schemes_bracket_des(branch_long):
    """Means and CDFs (two-sample DKW band) at the horizon: F_b - eps <= F_DES <= F_f + eps."""
    t = branch_long
    R = t["R"]
    se = lambda x: x.std() / math.sqrt(R)
    eps = 2 * math.sqrt(math.log(2 / 1e-3) / (2 * R))
    for i in range(t["net"].n):
        b, f, d = (t[k]["avg2"][:, i] for k in (oracle.BACKWARD, oracle.FORWARD, "des"))
        assert f.mean() - 3 * se(f) <= d.mean() + 3 * se(d)
        assert d.mean() - 3 * se(d) <= b.mean() + 3 * se(b)
        xs = np.arange(0, 60)
        F = {k: np.searchsorted(np.sort(t[k]["final"][:, i]), xs, side="right") / R
             for k in (oracle.BACKWARD, oracle.FORWARD, "des")}
        assert np.all(F[oracle.BACKWARD] - eps <= F["des"])
        assert np.all(F["des"] <= F[oracle.FORWARD] + eps)


def test_average_scheme_matches_erlang_c(branch_long):
    check_average_scheme_vs_erlang_c(branch_long)


# ---------------------------------------------------------------------------------------------
LOOP = "for (int32_t e = net->row_ptr[i]; e < net->row_ptr[i + 1] && rem > 0; ++e) {"
DRAW = "int32_t R = orc_binomial(rem, c->q[e], &S);"
PUSH = "Ain[net->col[e]] += R;"
NEXT = "(e + 1 < net->row_ptr[i + 1] ? e + 1 : net->row_ptr[i])"

MUTANTS = {
    "reverse_order": [(LOOP, "for (int32_t e = net->row_ptr[i + 1] - 1; e >= net->row_ptr[i] && rem > 0; --e) {")],
    "swapped_target": [(PUSH, f"Ain[net->col[{NEXT}]] += R;")],
    "next_edge_probability": [(DRAW, f"int32_t R = orc_binomial(rem, c->q[{NEXT}], &S);")],
    "unconditional_probability": [(DRAW, "int32_t R = orc_binomial(rem, net->prob[e], &S);")],
    "last_edge_takes_remainder": [(DRAW, "int32_t R = e + 1 == net->row_ptr[i + 1] ? rem : "
                                         "orc_binomial(rem, c->q[e], &S);")],
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_routing_mistakes_fail_a_pin(name, tmp_path):
    """A copy of the oracle with one planted mistake in the split fails at least one pin."""
    path = oracle.build_variant(MUTANTS[name], str(tmp_path), f"liboracle_{name}.so")
    failed = []
    with oracle.using_library(path):
        net, rec = record_branching()
        for label, check in (("joint", lambda: check_joint_multinomial(rec)), ("totals", lambda: check_edge_totals(rec)),
                             ("balance", lambda: check_balance(net, rec)),
                             ("erlang_c", lambda: check_average_scheme_vs_erlang_c(long_runs(K=2000, R=1000)))):
            try:
                check()
            except AssertionError:
                failed.append(label)
    assert failed, f"planted mistake {name} passed every routing pin"

"""Pins of the oracle's likelihood-ratio scores and gradient estimator.

The score of a draw is the parameter-derivative of the log-density of the random
variables the draw consumed (GenerateDeparture, Lemma 1 / Algorithm 3: a binomial, or an
Erlang time followed by a mu-free or a binomial split; arrivals: Poisson).  The pins do not
retype those formulas: they check E[S 1{D = d}] = dP(D = d)/dtheta against the exact
pure-death law differentiated numerically, the gradient of an exactly computed expected
cost of the Euler chain, and common-random-number finite differences of the simulator.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats as st

import netgen
import oracle


def death_law(x, m, mu, h):
    """P(D = d), d = 0..x, for a pure-death process from x with rates min(y, m) mu over h."""
    Q = np.zeros((x + 1, x + 1))
    for y in range(1, x + 1):
        Q[y, y - 1] = min(y, m) * mu
        Q[y, y] = -min(y, m) * mu
    row = scipy.linalg.expm(Q * h)[x]          # row[y] = P(state y at h)
    return np.array([row[x - d] for d in range(x + 1)])


def naive_law(x, m, mu, h):
    b = min(x, m)
    lam = b * mu * h
    p = st.poisson.pmf(np.arange(x + 1), lam)
    p[x] = st.poisson.sf(x - 1, lam)
    return p


def d_dtheta(fun, theta, rel=1e-5):
    d = theta * rel
    return (fun(theta + d) - fun(theta - d)) / (2 * d)


def check_score_identity(vals, scores, law, law_derivative, tol=4.5):
    """Per outcome d: mean of S 1{V = d} equals dP(V = d)/dtheta; and E[S] = 0.  Outcomes
    expected fewer than 30 times are not tested one by one."""
    M = len(vals)
    vals = vals.astype(int)
    sc = scores.astype(np.float64)
    assert abs(sc.mean()) < tol * sc.std() / math.sqrt(M)
    tested = 0
    for d, dp in enumerate(law_derivative):
        if law[d] * M < 30:
            continue
        tested += 1
        z = sc * (vals == d)
        se = z.std() / math.sqrt(M)
        assert abs(z.mean() - dp) < tol * se + 1e-9, (d, z.mean(), dp, se)
    assert tested >= 3


@pytest.mark.parametrize("x,m,mu,h", [(4, 6, 1.5, 0.2),      # x <= m: binomial
                                      (5, 3, 2.0, 0.5),      # x > m, T <= h mostly
                                      (9, 3, 2.0, 0.3),      # x > m, T > h mostly
                                      (7, 1, 0.8, 1.5)])     # single server, both cases
def test_departure_score_identity(x, m, mu, h):
    M = 400_000
    v, s = oracle.sample_score(oracle.SMP_GENDEP, M, seed=71, x=x, m=m, f0=mu, f1=h)
    mu32, h32 = float(np.float32(mu)), float(np.float32(h))
    deriv = d_dtheta(lambda t: death_law(x, m, t, h32), mu32)
    check_score_identity(v, s, death_law(x, m, mu32, h32), deriv)


def test_departure_score_zero_state():
    v, s = oracle.sample_score(oracle.SMP_GENDEP, 100, x=0, m=3, f0=1.0, f1=0.1)
    assert not v.any() and not s.any()


@pytest.mark.parametrize("x,m,mu,h", [(4, 6, 1.5, 0.2), (6, 2, 3.0, 0.4)])
def test_naive_departure_score_identity(x, m, mu, h):
    M = 400_000
    v, s = oracle.sample_score(oracle.SMP_GENDEP_NAIVE, M, seed=72, x=x, m=m, f0=mu, f1=h)
    mu32, h32 = float(np.float32(mu)), float(np.float32(h))
    deriv = d_dtheta(lambda t: naive_law(x, m, t, h32), mu32)
    check_score_identity(v, s, naive_law(x, m, mu32, h32), deriv)


@pytest.mark.parametrize("lam0,g", [(3.7, 0.4), (55.0, 0.25)])   # inversion and PTRS ranges
def test_arrival_score_identity(lam0, g):
    M = 400_000
    v, s = oracle.sample_score(oracle.SMP_POISSON, M, seed=73, sub=0, f0=lam0, f1=g)
    l32, g32 = float(np.float32(lam0)), float(np.float32(g))
    top = int(v.max()) + 1
    deriv = d_dtheta(lambda t: st.poisson.pmf(np.arange(top), t * g32), l32)
    check_score_identity(v, s, st.poisson.pmf(np.arange(top), l32 * g32), deriv)


def exact_mean_cost(lam, mu, c, h, K, scheme, naive=False, nmax=70):
    """(1/K) sum_{tau=1..K} E[(N_tau - c)^+] for one station, from the exact law of the chain."""
    arr_p = st.poisson.pmf(np.arange(nmax + 1), lam * h)
    dep = np.zeros((nmax + 1, nmax + 1))
    for x in range(nmax + 1):
        law = naive_law(x, c, mu, h) if naive else death_law(x, c, mu, h)
        for d in range(x + 1):
            dep[x, x - d] += law[d]
    arr = np.zeros((nmax + 1, nmax + 1))
    for x in range(nmax + 1):
        arr[x, x:] = arr_p[:nmax + 1 - x]
        arr[x, nmax] += 1.0 - arr_p[:nmax + 1 - x].sum()     # mass beyond the cut stays at nmax
    T = dep @ arr if scheme == oracle.BACKWARD else arr @ dep
    q = np.maximum(np.arange(nmax + 1) - c, 0).astype(float)
    p = np.zeros(nmax + 1)
    p[0] = 1.0
    tot = 0.0
    for _ in range(K):
        p = p @ T
        tot += p @ q
    return tot / K


@pytest.mark.parametrize("scheme,naive", [(0, False), (1, False), (0, True)])
def test_gradient_matches_exact_chain(scheme, naive):
    lam, mu, c, h, K = 6.0, 1.0, 5, 0.3, 25
    net = netgen.single_station(lam, mu, c)
    R = 120_000
    res = oracle.run(net, scheme, h, K, 404, np.arange(R), dep_mode=int(naive), scores=True)
    f = oracle.cost_per_rep(res["sumQ"], np.ones(1), K)
    g, se = oracle.lr_gradient(f, np.concatenate([res["score_mu"], res["score_lam"]], axis=1))
    l32, m32, h32 = (float(np.float32(v)) for v in (lam, mu, h))
    exact = exact_mean_cost(l32, m32, c, h32, K, scheme, naive)
    assert exact > 0.2                     # the cost is not degenerate
    assert abs(f.mean() - exact) < 4.5 * f.std() / math.sqrt(R)
    dmu = d_dtheta(lambda t: exact_mean_cost(l32, t, c, h32, K, scheme, naive), m32)
    dlam = d_dtheta(lambda t: exact_mean_cost(t, m32, c, h32, K, scheme, naive), l32)
    assert dmu < 0 < dlam
    assert abs(g[0] - dmu) < 4 * se[0], (g[0], dmu, se[0])
    assert abs(g[1] - dlam) < 4 * se[1], (g[1], dlam, se[1])
    assert se[0] < 0.2 * abs(dmu) and se[1] < 0.2 * abs(dlam)   # the check has power


def feedforward_net():
    return netgen.three_station()


def test_scores_leave_the_simulation_unchanged():
    net = feedforward_net()
    for scheme in (0, 1):
        a = oracle.run(net, scheme, 0.2, 30, 9, np.arange(50))
        b = oracle.run(net, scheme, 0.2, 30, 9, np.arange(50), scores=True)
        for k in ("final", "sumN", "sumQ", "sumD"):
            assert np.array_equal(a[k], b[k])


def test_scores_have_mean_zero():
    """E[S_j] = 0 for every parameter, with all departure branches visited."""
    net = feedforward_net()
    R = 40_000
    res = oracle.run(net, 1, 0.2, 40, 11, np.arange(R), scores=True)
    S = np.concatenate([res["score_mu"], res["score_lam"]], axis=1).astype(np.float64)
    assert (res["sumQ"] > 0).mean(axis=0).min() > 0.3       # x > m occurs at every station
    z = S.mean(axis=0) / (S.std(axis=0) / math.sqrt(R))
    assert np.abs(z).max() < 4.0, z


@pytest.mark.parametrize("scheme", [0, 1])
def test_gradient_matches_crn_finite_differences(scheme):
    """Each mu_i and lambda0_s: LR estimate vs central differences of the simulated cost
    with common random numbers (same seed, same replications), within 4 combined SE."""
    net = feedforward_net()
    h, K, R, seed = 0.2, 40, 60_000, 12
    hold = np.array([1.0, 2.0, 1.5])
    base = oracle.run(net, scheme, h, K, seed, np.arange(R), scores=True)
    f = oracle.cost_per_rep(base["sumQ"], hold, K)
    g, se = oracle.lr_gradient(f, np.concatenate([base["score_mu"], base["score_lam"]], axis=1))
    params = [("mu", i) for i in range(3)] + [("lambda0", s) for s in range(2)]
    for j, (name, i) in enumerate(params):
        arr = getattr(net, name).astype(np.float64)
        delta = 0.03 * arr[i]
        fs = []
        for sign in (+1, -1):
            a = arr.copy()
            a[i] += sign * delta
            net2 = net.replace(**{name: a.astype(np.float32)})
            d = float(np.float32(a[i])) - float(getattr(net, name)[i])
            r = oracle.run(net2, scheme, h, K, seed, np.arange(R))
            fs.append((oracle.cost_per_rep(r["sumQ"], hold, K), d))
        diff = (fs[0][0] - fs[1][0]) / (fs[0][1] - fs[1][1])
        fd, fd_se = diff.mean(), diff.std() / math.sqrt(R)
        assert abs(g[j] - fd) < 4 * math.hypot(se[j], fd_se), (name, i, g[j], se[j], fd, fd_se)


# ---------------------------------------------------------------------------------------------
# Reachability-pruned estimator: parameter j's score is correlated only with the cost of the
# stations that parameter j can reach (its station and everything downstream).  Pinned on the
# exact law of a two-station tandem, where the downstream station's cost depends on the upstream
# service rate (a pruning that drops it is biased) and the upstream cost does not depend on
# the downstream rate (keeping it only adds variance).
def tandem_exact_cost(lam, mu0, mu1, c0, c1, p, h, K, hold, nmax=40):
    """(1/K) sum_{tau=1..K} E[sum_i hold_i (N_tau,i - c_i)^+] for the backward scheme of the
    tandem 0 -> 1 (routing probability p, exit 1 - p; station 1 exits), from empty, by
    propagating the exact joint law of (N_0, N_1) (mass beyond nmax kept at nmax)."""
    N = nmax + 1
    arr = st.poisson.pmf(np.arange(N), lam * h)
    shift = np.zeros((N, N))                      # shift[y, x'] = P(y + A = x')
    for y in range(N):
        shift[y, y:] = arr[:N - y]
        shift[y, N - 1] += 1.0 - arr[:N - y].sum()
    U = np.zeros((N, N, N))                       # U[x0, r, x0'] = sum_d0 P(d0|x0) Bin(r; d0, p) shift[x0-d0, x0']
    for x0 in range(N):
        law = death_law(x0, c0, mu0, h)
        for d0 in range(x0 + 1):
            U[x0, :d0 + 1, :] += law[d0] * st.binom.pmf(np.arange(d0 + 1), d0, p)[:, None] * shift[x0 - d0][None, :]
    M1 = np.zeros((N, N, N))                      # M1[r, x1, x1'] = P(x1 - D1 + r = x1')
    for x1 in range(N):
        law = death_law(x1, c1, mu1, h)
        for d1 in range(x1 + 1):
            for r in range(N):
                M1[r, x1, min(x1 - d1 + r, N - 1)] += law[d1]
    P = np.zeros((N, N))
    P[0, 0] = 1.0
    q0 = hold[0] * np.maximum(np.arange(N) - c0, 0)
    q1 = hold[1] * np.maximum(np.arange(N) - c1, 0)
    tot = 0.0
    for _ in range(K):
        V = np.einsum("ab,rbc->arc", P, M1)
        P = np.einsum("arx,ary->xy", U, V)
        tot += q0 @ P.sum(1) + q1 @ P.sum(0)
    return tot / K


TANDEM2 = dict(lam=3.0, mu0=2.0, mu1=1.5, c0=2, c1=2, p=0.8, h=0.25, K=24, hold=(4.0, 1.0))


def tandem2_net():
    t = TANDEM2
    return netgen.tandem(2, p=t["p"], lam=t["lam"]).replace(mu=np.array([t["mu0"], t["mu1"]], np.float32),
                                                            servers=np.array([t["c0"], t["c1"]], np.int32))


@pytest.fixture(scope="module")
def tandem2_exact_and_sample():
    t = TANDEM2
    net = tandem2_net()
    l32, m0, m1, p32, h32 = (float(np.float32(v)) for v in (t["lam"], t["mu0"], t["mu1"], t["p"], t["h"]))
    q = float(net.prob[0])

    def J(lam=l32, mu0=m0, mu1=m1):
        return tandem_exact_cost(lam, mu0, mu1, t["c0"], t["c1"], q, h32, t["K"], t["hold"])

    exact = np.array([d_dtheta(lambda v: J(mu0=v), m0), d_dtheta(lambda v: J(mu1=v), m1),
                      d_dtheta(lambda v: J(lam=v), l32)])
    R = 200_000
    res = oracle.run(net, oracle.BACKWARD, t["h"], t["K"], 515, np.arange(R), scores=True)
    S = np.concatenate([res["score_mu"], res["score_lam"]], axis=1)
    return {"net": net, "J": J(), "exact": exact, "res": res, "S": S, "R": R}


def test_tandem2_exact_cost_matches_the_oracle(tandem2_exact_and_sample):
    t, d = TANDEM2, tandem2_exact_and_sample
    f = oracle.cost_per_rep(d["res"]["sumQ"], np.array(t["hold"]), t["K"])
    assert d["J"] > 0.3
    assert abs(f.mean() - d["J"]) < 4.5 * f.std() / math.sqrt(d["R"])


def test_reach_sets_of_the_tandem():
    reach = oracle.reach_sets(tandem2_net())
    assert reach.tolist() == [[True, True], [False, True], [True, True]]


def test_pruned_gradient_matches_exact_chain(tandem2_exact_and_sample):
    t, d = TANDEM2, tandem2_exact_and_sample
    hold = np.array(t["hold"])
    reach = oracle.reach_sets(d["net"])
    g, se = oracle.lr_gradient_reach(d["res"]["sumQ"], hold, t["K"], d["S"], reach)
    ex = d["exact"]
    assert ex[0] < 0 and ex[1] < 0 < ex[2]
    assert np.all(np.abs(g - ex) < 4 * se), (g, ex, se)
    assert np.all(se < 0.2 * np.abs(ex)), (se, ex)                      # the check has power
    # against the full-cost estimator: the same expectation, less variance where pruning applies
    gf, sef = oracle.lr_gradient(oracle.cost_per_rep(d["res"]["sumQ"], hold, t["K"]), d["S"])
    assert np.all(np.abs(gf - ex) < 4 * sef)
    assert se[1] < 0.5 * sef[1] and np.allclose(se[[0, 2]], sef[[0, 2]])


@pytest.mark.parametrize("mistake", ["ancestors", "without_self", "self_only"])
def test_planted_reach_mistakes_fail(tandem2_exact_and_sample, mistake):
    """A wrong reach set (ancestors in place of descendants, the parameter's own station left
    out, or only its own station) makes the estimate miss the exact derivative."""
    t, d = TANDEM2, tandem2_exact_and_sample
    n = d["net"].n
    reach = oracle.reach_sets(d["net"])
    if mistake == "ancestors":
        wrong = np.concatenate([reach[:n].T, reach[n:]], axis=0)
    elif mistake == "without_self":
        wrong = reach.copy()
        wrong[np.arange(n), np.arange(n)] = False
        wrong[n, 0] = False
    else:
        wrong = np.zeros_like(reach)
        wrong[np.arange(n), np.arange(n)] = True
        wrong[n, 0] = True
    g, se = oracle.lr_gradient_reach(d["res"]["sumQ"], np.array(t["hold"]), t["K"], d["S"], wrong)
    assert np.any(np.abs(g - d["exact"]) > 4 * se), (g, d["exact"], se)   # the pin's own threshold

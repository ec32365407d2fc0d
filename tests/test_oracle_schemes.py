"""Pins for the oracle's backward and forward schemes (Section 2 of the paper).

* The paper's 2-node tandem example (Section 2.3): one customer arriving within the first
  interval with service shorter than h at both nodes gives totals (0,1,1,0) under the
  backward scheme and (0,0,0,0) under the forward scheme.
* Exact flow conservation on a tandem with routing probability 1.
* M/M/inf special case (servers never all busy): with Poisson splitting the Euler states
  stay independent Poisson with means given by closed-form recursions, derived here from
  Lemma 1 (1) and the scheme definitions; checked for a 2-station tandem with constant
  and sinusoidal arrival rates (the arrival integrals computed by quadrature).
* Finite servers: the exact law of N_tau under each scheme from a brute-force Markov
  chain whose departure kernel is the matrix exponential of the pure-departure generator.
* Argument 3: E[N^b_tau] - E[N^f_tau] = E[D^f_tau].
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg
import scipy.stats as st

import netgen
import oracle
from test_oracle_samplers import gtest


def two_station(mu0, mu1, r, lam, c0=10**6, c1=10**6, shape_kind=0, amp=0.0, period=1.0):
    rp = np.array([0, 1, 1], np.int32)
    return netgen.Network(n=2, row_ptr=rp, col=np.array([1], np.int32), prob=np.array([r], np.float32),
                          servers=np.array([c0, c1], np.int32), mu=np.array([mu0, mu1], np.float32),
                          src=np.array([0], np.int32), lambda0=np.array([lam], np.float32),
                          shape_kind=shape_kind, amp=amp, period=period)


def test_paper_tandem_trace():
    """Section 2.3 example: service times shorter than h (mu h = 50 makes the departure
    probability exactly 1 in fp32) and a single arrival in the first interval."""
    net = two_station(5000.0, 5000.0, 1.0, 0.0, c0=1, c1=1)
    h = 0.01
    tot = {}
    for scheme in (oracle.BACKWARD, oracle.FORWARD):
        tot[scheme] = [0]
        for K in (1, 2, 3):
            inj = np.zeros((K, 2), np.int32)
            inj[0, 0] = 1
            r = oracle.run(net, scheme, h, K, 0, [0], inj_arr=inj)
            tot[scheme].append(int(r["final"].sum()))
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tandem_trace.json")))
    assert tot[oracle.BACKWARD] == gold["totals_backward"]
    assert tot[oracle.FORWARD] == gold["totals_forward"]


@pytest.mark.parametrize("scheme", [0, 1])
def test_flow_conservation_unit_routing(scheme):
    n = 3
    net = netgen.tandem(n, p=1.0, lam=40.0, mu=1.5, c=20)
    h, K = 0.05, 400
    r = oracle.run(net, scheme, h, K, 7, np.arange(64))
    sD, fin = r["sumD"], r["final"]
    assert np.all(fin >= 0)
    for j in range(1, n):
        # everything leaving j-1 enters j:  sum D_{j-1} = N_K(j) + sum D_j
        assert np.array_equal(sD[:, j - 1], fin[:, j] + sD[:, j])


def integrals(net, h, K):
    if net.shape_kind == netgen.SHAPE_PIECEWISE:    # non-periodic step function
        kt = np.asarray(net.knot_t)
        f = lambda t: float(net.knot_shape[int(np.searchsorted(kt, t, side="right")) - 1])
        return np.array([scipy.integrate.quad(f, (t - 1) * h, t * h, points=[x for x in kt if (t - 1) * h < x < t * h] or None)[0]
                         for t in range(1, K + 1)])
    f = lambda t: 1.0 + net.amp * math.sin(2 * math.pi * t / net.period + net.phase) if net.shape_kind else 1.0
    return np.array([scipy.integrate.quad(f, (t - 1) * h, t * h)[0] for t in range(1, K + 1)])


def mminf_means(net, h, K, scheme):
    """Closed-form means of (N0, N1) for the 2-station M/M/inf tandem."""
    lam = float(net.lambda0[0]) * integrals(net, float(np.float32(h)), K)
    mu0, mu1, r = float(net.mu[0]), float(net.mu[1]), float(net.prob[0])
    e0, e1 = math.exp(-mu0 * float(np.float32(h))), math.exp(-mu1 * float(np.float32(h)))
    a = b = 0.0
    A, B = [], []
    for t in range(K):
        if scheme == oracle.BACKWARD:
            a, b = a * e0 + lam[t], b * e1 + r * a * (1 - e0)
        else:
            a, b = (a + lam[t]) * e0, (b + r * (a + lam[t]) * (1 - e0)) * e1
        A.append(a)
        B.append(b)
    return np.array(A), np.array(B)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("shape", [0, 1, 2])
def test_mminf_tandem_closed_form(scheme, shape):
    net = two_station(1.3, 0.6, 0.7, 30.0, shape_kind=min(shape, 1), amp=0.8 if shape == 1 else 0.0, period=2.0)
    if shape == 2:
        net = net.with_piecewise_shape([0.0, 0.4, 1.13, 2.0], [0.3, 2.2, 0.0, 1.0], 0.0)
    h, K, R = 0.05, 60, 40000
    res = oracle.run(net, scheme, h, K, 101, np.arange(R))
    A, B = mminf_means(net, h, K, scheme)
    fin = res["final"].astype(float)
    for col, m in ((0, A[-1]), (1, B[-1])):
        x = fin[:, col]
        assert abs(x.mean() - m) < 4.5 * math.sqrt(m / R)
        assert abs(x.var() / m - 1.0) < 0.05            # Poisson dispersion
        pmf = st.poisson.pmf(np.arange(int(m + 10 * math.sqrt(m) + 20)), m)
        assert gtest(fin[:, col].astype(int), pmf) > 1e-4
    assert abs(np.corrcoef(fin[:, 0], fin[:, 1])[0, 1]) < 4.5 / math.sqrt(R)   # independent
    # time averages over tau = 1..K
    for col, M in ((0, A), (1, B)):
        avg = res["sumN"][:, col].astype(float) / K
        assert abs(avg.mean() - M.mean()) < 4.5 * avg.std() / math.sqrt(R)


def exact_single_station_pmf(lam, mu, c, h, K, scheme, nmax=90):
    """Exact law of N_K for one station from a truncated Markov chain on 0..nmax."""
    ps = st.poisson.pmf(np.arange(nmax + 1), lam * h)
    dep = np.zeros((nmax + 1, nmax + 1))   # dep[x, y]: P(x -> y by pure departures)
    Q = np.zeros((nmax + 1, nmax + 1))
    for y in range(1, nmax + 1):
        rr = min(y, c) * mu
        Q[y, y - 1] = rr
        Q[y, y] = -rr
    dep = scipy.linalg.expm(Q * h)
    arr = np.zeros((nmax + 1, nmax + 1))
    for x in range(nmax + 1):
        for a in range(nmax + 1 - x):
            arr[x, x + a] = ps[a]
    T = dep @ arr if scheme == oracle.BACKWARD else arr @ dep
    p = np.zeros(nmax + 1)
    p[0] = 1.0
    for _ in range(K):
        p = p @ T
    return p


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("lam,mu,c,h,K", [(3.0, 2.0, 2, 0.1, 30), (6.0, 1.0, 5, 0.3, 25), (2.5, 3.0, 1, 0.05, 80)])
def test_finite_server_exact_law(scheme, lam, mu, c, h, K):
    net = netgen.single_station(lam, mu, c)
    h32 = float(np.float32(h))
    R = 60000
    res = oracle.run(net, scheme, h, K, 202, np.arange(R))
    p = exact_single_station_pmf(float(np.float32(lam)), float(np.float32(mu)), c, h32, K, scheme)
    assert p[-5:].sum() < 1e-12
    assert gtest(res["final"][:, 0], p) > 1e-4


def test_argument3_gap_equals_forward_departures():
    """E[N^b_tau] - E[N^f_tau] = E[D^f_tau] (single station, every tau)."""
    net = netgen.single_station(4.0, 1.0, 5)
    h, R = 0.2, 60000
    lam = float(np.float32(4.0))
    for K in (3, 12):
        b = oracle.run(net, oracle.BACKWARD, h, K, 303, np.arange(R))
        f = oracle.run(net, oracle.FORWARD, h, K, 303, np.arange(R))
        f1 = oracle.run(net, oracle.FORWARD, h, K - 1, 303, np.arange(R))
        dK = (f["sumD"] - f1["sumD"])[:, 0].astype(float)      # D^f_K (same streams)
        gap = b["final"][:, 0].astype(float) - f["final"][:, 0]
        d = gap - dK
        assert abs(d.mean()) < 4.5 * d.std() / math.sqrt(R)
        # Theorem 1: the gap is at most m mu h
        assert gap.mean() <= 5 * 1.0 * h + 4.5 * gap.std() / math.sqrt(R)
    assert dK.mean() < lam * h + 0.05


@pytest.mark.parametrize("lam,mu,c,h", [(6.0, 1.0, 5, 0.3), (3.0, 2.0, 2, 0.1), (9.0, 1.0, 12, 0.5)])
def test_argument2_transient_stochastic_order(lam, mu, c, h):
    """Argument 2 (single station, from empty): N^f_tau <= N_tau <= N^b_tau in first-order
    stochastic dominance at every step.  The exact laws of the two Euler chains (the kernels the
    oracle's runs are pinned to) against the exact law of the M/M/c queue at tau h, from the
    matrix exponential of its generator: the tail probabilities are ordered at every level."""
    nmax = 160
    b, f = euler_kernels(lam, mu, c, h, nmax)
    G = np.zeros((nmax + 1, nmax + 1))
    for y in range(nmax + 1):
        if y < nmax:
            G[y, y + 1] = lam
        if y > 0:
            G[y, y - 1] = min(y, c) * mu
        G[y, y] = -G[y].sum()
    step = scipy.linalg.expm(G * h)
    pb = pf = pt = np.eye(nmax + 1)[0]
    for _ in range(30):
        pb, pf, pt = pb @ b, pf @ f, pt @ step
        assert pt[-10:].sum() < 1e-9
        tail = lambda p: p[::-1].cumsum()[::-1]          # P(N >= x), x = 0..nmax
        assert np.all(tail(pf) <= tail(pt) + 1e-12) and np.all(tail(pt) <= tail(pb) + 1e-12)
    # the ordering is strict in the mean, and the gap is of order lambda h
    mean = lambda p: float(p @ np.arange(nmax + 1))
    assert mean(pf) < mean(pt) < mean(pb) and mean(pb) - mean(pf) <= c * mu * h + 1e-9


def stationary_mean(T):
    """Mean of the stationary law of a finite transition matrix."""
    w, v = scipy.linalg.eig(T.T)
    p = np.real(v[:, np.argmin(np.abs(w - 1.0))])
    p = p / p.sum()
    return float(p @ np.arange(len(p)))


def euler_kernels(lam, mu, c, h, nmax):
    """Exact one-step kernels of the backward and forward schemes for one M/M/c station
    (departures from the matrix-exponential pure-death law, Poisson arrivals)."""
    ps = st.poisson.pmf(np.arange(nmax + 1), lam * h)
    Q = np.zeros((nmax + 1, nmax + 1))
    for y in range(1, nmax + 1):
        Q[y, y - 1] = min(y, c) * mu
        Q[y, y] = -min(y, c) * mu
    dep = scipy.linalg.expm(Q * h)
    arr = np.zeros((nmax + 1, nmax + 1))
    for x in range(nmax + 1):
        arr[x, x:] = ps[:nmax + 1 - x]
        arr[x, nmax] += 1.0 - ps[:nmax + 1 - x].sum()
    return dep @ arr, arr @ dep


def test_average_scheme_is_second_order():
    """Section 7's average scheme: the backward and forward steady-state means err by about
    +-lambda h (first order, opposite signs), their average by O(h^2)."""
    lam, mu, c, nmax = 8.0, 1.0, 10, 90
    rho = lam / (c * mu)
    # exact M/M/c mean (Erlang C)
    a = lam / mu
    p0 = 1.0 / (sum(a ** k / math.factorial(k) for k in range(c)) + a ** c / (math.factorial(c) * (1 - rho)))
    exact = a + p0 * a ** c * rho / (math.factorial(c) * (1 - rho) ** 2)
    errs = {}
    for h in (0.1, 0.05, 0.025):
        Tb, Tf = euler_kernels(lam, mu, c, h, nmax)
        eb, ef = stationary_mean(Tb) - exact, stationary_mean(Tf) - exact
        errs[h] = (eb, ef, 0.5 * (eb + ef))
        assert eb > 0 > ef                                   # the schemes bracket the truth
        assert abs((eb - ef) - lam * h) < 0.05 * lam * h     # Argument 3 in steady state
    for (h1, e1), (h2, e2) in zip(list(errs.items())[:-1], list(errs.items())[1:]):
        assert 1.7 < e1[0] / e2[0] < 2.3 and 1.7 < e1[1] / e2[1] < 2.3     # order 1
        assert 3.2 < e1[2] / e2[2] < 4.8                                   # order 2
        assert abs(e1[2]) < 0.2 * min(abs(e1[0]), abs(e1[1]))

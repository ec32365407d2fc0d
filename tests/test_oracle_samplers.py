"""Distribution pins for the oracle's samplers.

Each sampler is compared with an exact law computed independently of the oracle:
* Poisson and binomial draws against scipy's pmfs (G-test over binned support),
  on both sides of every algorithm switch (inversion / transformed rejection, p > 1/2).
* Gamma(k) draws (Erlang service completion time) against scipy's gamma cdf (KS).
* GenerateDeparture (Lemma 1 / Algorithm 3) against the transition law of the pure
  departure process obtained from the matrix exponential of its generator: states
  0..x, death rate min(y, m) mu in state y (Kolmogorov equations in the proof of
  Lemma 2).  This pins every branch of Algorithm 3 without re-deriving Lemma 1.
* The naive departure rule, Eq. (1): D = min(x, Poisson(min(x, m) mu h)).
The oracle is deterministic (counter-based streams with fixed seeds), so each test
either always passes or always fails.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats as st

import oracle

P_MIN = 1e-4


def gtest(samples: np.ndarray, pmf: np.ndarray, min_expected: float = 5.0) -> float:
    """Chi-square p-value of integer samples against pmf[0..len-1] (mass beyond the
    array is lumped into the last cell); low-expectation cells are merged."""
    samples = samples.astype(np.int64)
    N = len(samples)
    assert samples.min() >= 0
    K = len(pmf)
    counts = np.bincount(np.minimum(samples, K - 1), minlength=K).astype(float)
    probs = pmf.astype(float).copy()
    probs[-1] = max(0.0, 1.0 - probs[:-1].sum())
    exp = probs * N
    # merge cells left to right until each has expectation >= min_expected
    obs_m, exp_m = [], []
    o_acc = e_acc = 0.0
    for o, e in zip(counts, exp):
        o_acc += o
        e_acc += e
        if e_acc >= min_expected:
            obs_m.append(o_acc)
            exp_m.append(e_acc)
            o_acc = e_acc = 0.0
    if e_acc > 0 or o_acc > 0:
        if exp_m:
            obs_m[-1] += o_acc
            exp_m[-1] += e_acc
        else:
            obs_m.append(o_acc)
            exp_m.append(e_acc)
    obs_m, exp_m = np.array(obs_m), np.array(exp_m)
    if len(obs_m) < 2:
        return 1.0 if np.all(samples == np.argmax(pmf)) else 0.0
    chi2 = ((obs_m - exp_m) ** 2 / exp_m).sum()
    return float(st.chi2.sf(chi2, len(obs_m) - 1))


@pytest.mark.parametrize("lam", [0.05, 0.7, 3.3, 9.99, 10.0, 10.5, 37.2, 250.0, 4000.5])
def test_poisson(lam):
    N = 300000
    s = oracle.sample(oracle.SMP_POISSON, N, seed=17, sub=0, f0=lam)
    kmax = int(lam + 12 * math.sqrt(lam) + 30)
    pmf = st.poisson.pmf(np.arange(kmax + 1), lam)
    assert gtest(s, pmf) > P_MIN
    assert abs(s.mean() - lam) < 5 * math.sqrt(lam / N)


def test_poisson_zero_consumes_nothing():
    assert np.all(oracle.sample(oracle.SMP_POISSON, 100, f0=0.0) == 0)


@pytest.mark.parametrize("n,p", [(5, 0.3), (40, 0.2), (25, 0.41), (100, 0.099), (100, 0.1), (30, 0.34),
                                 (100, 0.5), (7, 0.5), (1000, 0.02), (10000, 0.005), (37, 0.9),
                                 (5000, 0.75), (2, 0.99), (100000, 0.3), (3000, 0.0034),
                                 (400, 0.0999), (400, 0.1), (80, 0.49), (200, 0.2), (1000, 0.035), (60, 0.55),
                                 (560, 0.0999), (560, 0.1), (114, 0.49), (115, 0.49), (1600, 0.035), (500, 0.112),
                                 (130, 0.43), (150, 0.627), (152, 0.63),
                                 # inversion with q^n below the normal fp32 range (scaled start), and
                                 # around the inversion / BTRS switch at n p = 80
                                 (140, 0.5), (158, 0.5), (161, 0.5), (400, 0.19), (186, 0.43), (800, 0.0999),
                                 (800, 0.1), (2300, 0.0347), (216, 0.63), (218, 0.634)])
def test_binomial(n, p):
    N = 300000
    s = oracle.sample(oracle.SMP_BINOMIAL, N, seed=23, i0=n, f0=p)
    assert s.min() >= 0 and s.max() <= n
    pmf = st.binom.pmf(np.arange(n + 1), n, np.float32(p).astype(np.float64))
    assert gtest(s, pmf) > P_MIN
    m = n * float(np.float32(p))
    assert abs(s.mean() - m) < 5 * math.sqrt(m * (1 - float(np.float32(p))) / N) + 1e-9


def _stirling_terms(j):
    """fc(j) = ln j! - ((j + 1/2) ln(j + 1) - (j + 1) + ln(2 pi)/2), fp64 from lgamma."""
    return math.lgamma(j + 1) - ((j + 0.5) * math.log(j + 1) - (j + 1) + 0.5 * math.log(2 * math.pi))


@pytest.mark.parametrize("n,p", [(115, 0.49), (130, 0.43), (200, 0.3), (1000, 0.2), (5000, 0.0125), (100000, 0.37),
                                 (10_000_000, 0.1), (134_000_001, 0.12)])
def test_btrs_log_ratio_against_lgamma(n, p):
    """BTRS accepts against ln f(k)/f(m), m = floor((n+1) p), which it evaluates by Stirling's
    series in log1p form.  Here that value is checked against ln f(k)/f(m) from lgamma in fp64,
    for k within 6 standard deviations of the mode, to the rounding the fp32 evaluation allows
    (a few ulp of its largest term).  A dropped or flipped Stirling remainder, or a wrong
    coefficient of a log term, moves it far beyond that (3e-3 and more at n = 115)."""
    p32 = np.float32(p)
    pf, qf = float(p32), 1.0 - float(p32)
    m = int(np.floor((np.float32(n) + np.float32(1.0)) * p32))
    sd = math.sqrt(n * pf * qf)
    ks = np.unique(np.clip(np.round(m + np.linspace(-6, 6, 49) * sd), 0, n).astype(np.int64))
    lr = math.log(pf / qf)
    for k in ks:
        k = int(k)
        exact = (math.lgamma(m + 1) + math.lgamma(n - m + 1) - math.lgamma(k + 1) - math.lgamma(n - k + 1)
                 + (k - m) * lr)
        got = oracle.btrs_log_ratio(n, pf, k)
        nk = n - k + 1
        scale = (abs((m + 0.5) * math.log1p((m + 1 - (pf / qf) * (n - m + 1)) / ((pf / qf) * (n - m + 1))))
                 + (n + 1) * abs(math.log1p((k - m) / nk)) + (k + 0.5) * abs(math.log((pf / qf) * nk / (k + 1)))
                 + 1.0)
        assert abs(got - exact) <= 16 * 2.0 ** -24 * scale, (n, p, k, got, exact, scale)


@pytest.mark.parametrize("lam", [10.0, 37.2, 250.0, 4000.5, 1.0e6, 1.6e7])
def test_ptrs_log_pmf_against_lgamma(lam):
    """PTRS accepts against ln f(k) = k ln lam - lam - ln k!, which it evaluates by Stirling's series
    in log1p form; checked against lgamma in fp64 for k within 6 standard deviations, to the
    rounding of the fp32 evaluation (a few ulp of its largest term)."""
    l32 = float(np.float32(lam))
    sd = math.sqrt(l32)
    ks = np.unique(np.clip(np.round(l32 + np.linspace(-6, 6, 49) * sd), 0, None).astype(np.int64))
    for k in ks:
        k = int(k)
        exact = k * math.log(l32) - l32 - math.lgamma(k + 1)
        got = oracle.ptrs_log_pmf(l32, k)
        t = k + 1 - l32
        scale = abs(t) + (k + 0.5) * abs(math.log1p(t / l32)) + 0.5 * abs(math.log(l32)) + 2.0
        assert abs(got - exact) <= 16 * 2.0 ** -24 * scale, (lam, k, got, exact, scale)


def test_binomial_degenerate():
    assert np.all(oracle.sample(oracle.SMP_BINOMIAL, 50, i0=0, f0=0.5) == 0)
    assert np.all(oracle.sample(oracle.SMP_BINOMIAL, 50, i0=9, f0=0.0) == 0)
    assert np.all(oracle.sample(oracle.SMP_BINOMIAL, 50, i0=9, f0=1.0) == 9)


@pytest.mark.parametrize("k", [1, 2, 5, 30, 1000, 20000, 1_000_000, 20_000_000])
def test_gamma(k):
    N = 200000
    s = oracle.sample(oracle.SMP_GAMMA, N, seed=5, i0=k).astype(np.float64)
    assert st.kstest(s, st.gamma(k).cdf).pvalue > P_MIN
    assert abs(s.mean() - k) < 5 * math.sqrt(k / N)


def pure_departure_pmf(x: int, m: int, mu: float, h: float) -> np.ndarray:
    """P(D = d), d = 0..x, for the pure departure process from x customers."""
    Q = np.zeros((x + 1, x + 1))
    for y in range(1, x + 1):
        r = min(y, m) * mu
        Q[y, y - 1] = r
        Q[y, y] = -r
    P = scipy.linalg.expm(Q * h)
    row = P[x]                      # distribution of the remaining count y
    return np.clip(row[::-1], 0.0, None)   # d = x - y


def host_tables(mu: float, m: int, h: float) -> tuple[float, float]:
    mu32, h32 = np.float32(mu), np.float32(h)
    pdep = np.float32(-math.expm1(-(float(mu32) * float(h32))))
    rate = np.float32(float(m) * float(mu32))
    return float(pdep), float(rate)


@pytest.mark.parametrize("x,m,mu,h", [(5, 10, 1.0, 0.5), (12, 12, 1.0, 0.1), (13, 12, 1.5, 0.2),
                                      (30, 10, 1.0, 0.05), (30, 10, 2.0, 0.6), (50, 3, 2.0, 0.3),
                                      (40, 20, 3.0, 0.5), (200, 150, 0.5, 0.02), (600, 500, 1.0, 0.02),
                                      (260, 250, 4.0, 0.05), (1, 1, 0.7, 0.9)])
def test_generate_departure_exact_law(x, m, mu, h):
    N = 200000
    pdep, rate = host_tables(mu, m, h)
    s = oracle.sample(oracle.SMP_GENDEP, N, seed=29, i0=x, i1=m, f0=float(np.float32(mu)), f1=float(np.float32(h)),
                      f2=pdep, f3=rate)
    assert s.min() >= 0 and s.max() <= x
    pmf = pure_departure_pmf(x, m, float(np.float32(mu)), float(np.float32(h)))
    assert gtest(s, pmf) > P_MIN


@pytest.mark.parametrize("x,m,mu,h", [(5, 10, 1.0, 0.5), (30, 10, 1.0, 0.05), (200, 150, 0.5, 0.3)])
def test_naive_departure_rule(x, m, mu, h):
    N = 200000
    mudt = float(np.float32(float(np.float32(mu)) * float(np.float32(h))))
    s = oracle.sample(oracle.SMP_GENDEP_NAIVE, N, seed=31, i0=x, i1=m, f0=mudt)
    lam = float(np.float32(min(x, m)) * np.float32(mudt))
    pmf = st.poisson.pmf(np.arange(x + 1), lam)
    pmf[x] = st.poisson.sf(x - 1, lam)
    assert gtest(s, pmf) > P_MIN


def test_naive_rule_overestimates_departures():
    # Section 4.1.1: the naive rule keeps min(x, m) servers busy all interval, so it
    # overestimates D when the busy count would drop within the interval
    x, m, mu, h = 12, 10, 2.0, 0.6
    pdep, rate = host_tables(mu, m, h)
    N = 100000
    exact = oracle.sample(oracle.SMP_GENDEP, N, seed=3, i0=x, i1=m, f0=mu, f1=h, f2=pdep, f3=rate)
    naive = oracle.sample(oracle.SMP_GENDEP_NAIVE, N, seed=3, i0=x, i1=m,
                          f0=float(np.float32(np.float32(mu) * np.float32(h))))
    pmf = pure_departure_pmf(x, m, mu, h)
    mean_exact = (np.arange(x + 1) * pmf).sum()
    assert abs(exact.mean() - mean_exact) < 0.05
    assert abs(naive.mean() - 10.6276) < 0.05      # E[min(x, Poisson(m mu h))]
    assert naive.mean() > mean_exact + 2.0


@pytest.mark.parametrize("n,p", [(1_000_000, 0.3), (30_000_001, 0.001), (20_000_003, 0.37), (100_000_000, 0.1),
                                 (134_000_001, 0.12)])
def test_binomial_beyond_2_24(n, p):
    """Large n p, and n above 2^24 where neither n nor n - k is an exact fp32 integer: the draws
    follow Binomial(n, p) (exact pmf on the window mean +- 8 sd, the mass outside negligible).
    A log-ratio that rounds a near-1 ratio, or n - k, to fp32 before its log fails this (at
    Binomial(2e7, 0.37) and Binomial(1e8, 0.1))."""
    N = 200000
    s = oracle.sample(oracle.SMP_BINOMIAL, N, seed=29, i0=n, f0=p).astype(np.int64)
    p64 = float(np.float32(p))
    mean, sd = n * p64, math.sqrt(n * p64 * (1 - p64))
    lo, hi = int(mean - 8 * sd), int(mean + 8 * sd)
    assert s.min() >= lo and s.max() <= hi
    pmf = st.binom.pmf(np.arange(lo, hi + 1), n, p64)
    assert gtest(s - lo, pmf) > P_MIN
    assert abs(s.mean() - mean) < 5 * sd / math.sqrt(N)


def test_out_of_range_draws_raise_the_flag():
    """Draws whose values fp32 cannot represent exactly raise the overflow flag, and only those:
    a binomial mode or a Poisson mean of 2^24 or more."""
    flagged = lambda **kw: oracle.sample(count=20, seed=3, return_flag=True, **kw)[1]
    assert flagged(kind=oracle.SMP_BINOMIAL, i0=100_000_000, f0=0.3)            # mode 3e7
    assert flagged(kind=oracle.SMP_BINOMIAL, i0=40_000_000, f0=0.5)
    assert not flagged(kind=oracle.SMP_BINOMIAL, i0=100_000_000, f0=0.1)        # mode 1e7
    assert not flagged(kind=oracle.SMP_BINOMIAL, i0=100_000_000, f0=0.9)        # Bin(n, 0.1) flipped
    assert flagged(kind=oracle.SMP_POISSON, f0=float(1 << 24))
    assert not flagged(kind=oracle.SMP_POISSON, f0=16_000_000.0)

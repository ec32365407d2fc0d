"""GPU parity of the likelihood-ratio gradient path, through the C ABI.

Score runs must leave the simulation unchanged (states and sums bit-identical to a plain
run) and reproduce the oracle's per-replication score sums and (N - m)^+ sums bit for bit;
the fp64 reductions must match the oracle's estimators on the same data to rounding, and the
gradient must agree with common-random-number central differences (relative step 1e-3)
within 3 combined standard errors, with a power check: where the check is stated to have
power, the combined standard error is below 0.3 |FD|.
"""
import math

import numpy as np
import pytest

import netgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_13259_amd import binding
    return binding


@pytest.fixture(scope="module")
def lr():
    from paper_2402_13259_amd import lr as lrmod
    return lrmod


def score_run(eb, netobj, scheme, dt, K, reps, seed=0, **kw):
    import torch
    net = eb.Net(netobj)
    res = eb.simulate_scores(net, scheme, dt, K, reps, seed, with_sums=True, **kw)
    torch.cuda.synchronize()
    return net, res


def assert_scores_equal(res, ref, n, rows=None):
    rows = np.arange(len(ref["final"])) if rows is None else np.asarray(rows)
    state = res.state.cpu().numpy().T
    sumq = res.sumq.cpu().numpy().T
    score = res.score.cpu().numpy().T
    assert np.array_equal(state[rows], ref["final"]), "states differ"
    assert np.array_equal(sumq[rows], ref["sumQ"]), "(N - m)^+ sums differ"
    assert np.array_equal(score[rows, :n].view(np.uint32), ref["score_mu"].view(np.uint32)), "mu scores differ"
    assert np.array_equal(score[rows, n:].view(np.uint32), ref["score_lam"].view(np.uint32)), "lambda0 scores differ"


SCORE_CASES = [
    (0, dict(f0=3.7, f1=0.4)), (0, dict(f0=55.0, f1=0.25)), (0, dict(f0=4321.0, f1=0.005)),
    (3, dict(x=5, m=10, f0=1.0, f1=0.5)), (3, dict(x=30, m=10, f0=1.0, f1=0.05)), (3, dict(x=40, m=20, f0=3.0, f1=0.5)),
    (3, dict(x=9000, m=8000, f0=1.1, f1=0.005)), (3, dict(x=8100, m=8000, f0=1.1, f1=0.005)),
    (3, dict(x=7, m=1, f0=0.8, f1=1.5)), (3, dict(x=0, m=3, f0=1.0, f1=0.1)),
    (4, dict(x=30, m=10, f0=1.0, f1=0.05)), (4, dict(x=6, m=2, f0=3.0, f1=0.4)),
]


@pytest.mark.parametrize("kind,kw", SCORE_CASES)
def test_score_samplers_bit_identical(eb, kind, kw):
    count = 100000
    sub = 0 if kind == 0 else 1
    v, s = eb.selftest_score(kind, count, seed=77, rep0=3, station=2, step0=5, sub=sub, **kw)
    rv, rs = oracle.sample_score(kind, count, seed=77, rep0=3, station=2, step0=5, sub=sub, **kw)
    assert np.array_equal(v.cpu().numpy().view(np.uint32), rv.view(np.uint32))
    assert np.array_equal(s.cpu().numpy().view(np.uint32), rs.view(np.uint32))


@pytest.mark.parametrize("scheme,dep_mode", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_score_run_matches_oracle(eb, scheme, dep_mode):
    """Three-station network, 60 steps, 200 replications (three full tiles and a ragged one)."""
    w = netgen.three_station()
    K, R, dt = 60, 200, 0.2
    net, res = score_run(eb, w, scheme, dt, K, R, seed=5, dep_mode=dep_mode)
    ref = oracle.run(w, scheme, dt, K, 5, np.arange(R), dep_mode=dep_mode, scores=True)
    assert_scores_equal(res, ref, w.n)
    # the plain run takes the same draws
    plain = eb.simulate(net, scheme, dt, K, R, 5, dep_mode=dep_mode, kernel=eb.EQ_KERNEL_SWEEP)
    assert np.array_equal(plain.state.cpu().numpy(), res.state.cpu().numpy())
    assert np.array_equal(plain.sums.cpu().numpy(), res.sums.cpu().numpy())


@pytest.mark.parametrize("scheme", [0, 1])
def test_score_run_dag1000_reduced_horizon(eb, scheme):
    """1000-station DAG, 300 steps, 100 replications: every replication bit-exact."""
    w = netgen.config3()
    K, R = 300, 100
    net, res = score_run(eb, w.net, scheme, w.dt, K, R, seed=9)
    ref = oracle.run(w.net, scheme, w.dt, K, 9, np.arange(R), scores=True)
    assert_scores_equal(res, ref, w.net.n)


def test_score_run_full_size_sampled_reps(eb):
    """The gradient workload at full size (1000 stations, 20000 steps, 8192 replications,
    backward scheme), as the benchmark runs it: sampled replications bit-exact, and the
    fp64 reductions equal to their definitions evaluated on the GPU's own outputs."""
    import torch
    w = netgen.config5()
    hold, staff = netgen.config5_costs(w.net.n)
    net, res = score_run(eb, w.net, 0, w.dt, w.K, w.reps, seed=0)
    wave = 93   # one wavefront's 64 replications: two whole 32-replication statistics tiles
    rows = np.r_[0, 1, 4095, 4096, 8191, wave * 64:(wave + 1) * 64]
    ref = oracle.run(w.net, 0, w.dt, w.K, 0, rows, scores=True)
    assert_scores_equal(res, ref, w.net.n, rows)
    for tile in (2 * wave, 2 * wave + 1):
        sums = res.sums.cpu().numpy()[:, :, tile]
        sel = rows // 32 == tile
        for k, name in enumerate(("sumN", "sumQ", "sumD")):
            assert np.array_equal(sums[k], ref[name][sel].sum(0)), (name, tile)
    assert (ref["sumQ"][rows // 64 == wave].sum(0) > 0).mean() > 0.5
    f, ms = eb.cost_reduce(torch.as_tensor(hold, device="cuda"), res.sumq, w.K)
    g, se = eb.grad_reduce(f, ms, res.score)
    f_np = res.sumq.cpu().numpy().T.astype(np.float64) @ hold / w.K
    assert np.allclose(f.cpu().numpy(), f_np, rtol=1e-13, atol=0)
    assert np.allclose(f.cpu().numpy()[rows], oracle.cost_per_rep(ref["sumQ"], hold, w.K), rtol=1e-13, atol=0)
    check_grad(g.cpu().numpy(), se.cpu().numpy(), f.cpu().numpy(), res.score.cpu().numpy().T)
    # the reachability-pruned estimator against its definition on the same outputs
    gr, ser = eb.grad_reduce_reach(net, torch.as_tensor(hold, device="cuda"), res.sumq, res.score, w.K)
    rg, rse = oracle.lr_gradient_reach(res.sumq.cpu().numpy().T, hold, w.K, res.score.cpu().numpy().T,
                                       oracle.reach_sets(w.net))
    assert np.all(np.abs(gr.cpu().numpy() - rg) <= 1e-9 * (np.abs(rg) + rse))
    assert np.allclose(ser.cpu().numpy(), rse, rtol=1e-6)


def check_grad(g, se, f, S):
    """GPU reduction against the oracle's estimator on the same f and scores [R, n_par]."""
    rg, rse = oracle.lr_gradient(f, S)
    scale = (np.abs(f - f.mean())[:, None] * np.abs(S.astype(np.float64))).sum(0) / (len(f) - 1)
    assert np.all(np.abs(g - rg) <= 1e-12 * scale + 1e-300)
    assert np.allclose(se, rse, rtol=1e-6, atol=1e-12 * scale.max())


@pytest.mark.parametrize("scheme,estimator", [(0, "reach"), (1, "reach"), (0, "full"), (1, "full")])
def test_cost_and_gradient_match_cpu_reference(eb, lr, scheme, estimator):
    """The autograd function's value and gradient (either estimator) against the oracle's
    estimator run on the CPU over the same replications."""
    import torch
    w = netgen.three_station()
    hold, staff = np.array([1.0, 2.0, 1.5]), np.array([0.3, 0.2, 0.5])
    K, R, dt = 40, 4000, 0.2
    prob = lr.CostProblem(w, hold, staff, dt, K, R, scheme=scheme, seed=21, estimator=estimator)
    mu = torch.tensor(w.mu, dtype=torch.float64, requires_grad=True)
    lam = torch.tensor(w.lambda0, dtype=torch.float64, requires_grad=True)
    J = lr.expected_cost(mu, lam, prob)
    J.backward()
    ref = oracle.run(w, scheme, dt, K, 21, np.arange(R), scores=True)
    f = oracle.cost_per_rep(ref["sumQ"], hold, K)
    stf = float(np.dot(staff, w.servers))
    assert abs(J.item() - (f.mean() + stf)) <= 1e-12 * (abs(f).mean() + stf)
    assert abs(prob.last["J_se"].item() - f.std(ddof=1) / math.sqrt(R)) <= 1e-9 * f.std()
    S = np.concatenate([ref["score_mu"], ref["score_lam"]], axis=1)
    if estimator == "reach":
        g_cpu, se_cpu = oracle.lr_gradient_reach(ref["sumQ"], hold, K, S, oracle.reach_sets(w))
    else:
        g_cpu, se_cpu = oracle.lr_gradient(f, S)
    g_gpu = np.concatenate([mu.grad.numpy(), lam.grad.numpy()])
    scale = np.abs(g_cpu) + se_cpu
    assert np.all(np.abs(g_gpu - g_cpu) <= 1e-9 * scale)
    assert np.allclose(prob.last["grad_se"].cpu().numpy(), se_cpu, rtol=1e-6)
    assert mu.grad.dtype == torch.float64 and mu.grad.device.type == "cpu"


@pytest.mark.parametrize("scheme", [0, 1])
def test_gradient_matches_crn_finite_differences(eb, lr, scheme):
    """Every mu_i and lambda0_s of the three-station network: the autograd gradient (pruned
    estimator) vs CRN central differences (same seed and replications, relative step 1e-3)
    within 3 combined standard errors, each check with power (combined SE < 0.3 |FD|)."""
    import torch
    w = netgen.three_station()
    hold, staff = np.array([1.0, 2.0, 1.5]), np.zeros(3)
    K, R, dt = 40, 200_000, 0.2
    prob = lr.CostProblem(w, hold, staff, dt, K, R, scheme=scheme, seed=33)
    mu = torch.tensor(w.mu, dtype=torch.float64, device="cuda", requires_grad=True)
    lam = torch.tensor(w.lambda0, dtype=torch.float64, device="cuda", requires_grad=True)
    lr.expected_cost(mu, lam, prob).backward()
    g, gse = prob.last["grad"].cpu().numpy(), prob.last["grad_se"].cpu().numpy()
    params = [("mu", i) for i in range(3)] + [("lambda0", s) for s in range(2)]
    for j, (name, i) in enumerate(params):
        base = getattr(w, name).astype(np.float64)
        fs = []
        for sign in (+1, -1):
            a = base.copy()
            a[i] = float(np.float32(base[i] * (1 + sign * 1e-3)))
            fs.append((lr.cost_samples(prob, **{name: a}), a[i]))
        diff = ((fs[0][0] - fs[1][0]) / (fs[0][1] - fs[1][1])).cpu().numpy()
        fd, fd_se = diff.mean(), diff.std() / math.sqrt(R)
        comb = math.hypot(gse[j], fd_se)
        assert abs(g[j] - fd) < 3 * comb, (name, i, g[j], gse[j], fd, fd_se)
        assert comb < 0.3 * abs(fd), (name, i, comb, fd)


def test_gradient_dag1000_directional_finite_differences(eb, lr):
    """1000-station DAG at a 2000-step horizon, 8192 replications: eight mu coordinates at
    spread DAG depths, four lambda0 coordinates and two random directions, the pruned
    estimate (as the autograd function returns it) against CRN central differences with a
    relative step of 1e-3, within 3 combined standard errors.  The lambda0 coordinates and the
    last station's mu carry power (combined SE < 0.3 |FD|); for the other mu the likelihood
    ratio's standard error stays above |FD| over 2000 steps and the check is one of agreement
    only.  On every coordinate checked, pruning does not widen the standard error of the
    full-cost estimator."""
    import torch
    w = netgen.config5()
    hold, staff = netgen.config5_costs(w.net.n)
    K, R = 2000, w.reps
    prob = lr.CostProblem(w.net, hold, staff, w.dt, K, R, seed=41)
    n = w.net.n
    mu = torch.tensor(w.net.mu, dtype=torch.float64, device="cuda", requires_grad=True)
    lam = torch.tensor(w.net.lambda0, dtype=torch.float64, device="cuda", requires_grad=True)
    J = lr.expected_cost(mu, lam, prob)
    J.backward()
    net = eb.Net(w.net)
    res = eb.simulate_scores(net, 0, w.dt, K, R, 41)
    hold_d = torch.as_tensor(hold, device="cuda")
    f, ms = eb.cost_reduce(hold_d, res.sumq, K)
    g, _ = eb.grad_reduce_reach(net, hold_d, res.sumq, res.score, K)
    assert torch.equal(torch.cat([mu.grad, lam.grad]), g)      # the autograd gradient is this estimator
    # per-replication products of both estimators, [R, n_par]
    S = res.score.double().T
    reach = torch.as_tensor(oracle.reach_sets(w.net), dtype=torch.float64, device="cuda")
    F = (res.sumq.double().T * (hold_d / K)[None, :]) @ reach.T
    P_reach = (F - F.mean(0)) * S * (R / (R - 1))
    P_full = (f - ms[0]).double()[:, None] * S * (R / (R - 1))
    assert torch.allclose(P_reach.mean(0), g, rtol=1e-9, atol=1e-9 * g.abs().max().item())
    theta = np.concatenate([w.net.mu, w.net.lambda0]).astype(np.float64)
    lev = net.levels()
    picks = [int(np.flatnonzero(lev == l)[0]) for l in np.linspace(1, lev.max(), 8).astype(int)]
    assert picks[-1] == n - 1
    dirs = []
    for j in picks + [n + s for s in (0, 17, 33, 49)]:
        v = np.zeros(len(theta))
        v[j] = 1.0
        dirs.append((j, v, j >= n or j == n - 1))
    rng = np.random.default_rng(8)
    for _ in range(2):
        dirs.append((-1, rng.standard_normal(len(theta)) / math.sqrt(len(theta)), False))
    for j, v, powered in dirs:
        wv = torch.as_tensor(theta * v, device="cuda")
        per, per_full = P_reach @ wv, P_full @ wv
        lr_d, lr_se = per.mean().item(), (per.std() / math.sqrt(R)).item()
        full_se = (per_full.std() / math.sqrt(R)).item()
        fs = []
        for sign in (+1, -1):
            t = (theta * (1 + sign * 1e-3 * v)).astype(np.float32)
            fs.append(lr.cost_samples(prob, mu=t[:n], lambda0=t[n:]))
        diff = ((fs[0] - fs[1]) / 2e-3).cpu().numpy()
        fd, fd_se = diff.mean(), diff.std() / math.sqrt(R)
        comb = math.hypot(lr_se, fd_se)
        assert abs(lr_d - fd) < 3 * comb, (j, lr_d, lr_se, fd, fd_se)
        if powered:
            assert comb < 0.3 * abs(fd), (j, comb, fd)
        if j >= 0:
            assert lr_se <= full_se * 1.0001, (j, lr_se, full_se)


def test_score_run_validation(eb):
    import torch
    w = netgen.three_station()
    net = eb.Net(w)
    desc = eb.make_desc(0, 0.2, 10, 64, kernel=eb.EQ_KERNEL_TILE)
    st = torch.empty((3, 64), dtype=torch.int32, device="cuda")
    sq = torch.empty((3, 64), dtype=torch.int64, device="cuda")
    sc = torch.empty((5, 64), dtype=torch.float32, device="cuda")
    import ctypes as C
    rc = eb.eq_sim_run_scores(net.handle, C.byref(desc), None, st.data_ptr(), None, sq.data_ptr(), sc.data_ptr(),
                              sc[3:].data_ptr(), None)
    assert rc == eb.EQ_EINVAL
    desc = eb.make_desc(0, 0.2, 10, 64)
    assert eb.eq_sim_run_scores(net.handle, C.byref(desc), None, st.data_ptr(), None, sq.data_ptr(), sc.data_ptr(),
                                None, None) == eb.EQ_EINVAL
    assert eb.eq_grad_reduce(5, 1, None, None, None, None, None, None) == eb.EQ_EINVAL


from hypothesis import HealthCheck, given, settings, strategies as hst  # noqa: E402

from net_strategies import random_networks, staffing_schedules  # noqa: E402


@settings(max_examples=30, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(random_networks(), hst.integers(0, 1), hst.integers(0, 1), hst.floats(0.01, 0.3), hst.integers(1, 40),
       hst.integers(2, 130), hst.booleans(), hst.data())
def test_random_score_runs_match_oracle(eb, net, scheme, dep_mode, dt, K, reps, staff, data):
    """Score runs on random networks (either rule, optionally under a random staffing
    schedule): states, (N - m)^+ sums and every fp32 score sum bit-equal to the oracle's."""
    if scheme == 1 and not net.is_index_dag():
        scheme = 0
    if staff:
        start, servers, period = data.draw(staffing_schedules(net.n))
        net = net.replace(staff_start=np.asarray(start, np.int32),
                          staff_servers=np.asarray(servers, np.int32).reshape(len(start), net.n),
                          staff_period=int(period))
    _, res = score_run(eb, net, scheme, dt, K, reps, seed=37, dep_mode=dep_mode)
    ref = oracle.run(net, scheme, dt, K, 37, np.arange(reps), dep_mode=dep_mode, scores=True)
    assert_scores_equal(res, ref, net.n)


@settings(max_examples=25, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(random_networks(), hst.integers(0, 1), hst.integers(0, 1), hst.floats(0.01, 0.3), hst.integers(1, 30),
       hst.integers(2, 300), hst.data())
def test_random_gradients_match_cpu_estimator(eb, lr, net, scheme, dep_mode, dt, K, reps, data):
    """The autograd function on random networks and cost weights: J, its standard error and
    the gradient in every mu_i and lambda0_s equal the oracle's estimator on the same draws,
    to fp64 rounding."""
    import torch
    if scheme == 1 and not net.is_index_dag():
        scheme = 0
    # few servers, so that most examples queue and the cost varies across replications
    net = net.replace(servers=np.array(data.draw(hst.lists(hst.integers(1, 8), min_size=net.n, max_size=net.n)),
                                       np.int32))
    hold = np.array(data.draw(hst.lists(hst.floats(0.0, 5.0), min_size=net.n, max_size=net.n)))
    staff = np.array(data.draw(hst.lists(hst.floats(0.0, 1.0), min_size=net.n, max_size=net.n)))
    prob = lr.CostProblem(net, hold, staff, dt, K, reps, scheme=scheme, seed=59, dep_mode=dep_mode)
    mu = torch.tensor(net.mu, dtype=torch.float64, requires_grad=True)
    lam = torch.tensor(net.lambda0, dtype=torch.float64, requires_grad=True)
    J = lr.expected_cost(mu, lam, prob)
    J.backward()
    ref = oracle.run(net, scheme, dt, K, 59, np.arange(reps), dep_mode=dep_mode, scores=True)
    f = oracle.cost_per_rep(ref["sumQ"], hold, K)
    stf = float(np.dot(staff, net.servers))
    assert abs(J.item() - (f.mean() + stf)) <= 1e-12 * (np.abs(f).mean() + stf) + 1e-300
    assert abs(prob.last["J_se"].item() - f.std(ddof=1) / math.sqrt(reps)) <= 1e-9 * f.std() + 1e-300
    g_cpu, se_cpu = oracle.lr_gradient_reach(ref["sumQ"], hold, K, np.concatenate([ref["score_mu"], ref["score_lam"]],
                                                                                  axis=1), oracle.reach_sets(net))
    g_gpu = np.concatenate([mu.grad.numpy(), lam.grad.numpy()])
    assert np.all(np.abs(g_gpu - g_cpu) <= 1e-9 * (np.abs(g_cpu) + se_cpu) + 1e-300)

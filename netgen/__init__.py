"""Seeded synthetic workloads: queueing networks of the shapes the paper studies.

This module only *builds inputs* (routing matrix in CSR form, server counts, service
rates, external-arrival rates and their time shape).  It holds none of the Euler
method's arithmetic, so both the oracle and the GPU library can consume it.

Networks follow the paper's model (Section 2.2 and Assumption 2): n stations, each a
multi-server FIFO queue with m_i servers of exponential rate mu_i; after service a
customer moves to j with probability p_ij or leaves with probability
1 - sum_j p_ij; station s receives external Poisson arrivals at rate
lambda0_s * shape(t), with shape(t) = 1, 1 + amp * sin(2 pi t / period + phase), or a
piecewise-constant function (heights knot_shape[k] from knot_t[k] on; repeated every
`period` when period > 0).

Random draws use numpy's PCG64 generator; because numpy does not promise stable
streams across versions, `fingerprint()` gives a SHA-256 over the arrays so a test
can tell if a regenerated network changed.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Optional

import numpy as np

SHAPE_CONST = 0
SHAPE_SINUSOID = 1
SHAPE_PIECEWISE = 2


@dataclasses.dataclass
class Network:
    n: int
    row_ptr: np.ndarray        # int32 [n+1]
    col: np.ndarray            # int32 [nnz]
    prob: np.ndarray           # float32 [nnz]
    servers: np.ndarray        # int32 [n]
    mu: np.ndarray             # float32 [n]
    src: np.ndarray            # int32 [n_src], strictly increasing
    lambda0: np.ndarray        # float32 [n_src]
    shape_kind: int = SHAPE_CONST
    amp: float = 0.0
    period: float = 1.0
    phase: float = 0.0
    name: str = ""
    # optional staffing schedule: segment k starts at interval index staff_start[k] (0-based
    # step tau - 1; staff_start[0] = 0, increasing) and gives every station the servers
    # staff_servers[k]; with staff_period > 0 the schedule repeats every staff_period steps
    staff_start: Optional[np.ndarray] = None      # int32 [n_seg]
    staff_servers: Optional[np.ndarray] = None    # int32 [n_seg, n]
    staff_period: int = 0
    # piecewise-constant arrival shape (shape_kind = SHAPE_PIECEWISE): knot_t[0] = 0, increasing
    knot_t: Optional[np.ndarray] = None           # float64 [n_knots]
    knot_shape: Optional[np.ndarray] = None       # float64 [n_knots], >= 0

    def with_piecewise_shape(self, knot_t, knot_shape, period: float = 0.0) -> "Network":
        """The same network with a piecewise-constant arrival shape (period 0: not repeated)."""
        return self.replace(shape_kind=SHAPE_PIECEWISE, amp=0.0, phase=0.0, period=float(period),
                            knot_t=np.asarray(knot_t, np.float64), knot_shape=np.asarray(knot_shape, np.float64))

    def servers_at(self, step0: int) -> np.ndarray:
        """Servers of every station during interval step0 + 1 (step0 = tau - 1)."""
        if self.staff_start is None:
            return self.servers
        t = step0 % self.staff_period if self.staff_period > 0 else step0
        k = int(np.searchsorted(self.staff_start, t, side="right")) - 1
        return self.staff_servers[k]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def exit_prob(self) -> np.ndarray:
        tot = np.zeros(self.n)
        for i in range(self.n):
            tot[i] = self.prob[self.row_ptr[i]:self.row_ptr[i + 1]].astype(np.float64).sum()
        return np.clip(1.0 - tot, 0.0, None)

    def dense_P(self) -> np.ndarray:
        P = np.zeros((self.n, self.n))
        for i in range(self.n):
            for e in range(self.row_ptr[i], self.row_ptr[i + 1]):
                P[i, self.col[e]] += float(self.prob[e])
        return P

    def lambda_ext(self) -> np.ndarray:
        lam = np.zeros(self.n)
        lam[self.src] = self.lambda0.astype(np.float64)
        return lam

    def total_rates(self) -> np.ndarray:
        """Time-average total arrival rates from the traffic equations
        lambda~ = lambda + P^T lambda~ (Theorem 2 of the paper)."""
        P = self.dense_P()
        return np.linalg.solve(np.eye(self.n) - P.T, self.lambda_ext())

    def is_index_dag(self) -> bool:
        for i in range(self.n):
            if np.any(self.col[self.row_ptr[i]:self.row_ptr[i + 1]] <= i):
                return False
        return True

    def fingerprint(self) -> str:
        h = hashlib.sha256()
        for a in (self.row_ptr, self.col, self.prob, self.servers, self.mu, self.src, self.lambda0):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(np.array([self.shape_kind, self.amp, self.period, self.phase]).tobytes())
        if self.knot_t is not None:
            h.update(np.ascontiguousarray(self.knot_t, np.float64).tobytes())
            h.update(np.ascontiguousarray(self.knot_shape, np.float64).tobytes())
        return h.hexdigest()

    def replace(self, **kw) -> "Network":
        return dataclasses.replace(self, **kw)


def _csr(n: int, rows: list[list[tuple[int, float]]]) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    cols, probs = [], []
    for i, r in enumerate(rows):
        r = sorted(r)
        row_ptr[i + 1] = row_ptr[i] + len(r)
        cols += [c for c, _ in r]
        probs += [p for _, p in r]
    return row_ptr, np.asarray(cols, dtype=np.int32), np.asarray(probs, dtype=np.float32)


def tandem(n: int = 4, p: float = 0.9, lam: float = 20.0, mu: float = 1.0, c: int = 25) -> Network:
    """Feedforward tandem 0 -> 1 -> ... -> n-1; each routes on with probability p and
    exits otherwise; the last station always exits.  Constant arrivals into station 0."""
    rows = [[(i + 1, p)] for i in range(n - 1)] + [[]]
    row_ptr, col, prob = _csr(n, rows)
    return Network(n=n, row_ptr=row_ptr, col=col, prob=prob,
                   servers=np.full(n, c, dtype=np.int32), mu=np.full(n, mu, dtype=np.float32),
                   src=np.array([0], dtype=np.int32), lambda0=np.array([lam], dtype=np.float32),
                   name=f"tandem{n}")


def three_station() -> Network:
    """Three stations with finite servers: 0 -> {1, 2}, 1 -> 2, sources 0 and 1, sinusoidal
    arrivals (a small feed-forward case that visits every departure branch)."""
    return Network(n=3, row_ptr=np.array([0, 2, 3, 3], np.int32), col=np.array([1, 2, 2], np.int32),
                   prob=np.array([0.5, 0.3, 0.8], np.float32), servers=np.array([4, 3, 5], np.int32),
                   mu=np.array([1.2, 1.5, 1.3], np.float32), src=np.array([0, 1], np.int32),
                   lambda0=np.array([4.0, 2.0], np.float32), shape_kind=SHAPE_SINUSOID, amp=0.5, period=3.0,
                   phase=0.0, name="three_station")


def branching() -> Network:
    """Five stations, feed-forward, every routing row with two or more edges of distinct
    probabilities: 0 -> {1: .5, 2: .25, 3: .15} (exit .1), 1 -> {3: .4, 4: .3} (exit .3),
    2 -> {4: .6} (exit .4), 3 -> {4: .5} (exit .5), 4 exits.  Constant arrivals at rate 20
    into station 0, mu = 1, servers (25, 13, 7, 9, 12): total rates (20, 10, 5, 7, 9.5), loads
    0.5 to 0.8.  A swapped target or a misordered split changes the total rates."""
    rows = [[(1, 0.5), (2, 0.25), (3, 0.15)], [(3, 0.4), (4, 0.3)], [(4, 0.6)], [(4, 0.5)], []]
    row_ptr, col, prob = _csr(5, rows)
    return Network(n=5, row_ptr=row_ptr, col=col, prob=prob, servers=np.array([25, 13, 7, 9, 12], np.int32),
                   mu=np.ones(5, np.float32), src=np.array([0], np.int32), lambda0=np.array([20.0], np.float32),
                   name="branching5")


def single_station(lam: float, mu: float, c: int, shape_kind: int = SHAPE_CONST, amp: float = 0.0,
                   period: float = 1.0) -> Network:
    return Network(n=1, row_ptr=np.array([0, 0], dtype=np.int32), col=np.zeros(0, dtype=np.int32),
                   prob=np.zeros(0, dtype=np.float32), servers=np.array([c], dtype=np.int32),
                   mu=np.array([mu], dtype=np.float32), src=np.array([0], dtype=np.int32),
                   lambda0=np.array([lam], dtype=np.float32), shape_kind=shape_kind, amp=amp,
                   period=period, name="single")


def layered(layers: int = 10, width: int = 10, seed: int = 2) -> Network:
    """Multi-layer feedforward network (the paper's Figure 2 structure): ids are
    layer-major; each station in layers 1..L-1 routes to 1-4 distinct stations of the
    next layer with (1-e) Dirichlet(1) probabilities, e ~ U(0.05, 0.2); the last layer
    exits.  A station below layer 1 left without an in-edge receives one from a random
    previous-layer station of degree < 4 (whose probabilities are redrawn).  Layer-1
    stations get lambda0 ~ U(50, 500) with a 24-period sinusoidal shape of amplitude 0.5;
    mu ~ U(0.5, 2); servers c_i = ceil(lambda~_i / (rho_i mu_i)), rho_i ~ U(0.8, 0.98)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = layers * width
    targets: list[list[int]] = [[] for _ in range(n)]
    exitp = np.zeros(n)
    for L in range(layers - 1):
        for w in range(width):
            i = L * width + w
            k = int(rng.integers(1, 5))
            targets[i] = sorted(int(t) for t in rng.choice(width, size=k, replace=False) + (L + 1) * width)
            exitp[i] = rng.uniform(0.05, 0.2)
    indeg = np.zeros(n, dtype=int)
    for i in range(n):
        for t in targets[i]:
            indeg[t] += 1
    for L in range(1, layers):
        for w in range(width):
            j = L * width + w
            if indeg[j] == 0:
                cands = [(L - 1) * width + v for v in range(width) if len(targets[(L - 1) * width + v]) < 4]
                i = int(rng.choice(cands))
                targets[i] = sorted(targets[i] + [j])
                indeg[j] += 1
    rows = []
    for i in range(n):
        if targets[i]:
            ps = (1.0 - exitp[i]) * rng.dirichlet(np.ones(len(targets[i])))
            rows.append(list(zip(targets[i], ps.tolist())))
        else:
            rows.append([])
    row_ptr, col, prob = _csr(n, rows)
    src = np.arange(width, dtype=np.int32)
    lam0 = rng.uniform(50.0, 500.0, size=width).astype(np.float32)
    mu = rng.uniform(0.5, 2.0, size=n).astype(np.float32)
    rho = rng.uniform(0.8, 0.98, size=n)
    net = Network(n=n, row_ptr=row_ptr, col=col, prob=prob, servers=np.ones(n, dtype=np.int32), mu=mu,
                  src=src, lambda0=lam0, shape_kind=SHAPE_SINUSOID, amp=0.5, period=24.0, phase=0.0,
                  name=f"layered{layers}x{width}")
    lt = net.total_rates()
    net.servers = np.maximum(1, np.ceil(lt / (rho * mu.astype(np.float64)))).astype(np.int32)
    return net


def jackson(layers: int = 10, width: int = 10, seed: int = 2, servers: int = 200,
            rho_range: tuple[float, float] = (0.8, 0.95)) -> Network:
    """The layered structure of `layered` with constant external rates and `servers`
    servers per station: rho_i ~ U(rho_range), mu_i = lambda~_i / (rho_i servers), the
    external rates scaled so that the median mu is 1.  A feed-forward Jackson network, so
    each station's steady-state law is that of an M/M/c queue with rate lambda~_i."""
    net = layered(layers, width, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    net.shape_kind, net.amp = SHAPE_CONST, 0.0
    net.servers = np.full(net.n, servers, dtype=np.int32)
    rho = rng.uniform(*rho_range, size=net.n)
    lt = net.total_rates()
    kappa = 1.0 / float(np.median(lt / (rho * servers)))
    net.lambda0 = (net.lambda0.astype(np.float64) * kappa).astype(np.float32)
    lt = net.total_rates()
    net.mu = (lt / (rho * servers)).astype(np.float32)
    net.name = f"jackson{layers}x{width}"
    return net


def sparse_dag(n: int = 1000, n_src: int = 50, seed: int = 3, max_deg: int = 8,
               c_range: tuple[int, int] = (1000, 10000), rho_range: tuple[float, float] = (0.85, 0.99),
               exit_range: tuple[float, float] = (0.05, 0.3), shape_kind: int = SHAPE_SINUSOID) -> Network:
    """Large sparse DAG: station k < n-1 routes to d ~ U{1..min(8, n-1-k)} distinct
    higher-index stations with (1-e) Dirichlet(1) probabilities, e ~ U(0.05, 0.3); the
    last station exits.  Stations >= n_src left without an in-edge get one from a random
    lower station of degree < 8 (any lower station if none has room).  Sources
    0..n_src-1 get lambda0 ~ U(50, 500) * kappa with a 24-period sinusoidal shape of
    amplitude 0.5.  c_i ~ U{1000..10000},
    rho_i ~ U(0.85, 0.99), mu_i = lambda~_i / (rho_i c_i), with kappa chosen so that
    the median mu is 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_src = max(1, min(n_src, n))
    targets: list[list[int]] = [[] for _ in range(n)]
    exitp = np.zeros(n)
    for k in range(n - 1):
        d = int(rng.integers(1, min(max_deg, n - 1 - k) + 1))
        targets[k] = sorted(int(t) for t in rng.choice(np.arange(k + 1, n), size=d, replace=False))
        exitp[k] = rng.uniform(*exit_range)
    indeg = np.zeros(n, dtype=int)
    for i in range(n):
        for t in targets[i]:
            indeg[t] += 1
    for j in range(n_src, n):
        if indeg[j] == 0:
            cands = [i for i in range(j) if len(targets[i]) < max_deg and j not in targets[i]]
            if not cands:          # tiny networks: every lower station is full; allow one more edge
                cands = [i for i in range(j) if j not in targets[i]]
            i = int(rng.choice(cands))
            targets[i] = sorted(targets[i] + [j])
            indeg[j] += 1
    rows = []
    for i in range(n):
        if targets[i]:
            ps = (1.0 - exitp[i]) * rng.dirichlet(np.ones(len(targets[i])))
            rows.append(list(zip(targets[i], ps.tolist())))
        else:
            rows.append([])
    row_ptr, col, prob = _csr(n, rows)
    src = np.arange(n_src, dtype=np.int32)
    lam_base = rng.uniform(50.0, 500.0, size=n_src)
    c = rng.integers(c_range[0], c_range[1] + 1, size=n).astype(np.int32)
    rho = rng.uniform(*rho_range, size=n)
    net = Network(n=n, row_ptr=row_ptr, col=col, prob=prob, servers=c, mu=np.ones(n, dtype=np.float32),
                  src=src, lambda0=lam_base.astype(np.float32), shape_kind=shape_kind,
                  amp=0.5 if shape_kind == SHAPE_SINUSOID else 0.0, period=24.0, phase=0.0,
                  name=f"dag{n}")
    lt = net.total_rates()
    mu1 = lt / (rho * c)
    kappa = 1.0 / float(np.median(mu1))
    net.lambda0 = (lam_base * kappa).astype(np.float32)
    lt = net.total_rates()
    net.mu = (lt / (rho * c)).astype(np.float32)
    return net


# --------------------------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    net: Network
    dt: float
    T: float
    reps: int
    seed: int = 0
    net_id: int = 0

    @property
    def K(self) -> int:
        return int(round(self.T / self.dt))

    @property
    def station_steps(self) -> int:
        return self.net.n * self.K * self.reps


def config1() -> Workload:
    """4-station tandem, lambda=20, mu=1, c=25, dt=0.01, T=10, 1000 replications."""
    return Workload("tandem4", tandem(4), dt=0.01, T=10.0, reps=1000)


def config2() -> Workload:
    """100 stations in 10 layers, sinusoidal arrivals, dt=0.01, T=48, 10^4 replications."""
    return Workload("layered100", layered(10, 10, seed=2), dt=0.01, T=48.0, reps=10000)


def config3() -> Workload:
    """1000-station sparse DAG, 50 sources, dt=0.005, T=100, 4096 replications."""
    return Workload("dag1000", sparse_dag(1000, 50, seed=3), dt=0.005, T=100.0, reps=4096)


def config4(count: int = 512, reps: int = 256, dt: float = 0.01, seed: int = 4) -> list[Workload]:
    """`count` independent DAG networks, n_k log-uniform in [10, 2000], T_k ~ U(10, 100)
    rounded to a multiple of dt, 256 replications each, network id k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(1, count + 1):
        nk = int(round(math.exp(rng.uniform(math.log(10), math.log(2000)))))
        Tk = round(float(rng.uniform(10.0, 100.0)) / dt) * dt
        net = sparse_dag(nk, max(1, int(round(0.05 * nk))), seed=k)
        net.name = f"dag{nk}_k{k}"
        out.append(Workload(net.name, net, dt=dt, T=Tk, reps=reps, net_id=k))
    return out


def config5_costs(n: int, seed: int = 5) -> tuple[np.ndarray, np.ndarray]:
    """Holding costs h_i ~ U(1, 5) and staffing costs k_i ~ U(0.1, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(1.0, 5.0, size=n), rng.uniform(0.1, 1.0, size=n)


def config5() -> Workload:
    w = config3()
    return Workload("dag1000_grad", w.net, dt=w.dt, T=w.T, reps=8192)


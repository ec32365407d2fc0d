"""Expected waiting-plus-staffing cost of a network as a differentiable torch function.

    J(mu, lambda0) = E[f],   f = sum_i hold_i (1/K) sum_{tau=1..K} (N_tau,i - m_i)^+  +  sum_i k_i m_i

where N is the Euler chain (backward or forward scheme) with per-server service rates mu and
external base rates lambda0.  The forward pass is one score run of the HIP library (the
simulation plus the per-replication sums of the likelihood-ratio scores of its Poisson and
binomial/Erlang draws) and the fp64 cost reduction; the backward pass is one of the library's
fp64 covariance reductions:

* "reach" (default): parameter j's score against the cost of the stations it can reach,
  grad_j = sum_r (f_{j,r} - mean f_j) S_{j,r} / (R - 1), f_{j,r} = sum_{i reachable from j}
  hold_i Q_{i,r} / K.  Stations outside that set do not depend on the parameter, so this is
  unbiased and leaves out their noise.
* "full": every score against the whole cost, grad_j = sum_r (f_r - mean f) S_{j,r} / (R - 1).

The simulation's integer path is the one a plain run takes: the same draws give the same states.

Only argument marshalling happens here; every step runs in the library.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import binding as eb


@dataclass
class CostProblem:
    """A network (netgen.Network-like: mu and lambda0 are replaced by the function's inputs),
    cost weights and the run: scheme, step dt, K steps, replications and Philox seed."""
    net: object
    hold: np.ndarray             # [n] holding cost per waiting customer and unit time
    staff: np.ndarray            # [n] staffing cost per server
    dt: float
    K: int
    reps: int
    scheme: int = eb.EQ_BACKWARD
    seed: int = 0
    dep_mode: int = eb.EQ_DEP_EXACT
    net_id: int = 0
    estimator: str = "reach"     # "reach" (pruned to reachable stations) or "full"
    # filled by each forward / backward pass: standard errors of J and of the gradient
    last: dict = field(default_factory=dict)

    def staffing(self) -> float:
        return float(np.dot(np.asarray(self.staff, np.float64), np.asarray(self.net.servers, np.float64)))


class ExpectedCost(torch.autograd.Function):
    """ExpectedCost.apply(mu [n], lambda0 [n_src], problem) -> J (0-dim float64 CUDA tensor)."""

    @staticmethod
    def forward(ctx, mu: torch.Tensor, lambda0: torch.Tensor, problem: CostProblem):
        p = problem
        net_np = p.net.replace(mu=mu.detach().to("cpu", torch.float32).numpy().copy(),
                               lambda0=lambda0.detach().to("cpu", torch.float32).numpy().copy())
        net = eb.Net(net_np)
        dev = torch.device("cuda", torch.cuda.current_device())
        res = eb.simulate_scores(net, p.scheme, p.dt, p.K, p.reps, p.seed, dep_mode=p.dep_mode, net_id=p.net_id)
        hold = torch.as_tensor(np.asarray(p.hold, np.float64), device=dev)
        f, mean_se = eb.cost_reduce(hold, res.sumq, p.K)
        J = mean_se[0] + p.staffing()
        p.last = {"J_se": mean_se[1]}
        if p.estimator not in ("reach", "full"):
            raise ValueError(f"estimator must be 'reach' or 'full', not {p.estimator!r}")
        ctx.save_for_backward(f, mean_se, res.score, res.sumq, hold)
        ctx.n = net.n
        ctx.net = net                      # keeps the device tables alive until backward
        ctx.problem = p
        ctx.in_meta = ((mu.dtype, mu.device), (lambda0.dtype, lambda0.device))
        return J

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        f, mean_se, score, sumq, hold = ctx.saved_tensors
        p = ctx.problem
        if p.estimator == "reach":
            g, se = eb.grad_reduce_reach(ctx.net, hold, sumq, score, p.K)
        else:
            g, se = eb.grad_reduce(f, mean_se, score)
        ctx.problem.last.update(grad=g, grad_se=se)
        n = ctx.n
        (mdt, mdev), (ldt, ldev) = ctx.in_meta
        gmu = (gJ * g[:n]).to(device=mdev, dtype=mdt)
        glam = (gJ * g[n:]).to(device=ldev, dtype=ldt)
        return gmu, glam, None


def expected_cost(mu: torch.Tensor, lambda0: torch.Tensor, problem: CostProblem) -> torch.Tensor:
    return ExpectedCost.apply(mu, lambda0, problem)


def cost_samples(problem: CostProblem, mu: Optional[np.ndarray] = None, lambda0: Optional[np.ndarray] = None,
                 seed: Optional[int] = None) -> torch.Tensor:
    """Per-replication costs f_r (float64 CUDA [reps], staffing included) of a plain run at
    (mu, lambda0): the building block of common-random-number finite differences."""
    p = problem
    kw = {}
    if mu is not None:
        kw["mu"] = np.asarray(mu, np.float32)
    if lambda0 is not None:
        kw["lambda0"] = np.asarray(lambda0, np.float32)
    net = eb.Net(p.net.replace(**kw) if kw else p.net)
    res = eb.simulate_scores(net, p.scheme, p.dt, p.K, p.reps, p.seed if seed is None else seed,
                             dep_mode=p.dep_mode, net_id=p.net_id)
    dev = res.sumq.device
    hold = torch.as_tensor(np.asarray(p.hold, np.float64), device=dev)
    f, _ = eb.cost_reduce(hold, res.sumq, p.K)
    return f + p.staffing()

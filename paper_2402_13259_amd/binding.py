"""ctypes binding of libeulerq.so (the C ABI in include/eulerq.h).

Argument marshalling only: every step of the simulation runs in the HIP library.  The
functions named eq_* mirror the C entry points one to one; `Net`, `simulate` and
`station_stats` are conveniences that allocate outputs as torch CUDA tensors and pass the
current torch stream.  Importing this module fails loudly when the library is missing:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeulerq.so")

from .abi import *  # noqa: F401,F403  (constants and structs of the C ABI)
from .abi import configure as _configure

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "(the simulator has no CPU fallback)")

_lib = C.CDLL(LIB_PATH)

globals().update(_configure(_lib))


class EqError(RuntimeError):
    """A negative return code of the library; `code` is the EQ_E* value, the message eq_last_error()."""
    def __init__(self, code: int, msg: str):
        super().__init__(f"eulerq error {code}: {msg}")
        self.code = code


def _check(rc: int) -> int:
    if rc < 0:
        raise EqError(rc, eq_last_error().decode())
    return rc


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _dev(t, dtype, shape, name: str):
    """A caller's tensor that the library will read or write through a raw device pointer: it
    must be a contiguous CUDA tensor of this dtype and shape (shape None: any) on the current
    device, else the kernels would be handed a host or foreign address."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} is on {t.device}; the current device is cuda:{torch.cuda.current_device()}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, not {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, not {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Net:
    """Owns an eq_net handle built from a netgen.Network-like object."""

    def __init__(self, net):
        self.n = int(net.n)
        self._keep = [np.ascontiguousarray(net.row_ptr, dtype=np.int32), np.ascontiguousarray(net.col, dtype=np.int32),
                      np.ascontiguousarray(net.prob, dtype=np.float32),
                      np.ascontiguousarray(net.servers, dtype=np.int32),
                      np.ascontiguousarray(net.mu, dtype=np.float32), np.ascontiguousarray(net.src, dtype=np.int32),
                      np.ascontiguousarray(net.lambda0, dtype=np.float32)]
        rp, col, prob, srv, mu, src, lam = self._keep
        self.nnz = int(rp[-1])
        self.n_src = len(src)
        kt = getattr(net, "knot_t", None)
        if kt is not None:
            self._keep += [np.ascontiguousarray(kt, dtype=np.float64),
                           np.ascontiguousarray(net.knot_shape, dtype=np.float64)]
            knots = (len(kt), _ptr(self._keep[-2]), _ptr(self._keep[-1]))
        else:
            knots = (0, None, None)
        arr = eq_arrivals(len(src), _ptr(src), _ptr(lam), int(net.shape_kind), float(net.amp), float(net.period),
                          float(net.phase), *knots)
        h = C.c_void_p()
        _check(eq_net_create(self.n, _ptr(rp), _ptr(col), _ptr(prob), _ptr(srv), _ptr(mu), C.byref(arr), C.byref(h)))
        self.handle = h
        if getattr(net, "staff_start", None) is not None:
            self.set_staffing(net.staff_start, net.staff_servers, getattr(net, "staff_period", 0))

    def set_params(self, mu=None, lambda0=None):
        """eq_net_set_params: new service rates [n] and/or base arrival rates [n_src]."""
        m = None if mu is None else np.ascontiguousarray(mu, dtype=np.float32).reshape(self.n)
        lam = None if lambda0 is None else np.ascontiguousarray(lambda0, dtype=np.float32).reshape(self.n_src)
        _check(eq_net_set_params(self.handle, _ptr(m), _ptr(lam)))

    def set_staffing(self, start, servers, period: int = 0):
        """eq_net_set_staffing; start=None clears the schedule."""
        if start is None:
            _check(eq_net_set_staffing(self.handle, 0, None, None, 0))
            return
        st = np.ascontiguousarray(start, dtype=np.int32)
        sv = np.ascontiguousarray(servers, dtype=np.int32).reshape(len(st), self.n)
        _check(eq_net_set_staffing(self.handle, len(st), _ptr(st), _ptr(sv), int(period)))

    def reach(self) -> np.ndarray:
        """eq_net_reach: bool [n + n_src, n], row j the stations parameter j can influence."""
        rows = _check(eq_net_reach(self.handle, None))
        out = np.zeros((rows, self.n), np.uint8)
        _check(eq_net_reach(self.handle, _ptr(out)))
        return out.astype(bool)

    def close(self):
        """eq_net_destroy (waits for queued device work first); later calls do nothing."""
        if getattr(self, "handle", None):
            eq_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tables(self, dt: float, K: int) -> dict:
        """eq_net_tables: the host tables for step dt and K steps (q, pdep, rate, mudt, kap, g)."""
        out = {"q": np.zeros(max(self.nnz, 1), np.float32), "pdep": np.zeros(self.n, np.float32),
               "rate": np.zeros(self.n, np.float32), "mudt": np.zeros(self.n, np.float32),
               "kap": np.zeros(self.n, np.float32), "g": np.zeros(max(K, 1), np.float32)}
        _check(eq_net_tables(self.handle, C.c_float(dt), int(K),
                             *(_ptr(out[k]) for k in ("q", "pdep", "rate", "mudt", "kap", "g"))))
        out["q"] = out["q"][:self.nnz]
        out["g"] = out["g"][:K]
        return out

    def levels(self) -> np.ndarray:
        """eq_net_levels: every station's longest-path level (EQ_ENOTDAG if not index-ordered)."""
        lev = np.zeros(self.n, np.int32)
        _check(eq_net_levels(self.handle, _ptr(lev)))
        return lev


@dataclass
class RunResult:
    """A run: final states [n, reps] int32, tile sums [3, n, tiles] int64 (or None) and its descriptor."""
    state: "object"      # torch int32 [n, reps]
    sums: "object"       # torch int64 [3, n, tiles] (32-replication statistics tiles) or None
    desc: eq_run_desc


def n_tiles(reps: int) -> int:
    """Number of statistics tiles (EQ_STAT_TILE_REPS replications each) of the sums."""
    return (int(reps) + STAT_TILE_REPS - 1) // STAT_TILE_REPS


def make_desc(scheme: int, dt: float, K: int, reps: int, seed: int = 0, dep_mode: int = EQ_DEP_EXACT,
              net_id: int = 0, rep0: int = 0, tile_reps: int = 0, block: int = 0,
              kernel: int = EQ_KERNEL_AUTO) -> eq_run_desc:
    """An eq_run_desc from keyword values (seed taken modulo 2^64)."""
    return eq_run_desc(int(scheme), int(dep_mode), float(dt), int(K), int(seed) & (2**64 - 1), int(net_id),
                       int(rep0), int(reps), int(kernel), int(tile_reps), int(block))


def simulate(net: Net, scheme: int, dt: float, K: int, reps: int, seed: int = 0, *, dep_mode: int = EQ_DEP_EXACT,
             net_id: int = 0, rep0: int = 0, init=None, with_sums: bool = True, tile_reps: int = 0, block: int = 0,
             kernel: int = EQ_KERNEL_AUTO, state=None, sums=None, stream=None, check: bool = True) -> RunResult:
    """Run one scheme on the GPU; outputs are torch tensors on the current device."""
    import torch
    desc = make_desc(scheme, dt, K, reps, seed, dep_mode, net_id, rep0, tile_reps, block, kernel)
    dev = torch.device("cuda", torch.cuda.current_device())
    if state is None:
        state = torch.empty((net.n, reps), dtype=torch.int32, device=dev)
    if with_sums and sums is None:
        sums = torch.empty((3, net.n, n_tiles(reps)), dtype=torch.int64, device=dev)
    _dev(state, torch.int32, (net.n, reps), "state")
    if with_sums:
        _dev(sums, torch.int64, (3, net.n, n_tiles(reps)), "sums")
    if init is not None:
        _dev(init, torch.int32, (net.n, reps), "init")
    _check(eq_sim_run(net.handle, C.byref(desc), _ptr(init), _ptr(state), _ptr(sums) if with_sums else None,
                      _stream(stream)))
    if check:
        _check(eq_sim_check(net.handle, _stream(stream)))
    return RunResult(state, sums if with_sums else None, desc)


@dataclass
class ScoreResult:
    """A score run: the run plus the per-replication (N-m)^+ sums and the fp32 score sums [n + n_src, reps]."""
    state: "object"      # torch int32 [n, reps]
    sums: "object"       # torch int64 [3, n, tiles] or None
    sumq: "object"       # torch int64 [n, reps]: sum over tau of (N - m)^+
    score: "object"      # torch float32 [n + n_src, reps]: mu rows, then lambda0 rows
    desc: eq_run_desc


def simulate_scores(net: Net, scheme: int, dt: float, K: int, reps: int, seed: int = 0, *,
                    dep_mode: int = EQ_DEP_EXACT, net_id: int = 0, rep0: int = 0, init=None, with_sums: bool = False,
                    state=None, sums=None, sumq=None, score=None, stream=None, check: bool = True) -> ScoreResult:
    """A score run (eq_sim_run_scores): the simulation plus per-replication score sums."""
    import torch
    desc = make_desc(scheme, dt, K, reps, seed, dep_mode, net_id, rep0, kernel=EQ_KERNEL_SWEEP)
    dev = torch.device("cuda", torch.cuda.current_device())
    if state is None:
        state = torch.empty((net.n, reps), dtype=torch.int32, device=dev)
    if with_sums and sums is None:
        sums = torch.empty((3, net.n, n_tiles(reps)), dtype=torch.int64, device=dev)
    if sumq is None:
        sumq = torch.empty((net.n, reps), dtype=torch.int64, device=dev)
    if score is None:
        score = torch.empty((net.n + net.n_src, reps), dtype=torch.float32, device=dev)
    _dev(state, torch.int32, (net.n, reps), "state")
    if with_sums:
        _dev(sums, torch.int64, (3, net.n, n_tiles(reps)), "sums")
    _dev(sumq, torch.int64, (net.n, reps), "sumq")
    _dev(score, torch.float32, (net.n + net.n_src, reps), "score")
    if init is not None:
        _dev(init, torch.int32, (net.n, reps), "init")
    slam = score[net.n:] if net.n_src else None
    _check(eq_sim_run_scores(net.handle, C.byref(desc), _ptr(init), _ptr(state), _ptr(sums) if with_sums else None,
                             _ptr(sumq), _ptr(score), _ptr(slam), _stream(stream)))
    if check:
        _check(eq_sim_check(net.handle, _stream(stream)))
    return ScoreResult(state, sums if with_sums else None, sumq, score, desc)


def cost_reduce(hold, sumq, K: int, stream=None):
    """(f [reps] float64, mean_se [2] float64) from eq_cost_reduce; hold float64 CUDA [n]."""
    import torch
    _dev(sumq, torch.int64, None, "sumq")
    if sumq.dim() != 2:
        raise ValueError("sumq must be [n, reps]")
    n, reps = sumq.shape
    _dev(hold, torch.float64, (n,), "hold")
    f = torch.empty(reps, dtype=torch.float64, device=sumq.device)
    ms = torch.empty(2, dtype=torch.float64, device=sumq.device)
    _check(eq_cost_reduce(int(n), int(reps), int(K), _ptr(hold), _ptr(sumq), _ptr(f), _ptr(ms), _stream(stream)))
    return f, ms


def grad_reduce(f, mean_se, score, stream=None):
    """(grad [n_par] float64, se [n_par] float64) from eq_grad_reduce over the rows of score."""
    import torch
    _dev(score, torch.float32, None, "score")
    if score.dim() != 2:
        raise ValueError("score must be [n_par, reps]")
    n_par, reps = score.shape
    _dev(f, torch.float64, (reps,), "f")
    _dev(mean_se, torch.float64, (2,), "mean_se")
    g = torch.empty(n_par, dtype=torch.float64, device=score.device)
    se = torch.empty(n_par, dtype=torch.float64, device=score.device)
    _check(eq_grad_reduce(int(n_par), int(reps), _ptr(f), _ptr(mean_se), _ptr(score), _ptr(g), _ptr(se),
                          _stream(stream)))
    return g, se


def grad_reduce_reach(net: Net, hold, sumq, score, K: int, stream=None):
    """(grad [n_par] float64, se [n_par] float64) from eq_grad_reduce_reach: each parameter's
    score against the waiting cost of the stations it can reach."""
    import torch
    _dev(score, torch.float32, None, "score")
    if score.dim() != 2 or score.shape[0] != net.n + net.n_src:
        raise ValueError("score must be [n + n_src, reps]")
    n_par, reps = score.shape
    _dev(sumq, torch.int64, (net.n, reps), "sumq")
    _dev(hold, torch.float64, (net.n,), "hold")
    g = torch.empty(n_par, dtype=torch.float64, device=score.device)
    se = torch.empty(n_par, dtype=torch.float64, device=score.device)
    _check(eq_grad_reduce_reach(net.handle, int(reps), int(K), _ptr(hold), _ptr(sumq), _ptr(score), _ptr(g), _ptr(se),
                                _stream(stream)))
    return g, se


def tune(net: Net, scheme: int, dt: float, K: int, reps: int, seed: int = 0, *, dep_mode: int = EQ_DEP_EXACT,
         trial_steps: int = 64, stream=None) -> dict:
    """Autotuned launch shape for this network and run shape (eq_sim_tune): a dict of the
    simulate() keywords kernel, tile_reps and block."""
    import torch
    desc = make_desc(scheme, dt, K, reps, seed, dep_mode)
    scratch = torch.empty((net.n, reps), dtype=torch.int32, device=torch.device("cuda", torch.cuda.current_device()))
    best = eq_run_desc()
    _check(eq_sim_tune(net.handle, C.byref(desc), int(trial_steps), _ptr(scratch), _stream(stream), C.byref(best)))
    return {"kernel": best.kernel, "tile_reps": best.tile_reps, "block": best.block}


@dataclass
class PairResult:
    """A pair run (average scheme): the backward and the forward RunResult."""
    backward: RunResult
    forward: RunResult


def simulate_pair(net: Net, dt: float, K: int, reps: int, seed: int = 0, *, dep_mode: int = EQ_DEP_EXACT,
                  net_id: int = 0, rep0: int = 0, init=None, block: int = 0, states=None, sums=None, stream=None,
                  check: bool = True) -> PairResult:
    """The average scheme's pair run (eq_sim_run_pair): backward and forward in one launch per step."""
    import torch
    desc = make_desc(EQ_BACKWARD, dt, K, reps, seed, dep_mode, net_id, rep0, block=block)
    dev = torch.device("cuda", torch.cuda.current_device())
    if states is None:
        states = [torch.empty((net.n, reps), dtype=torch.int32, device=dev) for _ in range(2)]
    if sums is None:
        sums = [torch.empty((3, net.n, n_tiles(reps)), dtype=torch.int64, device=dev) for _ in range(2)]
    for k in range(2):
        _dev(states[k], torch.int32, (net.n, reps), f"states[{k}]")
        _dev(sums[k], torch.int64, (3, net.n, n_tiles(reps)), f"sums[{k}]")
    if init is not None:
        _dev(init, torch.int32, (net.n, reps), "init")
    _check(eq_sim_run_pair(net.handle, C.byref(desc), _ptr(init), _ptr(states[0]), _ptr(states[1]), _ptr(sums[0]),
                           _ptr(sums[1]), _stream(stream)))
    if check:
        _check(eq_sim_check(net.handle, _stream(stream)))
    fdesc = make_desc(EQ_FORWARD, dt, K, reps, seed, dep_mode, net_id, rep0, block=block)
    return PairResult(RunResult(states[0], sums[0], desc), RunResult(states[1], sums[1], fdesc))


@dataclass
class RecordResult:
    """A recording run: the run, the first recorded step and the records N, D [len, n, reps], R [len, nnz, reps]."""
    run: RunResult
    rec_t0: int
    N: "object"          # torch int32 [rec_len, n, reps]
    D: "object"          # torch int32 [rec_len, n, reps]
    R: "object"          # torch int32 [rec_len, nnz, reps]


def simulate_host(net: Net, scheme: int, dt: float, K: int, reps: int, seed: int = 0, *,
                  dep_mode: int = EQ_DEP_EXACT, net_id: int = 0, rep0: int = 0, init=None, kernel: int = EQ_KERNEL_AUTO):
    """eq_sim_run_host: a synchronous run with host buffers; (final states int32 [n, reps],
    statistics float64 [6, n])."""
    desc = make_desc(scheme, dt, K, reps, seed, dep_mode, net_id, rep0, kernel=kernel)
    fin = np.zeros((net.n, reps), np.int32)
    stats = np.zeros((6, net.n), np.float64)
    ini = None if init is None else np.ascontiguousarray(init, dtype=np.int32).reshape(net.n, reps)
    _check(eq_sim_run_host(net.handle, C.byref(desc), _ptr(ini), _ptr(fin), _ptr(stats)))
    return fin, stats


def simulate_record(net: Net, scheme: int, dt: float, K: int, reps: int, seed: int = 0, *, rec_t0: int = 1,
                    rec_len: Optional[int] = None, dep_mode: int = EQ_DEP_EXACT, net_id: int = 0, rep0: int = 0,
                    init=None, with_sums: bool = True, stream=None, check: bool = True) -> RecordResult:
    """A recording run (eq_sim_run_record) over steps rec_t0 .. rec_t0 + rec_len - 1."""
    import torch
    rec_len = K - rec_t0 + 1 if rec_len is None else rec_len
    desc = make_desc(scheme, dt, K, reps, seed, dep_mode, net_id, rep0, kernel=EQ_KERNEL_SWEEP)
    dev = torch.device("cuda", torch.cuda.current_device())
    state = torch.empty((net.n, reps), dtype=torch.int32, device=dev)
    sums = torch.empty((3, net.n, n_tiles(reps)), dtype=torch.int64, device=dev) if with_sums else None
    rN = torch.empty((rec_len, net.n, reps), dtype=torch.int32, device=dev)
    rD = torch.empty((rec_len, net.n, reps), dtype=torch.int32, device=dev)
    rR = torch.empty((rec_len, max(net.nnz, 1), reps), dtype=torch.int32, device=dev)
    if init is not None:
        _dev(init, torch.int32, (net.n, reps), "init")
    _check(eq_sim_run_record(net.handle, C.byref(desc), _ptr(init), _ptr(state), _ptr(sums), int(rec_t0),
                             int(rec_len), _ptr(rN), _ptr(rD), _ptr(rR), _stream(stream)))
    if check:
        _check(eq_sim_check(net.handle, _stream(stream)))
    return RecordResult(RunResult(state, sums, desc), int(rec_t0), rN, rD, rR[:, :net.nnz])


def sojourn(net: Net, rec: RecordResult, i0, tau0, stream=None):
    """eq_sojourn: sojourn times in intervals, torch int32 [n_samples, reps] (-1: censored)."""
    import torch
    i0 = np.ascontiguousarray(i0, dtype=np.int32).reshape(-1)
    tau0 = np.ascontiguousarray(tau0, dtype=np.int32).reshape(-1)
    if len(i0) != len(tau0):
        raise ValueError("i0 and tau0 must have the same length")
    _dev(rec.N, torch.int32, None, "rec.N")
    if rec.N.dim() != 3 or rec.N.shape[1] != net.n:
        raise ValueError("rec.N must be [rec_len, n, reps]")
    rec_len, _, reps = rec.N.shape
    _dev(rec.D, torch.int32, (rec_len, net.n, reps), "rec.D")
    if tuple(rec.R.shape) != (rec_len, net.nnz, reps):
        raise ValueError(f"rec.R must have shape {(rec_len, net.nnz, reps)}")
    out = torch.empty((len(i0), reps), dtype=torch.int32, device=rec.N.device)
    rR = rec.R if rec.R.shape[1] else None
    _check(eq_sojourn(net.handle, C.byref(rec.run.desc), rec.rec_t0, rec.N.shape[0], _ptr(rec.N), _ptr(rec.D),
                      _ptr(rR.contiguous()) if rR is not None else None, len(i0), _ptr(i0), _ptr(tau0), _ptr(out),
                      _stream(stream)))
    return out


def pair_stats(net: Net, res: PairResult, init=None, stream=None):
    """[6, n] float64 statistics of the average scheme (eq_stats_reduce_pair)."""
    import torch
    b, f = res.backward, res.forward
    reps = b.desc.reps
    for k, r in enumerate((b, f)):
        _dev(r.state, torch.int32, (net.n, reps), f"state[{k}]")
        _dev(r.sums, torch.int64, (3, net.n, n_tiles(reps)), f"sums[{k}]")
    if init is not None:
        _dev(init, torch.int32, (net.n, reps), "init")
    out = torch.empty((6, net.n), dtype=torch.float64, device=b.state.device)
    _check(eq_stats_reduce_pair(net.handle, C.byref(b.desc), _ptr(b.sums), _ptr(f.sums), _ptr(b.state),
                                _ptr(f.state), _ptr(init), _ptr(out), _stream(stream)))
    return out


def station_stats(net: Net, res: RunResult, init=None, stream=None):
    """[6, n] float64: mean N, SE, mean (N-m)^+, SE, throughput, mean waiting time (Little)."""
    import torch
    reps = res.desc.reps
    _dev(res.state, torch.int32, (net.n, reps), "state")
    if res.sums is None:
        raise ValueError("station_stats needs a run made with sums")
    _dev(res.sums, torch.int64, (3, net.n, n_tiles(reps)), "sums")
    if init is not None:
        _dev(init, torch.int32, (net.n, reps), "init")
    out = torch.empty((6, net.n), dtype=torch.float64, device=res.state.device)
    _check(eq_stats_reduce(net.handle, C.byref(res.desc), _ptr(res.sums), _ptr(res.state), _ptr(init), _ptr(out),
                           _stream(stream)))
    return out


def selftest_math(kind: int, x):
    """eq_selftest_math: the device log (0), log1p (1), exp (2) or expm1 (3) of every element of x,
    or (4) the uniform the samplers take from the 32-bit word with the element's bits."""
    import torch
    _dev(x, torch.float32, None, "x")
    y = torch.empty_like(x)
    _check(eq_selftest_math(kind, _ptr(x), _ptr(y), x.numel(), _stream()))
    torch.cuda.synchronize()
    return y


def selftest_sample(kind: int, count: int, seed: int = 0, rep0: int = 0, station: int = 0, step0: int = 0,
                    sub: int = 1, i0: int = 0, i1: int = 0, f0: float = 0.0, f1: float = 0.0, f2: float = 0.0,
                    f3: float = 0.0):
    """eq_selftest_sample: `count` draws of one device sampler on the streams (rep0 + s, station, step0, sub)."""
    import torch
    out = torch.empty(count, dtype=torch.float32, device="cuda")
    _check(eq_selftest_sample(kind, count, seed, rep0, station, step0, sub, i0, i1, f0, f1, f2, f3, _ptr(out),
                              _stream()))
    return out


def selftest_score(kind: int, count: int, seed: int = 0, rep0: int = 0, station: int = 0, step0: int = 0,
                   sub: int = 1, x: int = 0, m: int = 0, f0: float = 0.0, f1: float = 0.0):
    """eq_selftest_score: `count` draws of one device sampler with their likelihood-ratio scores."""
    import torch
    val = torch.empty(count, dtype=torch.float32, device="cuda")
    sc = torch.empty(count, dtype=torch.float32, device="cuda")
    _check(eq_selftest_score(kind, count, seed, rep0, station, step0, sub, x, m, f0, f1, _ptr(val), _ptr(sc),
                             _stream()))
    return val, sc


def valu_peak(grid: int = 8192, iters: int = 1000, stream=None) -> float:
    """Measured non-packed fp32 FMA rate of the device, in lane-FMAs per second."""
    import torch
    out = torch.empty(grid * 256, dtype=torch.float32, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(eq_selftest_valu_peak(grid, iters, _ptr(out), s.cuda_stream))   # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    _check(eq_selftest_valu_peak(grid, iters, _ptr(out), s.cuda_stream))
    e1.record(s)
    e1.synchronize()
    return grid * 256.0 * iters * 128 / (e0.elapsed_time(e1) * 1e-3)


def selftest_philox(ctr, key):
    """eq_selftest_philox: the device Philox4x32-10 of every (counter [4], key [2]) row."""
    import torch
    _dev(ctr, torch.int32, None, "ctr")
    if ctr.dim() != 2 or ctr.shape[1] != 4:
        raise ValueError("ctr must be [rows, 4]")
    _dev(key, torch.int32, (ctr.shape[0], 2), "key")
    out = torch.empty_like(ctr)
    _check(eq_selftest_philox(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out), _stream()))
    torch.cuda.synchronize()
    return out


class Batch:
    """A group of Nets run together (eq_batch_*); keeps the Nets alive."""

    def __init__(self, nets):
        self.nets = list(nets)
        arr = (C.c_void_p * len(self.nets))(*[n.handle.value for n in self.nets])
        h = C.c_void_p()
        _check(eq_batch_create(len(self.nets), arr, C.byref(h)))
        self.handle = h

    def close(self):
        """eq_batch_destroy (waits for queued device work first); the networks stay valid."""
        if getattr(self, "handle", None):
            eq_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def layout(self, reps: int):
        """eq_batch_layout: offsets of every network's states and sums in the concatenated outputs."""
        so = np.zeros(len(self.nets) + 1, np.int64)
        mo = np.zeros(len(self.nets) + 1, np.int64)
        _check(eq_batch_layout(self.handle, int(reps), _ptr(so), _ptr(mo)))
        return so, mo

    def run(self, scheme: int, dt: float, n_steps, net_ids, reps: int, seed: int = 0, *,
            dep_mode: int = EQ_DEP_EXACT, waves_per_block: int = 0, use_graph: bool = True, with_sums: bool = True,
            states=None, sums=None, stream=None, check: bool = True):
        """Returns (states, sums) torch tensors (concatenated; see layout())."""
        import torch
        so, mo = self.layout(reps)
        if states is None:
            states = torch.empty(int(so[-1]), dtype=torch.int32, device="cuda")
        if with_sums and sums is None:
            sums = torch.empty(int(mo[-1]), dtype=torch.int64, device="cuda")
        _dev(states, torch.int32, (int(so[-1]),), "states")
        if with_sums:
            _dev(sums, torch.int64, (int(mo[-1]),), "sums")
        ks = np.ascontiguousarray(n_steps, dtype=np.int32).reshape(-1)
        ids = np.ascontiguousarray(net_ids, dtype=np.uint32).reshape(-1)
        if not len(ks) == len(self.nets) == len(ids):
            raise ValueError("n_steps and net_ids need one entry per network")
        d = eq_batch_desc(int(scheme), int(dep_mode), float(dt), int(seed) & (2**64 - 1), int(reps),
                          int(waves_per_block), int(bool(use_graph)))
        _check(eq_batch_run(self.handle, C.byref(d), _ptr(ks), _ptr(ids), _ptr(states),
                            _ptr(sums) if with_sums else None, _stream(stream)))
        if check:
            _check(eq_batch_check(self.handle, _stream(stream)))
        return states, (sums if with_sums else None)

    def tune(self, scheme: int, dt: float, n_steps, net_ids, reps: int, seed: int = 0, *,
             dep_mode: int = EQ_DEP_EXACT, trial_fraction: float = 0.02, stream=None) -> int:
        """eq_batch_tune: the fastest waves per workgroup, remembered by the batch."""
        import torch
        so, mo = self.layout(reps)
        states = torch.empty(int(so[-1]), dtype=torch.int32, device="cuda")
        ks = np.ascontiguousarray(n_steps, dtype=np.int32).reshape(-1)
        ids = np.ascontiguousarray(net_ids, dtype=np.uint32).reshape(-1)
        if not len(ks) == len(self.nets) == len(ids):
            raise ValueError("n_steps and net_ids need one entry per network")
        d = eq_batch_desc(int(scheme), int(dep_mode), float(dt), int(seed) & (2**64 - 1), int(reps), 0, 0)
        best = C.c_int32(0)
        _check(eq_batch_tune(self.handle, C.byref(d), _ptr(ks), _ptr(ids), C.c_float(trial_fraction), _ptr(states),
                             None, _stream(stream), C.byref(best)))
        return best.value

    def check(self, stream=None):
        """eq_batch_check: synchronise the stream and raise on a sticky device flag."""
        _check(eq_batch_check(self.handle, _stream(stream)))

    def split(self, states, sums, reps: int):
        """Per-network views: [(state [n, reps], sums [3, n, tiles]), ...]."""
        so, mo = self.layout(reps)
        t = n_tiles(reps)
        out = []
        for k, net in enumerate(self.nets):
            st = states[so[k]:so[k + 1]].view(net.n, reps)
            sm = None if sums is None else sums[mo[k]:mo[k + 1]].view(3, net.n, t)
            out.append((st, sm))
        return out


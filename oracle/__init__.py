"""Python access to the CPU oracle (plain C, see euler_oracle.c and des.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
cpu_baseline leg may import this package.  The GPU library never uses it.

`build()` compiles liboracle.so with gcc (-O2 -ffp-contract=off, no fast-math);
`lib()` loads it, building it first if it is missing.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "euler_oracle.c"), os.path.join(HERE, "des.c")]
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread", "-std=gnu11"]

BACKWARD, FORWARD = 0, 1
DEP_EXACT, DEP_NAIVE = 0, 1
SUB_ARRIVAL, SUB_DEPART, SUB_ROUTE = 0, 1, 2
SMP_POISSON, SMP_BINOMIAL, SMP_GAMMA, SMP_GENDEP, SMP_GENDEP_NAIVE = range(5)

_lib = None


def build() -> str:
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, *SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Net(C.Structure):
    _fields_ = [("n", C.c_int32), ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("prob", C.c_void_p),
                ("servers", C.c_void_p), ("mu", C.c_void_p), ("n_src", C.c_int32), ("src", C.c_void_p),
                ("lambda0", C.c_void_p), ("shape_kind", C.c_int32), ("amp", C.c_double),
                ("period", C.c_double), ("phase", C.c_double), ("n_seg", C.c_int32), ("seg_start", C.c_void_p),
                ("seg_servers", C.c_void_p), ("seg_period", C.c_int32), ("n_knots", C.c_int32),
                ("knot_t", C.c_void_p), ("knot_shape", C.c_void_p)]


def build_variant(substitutions, out_dir: str, name: str = "liboracle_variant.so", extra_flags=()) -> str:
    """Compile a copy of the oracle with textual substitutions [(old, new), ...] applied to
    euler_oracle.c (each `old` must occur exactly once) and optional extra compiler flags: the
    planted-mistake tests use this to check that their pins fail on a wrong oracle, the
    sanitizer tests to build it with AddressSanitizer.  Returns the library path."""
    src = open(SOURCES[0]).read()
    for old, new in substitutions:
        if src.count(old) != 1:
            raise ValueError(f"substitution target must occur once: {old!r}")
        src = src.replace(old, new)
    os.makedirs(out_dir, exist_ok=True)
    cpath = os.path.join(out_dir, "euler_oracle_variant.c")
    with open(cpath, "w") as fh:
        fh.write(src)
    out = os.path.join(out_dir, name)
    subprocess.run(["gcc", *CFLAGS, *extra_flags, "-o", out, cpath, SOURCES[1], "-lm"], check=True)
    return out


@contextlib.contextmanager
def using_library(path: str):
    """Route every call of this module to the oracle library at `path` for the duration."""
    global _lib
    saved = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _load(LIB_PATH)
    return _lib


def _load(path: str):
    L = C.CDLL(path)
    vp, i32, i64, u32, u64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float
    L.orc_run.argtypes = [C.POINTER(_Net), i32, i32, f32, i32, u64, u32, i32, vp, vp, vp, vp, vp, vp,
                          vp, vp, vp, i32]
    L.orc_tables.argtypes = [C.POINTER(_Net), f32, i32, vp, vp, vp, vp, vp, vp]
    L.orc_sample_score.argtypes = [i32, i64, u64, u32, u32, u32, u32, i32, i32, f32, f32, vp, vp]
    L.orc_run_record.argtypes = [C.POINTER(_Net), i32, i32, f32, i32, u64, u32, i32, vp, vp, vp, i32, i32, vp,
                                 vp, vp, i32]
    L.orc_sojourn.argtypes = [C.POINTER(_Net), i32, u64, u32, i32, vp, i32, i32, vp, vp, vp, i32, vp, vp, vp]
    L.orc_lemma3.argtypes = [i32, i32, i32]
    L.orc_lemma3.restype = f32
    L.orc_btrs_log_ratio.argtypes = [i32, f32, i32]
    L.orc_btrs_log_ratio.restype = f32
    L.orc_ptrs_log_pmf.argtypes = [f32, i32]
    L.orc_ptrs_log_pmf.restype = f32
    L.orc_sample.argtypes = [i32, i64, u64, u32, u32, u32, u32, i32, i32, f32, f32, f32, f32, vp]
    L.orc_math.argtypes = [i32, i64, vp, vp]
    L.orc_philox_batch.argtypes = [i64, vp, vp, vp]
    L.orc_get_tables.argtypes = [vp, vp]
    L.orc_get_tables.restype = None
    L.orc_philox_batch.restype = None
    L.orc_op_counts.argtypes = [vp, C.c_int]
    L.des_run.argtypes = [C.POINTER(_Net), C.c_double, i32, u64, i32, vp, i32, vp, vp, vp, vp, vp, vp,
                          i32]
    return L


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class _NetHolder:
    """Keeps contiguous copies of the network arrays alive while C uses them."""

    def __init__(self, net):
        self.arrs = [np.ascontiguousarray(net.row_ptr, dtype=np.int32), np.ascontiguousarray(net.col, dtype=np.int32),
                     np.ascontiguousarray(net.prob, dtype=np.float32),
                     np.ascontiguousarray(net.servers, dtype=np.int32), np.ascontiguousarray(net.mu, dtype=np.float32),
                     np.ascontiguousarray(net.src, dtype=np.int32),
                     np.ascontiguousarray(net.lambda0, dtype=np.float32)]
        rp, col, prob, srv, mu, src, lam = self.arrs
        start = getattr(net, "staff_start", None)
        if start is not None:
            self.arrs += [np.ascontiguousarray(start, dtype=np.int32),
                          np.ascontiguousarray(net.staff_servers, dtype=np.int32).reshape(-1)]
            nseg, pst, psv, per = len(start), _ptr(self.arrs[-2]), _ptr(self.arrs[-1]), int(net.staff_period)
        else:
            nseg, pst, psv, per = 0, None, None, 0
        kt = getattr(net, "knot_t", None)
        if kt is not None:
            self.arrs += [np.ascontiguousarray(kt, dtype=np.float64), np.ascontiguousarray(net.knot_shape, dtype=np.float64)]
            nk, pkt, pks = len(kt), _ptr(self.arrs[-2]), _ptr(self.arrs[-1])
        else:
            nk, pkt, pks = 0, None, None
        self.s = _Net(int(net.n), _ptr(rp), _ptr(col), _ptr(prob), _ptr(srv), _ptr(mu), int(len(src)), _ptr(src),
                      _ptr(lam), int(net.shape_kind), float(net.amp), float(net.period), float(net.phase), nseg, pst,
                      psv, per, nk, pkt, pks)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def run(net, scheme: int, dt: float, K: int, seed: int, rep_ids: Sequence[int], dep_mode: int = DEP_EXACT,
        net_id: int = 0, init_state=None, inj_arr=None, threads: Optional[int] = None, scores: bool = False) -> dict:
    """Simulate the listed global replication ids; returns final states and per-station
    sums over tau=1..K of N, (N-m)^+ and D, each [len(rep_ids), n].  With `scores`, also
    the fp32 sums of the departure-draw scores in mu_i ("score_mu", [R, n]) and of the
    arrival-draw scores in lambda0_s ("score_lam", [R, n_src])."""
    L = lib()
    h = _NetHolder(net)
    rep_ids = np.ascontiguousarray(rep_ids, dtype=np.int32)
    R, n = len(rep_ids), int(net.n)
    final = np.zeros((R, n), dtype=np.int32)
    sN = np.zeros((R, n), dtype=np.int64)
    sQ = np.zeros((R, n), dtype=np.int64)
    sD = np.zeros((R, n), dtype=np.int64)
    init = None if init_state is None else np.ascontiguousarray(init_state, dtype=np.int32)
    inj = None if inj_arr is None else np.ascontiguousarray(inj_arr, dtype=np.int32)
    if inj is not None:
        assert inj.shape == (K, n)
    smu = np.zeros((R, n), np.float32) if scores else None
    slam = np.zeros((R, max(len(net.src), 1)), np.float32) if scores else None
    rc = L.orc_run(C.byref(h.s), scheme, dep_mode, C.c_float(dt), int(K), C.c_uint64(seed), C.c_uint32(net_id), R,
                   _ptr(rep_ids), _ptr(init), _ptr(inj), _ptr(final), _ptr(sN), _ptr(sQ), _ptr(sD), _ptr(smu),
                   _ptr(slam), threads or default_threads())
    if rc not in (0, -5):
        raise ValueError(f"orc_run failed with code {rc}")
    out = {"final": final, "sumN": sN, "sumQ": sQ, "sumD": sD, "overflow": rc == -5}
    if scores:
        out["score_mu"] = smu
        out["score_lam"] = slam[:, :len(net.src)]
    return out


def run_record(net, scheme: int, dt: float, K: int, seed: int, rep_ids: Sequence[int], rec_t0: int, rec_len: int,
               dep_mode: int = DEP_EXACT, net_id: int = 0, init_state=None, threads: Optional[int] = None) -> dict:
    """A run that records N_tau, D_tau ([R, rec_len, n]) and the routed count of every edge
    ([R, rec_len, nnz]) for tau = rec_t0 .. rec_t0 + rec_len - 1."""
    L = lib()
    h = _NetHolder(net)
    rep_ids = np.ascontiguousarray(rep_ids, dtype=np.int32)
    R, n, nnz = len(rep_ids), int(net.n), int(net.row_ptr[-1])
    final = np.zeros((R, n), np.int32)
    rN = np.zeros((R, rec_len, n), np.int32)
    rD = np.zeros((R, rec_len, n), np.int32)
    rR = np.zeros((R, rec_len, max(nnz, 1)), np.int32)
    init = None if init_state is None else np.ascontiguousarray(init_state, dtype=np.int32)
    rc = L.orc_run_record(C.byref(h.s), scheme, dep_mode, C.c_float(dt), int(K), C.c_uint64(seed),
                          C.c_uint32(net_id), R, _ptr(rep_ids), _ptr(init), _ptr(final), int(rec_t0), int(rec_len),
                          _ptr(rN), _ptr(rD), _ptr(rR), threads or default_threads())
    if rc not in (0, -5):
        raise ValueError(f"orc_run_record failed with code {rc}")
    return {"final": final, "N": rN, "D": rD, "R": rR[:, :, :nnz], "rec_t0": rec_t0, "rep_ids": rep_ids}


def sojourn(net, scheme: int, seed: int, rec: dict, i0: Sequence[int], tau0: Sequence[int], net_id: int = 0) -> np.ndarray:
    """Algorithm 4 on a recorded path: sojourn times in intervals [R, n_samples], -1 where the
    record is too short."""
    L = lib()
    h = _NetHolder(net)
    i0 = np.ascontiguousarray(i0, dtype=np.int32)
    tau0 = np.ascontiguousarray(tau0, dtype=np.int32)
    rN, rD = np.ascontiguousarray(rec["N"]), np.ascontiguousarray(rec["D"])
    rR = np.ascontiguousarray(rec["R"]) if rec["R"].shape[2] else np.zeros(rN.shape[:2] + (1,), np.int32)
    R, rec_len = rN.shape[0], rN.shape[1]
    out = np.zeros((R, len(i0)), np.int32)
    rc = L.orc_sojourn(C.byref(h.s), scheme, C.c_uint64(seed), C.c_uint32(net_id), R, _ptr(rec["rep_ids"]),
                       int(rec["rec_t0"]), rec_len, _ptr(rN), _ptr(rD), _ptr(rR), len(i0), _ptr(i0), _ptr(tau0),
                       _ptr(out))
    if rc not in (0, -5):
        raise ValueError(f"orc_sojourn failed with code {rc}")
    return out


def lemma3(x: int, d: int, m: int) -> float:
    return float(lib().orc_lemma3(int(x), int(d), int(m)))


def btrs_log_ratio(n: int, p: float, k: int) -> float:
    """BTRS's acceptance log-ratio ln f(k)/f(m) of Binomial(n, p), 0 < p <= 1/2, m = floor((n+1) p),
    as the sampler computes it (Stirling series, fp32)."""
    return float(lib().orc_btrs_log_ratio(int(n), C.c_float(p), int(k)))


def ptrs_log_pmf(lam: float, k: int) -> float:
    """PTRS's acceptance bound ln f(k) of Poisson(lam), as the sampler computes it (Stirling series, fp32)."""
    return float(lib().orc_ptrs_log_pmf(C.c_float(lam), int(k)))


def tables(net, dt: float, K: int) -> dict:
    L = lib()
    h = _NetHolder(net)
    n, nnz = int(net.n), int(net.row_ptr[-1])
    out = {"q": np.zeros(max(nnz, 1), np.float32), "pdep": np.zeros(n, np.float32), "rate": np.zeros(n, np.float32),
           "mudt": np.zeros(n, np.float32), "kap": np.zeros(n, np.float32), "g": np.zeros(max(K, 1), np.float32)}
    L.orc_tables(C.byref(h.s), C.c_float(dt), int(K), _ptr(out["q"]), _ptr(out["pdep"]), _ptr(out["rate"]),
                 _ptr(out["mudt"]), _ptr(out["kap"]), _ptr(out["g"]))
    out["q"] = out["q"][:nnz]
    out["g"] = out["g"][:K]
    return out


def sampler_tables() -> tuple[np.ndarray, np.ndarray]:
    inv = np.zeros(256, np.float32)
    fc = np.zeros(10, np.float32)
    lib().orc_get_tables(_ptr(inv), _ptr(fc))
    return inv, fc


def sample(kind: int, count: int, seed: int = 0, rep0: int = 0, station: int = 0, step0: int = 0, sub: int = 1,
           i0: int = 0, i1: int = 0, f0: float = 0.0, f1: float = 0.0, f2: float = 0.0, f3: float = 0.0,
           return_flag: bool = False):
    """`count` draws of one sampler; with return_flag, also whether the overflow flag was raised
    (stream budget, retry cap, or a draw outside the samplers' exact fp32 range)."""
    out = np.zeros(count, np.float32)
    rc = lib().orc_sample(kind, count, C.c_uint64(seed), rep0, station, step0, sub, i0, i1, C.c_float(f0),
                          C.c_float(f1), C.c_float(f2), C.c_float(f3), _ptr(out))
    if rc not in (0, -5):
        raise ValueError(f"orc_sample failed with code {rc}")
    return (out, rc == -5) if return_flag else out


def sample_score(kind: int, count: int, seed: int = 0, rep0: int = 0, station: int = 0, step0: int = 0,
                 sub: int = 1, x: int = 0, m: int = 0, f0: float = 0.0, f1: float = 0.0) -> tuple[np.ndarray, np.ndarray]:
    """Draws with their likelihood-ratio scores: kind SMP_POISSON (f0 = lambda0, f1 = g;
    score in lambda0), SMP_GENDEP / SMP_GENDEP_NAIVE (x, m, f0 = mu, f1 = h; score in mu)."""
    val = np.zeros(count, np.float32)
    sc = np.zeros(count, np.float32)
    rc = lib().orc_sample_score(kind, count, C.c_uint64(seed), rep0, station, step0, sub, x, m, C.c_float(f0),
                                C.c_float(f1), _ptr(val), _ptr(sc))
    if rc not in (0, -5):
        raise ValueError(f"orc_sample_score failed with code {rc}")
    return val, sc


def cost_per_rep(sumQ: np.ndarray, hold: np.ndarray, K: int) -> np.ndarray:
    """Waiting cost of each replication, f_r = sum_i hold_i (1/K) sum_tau (N_{tau,i} - m_i)^+,
    in fp64 (the staffing term sum_i k_i m_i is a constant and is added by the caller)."""
    return (sumQ.astype(np.float64) @ np.asarray(hold, np.float64)) / K


def lr_gradient(f: np.ndarray, score: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Likelihood-ratio gradient estimate g_j = sum_r (f_r - mean f) S_{r,j} / (R - 1) in fp64,
    with its standard error (sample std of the per-replication products over sqrt(R))."""
    f = np.asarray(f, np.float64)
    S = np.asarray(score, np.float64)
    R = len(f)
    prod = (f - f.mean())[:, None] * S
    g = prod.sum(axis=0) / (R - 1)
    se = prod.std(axis=0, ddof=1) * R / (R - 1) / np.sqrt(R)
    return g, se


def reach_sets(net) -> np.ndarray:
    """reach[j, i] = True when the cost of station i can depend on parameter j: for j < n
    (mu_j) the stations reachable from station j along routing edges, station j itself
    included; for j = n + s (lambda0 of source s) those reachable from station src[s].  A
    station outside these sets evolves with draws whose laws do not involve the parameter, so
    its cost has zero covariance with the parameter's score in expectation."""
    n = int(net.n)
    adj = [net.col[net.row_ptr[i]:net.row_ptr[i + 1]] for i in range(n)]
    reach = np.zeros((n + len(net.src), n), bool)
    for j, start in enumerate(list(range(n)) + [int(s) for s in net.src]):
        seen = reach[j]
        stack = [start]
        seen[start] = True
        while stack:
            i = stack.pop()
            for t in adj[i]:
                if not seen[t]:
                    seen[t] = True
                    stack.append(int(t))
    return reach


def lr_gradient_reach(sumQ: np.ndarray, hold: np.ndarray, K: int, score: np.ndarray,
                      reach: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Likelihood-ratio gradient with each parameter's score correlated only with the cost of
    the stations it can reach: g_j = sum_r (f_{j,r} - mean f_j) S_{r,j} / (R - 1) with
    f_{j,r} = sum_{i in reach_j} hold_i Q_{r,i} / K, in fp64, and its standard error (sample
    std of the per-replication products over sqrt(R), times R / (R - 1))."""
    Q = np.asarray(sumQ, np.float64) * (np.asarray(hold, np.float64) / K)[None, :]    # [R, n]
    F = Q @ np.asarray(reach, np.float64).T                                          # [R, n_par]
    S = np.asarray(score, np.float64)
    R = len(F)
    prod = (F - F.mean(axis=0)) * S
    g = prod.sum(axis=0) / (R - 1)
    se = prod.std(axis=0, ddof=1) * R / (R - 1) / np.sqrt(R)
    return g, se


OP_EVENTS = ["station_step", "philox", "uniform", "pois_inv", "pois_inv_step", "ptrs", "ptrs_try", "ptrs_slow",
             "bin_inv", "bin_inv_step", "btrs", "btrs_try", "btrs_slow", "bin_prep", "gamma", "gamma_polar",
             "gamma_try", "gamma_slow", "expm1", "depart", "edge", "push"]


def op_counts(reset: bool = True) -> dict:
    """Event totals of the oracle's runs since the last reset (see the event list in
    euler_oracle.c): the algorithm's Philox blocks, sampler setups, search steps, rejection
    attempts, routed edges and station-steps."""
    L = lib()
    out = np.zeros(64, np.int64)
    k = L.orc_op_counts(_ptr(out), int(bool(reset)))
    assert k == len(OP_EVENTS)
    return {name: int(v) for name, v in zip(OP_EVENTS, out[:k])}


def math_fn(kind: int, x: np.ndarray) -> np.ndarray:
    """kind 0 log, 1 log1p, 2 exp, 3 expm1 (the oracle's own fp32 functions); 4 the uniform
    orc_u01 of the 32-bit word with each element's bits."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.zeros_like(x)
    lib().orc_math(kind, x.size, _ptr(x), _ptr(y))
    return y


def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros_like(ctr)
    lib().orc_philox_batch(len(ctr), _ptr(ctr), _ptr(key), _ptr(out))
    return out


def u01(x: np.ndarray) -> np.ndarray:
    """Same mapping as the oracle's orc_u01, vectorised (exact in fp32)."""
    x = np.asarray(x, dtype=np.uint32)
    j = ((x >> np.uint32(9)) << np.uint32(1)) | np.uint32(1)
    return j.astype(np.float32) * np.float32(2.0 ** -24)


def des(net, dt: float, K: int, seed: int, rep_ids: Sequence[int], snap_steps: Optional[Sequence[int]] = None,
        threads: Optional[int] = None) -> dict:
    """Exact Gillespie simulation; grid states at tau*dt, tau=1..K."""
    L = lib()
    h = _NetHolder(net)
    rep_ids = np.ascontiguousarray(rep_ids, dtype=np.int32)
    R, n = len(rep_ids), int(net.n)
    snaps_steps = None if snap_steps is None else np.ascontiguousarray(sorted(snap_steps), dtype=np.int32)
    ns = 0 if snaps_steps is None else len(snaps_steps)
    final = np.zeros((R, n), np.int32)
    sN = np.zeros((R, n), np.int64)
    sQ = np.zeros((R, n), np.int64)
    snaps = np.zeros((R, ns, n), np.int32) if ns else None
    events = np.zeros(R, np.int64)
    rc = L.des_run(C.byref(h.s), C.c_double(dt), int(K), C.c_uint64(seed), R, _ptr(rep_ids), ns, _ptr(snaps_steps),
                   _ptr(final), _ptr(sN), _ptr(sQ), _ptr(snaps), _ptr(events), threads or default_threads())
    if rc != 0:
        raise ValueError(f"des_run failed with code {rc}")
    return {"final": final, "sumN": sN, "sumQ": sQ, "snaps": snaps, "events": events}

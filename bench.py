"""Benchmark: Euler station-steps per second on one MI355X.

One benchmark step = one full simulation of the 1000-station sparse DAG (50 sinusoidal
sources, servers 1000..10000, h = 0.005, horizon 100 = 20000 steps, 4096 replications):
the backward scheme and the forward scheme, each followed by the per-station statistics
reduction, inputs resident on the GPU.  station-steps = n * K * reps per scheme.

Prints one JSON line with the throughput, the roofline of the dominant kernel (the
per-step sweep kernel, timed with HIP events on its own stream) and the CPU oracle timed
on the host's cores over a bounded sample of the same workload (all cores and one core, with
the exact discrete-event simulation of the 4-station tandem as context).  More measurements
ride along (--main-only leaves them out):
  average_scheme  the main workload as one pair run (both schemes per launch, pooled statistics);
  staffing        the main workload's backward scheme under 24 periodic staffing segments;
  host_buffers    the main workload's backward scheme through the host-buffer entry point
                  (allocation and PCIe copies included);
  sojourn         recording runs and sojourn-time sampling on a 100-station Jackson network;
  batching        512 feed-forward networks of 10..2000 stations (T ~ U(10, 100), h = 0.01, 256
                  replications each, backward scheme) in one autotuned, graph-captured batch,
                  against one autotuned run per network, every network one after another;
  gradient        the likelihood-ratio gradient of the expected waiting-plus-staffing cost of the
                  1000-station DAG (8192 replications, full horizon, backward scheme): score run
                  plus fp64 reductions (the reachability-pruned estimator the autograd function
                  uses), against the plain run of the same simulation; the full-cost estimator's
                  standard errors beside it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Counter-derived figures of the sweep kernel on this workload over the benchmark step's full
# horizon (rocprofv3 summaries in profiles/), valid for the kernel sources whose hash is recorded:
#   active = active VALU lane-operations per station-step
#          = SQ_INSTS_VALU * 64 * SQ_THREAD_CYCLES_VALU / (SQ_ACTIVE_INST_VALU * 64) / station-steps
#   slots  = issued VALU lane slots per station-step = SQ_INSTS_VALU * 64 / station-steps
#   bytes  = HBM bytes per station-step = (2.0 * FETCH_SIZE + 1.0 * WRITE_SIZE) / station-steps,
#            the factors from a plain 1 GiB device copy measured with the same counters.
KERNEL_COUNTERS = {"sources_sha256_16": "333cf0b41667b8b9", "active_lane_ops_per_station_step": 960.4,
                   "issued_lane_slots_per_station_step": 1680.2, "traffic_bytes_per_station_step": 33.08}
# The algorithm's own operations per station-step: the oracle's event counts on this workload
# (tests/golden/op_counts_dag1000.json) priced with the VALU instruction counts of each sampler
# building block in the gfx950 build (tests/isa/op_costs_gfx950.json).
OP_COUNTS_JSON = os.path.join(ROOT, "tests", "golden", "op_counts_dag1000.json")
OP_COSTS_JSON = os.path.join(ROOT, "tests", "isa", "op_costs_gfx950.json")
# The same events at the instruction costs of the first priced build, held fixed.
OP_COSTS_FIXED_JSON = os.path.join(ROOT, "tests", "isa", "op_costs_gfx950_first.json")
KERNEL_SOURCES = ["paper_2402_13259_amd/csrc/eq_device.h", "paper_2402_13259_amd/csrc/eq_internal.h",
                  "paper_2402_13259_amd/csrc/eq_sweep.h", "paper_2402_13259_amd/csrc/eq_kernels.hip"]
# VALU peak for the kernel's (non-packed) instructions: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# = 39.3e12 lane-operations per second.  The 157.3 TFLOP/s fp32 vector figure is this rate
# x 2 for packed fp32 x 2 for an FMA; the kernels are built without packed fp32.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def algorithmic_ops(costs_json: str = OP_COSTS_JSON) -> float:
    """Operations per station-step of the benchmark step (the mean of its two schemes)."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "isa"))
    import op_costs
    costs = json.load(open(costs_json))["events"]
    counts = json.load(open(OP_COUNTS_JSON))
    return 0.5 * sum(op_costs.algorithmic_ops(counts[s], costs) for s in ("backward", "forward"))


def summarize_counters(path: str, regex: str) -> None:
    """Sum every counter of rocprofv3's counter_collection CSV files under `path` over the
    dispatches of kernels matching `regex`; print the sums and the dispatch count as JSON."""
    import csv
    import glob
    import re
    sums, dispatches, per_kernel = {}, set(), {}
    pat = re.compile(regex)
    for f in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if not pat.search(row["Kernel_Name"]):
                    continue
                dispatches.add(row["Dispatch_Id"])
                name, v = row["Counter_Name"], float(row["Counter_Value"])
                sums[name] = sums.get(name, 0.0) + v
                k = per_kernel.setdefault(row["Kernel_Name"][:80], {"dispatches": set(), "sums": {}})
                k["dispatches"].add(row["Dispatch_Id"])
                k["sums"][name] = k["sums"].get(name, 0.0) + v
    per_kernel = {k: {"dispatches": len(v["dispatches"]), "sums": v["sums"]} for k, v in per_kernel.items()}
    print(json.dumps({"path": path, "kernels": regex, "dispatches": len(dispatches), "sums": sums,
                      "per_kernel": per_kernel}), flush=True)


def sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--horizon-steps", type=int, default=0, help="override K (profiling only; result is invalid)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="run only a plain device copy of MB megabytes 10 times (HBM counter calibration)")
    ap.add_argument("--skip-batch", action="store_true", help="leave out the batching measurement")
    ap.add_argument("--skip-grad", action="store_true", help="leave out the gradient measurement")
    ap.add_argument("--main-only", action="store_true",
                    help="only the main step and its roofline (no average-scheme, staffing, sojourn, batching "
                         "or gradient legs): the form the kernel profiles are taken with")
    ap.add_argument("--per-net-stride", type=int, default=1,
                    help="per-network baseline: every k-th network (1: all of them)")
    ap.add_argument("--error-order", action="store_true",
                    help="run only the error-order study of the backward, forward and average schemes")
    ap.add_argument("--fd-check", action="store_true",
                    help="run only the finite-difference check of the gradient at full size (several minutes)")
    ap.add_argument("--fd-seed", type=int, default=0,
                    help="Philox seed of the finite-difference check's runs (independent draws per seed)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("DIR", "KERNEL_REGEX"),
                    help="sum rocprofv3 counter CSVs under DIR over the kernels matching KERNEL_REGEX (no GPU)")
    return ap.parse_args()


def log(msg: str) -> None:
    """Progress on stderr (stdout carries only the result line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def copy_calibration(mb: int) -> None:
    """A plain copy kernel of known size, to scale rocprofv3 FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "copies": 10}), flush=True)


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: replications shard across GPUs by design (every draw is keyed "
              "by the global replication id), but this benchmark runs and reports a single MI355X only",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.fd_check:
        fd_check(seed=args.fd_seed)
        return
    if args.error_order:
        error_order()
        return
    import numpy as np
    import torch
    import netgen
    from paper_2402_13259_amd import binding as eb

    torch.cuda.set_device(0)
    w = netgen.config3()
    K = args.horizon_steps or w.K
    net = eb.Net(w.net)
    reps, n = w.reps, w.net.n
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    state = {s: torch.empty((n, reps), dtype=torch.int32, device=dev) for s in (0, 1)}
    sums = {s: torch.empty((3, n, eb.n_tiles(reps)), dtype=torch.int64, device=dev) for s in (0, 1)}
    stats = {s: torch.empty((6, n), dtype=torch.float64, device=dev) for s in (0, 1)}
    levels = int(net.levels().max()) + 1
    launches = {0: K, 1: K + levels - 1}

    def one_step(events=None):
        for s in (eb.EQ_BACKWARD, eb.EQ_FORWARD):
            if events is not None:
                events[s][0].record(stream)
            res = eb.simulate(net, s, w.dt, K, reps, 0, state=state[s], sums=sums[s], check=False,
                              kernel=eb.EQ_KERNEL_SWEEP)
            if events is not None:
                events[s][1].record(stream)
            eb.eq_stats_reduce(net.handle, eb.C.byref(res.desc), res.sums.data_ptr(), res.state.data_ptr(), None,
                               stats[s].data_ptr(), stream.cuda_stream)

    log(f"main workload: {args.warmup} warm-up and {args.steps} timed steps")
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    log("warm-up done")
    rc = eb.eq_sim_check(net.handle, stream.cuda_stream)
    if rc != 0:
        raise SystemExit(f"device flags after warmup: {eb.eq_last_error().decode()}")
    ev = [{s: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for s in (0, 1)}
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step(ev[k])
        log(f"timed step {k + 1} queued")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("timed steps done")
    if eb.eq_sim_check(net.handle, stream.cuda_stream) != 0:
        raise SystemExit(f"device flags: {eb.eq_last_error().decode()}")
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    station_steps = 2 * n * K * reps
    value = station_steps / ((t1 - t0) / args.steps)
    sweep_ms = {s: sum(e[s][0].elapsed_time(e[s][1]) for e in ev) / args.steps for s in (0, 1)}
    per_launch_ms = (sweep_ms[0] + sweep_ms[1]) / (launches[0] + launches[1])
    ss_per_launch = n * reps          # station-steps one sweep launch processes
    roof = {"bound": "alu", "unit": "TOP/s", "peak": round(VALU_PEAK_TOPS, 2),
            "kernel": "k_sweep (one launch per step)",
            "avg_launch_ms": round(per_launch_ms, 5),
            "station_steps_per_launch": ss_per_launch}
    roof["measured_fma_peak"] = round(eb.valu_peak() / 1e12, 2)   # non-packed fp32 FMA lanes, T/s
    launch_s = per_launch_ms * 1e-3
    alg = algorithmic_ops()
    achieved = alg * ss_per_launch / launch_s / 1e12
    roof.update(achieved=round(achieved, 3), frac=round(achieved / VALU_PEAK_TOPS, 4),
                ops_per_station_step=round(alg, 1),
                ops_basis="the algorithm's operations: oracle event counts on this workload (Philox blocks, "
                          "uniforms, sampler set-ups, search steps, rejection attempts, routed edges) x VALU "
                          "instructions of each building block in the gfx950 build")
    fixed = algorithmic_ops(OP_COSTS_FIXED_JSON)
    roof["fixed_prices"] = {"ops_per_station_step": round(fixed, 1),
                            "frac": round(fixed * ss_per_launch / launch_s / 1e12 / VALU_PEAK_TOPS, 4),
                            "basis": "the same event counts at the instruction costs of the first priced build "
                                     "(tests/isa/op_costs_gfx950_first.json), held fixed across builds"}
    if sources_hash() == KERNEL_COUNTERS["sources_sha256_16"]:
        act = KERNEL_COUNTERS["active_lane_ops_per_station_step"]
        slots = KERNEL_COUNTERS["issued_lane_slots_per_station_step"]
        traffic = KERNEL_COUNTERS["traffic_bytes_per_station_step"] * ss_per_launch
        roof["executed"] = {"active_lane_ops_per_station_step": act, "issued_lane_slots_per_station_step": slots,
                            "lane_utilisation": round(act / slots, 4),
                            "algorithmic_share_of_active": round(alg / act, 4),
                            "frac": round(act * ss_per_launch / launch_s / 1e12 / VALU_PEAK_TOPS, 4)}
        roof.update(traffic=round(traffic), hbm_gbs=round(traffic / launch_s / 1e9, 1),
                    hbm_frac=round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4))
    else:
        # counters were taken on other kernel sources: re-profile before quoting them
        roof.update(executed=None, traffic=None, note="kernel changed since the counters were taken")

    out = {
        "metric": "Euler station-steps/s at 1 GPU; batched vs per-net launch; grad/fwd time",
        "value": value, "unit": "station-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 samplers / i32 state", "data": "synthetic",
        "config": {"workload": "dag1000: 1000-station sparse DAG, 50 sinusoidal sources, c~U{1000..10000}, "
                               "load U(0.85,0.99), h=0.005, T=100 (20000 steps), 4096 replications, "
                               "backward + forward schemes + statistics per step",
                   "n": n, "K": K, "reps": reps, "schemes": ["backward", "forward"],
                   "kernel": "sweep", "network_sha256": w.net.fingerprint()},
        "per_scheme_station_steps_per_s": {"backward": n * K * reps / (sweep_ms[0] * 1e-3),
                                           "forward": n * K * reps / (sweep_ms[1] * 1e-3)},
        "roofline": roof,
    }
    if args.horizon_steps:
        out["note"] = "reduced horizon (testing only)"
    if not args.main_only:
        out["average_scheme"] = bench_pair(w, K, net, sweep_ms)
        log("average scheme done")
        out["staffing"] = bench_staffing(w, K, sweep_ms)
        out["host_buffers"] = bench_host_buffers(w, K, sweep_ms)
        log("staffing and host buffers done")
        out["sojourn"] = bench_sojourn()
        log("sojourn done")
    if not (args.skip_batch or args.main_only):
        out["batching"] = bench_batching(args.per_net_stride)
        log("batching done")
    if not (args.skip_grad or args.main_only):
        out["gradient"] = bench_gradient()
        log("gradient done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, K, args.cpu_seconds)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def bench_batching(stride: int) -> dict:
    """512 networks batched vs one run per network (sampled), both autotuned."""
    import numpy as np
    import torch
    import netgen
    from paper_2402_13259_amd import binding as eb
    stream = torch.cuda.current_stream()
    ws = netgen.config4()
    dt, reps = ws[0].dt, ws[0].reps
    nets = [eb.Net(w.net) for w in ws]
    ks = [w.K for w in ws]
    ids = [w.net_id for w in ws]
    batch = eb.Batch(nets)
    t = time.perf_counter()
    wpb = batch.tune(eb.EQ_BACKWARD, dt, ks, ids, reps, trial_fraction=0.02)
    tune_s = time.perf_counter() - t
    so, mo = batch.layout(reps)
    states = torch.empty(int(so[-1]), dtype=torch.int32, device="cuda")
    sums = torch.empty(int(mo[-1]), dtype=torch.int64, device="cuda")
    ss_all = sum(w.net.n * w.K for w in ws) * reps
    # timed: graph capture + instantiation + the whole horizon of every network
    e0, e1 = _events()
    torch.cuda.synchronize()
    t = time.perf_counter()
    e0.record(stream)
    batch.run(eb.EQ_BACKWARD, dt, ks, ids, reps, states=states, sums=sums, use_graph=True, check=False)
    e1.record(stream)
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t
    if eb.eq_batch_check(batch.handle, stream.cuda_stream) != 0:
        raise SystemExit(f"batch device flags: {eb.eq_last_error().decode()}")
    batched = ss_all / batch_s
    # per network: every `stride`-th network, its own autotuned launch shape, one after another
    sample = list(range(0, len(ws), stride))
    log(f"batch run done; tuning {len(sample)} networks for the per-network baseline")
    shapes = [eb.tune(nets[k], eb.EQ_BACKWARD, dt, ks[k], reps, 0, trial_steps=32) for k in sample]
    log("per-network tuning done")
    bufs = [(torch.empty((nets[k].n, reps), dtype=torch.int32, device="cuda"),
             torch.empty((3, nets[k].n, eb.n_tiles(reps)), dtype=torch.int64, device="cuda")) for k in sample]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i, ((st, sm), k, shape) in enumerate(zip(bufs, sample, shapes)):
        eb.simulate(nets[k], eb.EQ_BACKWARD, dt, ks[k], reps, 0, net_id=ids[k], state=st, sums=sm, check=False,
                    **shape)
        if i % 64 == 63:
            log(f"per-network runs queued: {i + 1} of {len(sample)}")
    torch.cuda.synchronize()
    per_s = time.perf_counter() - t
    ss_sample = sum(ws[k].net.n * ks[k] for k in sample) * reps
    per_net = ss_sample / per_s
    kinds = {"tile": sum(s["kernel"] == eb.EQ_KERNEL_TILE for s in shapes),
             "sweep": sum(s["kernel"] == eb.EQ_KERNEL_SWEEP for s in shapes)}
    return {"workload": "512 feed-forward networks, n log-uniform in [10, 2000], T ~ U(10, 100), h = 0.01, "
                        "256 replications each, backward scheme",
            "station_steps": ss_all, "batched_s": round(batch_s, 3), "batched_gpu_ms": round(e0.elapsed_time(e1), 1),
            "batched_station_steps_per_s": batched, "waves_per_block": wpb, "tune_s": round(tune_s, 2),
            "per_network_station_steps_per_s": per_net,
            "per_network_sample": f"networks {sample[0]}, {sample[0] + stride}, ..., {sample[-1]} ({len(sample)}), "
                                  f"full horizons, {ss_sample:.3g} station-steps, {per_s:.2f} s, each with its "
                                  f"autotuned shape ({kinds['tile']} tile, {kinds['sweep']} sweep)",
            "per_network_s": round(per_s, 3), "networks_sha256": batch_fingerprint(ws),
            "batched_over_per_network": batched / per_net}


def batch_fingerprint(ws) -> str:
    import hashlib
    h = hashlib.sha256()
    for w in ws:
        h.update(w.net.fingerprint().encode())
        h.update(repr((w.T, w.dt, w.reps, w.net_id)).encode())
    return h.hexdigest()


def bench_gradient() -> dict:
    """LR gradient of the expected cost: (score run + cost + gradient reductions) / plain run."""
    import numpy as np
    import torch
    import netgen
    from paper_2402_13259_amd import binding as eb
    stream = torch.cuda.current_stream()
    w = netgen.config5()
    hold, staff = netgen.config5_costs(w.net.n)
    net = eb.Net(w.net)
    n, R, K = w.net.n, w.reps, w.K
    state = torch.empty((n, R), dtype=torch.int32, device="cuda")
    sumq = torch.empty((n, R), dtype=torch.int64, device="cuda")
    score = torch.empty((n + net.n_src, R), dtype=torch.float32, device="cuda")
    hold_d = torch.as_tensor(hold, device="cuda")

    def plain():
        eb.simulate(net, eb.EQ_BACKWARD, w.dt, K, R, 0, state=state, with_sums=False, kernel=eb.EQ_KERNEL_SWEEP,
                    check=False)

    def scored():
        r = eb.simulate_scores(net, eb.EQ_BACKWARD, w.dt, K, R, 0, state=state, sumq=sumq, score=score, check=False)
        f, ms = eb.cost_reduce(hold_d, r.sumq, K)
        g, se = eb.grad_reduce_reach(net, hold_d, r.sumq, r.score, K)
        return ms, g, se, f

    # short warm-up of both paths (kernels loaded, tables for this horizon uploaded)
    eb.simulate(net, eb.EQ_BACKWARD, w.dt, K, R, 0, state=state, with_sums=False, kernel=eb.EQ_KERNEL_SWEEP)
    times = {}
    for name, fn in (("forward", plain), ("forward_score_reduce", scored)):
        e0, e1 = _events()
        torch.cuda.synchronize()
        e0.record(stream)
        out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1)
    if eb.eq_sim_check(net.handle, stream.cuda_stream) != 0:
        raise SystemExit(f"gradient run device flags: {eb.eq_last_error().decode()}")
    ms_d, g, se, f = out
    e0, e1 = _events()
    e0.record(stream)
    gf, sef = eb.grad_reduce(f, ms_d, score)
    e1.record(stream)
    gr0, gr1 = _events()
    gr0.record(stream)
    eb.grad_reduce_reach(net, hold_d, sumq, score, K)
    gr1.record(stream)
    torch.cuda.synchronize()
    full_ms, reach_ms = e0.elapsed_time(e1), gr0.elapsed_time(gr1)
    ms, g, se, gf, sef = (x.cpu().numpy() for x in (ms_d, g, se, gf, sef))
    staffing = float(np.dot(staff, w.net.servers))

    def med(se_, g_, sel=slice(None)):
        return float(np.median(se_[sel] / np.maximum(np.abs(g_[sel]), 1e-300)))

    def powered(se_, g_, sel=slice(None)):
        """share of the parameters whose estimate is at least 3.33 standard errors from zero"""
        return float(np.mean(se_[sel] < 0.3 * np.abs(g_[sel])))

    live = sef[:n] > 0           # parameters with a nonzero score somewhere (a station that served someone)
    return {"workload": "1000-station DAG, 8192 replications, 20000 steps, backward scheme; cost = sum_i hold_i "
                        "mean (N_i - m_i)^+ + sum_i k_i m_i, hold ~ U(1, 5), k ~ U(0.1, 1); 1000 mu + 50 lambda0",
            "forward_ms": round(times["forward"], 1), "grad_ms": round(times["forward_score_reduce"], 1),
            "grad_over_forward": times["forward_score_reduce"] / times["forward"],
            "J": float(ms[0] + staffing), "J_se": float(ms[1]),
            "estimator": "each score against the cost of the stations its parameter can reach",
            "grad_norm": float(np.linalg.norm(g)), "median_grad_se_over_abs": med(se, g),
            "median_grad_se_over_abs_mu": med(se, g, slice(0, n)),
            "median_grad_se_over_abs_lambda0": med(se, g, slice(n, None)),
            "reach_reduce_ms": round(reach_ms, 3), "full_reduce_ms": round(full_ms, 3),
            "share_powered_mu": powered(se, g, slice(0, n)), "share_powered_lambda0": powered(se, g, slice(n, None)),
            "full_cost_estimator": {"median_grad_se_over_abs": med(sef, gf),
                                    "median_grad_se_over_abs_mu": med(sef, gf, slice(0, n)),
                                    "share_powered_mu": powered(sef, gf, slice(0, n)),
                                    "share_powered_lambda0": powered(sef, gf, slice(n, None))},
            "se_ratio_reach_over_full_mu_quantiles": [float(q) for q in np.quantile(se[:n][live] / sef[:n][live],
                                                                                    [0.1, 0.5, 0.9])]}


def bench_pair(w, K, net, sweep_ms) -> dict:
    """The average scheme's pair run (both schemes in one launch per step) on the same workload,
    against the two schemes run one after the other (the sweep times of the main step)."""
    import torch
    from paper_2402_13259_amd import binding as eb
    stream = torch.cuda.current_stream()
    n, reps = w.net.n, w.reps
    states = [torch.empty((n, reps), dtype=torch.int32, device="cuda") for _ in range(2)]
    sums = [torch.empty((3, n, eb.n_tiles(reps)), dtype=torch.int64, device="cuda") for _ in range(2)]
    stats = torch.empty((6, n), dtype=torch.float64, device="cuda")
    e0, e1 = _events()
    torch.cuda.synchronize()
    e0.record(stream)
    res = eb.simulate_pair(net, w.dt, K, reps, 0, states=states, sums=sums, check=False)
    eb.eq_stats_reduce_pair(net.handle, eb.C.byref(res.backward.desc), sums[0].data_ptr(), sums[1].data_ptr(),
                            states[0].data_ptr(), states[1].data_ptr(), None, stats.data_ptr(), stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    if eb.eq_sim_check(net.handle, stream.cuda_stream) != 0:
        raise SystemExit(f"pair run device flags: {eb.eq_last_error().decode()}")
    ms = e0.elapsed_time(e1)
    seq = sweep_ms[0] + sweep_ms[1]
    return {"workload": "the main step's network and horizon, both schemes in one launch per step, pooled statistics",
            "pair_ms": round(ms, 1), "separate_ms": round(seq, 1),
            "station_steps_per_s": 2 * n * K * reps / (ms * 1e-3), "speedup_over_separate": seq / ms}


def bench_staffing(w, K, sweep_ms) -> dict:
    """The main workload's backward scheme under a 24-segment periodic staffing schedule (one
    segment per time unit, servers scaled by 1 + 0.2 sin over the 24-unit period of the
    arrivals), against the constant-servers backward sweep of the main step."""
    import numpy as np
    import torch
    from paper_2402_13259_amd import binding as eb, steprule
    n, reps = w.net.n, w.reps
    h, _ = steprule.fit_step(w.dt, w.T, [float(k) for k in range(1, 24)])
    starts = steprule.schedule_from_times([float(k) for k in range(1, 24)], h)
    factors = 1.0 + 0.2 * np.sin(2 * np.pi * (np.arange(24) + 0.5) / 24)
    servers = np.maximum(1, np.rint(factors[:, None] * w.net.servers[None, :])).astype(np.int32)
    net = eb.Net(w.net.replace(staff_start=starts, staff_servers=servers, staff_period=int(round(24 / h))))
    state = torch.empty((n, reps), dtype=torch.int32, device="cuda")
    sums = torch.empty((3, n, eb.n_tiles(reps)), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    e0, e1 = _events()
    torch.cuda.synchronize()
    e0.record(stream)
    eb.simulate(net, eb.EQ_BACKWARD, h, K, reps, 0, state=state, sums=sums, check=False, kernel=eb.EQ_KERNEL_SWEEP)
    e1.record(stream)
    torch.cuda.synchronize()
    if eb.eq_sim_check(net.handle, stream.cuda_stream) != 0:
        raise SystemExit(f"staffing run device flags: {eb.eq_last_error().decode()}")
    ms = e0.elapsed_time(e1)
    return {"workload": "main network, backward scheme, 24 hourly staffing segments repeating every 24 time units",
            "ms": round(ms, 1), "constant_servers_ms": round(sweep_ms[0], 1),
            "station_steps_per_s": n * K * reps / (ms * 1e-3)}


def bench_host_buffers(w, K, sweep_ms) -> dict:
    """eq_sim_run_host on the main workload's backward scheme: host initial state in, host
    final state and statistics out, timed on the wall clock around the call (device buffer
    allocation, both PCIe copies, the run, the statistics reduction and the flag check)."""
    import numpy as np
    from paper_2402_13259_amd import binding as eb
    n, reps = w.net.n, w.reps
    net = eb.Net(w.net)
    init = np.zeros((n, reps), np.int32)
    eb.simulate_host(net, eb.EQ_BACKWARD, w.dt, K, 64, 0, kernel=eb.EQ_KERNEL_SWEEP)   # tables for (h, K)
    t = time.perf_counter()
    eb.simulate_host(net, eb.EQ_BACKWARD, w.dt, K, reps, 0, init=init, kernel=eb.EQ_KERNEL_SWEEP)
    sec = time.perf_counter() - t
    return {"workload": "main network, backward scheme, through eq_sim_run_host (host buffers: initial "
                        "state in, final state and statistics out)",
            "ms": round(sec * 1e3, 1), "device_buffers_ms": round(sweep_ms[0], 1),
            "station_steps_per_s": n * K * reps / sec, "pcie_bytes": 2 * 4 * n * reps + 8 * 6 * n}


def bench_sojourn(samples: int = 64) -> dict:
    """Sojourn-time sampling (Algorithm 4): the Jackson network of the error-order study (100
    stations, 200 servers each), h = 0.01, T = 200, 1000 replications from empty; each scheme's
    run records N, D and the routed counts for t in [150, 200], and `samples` tagged customers
    per replication enter station 0 in the interval ending at t = 150.  Against the plain run
    of the same length, and the exact steady-state mean sojourn of the network (visits times
    M/M/c sojourn per station)."""
    import numpy as np
    import torch
    import netgen
    from paper_2402_13259_amd import binding as eb
    netw = netgen.jackson()
    h, T, reps, t_tag = 0.01, 200.0, 1000, 150.0
    K, tau0 = int(round(T / h)), int(round(t_tag / h))
    n = netw.n
    P = np.zeros((n, n))
    for i in range(n):
        for e in range(netw.row_ptr[i], netw.row_ptr[i + 1]):
            P[i, netw.col[e]] += netw.prob[e]
    visits = np.linalg.solve((np.eye(n) - P).T, np.eye(n)[0])
    lt = netw.total_rates()
    mu = netw.mu.astype(np.float64)
    per_station = np.array([erlang_c_mean(lt[i], mu[i], int(netw.servers[i])) / lt[i] for i in range(n)])
    exact = float(visits @ per_station)          # Little's law per station
    net = eb.Net(netw)
    stream = torch.cuda.current_stream()
    out = {"workload": "jackson10x10 (100 stations, 200 servers), h=0.01, T=200, 1000 replications, "
                       f"record t in [150, 200], {samples} tagged customers per replication at station 0, t=150",
           "exact_mean_sojourn": round(exact, 4)}
    means = {}
    for scheme, name in ((eb.EQ_BACKWARD, "backward"), (eb.EQ_FORWARD, "forward")):
        e0, e1 = _events()
        torch.cuda.synchronize()
        e0.record(stream)
        eb.simulate(net, scheme, h, K, reps, 3, check=False, kernel=eb.EQ_KERNEL_SWEEP)
        e1.record(stream)
        torch.cuda.synchronize()
        plain_ms = e0.elapsed_time(e1)
        e0.record(stream)
        rec = eb.simulate_record(net, scheme, h, K, reps, 3, rec_t0=tau0, rec_len=K - tau0 + 1, check=False)
        e1.record(stream)
        torch.cuda.synchronize()
        rec_ms = e0.elapsed_time(e1)
        if eb.eq_sim_check(net.handle, stream.cuda_stream) != 0:
            raise SystemExit(f"sojourn recording device flags: {eb.eq_last_error().decode()}")
        e0.record(stream)
        Ts = eb.sojourn(net, rec, [0] * samples, [tau0] * samples)
        e1.record(stream)
        torch.cuda.synchronize()
        soj_ms = e0.elapsed_time(e1)
        Tn = Ts.cpu().numpy()
        done = Tn >= 0
        means[name] = float(Tn[done].mean() * h)
        rec_bytes = (rec.N.numel() + rec.D.numel() + rec.R.numel()) * 4
        out[name] = {"plain_run_ms": round(plain_ms, 1), "record_run_ms": round(rec_ms, 1),
                     "record_bytes": rec_bytes, "sojourn_ms": round(soj_ms, 2),
                     "walks_per_s": Tn.size / (soj_ms * 1e-3),
                     "mean_sojourn": round(means[name], 4), "censored_frac": round(float(1 - done.mean()), 5),
                     "first_replication_quantiles": [round(float(q) * h, 3) for q in
                                                     np.quantile(Tn[:, 0][done[:, 0]], [0.1, 0.5, 0.9])]}
        del rec, Ts
    out["average_mean_sojourn"] = round(0.5 * (means["backward"] + means["forward"]), 4)
    return out


def erlang_c_mean(lam: float, mu: float, c: int) -> float:
    """Steady-state mean number in an M/M/c queue (Erlang B recursion, then Erlang C)."""
    a = lam / mu
    b = 1.0
    for k in range(1, c + 1):
        b = a * b / (k + a * b)
    rho = a / c
    pw = b / (1.0 - rho * (1.0 - b))
    return a + pw * rho / (1.0 - rho)


def error_order(T: float = 1000.0, reps: int = 1024) -> None:
    """Relative error of the long-run mean number in system under the backward, forward and
    average schemes on a feed-forward Jackson network (100 stations, 200 servers each,
    constant rates; exact means from the M/M/c formula at each station), for several h,
    with log-log slopes.  Runs start at the rounded exact station means."""
    import numpy as np
    import torch
    import netgen
    from paper_2402_13259_amd import binding as eb
    netw = netgen.jackson()
    lt = netw.total_rates()
    mu = netw.mu.astype(np.float64)
    exact = np.array([erlang_c_mean(lt[i], mu[i], int(netw.servers[i])) for i in range(netw.n)])
    total = float(exact.sum())
    net = eb.Net(netw)
    init = torch.as_tensor(np.repeat(np.rint(exact).astype(np.int32)[:, None], reps, axis=1), device="cuda")
    hs = [0.2, 0.1, 0.05, 0.025]
    errs = {"backward": [], "forward": [], "average": []}
    for h in hs:
        K = int(round(T / h))
        res = eb.simulate_pair(net, h, K, reps, 17, init=init)
        sb = eb.station_stats(net, res.backward, init=init).cpu().numpy()
        sf = eb.station_stats(net, res.forward, init=init).cpu().numpy()
        sa = eb.pair_stats(net, res, init=init).cpu().numpy()
        row = {"h": h, "K": K}
        for name, st in (("backward", sb), ("forward", sf), ("average", sa)):
            rel = (st[0].sum() - total) / total
            errs[name].append(rel)
            row[name] = rel
            row[name + "_se"] = float(np.sqrt((st[1] ** 2).sum())) / total
        print(json.dumps(row), flush=True)
    slopes = {name: float(np.polyfit(np.log(hs), np.log(np.abs(v)), 1)[0]) for name, v in errs.items()}
    print(json.dumps({"error_order": netw.name, "exact_mean_in_system": total, "T": T, "reps": reps,
                      "slopes": slopes}), flush=True)
    relative_error_vs_servers(T, reps)


def relative_error_vs_servers(T: float = 1000.0, reps: int = 1024) -> None:
    """Relative error of the long-run mean number in system of one M/M/m station against the
    Erlang C value, for m = 4 .. 4096 under square-root staffing (mu = 1, rho = 1 - 1/sqrt(m)),
    with the step of the selection rule h = alpha_m / mu, alpha_m = 0.4 / sqrt(m); backward,
    forward and average schemes, with the bound lambda h / E[N] of the relative-error theorem.
    Runs start at the rounded exact mean."""
    import numpy as np
    import torch
    import netgen
    from paper_2402_13259_amd import binding as eb, steprule
    rows = []
    for m in (4, 16, 64, 256, 1024, 4096):
        rho = 1.0 - 1.0 / np.sqrt(m)
        lam = rho * m
        w = netgen.single_station(lam, 1.0, m)
        h = steprule.selection_rule(w.mu, servers=w.servers)
        K = int(round(T / h))
        lam32, mu32 = float(np.float32(lam)), float(np.float32(1.0))
        exact = erlang_c_mean(lam32, mu32, m)
        net = eb.Net(w)
        init = torch.full((1, reps), int(round(exact)), dtype=torch.int32, device="cuda")
        res = eb.simulate_pair(net, h, K, reps, 23, init=init)
        row = {"m": m, "rho": round(rho, 5), "h": h, "K": K, "exact_mean": exact,
               "bound": lam32 * float(np.float32(h)) / exact}
        for name, st in (("backward", eb.station_stats(net, res.backward, init=init)),
                         ("forward", eb.station_stats(net, res.forward, init=init)),
                         ("average", eb.pair_stats(net, res, init=init))):
            st = st.cpu().numpy()
            row[name] = float((st[0, 0] - exact) / exact)
            row[name + "_se"] = float(st[1, 0] / exact)
        rows.append(row)
        print(json.dumps(row), flush=True)
    print(json.dumps({"relative_error_vs_servers": "single M/M/m station, rho = 1 - 1/sqrt(m), h = 0.4 / sqrt(m)",
                      "T": T, "reps": reps,
                      "backward": [r["backward"] for r in rows], "forward": [r["forward"] for r in rows],
                      "average": [r["average"] for r in rows], "bound": [r["bound"] for r in rows]}), flush=True)


def fd_check(rel: float = 1e-3, seed: int = 0) -> None:
    """Likelihood-ratio gradient of the 1000-station cost (8192 replications, full horizon,
    backward scheme) against common-random-number central differences: 8 mu coordinates at
    spread DAG depths, 4 lambda0 coordinates and 4 random directions v, each the derivative of
    J along theta * v with the parameters perturbed by +-rel relative.  The estimate is the
    reachability-pruned one (each score against the cost of the stations its parameter can
    reach); the full-cost estimate is reported beside it.  `seed` keys every run (the score run
    and both difference runs), so two seeds give independent repetitions of every check.  One
    JSON line per check, then a summary line."""
    import math
    import numpy as np
    import torch
    import netgen
    from paper_2402_13259_amd import binding as eb, lr
    w = netgen.config5()
    hold, staff = netgen.config5_costs(w.net.n)
    prob = lr.CostProblem(w.net, hold, staff, w.dt, w.K, w.reps, seed=seed)
    n, R, K = w.net.n, w.reps, w.K
    net = eb.Net(w.net)
    res = eb.simulate_scores(net, eb.EQ_BACKWARD, w.dt, K, R, seed)
    hold_d = torch.as_tensor(hold, device="cuda")
    f, ms = eb.cost_reduce(hold_d, res.sumq, K)
    g_reach, _ = eb.grad_reduce_reach(net, hold_d, res.sumq, res.score, K)
    # per-replication products of both estimators, [R, n_par]
    S = res.score.double().T
    reach = torch.as_tensor(net.reach(), dtype=torch.float64, device="cuda")
    F = (res.sumq.double().T * (hold_d / K)[None, :]) @ reach.T
    P_reach = (F - F.mean(0)) * S * (R / (R - 1))
    P_full = (f - ms[0]).double()[:, None] * S * (R / (R - 1))
    assert torch.allclose(P_reach.mean(0), g_reach, rtol=1e-9, atol=1e-9 * g_reach.abs().max().item())
    theta = np.concatenate([w.net.mu, w.net.lambda0]).astype(np.float64)
    lev = net.levels()
    mus = [int(np.flatnonzero(lev == l)[0]) for l in np.linspace(1, lev.max(), 8).astype(int)]
    checks = [("mu", i, None) for i in mus] + [("lambda0", s, None) for s in (0, 16, 33, 49)]
    rng = np.random.default_rng(11)
    for d in range(4):
        checks.append(("direction", d, rng.standard_normal(len(theta)) / math.sqrt(len(theta))))
    rows = []
    for kind, idx, vec in checks:
        v = np.zeros(len(theta))
        if kind == "mu":
            v[idx] = 1.0
        elif kind == "lambda0":
            v[n + idx] = 1.0
        else:
            v = vec
        wv = torch.as_tensor(theta * v, device="cuda")
        est = {}
        for name, P in (("lr", P_reach), ("lr_full", P_full)):
            per = P @ wv
            est[name] = (per.mean().item(), (per.std() / math.sqrt(R)).item())
        fs = []
        for sign in (+1, -1):
            t = (theta * (1 + sign * rel * v)).astype(np.float32)
            fs.append(lr.cost_samples(prob, mu=t[:n], lambda0=t[n:]))
        diff = ((fs[0] - fs[1]) / (2 * rel)).cpu().numpy()
        fd, fd_se = float(diff.mean()), float(diff.std() / math.sqrt(R))
        comb = math.hypot(est["lr"][1], fd_se)
        row = {"check": kind, "index": idx, "lr": est["lr"][0], "lr_se": est["lr"][1], "lr_full": est["lr_full"][0],
               "lr_full_se": est["lr_full"][1], "fd": fd, "fd_se": fd_se, "z": (est["lr"][0] - fd) / comb,
               "combined_se_over_abs_fd": comb / abs(fd) if fd else None}
        rows.append(row)
        print(json.dumps(row), flush=True)
    zs = [r["z"] for r in rows]
    print(json.dumps({"fd_check": "grad1000", "seed": seed, "checks": len(zs), "max_abs_z": max(abs(z) for z in zs),
                      "within_3_se": sum(abs(z) < 3 for z in zs), "relative_step": rel,
                      "with_power": sum(r["combined_se_over_abs_fd"] is not None and r["combined_se_over_abs_fd"] < 0.3
                                        for r in rows),
                      "units": "derivative of J along theta * v (relative perturbation)"}), flush=True)


def cpu_baseline(w, K, seconds):
    """The oracle on this host's cores, on replications 0..R-1 of the same workload."""
    import numpy as np
    import oracle
    threads = oracle.default_threads()
    # calibrate on a short horizon, then size the sample to about `seconds`
    t = time.perf_counter()
    oracle.run(w.net, 0, w.dt, 200, 0, np.arange(threads), threads=threads)
    per_ss = (time.perf_counter() - t) / (w.net.n * 200 * threads)
    steps = max(200, min(K, int(seconds / 2 / (per_ss * w.net.n * threads))))
    total = 0.0
    for scheme in (0, 1):
        t = time.perf_counter()
        oracle.run(w.net, scheme, w.dt, steps, 0, np.arange(threads), threads=threads)
        total += time.perf_counter() - t
    ss = 2 * w.net.n * steps * threads
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    out = {"value": ss / total, "unit": "station-steps/s", "cores": threads, "kind": "oracle", "cpu_model": model,
           "host_cpus": os.cpu_count(),
           "sample": f"both schemes, replications 0..{threads - 1}, first {steps} of {K} steps, "
                     f"{w.net.n} stations ({ss:.3g} station-steps, {total:.1f} s)"}
    # one core: replication 0, backward scheme, about a tenth of the time above
    steps1 = max(200, min(K, int(seconds / 10 / (per_ss * threads * w.net.n))))
    t = time.perf_counter()
    oracle.run(w.net, 0, w.dt, steps1, 0, np.arange(1), threads=1)
    t1 = time.perf_counter() - t
    out["single_core"] = {"value": w.net.n * steps1 / t1, "sample": f"backward scheme, replication 0, first {steps1} steps"}
    # context: the exact discrete-event simulation on the 4-station tandem (lambda 20, c 25, T 10)
    import netgen
    c1 = netgen.config1()
    t = time.perf_counter()
    d = oracle.des(c1.net, c1.dt, c1.K, 0, np.arange(c1.reps), threads=threads)
    td = time.perf_counter() - t
    out["des_tandem4"] = {"events_per_s": float(d["events"].sum()) / td, "replications": c1.reps,
                          "seconds": round(td, 2), "cores": threads}
    return out


if __name__ == "__main__":
    main()

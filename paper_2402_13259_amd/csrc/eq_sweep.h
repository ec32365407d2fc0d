// eq_sweep.h -- station-coherent "sweep" kernels for large networks (compiled as part of eq_kernels.hip).
//
// One wavefront = one station x 64 consecutive replications (a "tile"): the station's
// parameters and its CSR routing row are wave-uniform and live in scalar registers, and
// every branch that depends on the station (the departure law, the binomial algorithm,
// the number of edges) is taken by all lanes together.  The state N[station][rep] and the
// inflow slots live in HBM (cache resident for the tile's XCD); one kernel launch covers
// one step (one level-lagged step for the forward scheme) for every (station, tile) task.
//
// Backward scheme (Algorithm 1): launch tau runs step tau.  A task reads
// x = N_base + in[(tau-1) & 1] (the previous step's pushes), clears that slot, draws
// D = GenerateDeparture(x) and A, stores N_base = x - D + A and pushes its routed
// departures into in[tau & 1] of the targets.  Pushes of step tau are therefore only read
// in step tau + 1: arrivals land at the end of the interval, for any topology.  A finish
// launch folds the last pushes into N_K.
//
// Forward scheme (node by node along the customer flow, Section 2.2): station j at
// longest-path level l_j runs step tau in launch tau + l_j (launches numbered from 1).
// Every predecessor i of j has l_i < l_j, so its step-tau pushes were made in an earlier
// launch; j's own pushes for step tau are consumed by later launches.  Each station has a
// ring of D_j inflow slots (D_j = 1 + the largest level gap of an edge into j) indexed by
// step, so all stations advance in every launch and the DAG depth costs L - 1 extra
// launches instead of a barrier per level and step.
//
// Statistics: each task reduces N, (N - m)^+ and D over each half of its 64 lanes (64-bit
// shuffles) and lanes 0 and 32 add them to the int64 sums [3][n][stiles] of their 32-replication
// statistics tiles.
#pragma once
#include "eq_device.h"
#include "eq_internal.h"

namespace eq {

// Sum over each half (lanes 0..31, 32..63) of the wavefront.  Values are below 2^27, so
// groups of 16 lanes sum exactly in int32; the last level runs in int64.
__device__ __forceinline__ long long half_sum(int v) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
  long long w = v;
  w += __shfl_xor(w, 16, 64);
  return w;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ long long uniform_ll(long long v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

struct TaskPos {
  int s, t;
};

// XCD-aware task order: workgroup b runs on XCD b % 8; all tasks of tile t are given to
// XCD t % 8 so the tile's state and inflow slots stay in that XCD's L2.  Within an XCD,
// consecutive waves take the stations of one tile, heaviest (largest m mu) first, so that
// the short tasks fill the end of the launch.  Results do not depend on this order.
__device__ __forceinline__ bool task_of(const NetView &v, TaskPos &tp) {
  const int b = blockIdx.x, wave = threadIdx.x >> 6;
  const int xcd = b & 7, local = b >> 3;
  const int tl = uniform(local * (int)(blockDim.x >> 6) + wave);
  const int k = tl / v.n;
  tp.t = xcd + 8 * k;
  if (tp.t >= v.tiles) return false;
  tp.s = uniform(v.heavy[tl - k * v.n]);
  return true;
}

// Task (s, t) covers statistics tiles 2t and 2t + 1 (the second is absent when the last task
// holds 32 replications or fewer); each belongs to this task alone within a launch.  The sums
// are added with atomics whose result is not read: integer adds in any order give the same
// sums, and the task does not wait for a load of the old value (1.4 % on the 1000-station step).
__device__ __forceinline__ void add_tile_stats(const NetView &v, int s, int t, int xn, int xq, int xd,
                                               int lane) {
  const long long vn = half_sum(xn), vq = half_sum(xq), vd = half_sum(xd);
  const int st = 2 * t + (lane >> 5);
  if ((lane & 31) == 0 && st < v.stiles) {
    const long long plane = (long long)v.n * v.stiles;
    unsigned long long *p = reinterpret_cast<unsigned long long *>(v.tsums + (long long)s * v.stiles + st);
    atomicAdd(p, (unsigned long long)vn);
    atomicAdd(p + plane, (unsigned long long)vq);
    atomicAdd(p + 2 * plane, (unsigned long long)vd);
  }
}

// Score runs: adds (N - m)^+ to the replication's int64 sum (an atomic whose result is not read,
// like the statistics sums: the same sum, no wait for the old value).
__device__ __forceinline__ void add_sumq(long long *sq, int q) {
  if (q) atomicAdd(reinterpret_cast<unsigned long long *>(sq), (unsigned long long)q);
}

// One (station s, tile t) task of step tau.  SCORE runs also add each lane's draw scores
// and (N - m)^+ to its per-replication sums; REC runs store N_tau, D_tau and the routed
// counts of the recorded steps (backward: N_{tau-1} is complete only now, pushes included).
template <int SCHEME, bool SCORE, bool REC = false>
__device__ __forceinline__ void sweep_task(const NetView &v, int s, int t, int tau, int dep_mode, float dt,
                                           unsigned *dflags) {
  const int lane = threadIdx.x & 63;
  const int rep = t * 64 + lane;
  const bool valid = rep < v.reps;
  const StationParam p = v.sp[s];
  const StationRing ring = v.sp2[s];
  const long long reps = v.reps;
  // servers and m mu of this interval (staffing), and of the previous one for the backward
  // scheme's statistics of N_{tau-1}
  const int m = uniform(servers_in(v.segidx, v.seg_m, v.n, s, tau - 1, p.c));
  const float rate = rate_in(v.segidx, v.seg_rate, v.n, s, tau - 1, p.rate);
  const int m_prev = SCHEME == 0 && tau >= 2 ? uniform(servers_in(v.segidx, v.seg_m, v.n, s, tau - 2, p.c)) : m;
  uint32_t flags = 0;
  int x = 0, D = 0, q = 0, xn = 0;
  if (valid) {
    const uint32_t grep = (uint32_t)(v.rep0 + rep);
    int *Nrow = v.N + (long long)s * reps + rep;
    // Score runs: this lane owns its replication's score sums for the launch, so their old
    // values are read here, before the task stores anything, and the loads overlap the draws.
    float *sm = nullptr, *sl = nullptr;
    float sm0 = 0.0f, sl0 = 0.0f;
    if (SCORE) {
      sm = v.smu + (long long)s * reps + rep;
      sm0 = *sm;
      if (p.lam0 > 0.0f) {
        sl = v.slam + (long long)v.scp[s].src * reps + rep;
        sl0 = *sl;
      }
    }
    int A = 0;
    if (p.lam0 > 0.0f) {
      Stream S = make_stream(v.k0, v.k1, grep, (uint32_t)s, (uint32_t)(tau - 1), SUB_ARR);
      const float gt = v.g[tau - 1];
      A = poisson(p.lam0 * gt, S, flags);
      if (SCORE) *sl = sl0 + ((float)A / p.lam0 - gt);
    }
    const int slot = SCHEME == 0 ? ((tau - 1) & 1) : (tau % ring.depth);
    int *in = v.ring + ((long long)ring.off + slot) * reps + rep;
    const int inflow = *in;
    *in = 0;
    if (SCHEME == 0) {
      x = *Nrow + inflow;                        // N_{tau-1}
      xn = x;
      q = max(x - m_prev, 0);
    } else {
      x = *Nrow + A + inflow;                    // N_{tau-1} + A^ex + A^in
    }
    if (x >= kStateLimit) flags |= 1u;
    {
      Stream S = make_stream(v.k0, v.k1, grep, (uint32_t)s, (uint32_t)(tau - 1), SUB_DEP);
      if (SCORE) {
        float sc;
        D = dep_mode == 1 ? gendep_naive_score(x, m, p.mudt, p.mu, dt, S, flags, sc)
                          : gendep_score(x, m, p.mu, dt, v.dep[s], rate, v.scp[s].kap, S, flags, sc);
        if (x > 0) *sm = sm0 + sc;
      } else {
        D = dep_mode == 1 ? gendep_naive(x, m, p.mudt, S, flags)
                          : gendep(x, m, p.mu, dt, v.dep[s], rate, S, flags);
      }
    }
    if (SCHEME == 0) {
      *Nrow = x - D + A;
    } else {
      xn = x - D;
      *Nrow = xn;
      q = max(xn - m, 0);
    }
    if (SCORE && (SCHEME == 1 || tau >= 2)) add_sumq(v.sq + (long long)s * reps + rep, q);
    if (REC) {
      const int rt = tau - v.rec_t0;
      const int rn = SCHEME == 0 ? rt - 1 : rt;     // the step whose end state xn is
      if (rn >= 0 && rn < v.rec_len) v.rec_N[((long long)rn * v.n + s) * reps + rep] = xn;
      if (rt >= 0 && rt < v.rec_len) v.rec_D[((long long)rt * v.n + s) * reps + rep] = D;
    }
    if (D > 0) {
      Stream S = make_stream(v.k0, v.k1, grep, (uint32_t)s, (uint32_t)(tau - 1), SUB_ROUTE);
      int rem = D;
      for (int e = p.e0; e < p.e1 && rem > 0; ++e) {
        const Edge ed = v.edges[e];
        const int Rj = binomial_c(rem, BinomP{ed.ph, ed.r, ed.lq, ed.col2 & 1}, S, flags);
        if (REC) {
          const int rt = tau - v.rec_t0;
          if (rt >= 0 && rt < v.rec_len) v.rec_R[((long long)rt * v.nnz + e) * reps + rep] = Rj;
        }
        if (Rj) {
          const StationRing tr = v.sp2[ed.col2 >> 1];
          const int ts = SCHEME == 0 ? (tau & 1) : (tau % tr.depth);
          atomicAdd(v.ring + ((long long)tr.off + ts) * reps + rep, Rj);
        }
        rem -= Rj;
      }
    }
  }
  if (v.tsums) {
    // backward: statistics of N_{tau-1} (tau >= 2); forward: of N_tau
    const bool count_state = SCHEME == 1 || tau >= 2;
    add_tile_stats(v, s, t, count_state ? xn : 0, count_state ? q : 0, D, lane);
  }
  if (flags) atomicOr(dflags, flags);
}

// Backward only: N_K = N_base + in[K & 1]; statistics of N_K.
template <bool SCORE, bool REC = false>
__device__ __forceinline__ void finish_task(const NetView &v, int s, int t, unsigned *dflags) {
  const int lane = threadIdx.x & 63;
  const int rep = t * 64 + lane;
  int x = 0, q = 0;
  if (rep < v.reps) {
    int *Nrow = v.N + (long long)s * v.reps + rep;
    int *in = v.ring + ((long long)v.sp2[s].off + (v.K & 1)) * v.reps + rep;
    x = *Nrow + *in;
    *in = 0;
    *Nrow = x;
    q = v.K > 0 ? max(x - servers_in(v.segidx, v.seg_m, v.n, s, v.K - 1, v.sp[s].c), 0) : 0;
    if (x >= kStateLimit) atomicOr(dflags, 1u);
    if (SCORE && v.K > 0) add_sumq(v.sq + (long long)s * v.reps + rep, q);
    if (REC) {
      const int rn = v.K - v.rec_t0;
      if (v.K > 0 && rn >= 0 && rn < v.rec_len) v.rec_N[((long long)rn * v.n + s) * v.reps + rep] = x;
    }
  }
  if (v.tsums && v.K > 0) add_tile_stats(v, s, t, x, q, 0, lane);
}

// The network's read-only tables, passed again as kernel parameters of their own: marked
// __restrict__ (nothing writes them during a launch), their loads at wavefront-uniform
// addresses -- a station's records, each routing edge, the target's inflow ring, the step's
// arrival integral -- become scalar loads instead of vector loads of one address (4 % on the
// 1000-station step).  A pointer read from the argument struct carries no such guarantee.
struct Tables {
  const StationParam *sp;
  const BinomP *dep;
  const int *heavy;
  const StationRing *sp2;
  const Edge *edges;
  const float *g;
  const int *segidx, *seg_m;
  const float *seg_rate;
  const ScoreParam *scp;
};
#define EQ_TABLE_PARAMS                                                                              \
  const StationParam *__restrict__ t_sp, const BinomP *__restrict__ t_dep, const int *__restrict__ t_heavy, \
      const StationRing *__restrict__ t_sp2, const Edge *__restrict__ t_edges, const float *__restrict__ t_g, \
      const int *__restrict__ t_segidx, const int *__restrict__ t_seg_m, const float *__restrict__ t_seg_rate, \
      const ScoreParam *__restrict__ t_scp

__device__ __forceinline__ NetView bind_tables(NetView v, const StationParam *sp, const BinomP *dep, const int *heavy,
                                               const StationRing *sp2, const Edge *edges, const float *g,
                                               const int *segidx, const int *seg_m, const float *seg_rate,
                                               const ScoreParam *scp) {
  v.sp = sp; v.dep = dep; v.heavy = heavy; v.sp2 = sp2; v.edges = edges; v.g = g;
  v.segidx = segidx; v.seg_m = seg_m; v.seg_rate = seg_rate; v.scp = scp;
  return v;
}
#define EQ_BIND_TABLES(view) \
  bind_tables(view, t_sp, t_dep, t_heavy, t_sp2, t_edges, t_g, t_segidx, t_seg_m, t_seg_rate, t_scp)

inline Tables tables_of(const NetView &v) {
  return Tables{v.sp, v.dep, v.heavy, v.sp2, v.edges, v.g, v.segidx, v.seg_m, v.seg_rate, v.scp};
}
#define EQ_TABLE_ARGS(t) t.sp, t.dep, t.heavy, t.sp2, t.edges, t.g, t.segidx, t.seg_m, t.seg_rate, t.scp

template <int SCHEME, bool SCORE, bool REC>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a, EQ_TABLE_PARAMS) {
  const NetView v = EQ_BIND_TABLES(a.v);
  TaskPos tp;
  if (!task_of(v, tp)) return;
  const int lag = SCHEME == 0 ? 0 : uniform(v.sp2[tp.s].lag);
  const int tau = a.iter - lag;          // launches are numbered from 1
  if (tau < 1 || tau > v.K) return;
  sweep_task<SCHEME, SCORE, REC>(v, tp.s, tp.t, tau, a.dep_mode, a.dt, a.flags);
}

template <bool SCORE, bool REC>
__global__ __launch_bounds__(256) void k_sweep_finish(SweepArgs a, EQ_TABLE_PARAMS) {
  const NetView v = EQ_BIND_TABLES(a.v);
  TaskPos tp;
  if (!task_of(v, tp)) return;
  finish_task<SCORE, REC>(v, tp.s, tp.t, a.flags);
}

// Average scheme: the backward and the forward scheme of one network advance in the same
// launch (common random numbers come from the shared counters).  Within a tile's group the
// tasks alternate backward / forward over the stations, heaviest first; backward tasks run
// step iter, forward tasks step iter - level.
__global__ __launch_bounds__(256) void k_sweep_pair(PairArgs a, EQ_TABLE_PARAMS,
                                                    const StationRing *__restrict__ t_sp2f) {
  // both views read the same network's tables but their own inflow rings (t_sp2: backward)
  a.vb = EQ_BIND_TABLES(a.vb);
  a.vf = EQ_BIND_TABLES(a.vf);
  a.vf.sp2 = t_sp2f;
  const int b = blockIdx.x, wave = threadIdx.x >> 6;
  const int xcd = b & 7, local = b >> 3;
  const int tl = uniform(local * (int)(blockDim.x >> 6) + wave);
  const int n = a.vb.n;
  const int k = tl / (2 * n);
  const int t = xcd + 8 * k;
  if (t >= a.vb.tiles) return;
  const int r = tl - k * 2 * n;
  if ((r & 1) == 0) {
    const int s = uniform(a.vb.heavy[r >> 1]);
    if (a.iter >= 1 && a.iter <= a.vb.K) sweep_task<0, false>(a.vb, s, t, a.iter, a.dep_mode, a.dt, a.flags);
  } else {
    const int s = uniform(a.vf.heavy[r >> 1]);
    const int tau = a.iter - uniform(a.vf.sp2[s].lag);
    if (tau >= 1 && tau <= a.vf.K) sweep_task<1, false>(a.vf, s, t, tau, a.dep_mode, a.dt, a.flags);
  }
}

// Batched: global task id -> network (binary search over the active prefix) -> (s, t).
__device__ __forceinline__ bool batch_task(const BatchArgs &a, int &k, int &s, int &t) {
  const long long task = uniform_ll((long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  int lo = 0, hi = a.count - 1;
  if (task >= a.nets[hi].task0 + (long long)a.nets[hi].v.n * a.nets[hi].v.tiles) return false;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.nets[mid].task0 <= task) lo = mid; else hi = mid - 1;
  }
  k = lo;
  const int local = (int)(task - a.nets[k].task0);
  t = local / a.nets[k].v.n;
  s = uniform(a.nets[k].v.heavy[local - t * a.nets[k].v.n]);
  return true;
}

// Batch kernels take 1..16 wavefronts per workgroup (chosen by the autotuner).
template <int SCHEME>
__global__ __launch_bounds__(1024) void k_batch_step(BatchArgs a) {
  int k, s, t;
  if (!batch_task(a, k, s, t)) return;
  // A copy, read once at the start (before the task stores anything): the fields and the
  // table records read through them at wavefront-uniform addresses become scalar loads; through
  // a reference the compiler reloads them after every store, with vector loads (8 % of the
  // batch step).
  const NetView v = a.nets[k].v;
  const int lag = SCHEME == 0 ? 0 : uniform(v.sp2[s].lag);
  const int tau = a.iter - lag;
  if (tau < 1 || tau > v.K) return;
  sweep_task<SCHEME, false>(v, s, t, tau, a.dep_mode, a.dt, a.flags);
}

__global__ __launch_bounds__(1024) void k_batch_finish(BatchArgs a) {
  int k, s, t;
  if (!batch_task(a, k, s, t)) return;
  const NetView v = a.nets[k].v;
  finish_task<false, false>(v, s, t, a.flags);
}

// N = init (or 0), inflow slots = 0, tile sums = 0.
__global__ void k_sweep_init(int *N, const int *init, long long nstate, int *ring, long long nring,
                             long long *tsums, long long nsums) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nstate; i += stride)
    N[i] = init ? init[i] : 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nring; i += stride) ring[i] = 0;
  if (tsums)
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nsums; i += stride) tsums[i] = 0;
}

// Workgroups of `wpb` wavefronts, a multiple of 8 of them so that every XCD gets the same
// number of tasks.
int sweep_grid(const NetView &v, int wpb) {
  const int per_xcd_tiles = (v.tiles + 7) / 8;
  const int tasks_per_xcd = per_xcd_tiles * v.n;
  return 8 * ((tasks_per_xcd + wpb - 1) / wpb);
}

hipError_t launch_sweep_init(int *N, const int *init, long long nstate, int *ring, long long nring,
                             long long *tsums, long long nsums, hipStream_t st) {
  hipLaunchKernelGGL(k_sweep_init, dim3(1024), dim3(256), 0, st, N, init, nstate, ring, nring, tsums, nsums);
  return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs &a, int scheme, int mode, int wpb, hipStream_t st) {
  const Tables t = tables_of(a.v);
  const int grid = sweep_grid(a.v, wpb);
  const dim3 blk(64 * wpb);
  if (scheme == 0) {
    if (mode == 1) hipLaunchKernelGGL((k_sweep<0, true, false>), dim3(grid), blk, 0, st, a, EQ_TABLE_ARGS(t));
    else if (mode == 2) hipLaunchKernelGGL((k_sweep<0, false, true>), dim3(grid), blk, 0, st, a, EQ_TABLE_ARGS(t));
    else hipLaunchKernelGGL((k_sweep<0, false, false>), dim3(grid), blk, 0, st, a, EQ_TABLE_ARGS(t));
  } else {
    if (mode == 1) hipLaunchKernelGGL((k_sweep<1, true, false>), dim3(grid), blk, 0, st, a, EQ_TABLE_ARGS(t));
    else if (mode == 2) hipLaunchKernelGGL((k_sweep<1, false, true>), dim3(grid), blk, 0, st, a, EQ_TABLE_ARGS(t));
    else hipLaunchKernelGGL((k_sweep<1, false, false>), dim3(grid), blk, 0, st, a, EQ_TABLE_ARGS(t));
  }
  return hipGetLastError();
}

hipError_t launch_sweep_finish(const SweepArgs &a, int mode, int wpb, hipStream_t st) {
  const Tables t = tables_of(a.v);
  const dim3 blk(64 * wpb), grid(sweep_grid(a.v, wpb));
  if (mode == 1) hipLaunchKernelGGL((k_sweep_finish<true, false>), grid, blk, 0, st, a, EQ_TABLE_ARGS(t));
  else if (mode == 2) hipLaunchKernelGGL((k_sweep_finish<false, true>), grid, blk, 0, st, a, EQ_TABLE_ARGS(t));
  else hipLaunchKernelGGL((k_sweep_finish<false, false>), grid, blk, 0, st, a, EQ_TABLE_ARGS(t));
  return hipGetLastError();
}

// Zero a buffer of 32-bit words (a kernel, so that it can sit inside a captured graph).
__global__ void k_zero32(uint32_t *p, long long count) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0u;
}

// Per-edge and per-station binomial constants (binom_prep on the device).
__global__ void k_prep_edges(const int *col, const float *q, Edge *edges, int nnz) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const BinomP b = binom_prep(q[e]);
  edges[e] = Edge{2 * col[e] + b.flip, b.ph, b.r, b.lq};
}

__global__ void k_prep_dep(const StationParam *sp, BinomP *dep, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dep[i] = binom_prep(sp[i].pdep);
}

hipError_t launch_prep_edges(const int *col, const float *q, Edge *edges, int nnz, hipStream_t st) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep_edges, dim3((nnz + 255) / 256), dim3(256), 0, st, col, q, edges, nnz);
  return hipGetLastError();
}

hipError_t launch_prep_dep(const StationParam *sp, BinomP *dep, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep_dep, dim3((n + 255) / 256), dim3(256), 0, st, sp, dep, n);
  return hipGetLastError();
}

hipError_t launch_zero(void *p, long long words32, hipStream_t st) {
  if (words32 <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero32, dim3(1024), dim3(256), 0, st, (uint32_t *)p, words32);
  return hipGetLastError();
}

hipError_t launch_sweep_pair(const PairArgs &a, int wpb, hipStream_t st) {
  const int per_xcd_tiles = (a.vb.tiles + 7) / 8;
  const int tasks_per_xcd = per_xcd_tiles * 2 * a.vb.n;
  const int grid = 8 * ((tasks_per_xcd + wpb - 1) / wpb);
  const Tables t = tables_of(a.vb);
  hipLaunchKernelGGL(k_sweep_pair, dim3(grid), dim3(64 * wpb), 0, st, a, EQ_TABLE_ARGS(t), a.vf.sp2);
  return hipGetLastError();
}

hipError_t launch_batch_step(const BatchArgs &a, long long tasks, int scheme, int waves_per_block, hipStream_t st) {
  const long long grid = (tasks + waves_per_block - 1) / waves_per_block;
  if (grid <= 0) return hipSuccess;
  const dim3 blk(64 * waves_per_block);
  if (scheme == 0) hipLaunchKernelGGL(k_batch_step<0>, dim3((unsigned)grid), blk, 0, st, a);
  else hipLaunchKernelGGL(k_batch_step<1>, dim3((unsigned)grid), blk, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_batch_finish(const BatchArgs &a, long long tasks, int waves_per_block, hipStream_t st) {
  const long long grid = (tasks + waves_per_block - 1) / waves_per_block;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)grid), dim3(64 * waves_per_block), 0, st, a);
  return hipGetLastError();
}

}  // namespace eq

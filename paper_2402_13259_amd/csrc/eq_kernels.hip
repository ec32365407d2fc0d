// eq_kernels.hip -- simulation kernels of the Euler-approximation schemes on gfx950.
//
// Layout.  A workgroup owns a tile of R replications (R a power of two) and the whole
// network for that tile.  Everything per (station, rep) item lives in LDS for the whole
// horizon -- the state N (int32, replication fastest), the step's departures, and int32
// partial sums of N, (N - m)^+ and D -- so the hot loop touches HBM only for the read-only
// network tables (cache resident) and for statistics flushes every 16 steps into the
// int64 per-(station, 32-replication statistics tile) sums [3][n][tiles] (atomic integer
// adds).  This path suits networks small enough for a tile of >= 16 replications to fit in
// LDS.  Items are (station, rep) pairs, consecutive lanes taking consecutive replications of
// one station; a thread walks items tid, tid + B, ...
//
// Backward scheme (Algorithm 1), two phases per step separated by barriers:
//   1. each item reads x = N_{tau-1} (its own entry only), draws D = GenerateDeparture(x)
//      and the external arrivals A, and writes N = x - D + A and D;
//   2. each item splits its D over the CSR row (conditional binomials) and pushes the
//      routed counts into the targets with LDS atomics.
// No entry is read in phase 1 by anyone but its owner and pushes only start after the
// barrier, so every departure is drawn from N_{tau-1} and every arrival lands at the end
// of the interval, for any topology (feedback included).
//
// Forward scheme (Section 2.2, node by node along the customer flow): stations are swept
// level by level (longest-path depth in the DAG), one barrier per level; a station adds
// its external arrivals, departs from N_{tau-1} + A^ex + A^in and pushes its routed
// customers into stations of later levels, which have not yet departed in this step.
#include "eq_device.h"
#include "eq_internal.h"

namespace eq {

__constant__ float4 c_rcp4[kRcpTab / 4];
__constant__ float c_fc[10];

// int32 statistics partials are flushed every kFlushEvery steps; a state at or above
// kStateLimit sets the sticky flag (it would overflow a partial).  States below 2^24 are exact
// in fp32; between 2^24 and the limit the samplers use fp32(x), rounded identically everywhere.
constexpr int kFlushEvery = 16;

__device__ __forceinline__ Stream stream_for(const SimArgs &a, uint32_t rep, uint32_t s,
                                             int tau, uint32_t sub) {
  return make_stream(a.k0, a.k1, rep, s, (uint32_t)(tau - 1), sub);
}

// Departures of interval tau with that interval's servers (staffing) and fp32(m mu).
__device__ __forceinline__ int draw_departures(const SimArgs &a, const StationParam &p, int x,
                                               uint32_t rep, uint32_t s, int tau, uint32_t &flags) {
  Stream S = stream_for(a, rep, s, tau, SUB_DEP);
  const int m = servers_in(a.segidx, a.seg_m, a.n, (int)s, tau - 1, p.c);
  if (a.dep_mode == 1) return gendep_naive(x, m, p.mudt, S, flags);
  return gendep(x, m, p.mu, a.dt, a.dep[s], rate_in(a.segidx, a.seg_rate, a.n, (int)s, tau - 1, p.rate), S, flags);
}

__device__ __forceinline__ int draw_arrivals(const SimArgs &a, const StationParam &p, float gt,
                                             uint32_t rep, uint32_t s, int tau, uint32_t &flags) {
  if (!(p.lam0 > 0.0f)) return 0;
  Stream S = stream_for(a, rep, s, tau, SUB_ARR);
  return poisson(p.lam0 * gt, S, flags);
}

// Multinomial split of D over the row: Binomial(rem, q_e) edge by edge, remainder exits.
__device__ __forceinline__ void route_push(const SimArgs &a, const StationParam &p, int D,
                                           uint32_t rep, uint32_t s, int tau, int r, int *N,
                                           uint32_t &flags) {
  if (D <= 0) return;
  Stream S = stream_for(a, rep, s, tau, SUB_ROUTE);
  int rem = D;
  for (int e = p.e0; e < p.e1 && rem > 0; ++e) {
    const Edge ed = a.edges[e];
    const int Rj = binomial_c(rem, BinomP{ed.ph, ed.r, ed.lq, ed.col2 & 1}, S, flags);
    if (Rj) atomicAdd(&N[((ed.col2 >> 1) << a.log2R) | r], Rj);
    rem -= Rj;
  }
}

__device__ __forceinline__ void flush_add(long long *dst, int v) {
  if (v) atomicAdd((unsigned long long *)dst, (unsigned long long)(long long)v);
}

// Statistics partials of one item: add this step's state; flush into HBM when due.
__device__ __forceinline__ void stats_step(const SimArgs &a, int *PN, int *PQ, int *PD, int item,
                                           int x, int c, bool flush, long long g, long long plane) {
  int vn = PN[item] + x, vq = PQ[item] + max(x - c, 0), vd = PD[item];
  if (flush) {
    flush_add(a.sums + g, vn);
    flush_add(a.sums + g + plane, vq);
    flush_add(a.sums + g + 2 * plane, vd);
    vn = vq = vd = 0;
  }
  PN[item] = vn; PQ[item] = vq; PD[item] = vd;
}

__device__ __forceinline__ void init_tile(const SimArgs &a, int *N, int *PN, int *PQ, int *PD,
                                          int rep_base) {
  for (int item = threadIdx.x; item < a.items; item += blockDim.x) {
    const int s = item >> a.log2R, r = item & (a.R - 1), rep = rep_base + r;
    const bool valid = rep < a.reps;
    N[item] = (valid && a.init) ? a.init[(long long)s * a.reps + rep] : 0;
    PN[item] = PQ[item] = PD[item] = 0;
  }
}

// index of the (station, tile) statistics sum of an item
__device__ __forceinline__ long long tile_index(const SimArgs &a, int s, int rep) {
  return (long long)s * a.tiles + rep / kStatReps;
}

__global__ __launch_bounds__(1024) void k_backward(SimArgs a) {
  extern __shared__ int lds[];
  int *N = lds, *Dd = lds + a.items, *PN = lds + 2 * a.items, *PQ = lds + 3 * a.items,
      *PD = lds + 4 * a.items;
  const int tid = threadIdx.x, B = blockDim.x;
  const int rep_base = blockIdx.x * a.R;
  const long long plane = (long long)a.n * a.tiles;
  uint32_t flags = 0;
  init_tile(a, N, PN, PQ, PD, rep_base);
  __syncthreads();

  for (int tau = 1; tau <= a.K; ++tau) {
    const float gt = a.g[tau - 1];
    const bool flush = a.sums && ((tau - 1) % kFlushEvery) == 0 && tau > 1;
    // phase 1: departures from N_{tau-1}, external arrivals; statistics of N_{tau-1}
    for (int item = tid; item < a.items; item += B) {
      const int s = item >> a.log2R, r = item & (a.R - 1), rep = rep_base + r;
      if (rep >= a.reps) continue;
      const StationParam p = a.sp[s];
      const int x = N[item];
      if (x >= kStateLimit) flags |= 1u;
      if (tau > 1)
        stats_step(a, PN, PQ, PD, item, x, servers_in(a.segidx, a.seg_m, a.n, s, tau - 2, p.c), flush,
                   tile_index(a, s, rep), plane);
      const uint32_t grep = (uint32_t)(a.rep0 + rep);
      const int D = draw_departures(a, p, x, grep, (uint32_t)s, tau, flags);
      const int A = draw_arrivals(a, p, gt, grep, (uint32_t)s, tau, flags);
      N[item] = x - D + A;
      Dd[item] = D;
      PD[item] += D;
    }
    __syncthreads();
    // phase 2: multinomial routing, pushes land at the end of the interval
    for (int item = tid; item < a.items; item += B) {
      const int s = item >> a.log2R, r = item & (a.R - 1), rep = rep_base + r;
      if (rep >= a.reps) continue;
      const int D = Dd[item];
      if (D > 0) {
        const StationParam p = a.sp[s];
        route_push(a, p, D, (uint32_t)(a.rep0 + rep), (uint32_t)s, tau, r, N, flags);
      }
    }
    __syncthreads();
  }

  for (int item = tid; item < a.items; item += B) {
    const int s = item >> a.log2R, r = item & (a.R - 1), rep = rep_base + r;
    if (rep >= a.reps) continue;
    const int x = N[item];
    if (x >= kStateLimit) flags |= 1u;
    a.state[(long long)s * a.reps + rep] = x;
    if (a.sums) {
      if (a.K > 0)
        stats_step(a, PN, PQ, PD, item, x, servers_in(a.segidx, a.seg_m, a.n, s, a.K - 1, a.sp[s].c), true,
                   tile_index(a, s, rep), plane);
      else stats_step(a, PN, PQ, PD, item, 0, 0, true, tile_index(a, s, rep), plane);
    }
  }
  if (flags) atomicOr(a.flags, flags);
}

__global__ __launch_bounds__(1024) void k_forward(SimArgs a) {
  extern __shared__ int lds[];
  int *N = lds, *PN = lds + a.items, *PQ = lds + 2 * a.items, *PD = lds + 3 * a.items;
  const int tid = threadIdx.x, B = blockDim.x;
  const int rep_base = blockIdx.x * a.R;
  const long long plane = (long long)a.n * a.tiles;
  uint32_t flags = 0;
  init_tile(a, N, PN, PQ, PD, rep_base);
  __syncthreads();

  for (int tau = 1; tau <= a.K; ++tau) {
    const float gt = a.g[tau - 1];
    for (int lev = 0; lev < a.n_levels; ++lev) {
      const int p0 = a.level_ptr[lev];
      const int cnt = (a.level_ptr[lev + 1] - p0) << a.log2R;
      for (int k = tid; k < cnt; k += B) {
        const int r = k & (a.R - 1), rep = rep_base + r;
        if (rep >= a.reps) continue;
        const int s = a.order[p0 + (k >> a.log2R)];
        const int item = (s << a.log2R) | r;
        const StationParam p = a.sp[s];
        const uint32_t grep = (uint32_t)(a.rep0 + rep);
        const int A = draw_arrivals(a, p, gt, grep, (uint32_t)s, tau, flags);
        const int x = N[item] + A;
        if (x >= kStateLimit) flags |= 1u;
        const int D = draw_departures(a, p, x, grep, (uint32_t)s, tau, flags);
        N[item] = x - D;
        PD[item] += D;
        route_push(a, p, D, grep, (uint32_t)s, tau, r, N, flags);
      }
      __syncthreads();
    }
    const bool flush = a.sums && ((tau % kFlushEvery) == 0 || tau == a.K);
    for (int item = tid; item < a.items; item += B) {
      const int s = item >> a.log2R, r = item & (a.R - 1), rep = rep_base + r;
      if (rep >= a.reps) continue;
      if (a.sums)
        stats_step(a, PN, PQ, PD, item, N[item], servers_in(a.segidx, a.seg_m, a.n, s, tau - 1, a.sp[s].c),
                   flush, tile_index(a, s, rep), plane);
    }
    __syncthreads();
  }

  for (int item = tid; item < a.items; item += B) {
    const int s = item >> a.log2R, r = item & (a.R - 1), rep = rep_base + r;
    if (rep < a.reps) a.state[(long long)s * a.reps + rep] = N[item];
  }
  if (flags) atomicOr(a.flags, flags);
}

// Per-station reduction over the 32-replication statistics tiles; one workgroup per station, fixed
// tree order.  Means are exact integer totals divided once; the standard error treats the
// tile means as independent samples, weighted by tile size (equal weights for full tiles).
constexpr int kStatThreads = 256;

// With a second run (tsums2, state2: the other scheme on the same replications) the sums of
// both are pooled, which gives the statistics of the average scheme: means over 2K station-
// steps per replication, tile means of the pooled sums, pooled arrivals.
__global__ __launch_bounds__(kStatThreads) void k_stats(const long long *tsums, const int *state,
                                                        const long long *tsums2, const int *state2,
                                                        const int *init, int n, int reps, int K,
                                                        float dt, double *out) {
  __shared__ long long red_i[4][kStatThreads];
  __shared__ double red_d[2][kStatThreads];
  const int s = blockIdx.x, tid = threadIdx.x;
  const int tiles = stat_tiles(reps);
  const long long plane = (long long)n * tiles;
  const long long *sN = tsums + (long long)s * tiles, *sQ = sN + plane, *sD = sN + 2 * plane;
  const long long *sN2 = tsums2 ? tsums2 + (long long)s * tiles : nullptr;
  const long long *sQ2 = sN2 ? sN2 + plane : nullptr, *sD2 = sN2 ? sN2 + 2 * plane : nullptr;
  const int runs = tsums2 ? 2 : 1;
  auto tile_n = [&](int t) { return sN[t] + (sN2 ? sN2[t] : 0); };
  auto tile_q = [&](int t) { return sQ[t] + (sQ2 ? sQ2[t] : 0); };
  long long tn = 0, tq = 0, td = 0, ta = 0;
  for (int t = tid; t < tiles; t += kStatThreads) { tn += tile_n(t); tq += tile_q(t); td += sD[t] + (sD2 ? sD2[t] : 0); }
  for (int r = tid; r < reps; r += kStatThreads) {
    const long long g = (long long)s * reps + r;
    ta += (long long)state[g] + (state2 ? state2[g] : 0) - (long long)runs * (init ? init[g] : 0);
  }
  red_i[0][tid] = tn; red_i[1][tid] = tq; red_i[2][tid] = td; red_i[3][tid] = ta;
  __syncthreads();
  for (int w = kStatThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int k = 0; k < 4; ++k) red_i[k][tid] += red_i[k][tid + w];
    __syncthreads();
  }
  const double R = (double)reps;
  const double Ke = (double)K * runs;   // station-steps per replication and station
  const double mN = K > 0 ? (double)red_i[0][0] / (R * Ke) : 0.0;
  const double mQ = K > 0 ? (double)red_i[1][0] / (R * Ke) : 0.0;
  double vn = 0.0, vq = 0.0;
  if (K > 0) {
    for (int t = tid; t < tiles; t += kStatThreads) {
      const double c = (double)min(kStatReps, reps - kStatReps * t);
      const double w = c / R;
      const double dn = (double)tile_n(t) / (c * Ke) - mN;
      const double dq = (double)tile_q(t) / (c * Ke) - mQ;
      vn += w * w * dn * dn;
      vq += w * w * dq * dq;
    }
  }
  red_d[0][tid] = vn; red_d[1][tid] = vq;
  __syncthreads();
  for (int w = kStatThreads / 2; w > 0; w >>= 1) {
    if (tid < w) { red_d[0][tid] += red_d[0][tid + w]; red_d[1][tid] += red_d[1][tid + w]; }
    __syncthreads();
  }
  if (tid == 0) {
    const double T = (double)tiles;
    const double corr = tiles > 1 ? T / (T - 1.0) : 0.0;
    const double horizon = Ke * (double)dt;
    const long long arrivals = red_i[3][0] + red_i[2][0];
    out[s] = mN;
    out[s + n] = sqrt(red_d[0][0] * corr);
    out[s + 2 * n] = mQ;
    out[s + 3 * n] = sqrt(red_d[1][0] * corr);
    out[s + 4 * n] = K > 0 ? (double)red_i[2][0] / (R * horizon) : 0.0;
    out[s + 5 * n] = arrivals > 0 ? (double)red_i[1][0] * (double)dt / (double)arrivals : 0.0;
  }
}

// ---- diagnostics ------------------------------------------------------------------------
__global__ void k_selftest_math(int kind, const float *x, float *y, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float v = x[i];
  float r = 0.0f;
  switch (kind) {
    case 0: r = ln(v); break;
    case 1: r = ln1p(v); break;
    case 2: r = ex(v); break;
    case 3: r = exm1(v); break;
    default: r = to_unit(__float_as_uint(v)); break;
  }
  y[i] = r;
}

__global__ void k_selftest_sample(int kind, long long count, uint32_t k0, uint32_t k1, uint32_t rep0,
                                  uint32_t station, uint32_t step0, uint32_t sub, int i0, int i1,
                                  float f0, float f1, float f2, float f3, float *out,
                                  unsigned *dflags) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t flags = 0;
  Stream S = make_stream(k0, k1, rep0 + (uint32_t)i, station, step0, sub);
  float v = 0.0f;
  switch (kind) {
    case 0: v = (float)poisson(f0, S, flags); break;
    case 1: v = (float)binomial(i0, f0, S, flags); break;
    case 2: v = gamma_int(i0, S, flags); break;
    case 3: v = (float)gendep(i0, i1, f0, f1, binom_prep(f2), f3, S, flags); break;
    default: v = (float)gendep_naive(i0, i1, f0, S, flags); break;
  }
  out[i] = v;
  if (flags) atomicOr(dflags, flags);
}

// kind 0: A ~ Poisson(f0 f1) with its score in lambda0 = f0 (f1 = g); kind 3: GenerateDeparture
// (x, m, mu = f0, dt = f1) with its score in mu; kind 4: naive departures, same arguments.
__global__ void k_selftest_score(int kind, long long count, uint32_t k0, uint32_t k1, uint32_t rep0,
                                 uint32_t station, uint32_t step0, uint32_t sub, int x, int m, float f0,
                                 float f1, float pdep, float rate, float mudt, float kap, float *val,
                                 float *score, unsigned *dflags) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t flags = 0;
  Stream S = make_stream(k0, k1, rep0 + (uint32_t)i, station, step0, sub);
  float sc = 0.0f;
  int v;
  switch (kind) {
    case 0:
      v = poisson(f0 * f1, S, flags);
      sc = (float)v / f0 - f1;
      break;
    case 3: v = gendep_score(x, m, f0, f1, binom_prep(pdep), rate, kap, S, flags, sc); break;
    default: v = gendep_naive_score(x, m, mudt, f0, f1, S, flags, sc); break;
  }
  val[i] = (float)v;
  score[i] = sc;
  if (flags) atomicOr(dflags, flags);
}

__global__ void k_selftest_philox(long long count, const uint32_t *ctr, const uint32_t *key,
                                  uint32_t *out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const U4 o = philox10(U4{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]},
                        key[2 * i], key[2 * i + 1]);
  out[4 * i] = o.x; out[4 * i + 1] = o.y; out[4 * i + 2] = o.z; out[4 * i + 3] = o.w;
}

// ---- launch helpers (host) ---------------------------------------------------------------
static_assert(kRcpTab == kRcpTabHost, "reciprocal table of the host and the samplers");

hipError_t upload_sampler_tables(const float *inv, const float *fc) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_rcp4), inv, sizeof(float) * kRcpTab);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_fc), fc, sizeof(float) * 10);
}

hipError_t launch_backward(const SimArgs &a, int grid, int block, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_backward, dim3(grid), dim3(block), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_forward(const SimArgs &a, int grid, int block, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_forward, dim3(grid), dim3(block), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_stats(const long long *tsums, const int *state, const long long *tsums2,
                        const int *state2, const int *init, int n, int reps, int K, float dt, double *out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_stats, dim3(n), dim3(kStatThreads), 0, st, tsums, state, tsums2, state2, init, n,
                     reps, K, dt, out);
  return hipGetLastError();
}

hipError_t launch_selftest_math(int kind, const float *x, float *y, long long count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int blk = 256;
  const long long grid = (count + blk - 1) / blk;
  hipLaunchKernelGGL(k_selftest_math, dim3((unsigned)grid), dim3(blk), 0, st, kind, x, y, count);
  return hipGetLastError();
}

hipError_t launch_selftest_sample(int kind, long long count, uint32_t k0, uint32_t k1, uint32_t rep0,
                                  uint32_t station, uint32_t step0, uint32_t sub, int i0, int i1,
                                  float f0, float f1, float f2, float f3, float *out,
                                  unsigned *dflags, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int blk = 256;
  const long long grid = (count + blk - 1) / blk;
  hipLaunchKernelGGL(k_selftest_sample, dim3((unsigned)grid), dim3(blk), 0, st, kind, count, k0, k1,
                     rep0, station, step0, sub, i0, i1, f0, f1, f2, f3, out, dflags);
  return hipGetLastError();
}

hipError_t launch_selftest_score(int kind, long long count, uint32_t k0, uint32_t k1, uint32_t rep0,
                                 uint32_t station, uint32_t step0, uint32_t sub, int x, int m, float f0,
                                 float f1, float pdep, float rate, float mudt, float kap, float *val,
                                 float *score, unsigned *dflags, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int blk = 256;
  const long long grid = (count + blk - 1) / blk;
  hipLaunchKernelGGL(k_selftest_score, dim3((unsigned)grid), dim3(blk), 0, st, kind, count, k0, k1, rep0,
                     station, step0, sub, x, m, f0, f1, pdep, rate, mudt, kap, val, score, dflags);
  return hipGetLastError();
}

hipError_t launch_selftest_philox(long long count, const uint32_t *ctr, const uint32_t *key,
                                  uint32_t *out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int blk = 256;
  const long long grid = (count + blk - 1) / blk;
  hipLaunchKernelGGL(k_selftest_philox, dim3((unsigned)grid), dim3(blk), 0, st, count, ctr, key, out);
  return hipGetLastError();
}

}  // namespace eq

// The sweep kernels share this translation unit (and its __constant__ sampler tables).
#include "eq_sweep.h"

namespace eq {

// The inflow slots of eq_sim_run_noalloc's sweep kernels live here instead of in a workspace
// the library allocates.  Each device holds its own copy; host code uses only the address that
// hipGetSymbolAddress returns for it on that device, never the name.
constexpr int kScratchDevices = 64;
static __device__ __align__(256) int scratch[kNoAllocScratchBytes / sizeof(int)];
static int *g_scratch_ptr[kScratchDevices];

hipError_t setup_noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = static_cast<int *>(p);
  return hipSuccess;
}

int *noalloc_scratch(int dev) { return dev >= 0 && dev < kScratchDevices ? g_scratch_ptr[dev] : nullptr; }

}  // namespace eq

// eq_capi.cpp -- host side of the C ABI declared in include/eulerq.h.
//
// Network validation, the host tables of the method (routing conditionals for the
// sequential-binomial multinomial, departure probabilities, arrival-rate integrals,
// topological levels), device residency of those tables, launch-shape selection and the
// error convention (negative codes + thread-local message).  Host tables are computed in
// fp64 with libm and rounded once to fp32.
#include "eulerq.h"
#include "eq_internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <new>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(EQ_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr int kMaxDevices = 64;
std::mutex g_dev_mu;
bool g_dev_ready[kMaxDevices];

// fp32(1/k) for k = 1..63 and the Stirling-series remainders fc(0..9).
// rcp[i] = fp32(1/(i+1)); fc[j] = Stirling remainder of ln j!, j < 10.
void sampler_tables(float *rcp, float *fc) {
  for (int i = 0; i < eq::kRcpTabHost; ++i) rcp[i] = 1.0f / (float)(i + 1);
  for (int j = 0; j < 10; ++j) {
    const double jd = (double)j;
    const double lf = std::lgamma(jd + 1.0);
    const double st = (jd + 0.5) * std::log(jd + 1.0) - (jd + 1.0) + 0.5 * std::log(2.0 * M_PI);
    fc[j] = (float)(lf - st);
  }
}

// Current device must be gfx950; upload the sampler tables once per device.
int ensure_device(int *dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(EQ_EDEVICE, "device index %d unsupported", dev);
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (!g_dev_ready[dev]) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(EQ_EDEVICE, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
    float rcp[eq::kRcpTabHost], fc[10];
    sampler_tables(rcp, fc);
    e = eq::upload_sampler_tables(rcp, fc);
    if (e != hipSuccess) return hip_fail(e, "upload sampler tables");
    e = eq::setup_noalloc_scratch(dev);
    if (e != hipSuccess) return hip_fail(e, "address of the allocation-free scratch");
    g_dev_ready[dev] = true;
  }
  *dev_out = dev;
  return EQ_OK;
}

uint32_t bits_of(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

int pow2_floor(long long v) {
  int p = 1;
  while ((long long)p * 2 <= v) p *= 2;
  return p;
}

int log2_exact(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

}  // namespace

struct eq_net {
  int32_t n = 0;
  std::vector<int32_t> row_ptr, col, servers;
  std::vector<float> prob, mu, lam0, q;
  std::vector<int32_t> src_list;                 // stations with external arrivals, increasing
  // staffing schedule (n_seg = 0: constant servers)
  int32_t n_seg = 0, seg_period = 0;
  std::vector<int32_t> seg_start, seg_servers;   // [n_seg], [n_seg][n]
  int32_t shape_kind = EQ_SHAPE_CONST;
  double amp = 0.0, period = 1.0, phase = 0.0;
  std::vector<double> knot_t, knot_shape;        // piecewise-constant shape
  bool index_dag = false;
  std::vector<int32_t> level, order, level_ptr;
  std::vector<eq::StationRing> ring_b, ring_f;   // sweep-kernel inflow rings
  int64_t ring_f_slots = 0;
  // device residency
  int device = -1;
  eq::StationParam *d_sp = nullptr;
  eq::BinomP *d_dep = nullptr;
  eq::ScoreParam *d_scp = nullptr;
  eq::Edge *d_edges = nullptr;
  float *d_g = nullptr;
  int *d_order = nullptr, *d_level_ptr = nullptr, *d_heavy = nullptr;
  int *d_segidx = nullptr, *d_seg_m = nullptr;   // staffing: [K+1] segment per interval, [n_seg][n]
  float *d_seg_rate = nullptr;                   // [n_seg][n] fp32(m mu)
  unsigned *d_flags = nullptr;
  eq::StationRing *d_ring_b = nullptr, *d_ring_f = nullptr;
  int *d_ws = nullptr;
  size_t ws_cap = 0;
  int32_t *d_soj = nullptr;    // sojourn sample table (i0, tau0)
  size_t soj_cap = 0;
  // reachability-pruned gradient: reach[j][i] for the n + n_src parameters (host, made at the
  // first such reduction), its device copy and the reduction's workspace
  std::vector<uint8_t> reach;
  unsigned char *d_reach = nullptr;
  double *d_gws = nullptr;
  size_t gws_cap = 0;
  size_t g_cap = 0;
  bool dev_valid = false;
  uint64_t tables_gen = 0;   // bumped at every rebuild of the device tables (batch graph key)
  float dev_dt = 0.0f;
  int32_t dev_K = -1;

  ~eq_net() { release(); }
  void release() {
    if (device >= 0) {
      int cur = -1;
      (void)hipGetDevice(&cur);
      if (cur != device) (void)hipSetDevice(device);
      (void)hipDeviceSynchronize();   // runs still queued on any stream may read these tables
      (void)hipFree(d_sp); (void)hipFree(d_dep); (void)hipFree(d_scp); (void)hipFree(d_edges); (void)hipFree(d_g);
      (void)hipFree(d_order); (void)hipFree(d_level_ptr); (void)hipFree(d_heavy); (void)hipFree(d_flags);
      (void)hipFree(d_segidx); (void)hipFree(d_seg_m); (void)hipFree(d_seg_rate); (void)hipFree(d_soj);
      (void)hipFree(d_ring_b); (void)hipFree(d_ring_f); (void)hipFree(d_ws);
      (void)hipFree(d_reach); (void)hipFree(d_gws);
      if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    }
    d_reach = nullptr; d_gws = nullptr; gws_cap = 0;
    d_sp = nullptr; d_dep = nullptr; d_scp = nullptr; d_edges = nullptr; d_g = nullptr; d_order = nullptr; d_level_ptr = nullptr; d_heavy = nullptr;
    d_segidx = nullptr; d_seg_m = nullptr; d_seg_rate = nullptr; d_soj = nullptr; soj_cap = 0;
    d_flags = nullptr; d_ring_b = nullptr; d_ring_f = nullptr; d_ws = nullptr; ws_cap = 0;
    device = -1; g_cap = 0; dev_valid = false;
  }
};

namespace {

// q_e = p_e / (p_exit + sum_{l >= e} p_l): the probability that a customer not routed to the
// earlier edges of the row takes edge e (sequential conditional binomials, exit last).
void routing_conditionals(eq_net &net) {
  net.q.assign(net.col.size(), 0.0f);
  for (int32_t i = 0; i < net.n; ++i) {
    const int32_t b = net.row_ptr[i], e = net.row_ptr[i + 1];
    double tot = 0.0;
    for (int32_t j = b; j < e; ++j) tot += (double)net.prob[j];
    double pexit = 1.0 - tot;
    if (pexit < 0.0) pexit = 0.0;
    double suffix = pexit;
    for (int32_t j = e - 1; j >= b; --j) {
      suffix += (double)net.prob[j];
      double qq = suffix > 0.0 ? (double)net.prob[j] / suffix : 1.0;
      qq = std::min(1.0, std::max(0.0, qq));
      net.q[j] = (float)qq;
    }
  }
}

// Per-station constants for step dt: 1 - e^{-mu dt}, m mu, mu dt, and the score constant
// kap = dt e^{-mu dt} / (1 - e^{-mu dt}) = d/dmu log(1 - e^{-mu dt}).
void station_tables(const eq_net &net, float dt, float *pdep, float *rate, float *mudt, float *kap) {
  const double dtd = (double)dt;
  for (int32_t i = 0; i < net.n; ++i) {
    const double mud = (double)net.mu[i];
    if (pdep) pdep[i] = (float)(-std::expm1(-(mud * dtd)));
    if (rate) rate[i] = (float)((double)net.servers[i] * mud);
    if (mudt) mudt[i] = (float)(mud * dtd);
    if (kap) kap[i] = (float)(dtd * std::exp(-(mud * dtd)) / -std::expm1(-(mud * dtd)));
  }
}

// Integral of a piecewise-constant shape over [t0, t1]: the positive overlaps c (min(t1, hi) -
// max(t0, lo)) of its pieces [lo, hi), summed in time order.  In period j (the knots repeat
// with period P > 0; P = 0: one unbounded pass) piece k spans j P + t_k .. j P + t_{k+1}, the
// last ending at (j + 1) P (or never).  The first piece to visit comes from a binary search
// started two pieces early; pieces before it end before t0 and add nothing.
double piecewise_integral(const eq_net &net, double t0, double t1) {
  const int32_t nk = (int32_t)net.knot_t.size();
  const bool periodic = net.period > 0.0;
  const long long j0 = periodic ? (long long)std::floor(t0 / net.period) : 0;
  const long long j1 = periodic ? (long long)std::floor(t1 / net.period) : 0;
  double val = 0.0;
  for (long long j = j0; j <= j1; ++j) {
    const double base = periodic ? (double)j * net.period : 0.0;
    int32_t k = (int32_t)(std::upper_bound(net.knot_t.begin(), net.knot_t.end(), t0 - base) - net.knot_t.begin()) - 3;
    for (k = std::max(k, 0); k < nk; ++k) {
      const double lo = base + net.knot_t[k];
      if (!(lo < t1)) break;
      const double hi = k + 1 < nk ? base + net.knot_t[k + 1]
                                   : (periodic ? (double)(j + 1) * net.period : HUGE_VAL);
      const double a = lo > t0 ? lo : t0;
      const double b = hi < t1 ? hi : t1;
      if (b > a) val += net.knot_shape[k] * (b - a);
    }
  }
  return val;
}

// g[tau-1] = integral over ((tau-1) dt, tau dt] of the arrival shape (Section 2.1.1).
void shape_integrals(const eq_net &net, float dt, int32_t K, float *g) {
  const double dtd = (double)dt;
  if (net.shape_kind == EQ_SHAPE_CONST) {
    for (int32_t t = 0; t < K; ++t) g[t] = (float)dtd;
    return;
  }
  if (net.shape_kind == EQ_SHAPE_PIECEWISE) {
    for (int32_t t = 0; t < K; ++t) g[t] = (float)piecewise_integral(net, (double)t * dtd, (double)(t + 1) * dtd);
    return;
  }
  const double w = 2.0 * M_PI / net.period;
  for (int32_t t = 0; t < K; ++t) {
    const double t0 = (double)t * dtd, t1 = (double)(t + 1) * dtd;
    const double val = (t1 - t0) + net.amp / w * (std::cos(w * t0 + net.phase) - std::cos(w * t1 + net.phase));
    g[t] = (float)val;
  }
}

void compute_levels(eq_net &net) {
  net.index_dag = true;
  for (int32_t i = 0; i < net.n && net.index_dag; ++i)
    for (int32_t e = net.row_ptr[i]; e < net.row_ptr[i + 1]; ++e)
      if (net.col[e] <= i) { net.index_dag = false; break; }
  net.level.assign(net.n, 0);
  net.order.clear();
  net.level_ptr.clear();
  if (!net.index_dag) return;
  int32_t maxl = 0;
  for (int32_t i = 0; i < net.n; ++i) {
    for (int32_t e = net.row_ptr[i]; e < net.row_ptr[i + 1]; ++e)
      net.level[net.col[e]] = std::max(net.level[net.col[e]], net.level[i] + 1);
    maxl = std::max(maxl, net.level[i]);
  }
  net.level_ptr.assign(maxl + 2, 0);
  for (int32_t i = 0; i < net.n; ++i) net.level_ptr[net.level[i] + 1]++;
  for (int32_t l = 0; l <= maxl; ++l) net.level_ptr[l + 1] += net.level_ptr[l];
  net.order.assign(net.n, 0);
  std::vector<int32_t> fill(net.level_ptr.begin(), net.level_ptr.end() - 1);
  for (int32_t i = 0; i < net.n; ++i) net.order[fill[net.level[i]]++] = i;
}

// Inflow rings of the sweep kernels.  Backward: two slots per station (pushes of step tau
// are read in step tau + 1).  Forward: station j runs step tau in launch tau + l_j,
// a push along i -> j waits l_j - l_i iterations, so j needs 1 + max(l_j - l_i) slots.
void compute_rings(eq_net &net) {
  net.ring_b.resize(net.n);
  for (int32_t i = 0; i < net.n; ++i) net.ring_b[i] = eq::StationRing{2 * i, 2, 0, 0};
  net.ring_f.clear();
  net.ring_f_slots = 0;
  if (!net.index_dag) return;
  std::vector<int32_t> depth(net.n, 1);
  for (int32_t i = 0; i < net.n; ++i)
    for (int32_t e = net.row_ptr[i]; e < net.row_ptr[i + 1]; ++e) {
      const int32_t j = net.col[e];
      depth[j] = std::max(depth[j], net.level[j] - net.level[i] + 1);
    }
  net.ring_f.resize(net.n);
  int64_t off = 0;
  for (int32_t i = 0; i < net.n; ++i) {
    net.ring_f[i] = eq::StationRing{(int)off, depth[i], net.level[i], 0};
    off += depth[i];
  }
  net.ring_f_slots = off;
}

// reach[j][i] = 1 when station i is reachable from parameter j's station along routing edges
// (itself included): station j for mu_j (j < n), the source's station for lambda0 (j = n + s).
void compute_reach(eq_net &net) {
  const int32_t n = net.n;
  const size_t n_par = (size_t)n + net.src_list.size();
  net.reach.assign(n_par * (size_t)n, 0);
  std::vector<int32_t> stack;
  for (size_t j = 0; j < n_par; ++j) {
    uint8_t *row = net.reach.data() + j * (size_t)n;
    const int32_t start = j < (size_t)n ? (int32_t)j : net.src_list[j - n];
    row[start] = 1;
    stack.assign(1, start);
    while (!stack.empty()) {
      const int32_t i = stack.back();
      stack.pop_back();
      for (int32_t e = net.row_ptr[i]; e < net.row_ptr[i + 1]; ++e)
        if (!row[net.col[e]]) {
          row[net.col[e]] = 1;
          stack.push_back(net.col[e]);
        }
    }
  }
}

// Milliseconds of GPU time `fn` enqueues on `st` (events on the same stream).
template <class F>
int time_on_stream(hipStream_t st, F fn, float *ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(e, "hipEventCreate"); }
  int rc = EQ_OK;
  if ((e = hipEventRecord(e0, st)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
  if (!rc) rc = fn();
  if (!rc && (e = hipEventRecord(e1, st)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
  if (!rc && (e = hipEventSynchronize(e1)) != hipSuccess) rc = hip_fail(e, "hipEventSynchronize");
  if (!rc && (e = hipEventElapsedTime(ms, e0, e1)) != hipSuccess) rc = hip_fail(e, "hipEventElapsedTime");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

template <class T>
hipError_t dev_alloc(T **p, size_t count) {
  return hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1));
}

// Make the network's device tables current for (dt, K) on the current device.
int ensure_net_device(eq_net &net, float dt, int32_t K) {
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  hipError_t e;
  if (net.device != dev) {
    net.release();
    net.device = dev;
    const size_t nnz = net.col.size();
    if ((e = dev_alloc(&net.d_sp, net.n)) != hipSuccess ||
        (e = dev_alloc(&net.d_dep, net.n)) != hipSuccess ||
        (e = dev_alloc(&net.d_scp, net.n)) != hipSuccess ||
        (e = dev_alloc(&net.d_edges, nnz)) != hipSuccess ||
        (e = dev_alloc(&net.d_order, net.n)) != hipSuccess ||
        (e = dev_alloc(&net.d_heavy, net.n)) != hipSuccess ||
        (e = dev_alloc(&net.d_level_ptr, net.level_ptr.size() + 1)) != hipSuccess ||
        (e = dev_alloc(&net.d_flags, 1)) != hipSuccess ||
        (e = dev_alloc(&net.d_ring_b, net.n)) != hipSuccess ||
        (e = dev_alloc(&net.d_ring_f, net.n)) != hipSuccess) {
      net.release();
      return fail(EQ_ENOMEM, "device allocation for network tables: %s", hipGetErrorString(e));
    }
    // routing edges: raw (target, q_e) up, then the binomial constants made on the device
    {
      int *d_col = nullptr;
      float *d_q = nullptr;
      if ((e = dev_alloc(&d_col, nnz)) != hipSuccess || (e = dev_alloc(&d_q, nnz)) != hipSuccess) {
        (void)hipFree(d_col);
        net.release();
        return fail(EQ_ENOMEM, "device allocation for routing table: %s", hipGetErrorString(e));
      }
      e = hipMemcpy(d_col, net.col.data(), sizeof(int) * nnz, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(d_q, net.q.data(), sizeof(float) * nnz, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = eq::launch_prep_edges(d_col, d_q, net.d_edges, (int)nnz, nullptr);
      if (e == hipSuccess) e = hipDeviceSynchronize();
      (void)hipFree(d_col);
      (void)hipFree(d_q);
      if (e == hipSuccess) e = hipMemset(net.d_flags, 0, sizeof(unsigned));
    }
    // a failed upload leaves no device state behind: the next call starts over
    const char *what = nullptr;
    if (e != hipSuccess) what = "upload routing table";
    if (!what && (e = hipMemcpy(net.d_ring_b, net.ring_b.data(), sizeof(eq::StationRing) * net.n,
                                hipMemcpyHostToDevice)) != hipSuccess)
      what = "upload rings";
    if (!what && net.index_dag) {
      if ((e = hipMemcpy(net.d_ring_f, net.ring_f.data(), sizeof(eq::StationRing) * net.n, hipMemcpyHostToDevice)) !=
          hipSuccess)
        what = "upload rings";
      else if ((e = hipMemcpy(net.d_order, net.order.data(), sizeof(int) * net.n, hipMemcpyHostToDevice)) !=
                   hipSuccess ||
               (e = hipMemcpy(net.d_level_ptr, net.level_ptr.data(), sizeof(int) * net.level_ptr.size(),
                              hipMemcpyHostToDevice)) != hipSuccess)
        what = "upload levels";
    }
    if (what) {
      const int rc_fail = hip_fail(e, what);
      net.release();
      return rc_fail;
    }
  }
  if (net.dev_valid && net.dev_dt == dt && net.dev_K == K) return EQ_OK;
  // tables change: make sure no queued run still reads the old ones; until the rebuild
  // completes the tables match no (dt, K)
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  net.dev_valid = false;
  std::vector<float> pdep(net.n), rate(net.n), mudt(net.n), kap(net.n), g(std::max<int32_t>(K, 1));
  station_tables(net, dt, pdep.data(), rate.data(), mudt.data(), kap.data());
  shape_integrals(net, dt, K, g.data());
  std::vector<eq::StationParam> sp(net.n);
  for (int32_t i = 0; i < net.n; ++i)
    sp[i] = eq::StationParam{net.servers[i], net.mu[i], pdep[i], rate[i], mudt[i], net.lam0[i],
                             net.row_ptr[i], net.row_ptr[i + 1]};
  if ((e = hipMemcpy(net.d_sp, sp.data(), sizeof(eq::StationParam) * net.n, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "upload station table");
  // sweep task order: stations by decreasing service capacity m mu (ties by index); results do
  // not depend on it
  {
    std::vector<int> heavy(net.n);
    std::iota(heavy.begin(), heavy.end(), 0);
    std::stable_sort(heavy.begin(), heavy.end(), [&](int x, int y) {
      return (double)net.servers[x] * net.mu[x] > (double)net.servers[y] * net.mu[y];
    });
    if ((e = hipMemcpy(net.d_heavy, heavy.data(), sizeof(int) * net.n, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "upload task order");
  }
  if ((e = eq::launch_prep_dep(net.d_sp, net.d_dep, net.n, nullptr)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess)
    return hip_fail(e, "departure constants");
  std::vector<eq::ScoreParam> scp(net.n, eq::ScoreParam{0.0f, -1});
  for (int32_t i = 0; i < net.n; ++i) scp[i].kap = kap[i];
  for (size_t k = 0; k < net.src_list.size(); ++k) scp[net.src_list[k]].src = (int)k;
  if ((e = hipMemcpy(net.d_scp, scp.data(), sizeof(eq::ScoreParam) * net.n, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "upload score table");
  if ((size_t)std::max<int32_t>(K, 1) > net.g_cap) {
    (void)hipFree(net.d_g);
    net.d_g = nullptr;
    if ((e = dev_alloc(&net.d_g, (size_t)std::max<int32_t>(K, 1))) != hipSuccess) {
      net.g_cap = 0;
      return fail(EQ_ENOMEM, "device allocation for rate integrals: %s", hipGetErrorString(e));
    }
    net.g_cap = (size_t)std::max<int32_t>(K, 1);
  }
  if ((e = hipMemcpy(net.d_g, g.data(), sizeof(float) * g.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "upload rate integrals");
  // staffing: segment of every interval, servers and fp32(m mu) of every segment
  (void)hipFree(net.d_segidx); (void)hipFree(net.d_seg_m); (void)hipFree(net.d_seg_rate);
  net.d_segidx = nullptr; net.d_seg_m = nullptr; net.d_seg_rate = nullptr;
  if (net.n_seg > 0) {
    // one entry per interval 1..K, plus interval K+1: the sojourn walk looks up the servers of
    // the interval after the last recorded one before it finds that interval missing
    const size_t Kc = (size_t)K + 1, cells = (size_t)net.n_seg * net.n;
    std::vector<int> segidx(Kc, 0);
    for (int32_t t = 0; t <= K; ++t) {
      const int32_t tt = net.seg_period > 0 ? t % net.seg_period : t;
      int k = 0;
      while (k + 1 < net.n_seg && net.seg_start[k + 1] <= tt) ++k;
      segidx[t] = k;
    }
    std::vector<float> seg_rate(cells);
    for (int32_t k = 0; k < net.n_seg; ++k)
      for (int32_t i = 0; i < net.n; ++i)
        seg_rate[(size_t)k * net.n + i] = (float)((double)net.seg_servers[(size_t)k * net.n + i] * (double)net.mu[i]);
    if ((e = dev_alloc(&net.d_segidx, Kc)) != hipSuccess || (e = dev_alloc(&net.d_seg_m, cells)) != hipSuccess ||
        (e = dev_alloc(&net.d_seg_rate, cells)) != hipSuccess)
      return fail(EQ_ENOMEM, "device allocation for staffing: %s", hipGetErrorString(e));
    if ((e = hipMemcpy(net.d_segidx, segidx.data(), sizeof(int) * Kc, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(net.d_seg_m, net.seg_servers.data(), sizeof(int) * cells, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(net.d_seg_rate, seg_rate.data(), sizeof(float) * cells, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "upload staffing");
  }
  net.dev_valid = true;
  net.dev_dt = dt;
  net.dev_K = K;
  net.tables_gen += 1;
  return EQ_OK;
}

int check_desc(const eq_net *net, const eq_run_desc *d) {
  if (!net || !d) return fail(EQ_EINVAL, "null network or run descriptor");
  if (d->scheme != EQ_BACKWARD && d->scheme != EQ_FORWARD) return fail(EQ_EINVAL, "scheme %d", d->scheme);
  if (d->dep_mode != EQ_DEP_EXACT && d->dep_mode != EQ_DEP_NAIVE) return fail(EQ_EINVAL, "dep_mode %d", d->dep_mode);
  if (!(d->dt > 0.0f) || !std::isfinite(d->dt)) return fail(EQ_EINVAL, "dt must be finite and > 0");
  if (d->n_steps < 0) return fail(EQ_EINVAL, "n_steps must be >= 0");
  if (d->reps < 1) return fail(EQ_EINVAL, "reps must be >= 1");
  if (d->rep0 < 0 || (long long)d->rep0 + d->reps > 0xFFFFFFFFll) return fail(EQ_EINVAL, "rep0 out of range");
  if (d->kernel < EQ_KERNEL_AUTO || d->kernel > EQ_KERNEL_SWEEP) return fail(EQ_EINVAL, "kernel %d", d->kernel);
  if (d->tile_reps < 0 || d->tile_reps > 64 || (d->tile_reps & (d->tile_reps - 1)))
    return fail(EQ_EINVAL, "tile_reps must be 0 or a power of two <= 64");
  if (d->block < 0 || d->block > 1024 || d->block % 64) return fail(EQ_EINVAL, "block must be 0 or a multiple of 64 <= 1024");
  if (d->kernel == EQ_KERNEL_SWEEP && d->block > 256) return fail(EQ_EINVAL, "sweep kernel block must be 64..256");
  if (d->scheme == EQ_FORWARD && !net->index_dag)
    return fail(EQ_ENOTDAG, "forward scheme needs every routing edge i -> j to have j > i");
  return EQ_OK;
}

constexpr long long kLdsBudget = 65536;   // bytes of LDS per workgroup
// Sweep workgroups: one wavefront each unless the run asks otherwise; the finest grain packs
// the end of each launch best (measured on the 1000-station DAG).
constexpr int kSweepWavesPerBlock = 1;

struct Shape { int R, block, grid; size_t lds; };

// Replications per workgroup: the largest power of two (<= 64, <= what the replication
// count needs) whose tile fits the LDS budget; per-item LDS bytes are 20 for the backward
// kernel (state, departures, three statistics partials) and 16 for the forward kernel.
int choose_shape(const eq_net &net, const eq_run_desc &d, Shape *sh) {
  const long long n = net.n;
  const long long per_item = d.scheme == EQ_BACKWARD ? 20 : 16;
  const int reps_p2 = d.reps >= 64 ? 64 : (1 << log2_exact(d.reps));
  const long long rmax = std::min<long long>(64, kLdsBudget / (per_item * n));
  if (rmax < 1 && !d.tile_reps)
    return fail(EQ_EINVAL, "network of %lld stations exceeds the LDS-resident kernel", n);
  const int R = d.tile_reps ? d.tile_reps : std::min(pow2_floor(rmax), reps_p2);
  const long long items = n * R;
  if (items * per_item > kLdsBudget)
    return fail(EQ_EINVAL, "tile of %d replications x %lld stations exceeds %lld bytes of LDS", R, n, kLdsBudget);
  int block = d.block;
  if (!block) {
    const long long want = d.scheme == EQ_BACKWARD ? 512 : 256;
    block = (int)std::min<long long>(want, (items + 63) / 64 * 64);
  }
  sh->R = R;
  sh->block = block;
  sh->lds = (size_t)(items * per_item);
  sh->grid = (d.reps + R - 1) / R;
  return EQ_OK;
}

// The sweep kernels' view of one network for one run (device tables must be current).
eq::NetView make_view(const eq_net &net, const eq_run_desc &d, int32_t *state, int *ring, long long *tsums) {
  eq::NetView v;
  std::memset(&v, 0, sizeof v);
  v.sp = net.d_sp;
  v.dep = net.d_dep;
  v.segidx = net.d_segidx;
  v.seg_m = net.d_seg_m;
  v.seg_rate = net.d_seg_rate;
  v.heavy = net.d_heavy;
  v.sp2 = d.scheme == EQ_BACKWARD ? net.d_ring_b : net.d_ring_f;
  v.edges = net.d_edges;
  v.g = net.d_g;
  v.N = state;
  v.ring = ring;
  v.tsums = tsums;
  v.n = net.n;
  v.K = d.n_steps;
  v.reps = d.reps;
  v.rep0 = d.rep0;
  v.tiles = (d.reps + eq::kTileReps - 1) / eq::kTileReps;
  v.stiles = eq::stat_tiles(d.reps);
  v.extra = d.scheme == EQ_FORWARD ? (int)net.level_ptr.size() - 2 : 0;
  v.k0 = (uint32_t)d.seed;
  v.k1 = (uint32_t)(d.seed >> 32) ^ d.net_id;
  return v;
}

int64_t ring_slots(const eq_net &net, int scheme) {
  return scheme == EQ_BACKWARD ? 2 * (int64_t)net.n : net.ring_f_slots;
}

// SWEEP when one step gives the chip enough station-coherent wavefronts (>= 2048, i.e. 8
// per CU); otherwise (tiny networks or few replications, where per-step launches would be
// latency bound) TILE if the tile fits in LDS.
int pick_kernel(const eq_net &net, const eq_run_desc &d) {
  if (d.kernel != EQ_KERNEL_AUTO) return d.kernel;
  const long long waves = (long long)net.n * ((d.reps + eq::kTileReps - 1) / eq::kTileReps);
  const long long per_item = d.scheme == EQ_BACKWARD ? 20 : 16;
  if (waves >= 2048 || (long long)net.n * per_item > kLdsBudget) return EQ_KERNEL_SWEEP;
  return EQ_KERNEL_TILE;
}

}  // namespace

// ------------------------------------------------------------------------------------------
extern "C" {

const char *eq_last_error(void) { return g_err.c_str(); }

int eq_net_create(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
                  const int32_t *servers, const float *mu, const eq_arrivals *arr, eq_net **out) {
  if (!out) return fail(EQ_EINVAL, "out is null");
  *out = nullptr;
  if (n <= 0) return fail(EQ_EINVAL, "n must be > 0");
  if (!row_ptr || !servers || !mu || !arr) return fail(EQ_EINVAL, "null array argument");
  if (row_ptr[0] != 0) return fail(EQ_EINVAL, "row_ptr[0] must be 0");
  for (int32_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return fail(EQ_EINVAL, "row_ptr not monotone at %d", i);
  const int32_t nnz = row_ptr[n];
  if (nnz > 0 && (!col || !prob)) return fail(EQ_EINVAL, "null col or prob");
  for (int32_t i = 0; i < n; ++i) {
    double tot = 0.0;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) return fail(EQ_EINVAL, "col[%d] = %d out of range", e, col[e]);
      if (!(prob[e] >= 0.0f) || !std::isfinite(prob[e])) return fail(EQ_EINVAL, "prob[%d] invalid", e);
      tot += prob[e];
    }
    if (tot > 1.0 + 1e-6) return fail(EQ_EINVAL, "routing row %d sums to %.9g > 1", i, tot);
    if (servers[i] < 1) return fail(EQ_EINVAL, "servers[%d] = %d < 1", i, servers[i]);
    if (!(mu[i] > 0.0f) || !std::isfinite(mu[i])) return fail(EQ_EINVAL, "mu[%d] must be finite and > 0", i);
  }
  if (arr->n_src < 0 || (arr->n_src > 0 && (!arr->src || !arr->lambda0)))
    return fail(EQ_EINVAL, "bad arrival sources");
  for (int32_t k = 0; k < arr->n_src; ++k) {
    if (arr->src[k] < 0 || arr->src[k] >= n) return fail(EQ_EINVAL, "src[%d] out of range", k);
    if (k > 0 && arr->src[k] <= arr->src[k - 1]) return fail(EQ_EINVAL, "src must be strictly increasing");
    if (!(arr->lambda0[k] >= 0.0f) || !std::isfinite(arr->lambda0[k])) return fail(EQ_EINVAL, "lambda0[%d] invalid", k);
  }
  if (arr->shape_kind != EQ_SHAPE_CONST && arr->shape_kind != EQ_SHAPE_SINUSOID &&
      arr->shape_kind != EQ_SHAPE_PIECEWISE)
    return fail(EQ_EINVAL, "shape_kind %d", arr->shape_kind);
  if (arr->shape_kind == EQ_SHAPE_PIECEWISE) {
    if (arr->n_knots < 1 || !arr->knot_t || !arr->knot_shape) return fail(EQ_EINVAL, "piecewise shape needs knots");
    if (arr->knot_t[0] != 0.0) return fail(EQ_EINVAL, "knot_t[0] must be 0");
    if (!(arr->period >= 0.0) || !std::isfinite(arr->period)) return fail(EQ_EINVAL, "period must be >= 0");
    for (int32_t k = 0; k < arr->n_knots; ++k) {
      if (!std::isfinite(arr->knot_t[k]) || !(arr->knot_shape[k] >= 0.0) || !std::isfinite(arr->knot_shape[k]))
        return fail(EQ_EINVAL, "knot %d invalid", k);
      if (k > 0 && !(arr->knot_t[k] > arr->knot_t[k - 1])) return fail(EQ_EINVAL, "knot_t must increase");
    }
    if (arr->period > 0.0 && !(arr->knot_t[arr->n_knots - 1] < arr->period))
      return fail(EQ_EINVAL, "knots must lie inside the period");
  }
  if (arr->shape_kind == EQ_SHAPE_SINUSOID &&
      (!(std::fabs(arr->amp) <= 1.0) || !(arr->period > 0.0) || !std::isfinite(arr->period) || !std::isfinite(arr->phase)))
    return fail(EQ_EINVAL, "sinusoid needs |amp| <= 1 and period > 0");

  eq_net *net = new (std::nothrow) eq_net();
  if (!net) return fail(EQ_ENOMEM, "host allocation");
  try {
    net->n = n;
    net->row_ptr.assign(row_ptr, row_ptr + n + 1);
    net->col.assign(col, col + nnz);
    net->prob.assign(prob, prob + nnz);
    net->servers.assign(servers, servers + n);
    net->mu.assign(mu, mu + n);
    net->lam0.assign(n, 0.0f);
    for (int32_t k = 0; k < arr->n_src; ++k) net->lam0[arr->src[k]] = arr->lambda0[k];
    net->src_list.assign(arr->src, arr->src + arr->n_src);
    net->shape_kind = arr->shape_kind;
    net->amp = arr->amp;
    net->period = arr->period;
    net->phase = arr->phase;
    if (arr->shape_kind == EQ_SHAPE_PIECEWISE) {
      net->knot_t.assign(arr->knot_t, arr->knot_t + arr->n_knots);
      net->knot_shape.assign(arr->knot_shape, arr->knot_shape + arr->n_knots);
    }
    routing_conditionals(*net);
    compute_levels(*net);
    compute_rings(*net);
  } catch (...) {
    delete net;
    return fail(EQ_ENOMEM, "host allocation");
  }
  *out = net;
  return EQ_OK;
}

void eq_net_destroy(eq_net *net) { delete net; }

int eq_net_set_staffing(eq_net *net, int32_t n_seg, const int32_t *seg_start, const int32_t *servers,
                        int32_t period) {
  if (!net) return fail(EQ_EINVAL, "null network");
  if (n_seg < 0 || period < 0) return fail(EQ_EINVAL, "n_seg and period must be >= 0");
  if (n_seg > 0) {
    if (!seg_start || !servers) return fail(EQ_EINVAL, "null schedule array");
    if (seg_start[0] != 0) return fail(EQ_EINVAL, "the first segment must start at interval 0");
    for (int32_t k = 1; k < n_seg; ++k)
      if (seg_start[k] <= seg_start[k - 1]) return fail(EQ_EINVAL, "segment starts must increase");
    if (period > 0 && seg_start[n_seg - 1] >= period) return fail(EQ_EINVAL, "segment start beyond the period");
    for (int64_t j = 0; j < (int64_t)n_seg * net->n; ++j)
      if (servers[j] < 1) return fail(EQ_EINVAL, "servers must be >= 1");
  }
  try {
    // copies first, so that a failed allocation leaves the old schedule whole
    std::vector<int32_t> st(seg_start, seg_start + n_seg), sv(servers, servers + (size_t)n_seg * net->n);
    net->seg_start.swap(st);
    net->seg_servers.swap(sv);
  } catch (...) {
    return fail(EQ_ENOMEM, "host allocation");
  }
  net->n_seg = n_seg;
  net->seg_period = n_seg > 0 ? period : 0;
  net->dev_valid = false;   // tables are rebuilt (after a device synchronisation) by the next run
  return EQ_OK;
}

int eq_net_set_params(eq_net *net, const float *mu, const float *lambda0) {
  if (!net) return fail(EQ_EINVAL, "null network");
  if (mu)
    for (int32_t i = 0; i < net->n; ++i)
      if (!(mu[i] > 0.0f) || !std::isfinite(mu[i])) return fail(EQ_EINVAL, "mu[%d] must be finite and > 0", i);
  if (lambda0)
    for (size_t k = 0; k < net->src_list.size(); ++k)
      if (!(lambda0[k] >= 0.0f) || !std::isfinite(lambda0[k])) return fail(EQ_EINVAL, "lambda0[%zu] invalid", k);
  if (mu) std::copy(mu, mu + net->n, net->mu.begin());
  if (lambda0)
    for (size_t k = 0; k < net->src_list.size(); ++k) net->lam0[net->src_list[k]] = lambda0[k];
  if (mu || lambda0) net->dev_valid = false;
  return EQ_OK;
}

int eq_net_tables(const eq_net *net, float dt, int32_t K, float *q, float *pdep, float *rate,
                  float *mudt, float *kap, float *g) {
  if (!net) return fail(EQ_EINVAL, "null network");
  if (!(dt > 0.0f) || K < 0) return fail(EQ_EINVAL, "dt must be > 0 and K >= 0");
  if (q) std::copy(net->q.begin(), net->q.end(), q);
  station_tables(*net, dt, pdep, rate, mudt, kap);
  if (g) shape_integrals(*net, dt, K, g);
  return EQ_OK;
}

int eq_net_reach(eq_net *net, uint8_t *reach) {
  if (!net) return fail(EQ_EINVAL, "null network");
  try {
    if (net->reach.empty()) compute_reach(*net);
  } catch (...) {
    return fail(EQ_ENOMEM, "host allocation");
  }
  if (reach) std::copy(net->reach.begin(), net->reach.end(), reach);
  return net->n + (int)net->src_list.size();
}

int eq_net_levels(const eq_net *net, int32_t *level) {
  if (!net) return fail(EQ_EINVAL, "null network");
  if (!net->index_dag) return fail(EQ_ENOTDAG, "network has an edge i -> j with j <= i");
  if (level) std::copy(net->level.begin(), net->level.end(), level);
  return (int)net->level_ptr.size() - 1;
}

size_t eq_sim_workspace_bytes(const eq_net *net, const eq_run_desc *desc) {
  if (!net || !desc || desc->reps < 1) return 0;
  if (pick_kernel(*net, *desc) != EQ_KERNEL_SWEEP) return 0;
  return (size_t)(ring_slots(*net, desc->scheme) * desc->reps) * sizeof(int32_t);
}

}  // extern "C"

namespace {

struct ScoreBufs {
  int64_t *sumq;
  float *smu, *slam;
};

struct RecBufs {
  int32_t t0, len;
  int32_t *N, *D, *R;
};

// scratch: inflow slots of the sweep kernels supplied by the caller (the allocation-free entry
// point), big enough for the run; nullptr: the network's own workspace, grown as needed.
int run_sim(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state, int64_t *d_sums,
            const ScoreBufs *sc, hipStream_t st, const RecBufs *rec = nullptr, int *scratch = nullptr) {
  int rc = check_desc(net, desc);
  if (rc) return rc;
  if (!d_state) return fail(EQ_EINVAL, "d_state is null");
  if (d_init && d_init == d_state) return fail(EQ_EINVAL, "d_init must not alias d_state");
  const int kernel = sc || rec ? EQ_KERNEL_SWEEP : pick_kernel(*net, *desc);
  if ((sc || rec) && desc->kernel == EQ_KERNEL_TILE)
    return fail(EQ_EINVAL, "score and recording runs use the sweep kernel (kernel must be AUTO or SWEEP)");
  Shape sh{};
  if (kernel == EQ_KERNEL_TILE && (rc = choose_shape(*net, *desc, &sh))) return rc;
  if ((rc = ensure_net_device(*net, desc->dt, desc->n_steps))) return rc;
  const int tiles = eq::stat_tiles(desc->reps);
  const long long nsums = 3LL * net->n * tiles;
  const uint32_t k0 = (uint32_t)desc->seed, k1 = (uint32_t)(desc->seed >> 32) ^ desc->net_id;
  hipError_t e;
  if (kernel == EQ_KERNEL_TILE) {
    if (d_sums && (e = eq::launch_sweep_init(nullptr, nullptr, 0, nullptr, 0, reinterpret_cast<long long *>(d_sums),
                                             nsums, st)) != hipSuccess)
      return hip_fail(e, "init launch");
    eq::SimArgs a;
    std::memset(&a, 0, sizeof a);
    a.sp = net->d_sp; a.dep = net->d_dep; a.edges = net->d_edges; a.g = net->d_g;
    a.segidx = net->d_segidx; a.seg_m = net->d_seg_m; a.seg_rate = net->d_seg_rate;
    a.order = net->d_order; a.level_ptr = net->d_level_ptr;
    a.init = d_init; a.state = d_state; a.sums = reinterpret_cast<long long *>(d_sums);
    a.flags = net->d_flags;
    a.n = net->n; a.K = desc->n_steps; a.reps = desc->reps; a.rep0 = desc->rep0;
    a.R = sh.R; a.log2R = log2_exact(sh.R); a.items = net->n * sh.R;
    a.n_levels = net->index_dag ? (int)net->level_ptr.size() - 1 : 0;
    a.dep_mode = desc->dep_mode; a.dt = desc->dt; a.tiles = tiles;
    a.k0 = k0; a.k1 = k1;
    e = desc->scheme == EQ_BACKWARD ? eq::launch_backward(a, sh.grid, sh.block, sh.lds, st)
                                    : eq::launch_forward(a, sh.grid, sh.block, sh.lds, st);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return EQ_OK;
  }
  // sweep kernel: workspace of inflow slots
  const size_t ws = (size_t)(ring_slots(*net, desc->scheme) * desc->reps) * sizeof(int32_t);
  if (!scratch && ws > net->ws_cap) {
    // runs queued earlier on any stream may still use the old workspace
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    (void)hipFree(net->d_ws);
    net->d_ws = nullptr;
    net->ws_cap = 0;
    if ((e = hipMalloc((void **)&net->d_ws, ws)) != hipSuccess)
      return fail(EQ_ENOMEM, "workspace of %zu bytes: %s", ws, hipGetErrorString(e));
    net->ws_cap = ws;
  }
  eq::SweepArgs a;
  std::memset(&a, 0, sizeof a);
  int *const ring = scratch ? scratch : net->d_ws;
  a.v = make_view(*net, *desc, d_state, ring, reinterpret_cast<long long *>(d_sums));
  if (sc) {
    const long long per = (long long)net->n * desc->reps;
    a.v.scp = net->d_scp;
    a.v.smu = sc->smu;
    a.v.slam = sc->slam;
    a.v.sq = reinterpret_cast<long long *>(sc->sumq);
    if ((e = eq::launch_zero(sc->sumq, 2 * per, st)) != hipSuccess ||
        (e = eq::launch_zero(sc->smu, per, st)) != hipSuccess ||
        (e = eq::launch_zero(sc->slam, (long long)net->src_list.size() * desc->reps, st)) != hipSuccess)
      return hip_fail(e, "zero launch");
  }
  if (rec) {
    const long long nn = (long long)rec->len * net->n * desc->reps;
    const long long ne = (long long)rec->len * (long long)net->col.size() * desc->reps;
    a.v.rec_N = rec->N;
    a.v.rec_D = rec->D;
    a.v.rec_R = rec->R;
    a.v.rec_t0 = rec->t0;
    a.v.rec_len = rec->len;
    a.v.nnz = (int)net->col.size();
    if ((e = eq::launch_zero(rec->N, nn, st)) != hipSuccess || (e = eq::launch_zero(rec->D, nn, st)) != hipSuccess ||
        (e = eq::launch_zero(rec->R, ne, st)) != hipSuccess)
      return hip_fail(e, "zero launch");
  }
  a.flags = net->d_flags;
  a.dep_mode = desc->dep_mode;
  a.dt = desc->dt;
  if ((e = eq::launch_sweep_init(d_state, d_init, (long long)net->n * desc->reps, ring,
                                 (long long)(ws / sizeof(int32_t)), a.v.tsums, d_sums ? nsums : 0, st)) != hipSuccess)
    return hip_fail(e, "init launch");
  const int iters = desc->n_steps > 0 ? desc->n_steps + a.v.extra : 0;
  const int wpb = desc->block >= 64 && desc->block <= 256 ? desc->block / 64 : kSweepWavesPerBlock;
  const int mode = sc ? 1 : rec ? 2 : 0;
  for (int it = 1; it <= iters; ++it) {
    a.iter = it;
    if ((e = eq::launch_sweep(a, desc->scheme, mode, wpb, st)) != hipSuccess) return hip_fail(e, "sweep launch");
  }
  if (desc->scheme == EQ_BACKWARD && (e = eq::launch_sweep_finish(a, mode, wpb, st)) != hipSuccess)
    return hip_fail(e, "finish launch");
  return EQ_OK;
}

}  // namespace

extern "C" {

int eq_sim_run(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state,
               int64_t *d_sums, void *stream) {
  return run_sim(net, desc, d_init, d_state, d_sums, nullptr, (hipStream_t)stream);
}

static_assert(EQ_NOALLOC_SCRATCH_BYTES == eq::kNoAllocScratchBytes, "scratch size of the header and the kernels");
static_assert(EQ_STAT_TILE_REPS == eq::kStatReps, "statistics tile of the header and the kernels");

int eq_sim_run_noalloc(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state,
                       int64_t *d_sums, void *stream) {
  int rc = check_desc(net, desc);
  if (rc) return rc;
  if (!d_state) return fail(EQ_EINVAL, "d_state is null");
  if (d_init && d_init == d_state) return fail(EQ_EINVAL, "d_init must not alias d_state");
  int dev = 0;
  if ((rc = ensure_device(&dev))) return rc;
  // building the device tables allocates: they must already hold this run's (h, K)
  if (net->device != dev || !net->dev_valid || net->dev_dt != desc->dt || net->dev_K != desc->n_steps)
    return fail(EQ_EINVAL, "the network's device tables are not built for this device, h and n_steps "
                           "(one eq_sim_run with the same h and n_steps builds them)");
  int *scratch = eq::noalloc_scratch(dev);
  if (!scratch) return fail(EQ_EDEVICE, "the allocation-free scratch is not set up on device %d", dev);
  if (pick_kernel(*net, *desc) == EQ_KERNEL_SWEEP) {
    const long long need = (long long)ring_slots(*net, desc->scheme) * desc->reps * (long long)sizeof(int32_t);
    if (need > eq::kNoAllocScratchBytes)
      return fail(EQ_EINVAL, "this run needs %lld bytes of scratch; the allocation-free entry point has %lld",
                  need, eq::kNoAllocScratchBytes);
  }
  return run_sim(net, desc, d_init, d_state, d_sums, nullptr, (hipStream_t)stream, nullptr, scratch);
}

int eq_sim_run_host(eq_net *net, const eq_run_desc *desc, const int32_t *init, int32_t *final_state,
                    double *stats) {
  int rc = check_desc(net, desc);
  if (rc) return rc;
  const size_t cells = (size_t)net->n * (size_t)desc->reps;
  const size_t tiles = (size_t)eq::stat_tiles(desc->reps);
  int32_t *d_init = nullptr, *d_state = nullptr;
  int64_t *d_sums = nullptr;
  double *d_stats = nullptr;
  hipError_t e = hipSuccess;
  auto release = [&]() {
    (void)hipFree(d_init); (void)hipFree(d_state); (void)hipFree(d_sums); (void)hipFree(d_stats);
  };
  int dev = 0;
  if ((rc = ensure_device(&dev))) return rc;
  if ((init && (e = hipMalloc((void **)&d_init, sizeof(int32_t) * cells)) != hipSuccess) ||
      (e = hipMalloc((void **)&d_state, sizeof(int32_t) * cells)) != hipSuccess ||
      (stats && (e = hipMalloc((void **)&d_sums, sizeof(int64_t) * 3 * net->n * tiles)) != hipSuccess) ||
      (stats && (e = hipMalloc((void **)&d_stats, sizeof(double) * 6 * net->n)) != hipSuccess)) {
    release();
    return fail(EQ_ENOMEM, "device buffers for a host-output run: %s", hipGetErrorString(e));
  }
  if (init && (e = hipMemcpy(d_init, init, sizeof(int32_t) * cells, hipMemcpyHostToDevice)) != hipSuccess) {
    release();
    return hip_fail(e, "upload initial state");
  }
  rc = run_sim(net, desc, d_init, d_state, d_sums, nullptr, nullptr);
  if (!rc && stats) rc = eq_stats_reduce(net, desc, d_sums, d_state, d_init, d_stats, nullptr);
  if (!rc) rc = eq_sim_check(net, nullptr);
  if (!rc && final_state && (e = hipMemcpy(final_state, d_state, sizeof(int32_t) * cells, hipMemcpyDeviceToHost)) !=
                                hipSuccess)
    rc = hip_fail(e, "download final state");
  if (!rc && stats && (e = hipMemcpy(stats, d_stats, sizeof(double) * 6 * net->n, hipMemcpyDeviceToHost)) !=
                          hipSuccess)
    rc = hip_fail(e, "download statistics");
  release();
  return rc;
}

int eq_sim_run_scores(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state,
                      int64_t *d_sums, int64_t *d_sumq, float *d_score_mu, float *d_score_lam, void *stream) {
  if (!net) return fail(EQ_EINVAL, "null network");
  if (!d_sumq || !d_score_mu || (!d_score_lam && !net->src_list.empty()))
    return fail(EQ_EINVAL, "null score buffer");
  const ScoreBufs sc{d_sumq, d_score_mu, d_score_lam};
  return run_sim(net, desc, d_init, d_state, d_sums, &sc, (hipStream_t)stream);
}

int eq_sim_run_record(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state,
                      int64_t *d_sums, int32_t rec_t0, int32_t rec_len, int32_t *d_rec_N, int32_t *d_rec_D,
                      int32_t *d_rec_R, void *stream) {
  if (!net) return fail(EQ_EINVAL, "null network");
  if (rec_t0 < 1 || rec_len < 1) return fail(EQ_EINVAL, "rec_t0 and rec_len must be >= 1");
  if (!d_rec_N || !d_rec_D || (!d_rec_R && !net->col.empty())) return fail(EQ_EINVAL, "null record buffer");
  const RecBufs rec{rec_t0, rec_len, d_rec_N, d_rec_D, d_rec_R};
  return run_sim(net, desc, d_init, d_state, d_sums, nullptr, (hipStream_t)stream, &rec);
}

int eq_sojourn(eq_net *net, const eq_run_desc *desc, int32_t rec_t0, int32_t rec_len, const int32_t *d_rec_N,
               const int32_t *d_rec_D, const int32_t *d_rec_R, int32_t n_samples, const int32_t *i0,
               const int32_t *tau0, int32_t *d_out, void *stream) {
  int rc = check_desc(net, desc);
  if (rc) return rc;
  if (rec_t0 < 1 || rec_len < 1 || n_samples < 0) return fail(EQ_EINVAL, "bad record window or sample count");
  if ((long long)rec_t0 + rec_len - 1 > desc->n_steps)
    return fail(EQ_EINVAL, "the record must lie within the run's n_steps");
  if (!d_rec_N || !d_rec_D || (!d_rec_R && !net->col.empty()) || !d_out || (n_samples > 0 && (!i0 || !tau0)))
    return fail(EQ_EINVAL, "null argument");
  for (int32_t k = 0; k < n_samples; ++k)
    if (i0[k] < 0 || i0[k] >= net->n) return fail(EQ_EINVAL, "i0[%d] = %d out of range", k, i0[k]);
  if ((rc = ensure_net_device(*net, desc->dt, desc->n_steps))) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  // sample table (host -> library buffer)
  const size_t need = 2 * (size_t)std::max(n_samples, 1) * sizeof(int32_t);
  if (need > net->soj_cap) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    (void)hipFree(net->d_soj);
    net->d_soj = nullptr;
    net->soj_cap = 0;
    if ((e = hipMalloc((void **)&net->d_soj, need)) != hipSuccess) return fail(EQ_ENOMEM, "sample table");
    net->soj_cap = need;
  }
  if (n_samples > 0 &&
      ((e = hipMemcpyAsync(net->d_soj, i0, sizeof(int32_t) * n_samples, hipMemcpyHostToDevice, st)) != hipSuccess ||
       (e = hipMemcpyAsync(net->d_soj + n_samples, tau0, sizeof(int32_t) * n_samples, hipMemcpyHostToDevice, st)) !=
           hipSuccess))
    return hip_fail(e, "upload samples");
  eq::SojournArgs a;
  std::memset(&a, 0, sizeof a);
  a.sp = net->d_sp; a.edges = net->d_edges; a.segidx = net->d_segidx; a.seg_m = net->d_seg_m;
  a.rec_N = d_rec_N; a.rec_D = d_rec_D; a.rec_R = d_rec_R; a.i0 = net->d_soj; a.tau0 = net->d_soj + n_samples;
  a.out = d_out;
  a.n = net->n; a.nnz = (int)net->col.size(); a.reps = desc->reps; a.rep0 = desc->rep0;
  a.rec_t0 = rec_t0; a.rec_len = rec_len; a.n_samples = n_samples; a.scheme = desc->scheme;
  a.k0 = (uint32_t)desc->seed;
  a.k1 = (uint32_t)(desc->seed >> 32) ^ desc->net_id;
  if ((e = eq::launch_sojourn(a, st)) != hipSuccess) return hip_fail(e, "sojourn launch");
  // the sample table must outlive the launch: synchronise before the caller may reuse it
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return EQ_OK;
}

int eq_cost_reduce(int32_t n, int32_t reps, int32_t n_steps, const double *d_hold, const int64_t *d_sumq,
                   double *d_f, double *d_mean_se, void *stream) {
  if (n < 1 || reps < 1 || n_steps < 1) return fail(EQ_EINVAL, "n, reps and n_steps must be >= 1");
  if (!d_hold || !d_sumq || !d_f || !d_mean_se) return fail(EQ_EINVAL, "null argument");
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  hipError_t e = eq::launch_cost(d_hold, reinterpret_cast<const long long *>(d_sumq), n, reps, n_steps, d_f,
                                 d_mean_se, (hipStream_t)stream);
  return e == hipSuccess ? EQ_OK : hip_fail(e, "cost launch");
}

int eq_grad_reduce(int32_t n_par, int32_t reps, const double *d_f, const double *d_mean_se, const float *d_score,
                   double *d_grad, double *d_se, void *stream) {
  if (n_par < 0 || reps < 2) return fail(EQ_EINVAL, "n_par must be >= 0 and reps >= 2");
  if (n_par > 0 && (!d_f || !d_mean_se || !d_score || !d_grad || !d_se)) return fail(EQ_EINVAL, "null argument");
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  hipError_t e = eq::launch_grad(d_f, d_mean_se, d_score, reps, n_par, d_grad, d_se, (hipStream_t)stream);
  return e == hipSuccess ? EQ_OK : hip_fail(e, "gradient launch");
}

int eq_grad_reduce_reach(eq_net *net, int32_t reps, int32_t n_steps, const double *d_hold, const int64_t *d_sumq,
                         const float *d_score, double *d_grad, double *d_se, void *stream) {
  if (!net) return fail(EQ_EINVAL, "null network");
  if (reps < 2 || n_steps < 1) return fail(EQ_EINVAL, "reps must be >= 2 and n_steps >= 1");
  if (!d_hold || !d_sumq || !d_score || !d_grad || !d_se) return fail(EQ_EINVAL, "null argument");
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  if (net->device != dev)
    return fail(EQ_EINVAL, "the network has no tables on device %d: reduce on the device its score run used", dev);
  const int n = net->n, n_par = net->n + (int)net->src_list.size();
  hipError_t e;
  try {
    if (net->reach.empty()) compute_reach(*net);
  } catch (...) {
    return fail(EQ_ENOMEM, "host allocation");
  }
  if (!net->d_reach) {
    if ((e = hipMalloc((void **)&net->d_reach, net->reach.size())) != hipSuccess) {
      net->d_reach = nullptr;
      return fail(EQ_ENOMEM, "reach table: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(net->d_reach, net->reach.data(), net->reach.size(), hipMemcpyHostToDevice)) != hipSuccess) {
      (void)hipFree(net->d_reach);
      net->d_reach = nullptr;
      return hip_fail(e, "upload reach table");
    }
  }
  const size_t ws = eq::grad_reach_workspace_bytes(n, n_par, reps);
  if (ws > net->gws_cap) {
    // an earlier reduction on any stream may still use the old workspace
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    (void)hipFree(net->d_gws);
    net->d_gws = nullptr;
    net->gws_cap = 0;
    if ((e = hipMalloc((void **)&net->d_gws, ws)) != hipSuccess)
      return fail(EQ_ENOMEM, "gradient workspace of %zu bytes: %s", ws, hipGetErrorString(e));
    net->gws_cap = ws;
  }
  e = eq::launch_grad_reach(net->d_reach, d_hold, reinterpret_cast<const long long *>(d_sumq), d_score, n, n_par,
                            reps, n_steps, net->d_gws, d_grad, d_se, (hipStream_t)stream);
  return e == hipSuccess ? EQ_OK : hip_fail(e, "gradient launch");
}

int eq_sim_tune(eq_net *net, const eq_run_desc *desc, int32_t trial_steps, int32_t *d_state, void *stream,
                eq_run_desc *best) {
  int rc = check_desc(net, desc);
  if (rc) return rc;
  if (!d_state || !best) return fail(EQ_EINVAL, "null d_state or best");
  if (trial_steps < 1) return fail(EQ_EINVAL, "trial_steps must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  eq_run_desc td = *desc;
  td.n_steps = std::min(std::max(desc->n_steps, 1), trial_steps);
  // candidates: the LDS tile kernel at every replication count per workgroup that fits, and
  // the sweep kernel
  // (kernel, tile_reps, block)
  std::vector<std::array<int, 3>> cands;
  const long long per_item = desc->scheme == EQ_BACKWARD ? 20 : 16;
  for (int R = 1; R <= 64 && R <= 2 * desc->reps; R <<= 1)
    if ((long long)net->n * R * per_item <= kLdsBudget) cands.push_back({EQ_KERNEL_TILE, R, 0});
  for (int blk : {64, 128, 256}) cands.push_back({EQ_KERNEL_SWEEP, 0, blk});
  float best_ms = 0.0f;
  int bi = -1;
  for (size_t c = 0; c < cands.size(); ++c) {
    td.kernel = cands[c][0];
    td.tile_reps = cands[c][1];
    td.block = cands[c][2];
    if ((rc = run_sim(net, &td, nullptr, d_state, nullptr, nullptr, st))) return rc;   // warm-up
    float ms = 0.0f;
    rc = time_on_stream(st, [&] { return run_sim(net, &td, nullptr, d_state, nullptr, nullptr, st); }, &ms);
    if (rc) return rc;
    if (bi < 0 || ms < best_ms) { best_ms = ms; bi = (int)c; }
  }
  *best = *desc;
  best->kernel = cands[bi][0];
  best->tile_reps = cands[bi][1];
  best->block = cands[bi][2];
  return eq_sim_check(net, stream);
}

int eq_stats_reduce(const eq_net *net, const eq_run_desc *desc, const int64_t *d_sums,
                    const int32_t *d_state, const int32_t *d_init, double *d_out, void *stream) {
  if (!net || !desc || !d_sums || !d_state || !d_out) return fail(EQ_EINVAL, "null argument");
  if (desc->reps < 1 || desc->n_steps < 0 || !(desc->dt > 0.0f)) return fail(EQ_EINVAL, "bad run descriptor");
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  hipError_t e = eq::launch_stats(reinterpret_cast<const long long *>(d_sums), d_state, nullptr, nullptr, d_init,
                                  net->n, desc->reps, desc->n_steps, desc->dt, d_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stats launch");
  return EQ_OK;
}

int eq_sim_run_pair(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state_b,
                    int32_t *d_state_f, int64_t *d_sums_b, int64_t *d_sums_f, void *stream) {
  eq_run_desc fd;
  if (desc) { fd = *desc; fd.scheme = EQ_FORWARD; fd.kernel = EQ_KERNEL_AUTO; }
  int rc = check_desc(net, desc ? &fd : nullptr);
  if (rc) return rc;
  if (!d_state_b || !d_state_f || d_state_b == d_state_f) return fail(EQ_EINVAL, "need two distinct state buffers");
  if ((d_sums_b == nullptr) != (d_sums_f == nullptr) || (d_sums_b && d_sums_b == d_sums_f))
    return fail(EQ_EINVAL, "give both or neither statistics buffers, distinct");
  if (d_init && (d_init == d_state_b || d_init == d_state_f)) return fail(EQ_EINVAL, "d_init must not alias a state");
  if ((rc = ensure_net_device(*net, desc->dt, desc->n_steps))) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  const long long slots_b = ring_slots(*net, EQ_BACKWARD), slots_f = ring_slots(*net, EQ_FORWARD);
  const size_t ws = (size_t)((slots_b + slots_f) * desc->reps) * sizeof(int32_t);
  if (ws > net->ws_cap) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    (void)hipFree(net->d_ws);
    net->d_ws = nullptr;
    net->ws_cap = 0;
    if ((e = hipMalloc((void **)&net->d_ws, ws)) != hipSuccess)
      return fail(EQ_ENOMEM, "workspace of %zu bytes: %s", ws, hipGetErrorString(e));
    net->ws_cap = ws;
  }
  eq_run_desc bd = fd;
  bd.scheme = EQ_BACKWARD;
  int *ring_b = net->d_ws, *ring_f = net->d_ws + slots_b * desc->reps;
  eq::PairArgs a;
  std::memset(&a, 0, sizeof a);
  a.vb = make_view(*net, bd, d_state_b, ring_b, reinterpret_cast<long long *>(d_sums_b));
  a.vf = make_view(*net, fd, d_state_f, ring_f, reinterpret_cast<long long *>(d_sums_f));
  a.flags = net->d_flags;
  a.dep_mode = desc->dep_mode;
  a.dt = desc->dt;
  const long long nstate = (long long)net->n * desc->reps;
  const long long nsums = d_sums_b ? 3LL * net->n * a.vb.stiles : 0;
  if ((e = eq::launch_sweep_init(d_state_b, d_init, nstate, ring_b, slots_b * desc->reps, a.vb.tsums, nsums, st)) !=
          hipSuccess ||
      (e = eq::launch_sweep_init(d_state_f, d_init, nstate, ring_f, slots_f * desc->reps, a.vf.tsums, nsums, st)) !=
          hipSuccess)
    return hip_fail(e, "init launch");
  const int iters = desc->n_steps > 0 ? desc->n_steps + a.vf.extra : 0;
  const int wpb = desc->block >= 64 && desc->block <= 256 ? desc->block / 64 : kSweepWavesPerBlock;
  for (int it = 1; it <= iters; ++it) {
    a.iter = it;
    if ((e = eq::launch_sweep_pair(a, wpb, st)) != hipSuccess) return hip_fail(e, "pair launch");
  }
  eq::SweepArgs fin;
  std::memset(&fin, 0, sizeof fin);
  fin.v = a.vb;
  fin.flags = net->d_flags;
  if ((e = eq::launch_sweep_finish(fin, 0, wpb, st)) != hipSuccess) return hip_fail(e, "finish launch");
  return EQ_OK;
}

int eq_stats_reduce_pair(const eq_net *net, const eq_run_desc *desc, const int64_t *d_sums_b,
                         const int64_t *d_sums_f, const int32_t *d_state_b, const int32_t *d_state_f,
                         const int32_t *d_init, double *d_out, void *stream) {
  if (!net || !desc || !d_sums_b || !d_sums_f || !d_state_b || !d_state_f || !d_out)
    return fail(EQ_EINVAL, "null argument");
  if (desc->reps < 1 || desc->n_steps < 0 || !(desc->dt > 0.0f)) return fail(EQ_EINVAL, "bad run descriptor");
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  hipError_t e = eq::launch_stats(reinterpret_cast<const long long *>(d_sums_b), d_state_b,
                                  reinterpret_cast<const long long *>(d_sums_f), d_state_f, d_init, net->n,
                                  desc->reps, desc->n_steps, desc->dt, d_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stats launch");
  return EQ_OK;
}

int eq_sim_check(eq_net *net, void *stream) {
  if (!net) return fail(EQ_EINVAL, "null network");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (!net->d_flags) return EQ_OK;
  unsigned flags = 0;
  if ((e = hipMemcpy(&flags, net->d_flags, sizeof flags, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "read flags");
  if (flags) {
    if ((e = hipMemset(net->d_flags, 0, sizeof(unsigned))) != hipSuccess) return hip_fail(e, "clear flags");
    return fail(EQ_EOVERFLOW, "device flags 0x%x: %s%s%s", flags, (flags & 1u) ? "state at 2^27 or stream budget; " : "",
                (flags & 2u) ? "sampler retry cap; " : "",
                (flags & 4u) ? "a draw outside the samplers' exact fp32 range" : "");
  }
  return EQ_OK;
}

int eq_selftest_math(int32_t kind, const float *d_x, float *d_y, int64_t count, void *stream) {
  if (kind < 0 || kind > 4 || count < 0 || (count > 0 && (!d_x || !d_y))) return fail(EQ_EINVAL, "bad arguments");
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  hipError_t e = eq::launch_selftest_math(kind, d_x, d_y, count, (hipStream_t)stream);
  return e == hipSuccess ? EQ_OK : hip_fail(e, "selftest launch");
}

int eq_selftest_sample(int32_t kind, int64_t count, uint64_t seed, uint32_t rep0, uint32_t station,
                       uint32_t step0, uint32_t sub, int32_t i0, int32_t i1, float f0, float f1,
                       float f2, float f3, float *d_out, void *stream) {
  if (kind < 0 || kind > 4 || count < 0 || (count > 0 && !d_out) || sub > 255) return fail(EQ_EINVAL, "bad arguments");
  if ((kind == 2 && i0 < 1) || (kind == 3 && i1 < 1)) return fail(EQ_EINVAL, "bad sampler parameters");
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  unsigned *dflags = nullptr;
  hipError_t e = hipMalloc((void **)&dflags, sizeof(unsigned));
  if (e != hipSuccess) return fail(EQ_ENOMEM, "flag allocation");
  (void)hipMemsetAsync(dflags, 0, sizeof(unsigned), (hipStream_t)stream);
  e = eq::launch_selftest_sample(kind, count, (uint32_t)seed, (uint32_t)(seed >> 32), rep0, station, step0, sub,
                                 i0, i1, f0, f1, f2, f3, d_out, dflags, (hipStream_t)stream);
  unsigned flags = 0;
  hipError_t e2 = hipMemcpyAsync(&flags, dflags, sizeof flags, hipMemcpyDeviceToHost, (hipStream_t)stream);
  hipError_t e3 = hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(dflags);
  if (e != hipSuccess) return hip_fail(e, "selftest launch");
  if (e2 != hipSuccess || e3 != hipSuccess) return hip_fail(e2 != hipSuccess ? e2 : e3, "selftest sync");
  if (flags) return fail(EQ_EOVERFLOW, "sampler flags 0x%x", flags);
  return EQ_OK;
}

int eq_selftest_score(int32_t kind, int64_t count, uint64_t seed, uint32_t rep0, uint32_t station,
                      uint32_t step0, uint32_t sub, int32_t x, int32_t m, float f0, float f1, float *d_value,
                      float *d_score, void *stream) {
  if ((kind != 0 && kind != 3 && kind != 4) || count < 0 || (count > 0 && (!d_value || !d_score)) || sub > 255)
    return fail(EQ_EINVAL, "bad arguments");
  if (kind != 0 && (m < 1 || !(f0 > 0.0f) || !(f1 > 0.0f))) return fail(EQ_EINVAL, "bad sampler parameters");
  if (kind == 0 && !(f0 > 0.0f)) return fail(EQ_EINVAL, "lambda0 must be > 0");
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  // the constants a network's tables would hold for (mu = f0, dt = f1, m servers)
  const double mud = (double)f0, dtd = (double)f1;
  const float pdep = (float)(-std::expm1(-(mud * dtd)));
  const float rate = (float)((double)m * mud);
  const float mudt = (float)(mud * dtd);
  const float kap = (float)(dtd * std::exp(-(mud * dtd)) / -std::expm1(-(mud * dtd)));
  unsigned *dflags = nullptr;
  hipError_t e = hipMalloc((void **)&dflags, sizeof(unsigned));
  if (e != hipSuccess) return fail(EQ_ENOMEM, "flag allocation");
  (void)hipMemsetAsync(dflags, 0, sizeof(unsigned), (hipStream_t)stream);
  e = eq::launch_selftest_score(kind, count, (uint32_t)seed, (uint32_t)(seed >> 32), rep0, station, step0, sub, x,
                                m, f0, f1, pdep, rate, mudt, kap, d_value, d_score, dflags, (hipStream_t)stream);
  unsigned flags = 0;
  hipError_t e2 = hipMemcpyAsync(&flags, dflags, sizeof flags, hipMemcpyDeviceToHost, (hipStream_t)stream);
  hipError_t e3 = hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(dflags);
  if (e != hipSuccess) return hip_fail(e, "selftest launch");
  if (e2 != hipSuccess || e3 != hipSuccess) return hip_fail(e2 != hipSuccess ? e2 : e3, "selftest sync");
  if (flags) return fail(EQ_EOVERFLOW, "sampler flags 0x%x", flags);
  return EQ_OK;
}

int eq_selftest_valu_peak(int32_t grid, int32_t iters, float *d_out, void *stream) {
  if (grid < 1 || iters < 1 || !d_out) return fail(EQ_EINVAL, "bad arguments");
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  hipError_t e = eq::launch_valu_peak(d_out, grid, iters, (hipStream_t)stream);
  return e == hipSuccess ? EQ_OK : hip_fail(e, "peak launch");
}

int eq_selftest_philox(int64_t count, const uint32_t *d_ctr, const uint32_t *d_key, uint32_t *d_out,
                       void *stream) {
  if (count < 0 || (count > 0 && (!d_ctr || !d_key || !d_out))) return fail(EQ_EINVAL, "bad arguments");
  int dev = 0;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  hipError_t e = eq::launch_selftest_philox(count, d_ctr, d_key, d_out, (hipStream_t)stream);
  return e == hipSuccess ? EQ_OK : hip_fail(e, "selftest launch");
}

}  // extern "C"

// ---- batches of networks (row a8) ---------------------------------------------------------
struct eq_batch {
  std::vector<eq_net *> nets;
  int device = -1;
  eq::BatchNet *d_nets = nullptr;
  int *d_ws = nullptr;
  size_t ws_cap = 0;
  // waves per block picked by eq_batch_tune for (scheme, dep_mode, reps)
  std::vector<std::array<int, 4>> tuned;
  // cached instantiated graph of the last run shape
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<int64_t> gkey;
  // the descriptors in d_nets may be read by work still queued (a run without a graph on a
  // stream the library does not wait on): set by every enqueue, cleared by a synchronisation
  bool nets_in_use = false;

  ~eq_batch() { release(); }
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    gkey.clear();
  }
  void release() {
    if (device >= 0) (void)hipDeviceSynchronize();   // a replay may still be running
    drop_graph();
    if (device >= 0) {
      (void)hipFree(d_nets);
      (void)hipFree(d_ws);
    }
    d_nets = nullptr;
    d_ws = nullptr;
    ws_cap = 0;
    device = -1;
  }
};

namespace {

// Without tuning, one wavefront per workgroup: on uneven batches the finest grain balances
// the CUs best (measured on 512 networks of 10..2000 stations).
constexpr int kDefaultWavesPerBlock = 1;

int check_batch_desc(const eq_batch *b, const eq_batch_desc *d) {
  if (!b || !d) return fail(EQ_EINVAL, "null batch or descriptor");
  if (d->scheme != EQ_BACKWARD && d->scheme != EQ_FORWARD) return fail(EQ_EINVAL, "scheme %d", d->scheme);
  if (d->dep_mode != EQ_DEP_EXACT && d->dep_mode != EQ_DEP_NAIVE) return fail(EQ_EINVAL, "dep_mode %d", d->dep_mode);
  if (!(d->dt > 0.0f) || !std::isfinite(d->dt)) return fail(EQ_EINVAL, "dt must be finite and > 0");
  if (d->reps < 1) return fail(EQ_EINVAL, "reps must be >= 1");
  const int w = d->waves_per_block;
  if (w != 0 && w != 1 && w != 2 && w != 4 && w != 8 && w != 16)
    return fail(EQ_EINVAL, "waves_per_block must be 0, 1, 2, 4, 8 or 16");
  if (d->scheme == EQ_FORWARD)
    for (size_t k = 0; k < b->nets.size(); ++k)
      if (!b->nets[k]->index_dag) return fail(EQ_ENOTDAG, "network %zu: forward scheme needs an index-ordered DAG", k);
  return EQ_OK;
}

}  // namespace

extern "C" {

int eq_batch_create(int32_t count, eq_net *const *nets, eq_batch **out) {
  if (!out) return fail(EQ_EINVAL, "out is null");
  *out = nullptr;
  if (count < 1 || !nets) return fail(EQ_EINVAL, "count must be >= 1 and nets non-null");
  for (int32_t k = 0; k < count; ++k)
    if (!nets[k]) return fail(EQ_EINVAL, "nets[%d] is null", k);
  // a network's device tables exist for one (h, K) at a time, so a handle may appear once
  try {
    std::vector<eq_net *> seen(nets, nets + count);
    std::sort(seen.begin(), seen.end());
    for (size_t k = 1; k < seen.size(); ++k)
      if (seen[k] == seen[k - 1]) return fail(EQ_EINVAL, "a network handle appears more than once in the batch");
  } catch (...) {
    return fail(EQ_ENOMEM, "host allocation");
  }
  eq_batch *b = new (std::nothrow) eq_batch();
  if (!b) return fail(EQ_ENOMEM, "host allocation");
  b->nets.assign(nets, nets + count);
  *out = b;
  return EQ_OK;
}

void eq_batch_destroy(eq_batch *b) { delete b; }

int eq_batch_layout(const eq_batch *b, int32_t reps, int64_t *state_off, int64_t *sums_off) {
  if (!b || reps < 1) return fail(EQ_EINVAL, "null batch or reps < 1");
  const int64_t tiles = eq::stat_tiles(reps);
  int64_t so = 0, mo = 0;
  for (size_t k = 0; k < b->nets.size(); ++k) {
    if (state_off) state_off[k] = so;
    if (sums_off) sums_off[k] = mo;
    so += (int64_t)b->nets[k]->n * reps;
    mo += 3 * (int64_t)b->nets[k]->n * tiles;
  }
  if (state_off) state_off[b->nets.size()] = so;
  if (sums_off) sums_off[b->nets.size()] = mo;
  return EQ_OK;
}

int eq_batch_run(eq_batch *b, const eq_batch_desc *d, const int32_t *n_steps, const uint32_t *net_ids,
                 int32_t *d_states, int64_t *d_sums, void *stream) {
  int rc = check_batch_desc(b, d);
  if (rc) return rc;
  const size_t count = b->nets.size();
  if (!n_steps || !net_ids || !d_states) return fail(EQ_EINVAL, "null n_steps, net_ids or d_states");
  for (size_t k = 0; k < count; ++k)
    if (n_steps[k] < 0) return fail(EQ_EINVAL, "n_steps[%zu] < 0", k);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  // device tables of every network for its (dt, K)
  for (size_t k = 0; k < count; ++k)
    if ((rc = ensure_net_device(*b->nets[k], d->dt, n_steps[k]))) return rc;
  int dev = 0;
  if ((rc = ensure_device(&dev))) return rc;
  if (b->device != dev) {
    b->release();
    b->device = dev;
  }
  // layout: outputs (caller buffers) and inflow slots (batch workspace)
  std::vector<int64_t> state_off(count + 1), sums_off(count + 1), ws_off(count + 1, 0);
  eq_batch_layout(b, d->reps, state_off.data(), sums_off.data());
  for (size_t k = 0; k < count; ++k) ws_off[k + 1] = ws_off[k] + ring_slots(*b->nets[k], d->scheme) * d->reps;
  const size_t ws = (size_t)ws_off[count] * sizeof(int32_t);
  if (ws > b->ws_cap) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    b->drop_graph();
    (void)hipFree(b->d_ws);
    b->d_ws = nullptr;
    b->ws_cap = 0;
    if ((e = hipMalloc((void **)&b->d_ws, std::max<size_t>(ws, 4))) != hipSuccess)
      return fail(EQ_ENOMEM, "batch workspace of %zu bytes: %s", ws, hipGetErrorString(e));
    b->ws_cap = std::max<size_t>(ws, 4);
  }
  // networks sorted by launches needed, longest first: the running ones form a prefix
  std::vector<eq::BatchNet> bn(count);
  std::vector<int> launches(count);
  for (size_t k = 0; k < count; ++k) {
    eq_run_desc rd;
    std::memset(&rd, 0, sizeof rd);
    rd.scheme = d->scheme; rd.dep_mode = d->dep_mode; rd.dt = d->dt; rd.n_steps = n_steps[k];
    rd.seed = d->seed; rd.net_id = net_ids[k]; rd.rep0 = 0; rd.reps = d->reps;
    bn[k].v = make_view(*b->nets[k], rd, d_states + state_off[k], b->d_ws + ws_off[k],
                        d_sums ? reinterpret_cast<long long *>(d_sums) + sums_off[k] : nullptr);
    launches[k] = n_steps[k] > 0 ? n_steps[k] + bn[k].v.extra : 0;
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return launches[x] > launches[y]; });
  std::vector<eq::BatchNet> sorted(count);
  std::vector<int64_t> prefix(count + 1, 0);
  for (size_t i = 0; i < count; ++i) {
    sorted[i] = bn[order[i]];
    sorted[i].task0 = prefix[i];
    prefix[i + 1] = prefix[i] + (int64_t)sorted[i].v.n * sorted[i].v.tiles;
  }
  int wpb = d->waves_per_block;
  if (!wpb) {
    wpb = kDefaultWavesPerBlock;
    for (const auto &t : b->tuned)
      if (t[0] == d->scheme && t[1] == d->dep_mode && t[2] == d->reps) wpb = t[3];
  }
  // graph cache key: everything that shapes the launches or their arguments
  std::vector<int64_t> key = {d->scheme, d->dep_mode, (int64_t)bits_of(d->dt), (int64_t)d->seed, d->reps, wpb,
                              (int64_t)(intptr_t)d_states, (int64_t)(intptr_t)d_sums, (int64_t)(intptr_t)b->d_ws};
  for (size_t k = 0; k < count; ++k) {
    key.push_back(n_steps[k]);
    key.push_back(net_ids[k]);
    key.push_back((int64_t)b->nets[k]->tables_gen);   // tables rebuilt: new pointers and contents
  }
  const bool replay = d->use_graph && b->gexec && key == b->gkey;
  if (!replay) {
    if (b->gexec || b->nets_in_use) {
      // a replay or an earlier run (on any stream) may still read the descriptors
      if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      b->drop_graph();
      b->nets_in_use = false;
    }
    if (!b->d_nets && (e = hipMalloc((void **)&b->d_nets, sizeof(eq::BatchNet) * count)) != hipSuccess)
      return fail(EQ_ENOMEM, "batch descriptor allocation");
    if ((e = hipMemcpy(b->d_nets, sorted.data(), sizeof(eq::BatchNet) * count, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "upload batch descriptors");
  }
  eq::BatchArgs a;
  std::memset(&a, 0, sizeof a);
  a.nets = b->d_nets;
  a.dep_mode = d->dep_mode;
  a.dt = d->dt;
  a.flags = b->nets[0]->d_flags;
  const int max_launch = count ? launches[order[0]] : 0;
  auto enqueue = [&](hipStream_t s) -> hipError_t {
    hipError_t err = eq::launch_sweep_init(d_states, nullptr, state_off[count], b->d_ws, ws_off[count],
                                           reinterpret_cast<long long *>(d_sums), d_sums ? sums_off[count] : 0, s);
    if (err != hipSuccess) return err;
    size_t active = count;
    for (int it = 1; it <= max_launch; ++it) {
      while (active > 0 && launches[order[active - 1]] < it) --active;
      a.count = (int)active;
      a.iter = it;
      if ((err = eq::launch_batch_step(a, prefix[active], d->scheme, wpb, s)) != hipSuccess) return err;
    }
    if (d->scheme == EQ_BACKWARD) {
      a.count = (int)count;
      a.iter = 0;
      if ((err = eq::launch_batch_finish(a, prefix[count], wpb, s)) != hipSuccess) return err;
    }
    return hipSuccess;
  };
  if (!d->use_graph) {
    b->nets_in_use = true;
    if ((e = enqueue(st)) != hipSuccess) return hip_fail(e, "batch launch");
    return EQ_OK;
  }
  if (!replay) {
    hipStream_t cs = nullptr;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "capture stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e1 = enqueue(cs);
      hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
      e = e1 != hipSuccess ? e1 : e2;
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) { b->drop_graph(); return hip_fail(e, "graph capture"); }
    if ((e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
      b->drop_graph();
      return hip_fail(e, "graph instantiate");
    }
    b->gkey = key;
  }
  if ((e = hipGraphLaunch(b->gexec, st)) != hipSuccess) return hip_fail(e, "graph launch");
  return EQ_OK;
}

int eq_batch_tune(eq_batch *b, const eq_batch_desc *d, const int32_t *n_steps, const uint32_t *net_ids,
                  float trial_fraction, int32_t *d_states, int64_t *d_sums, void *stream, int32_t *best) {
  int rc = check_batch_desc(b, d);
  if (rc) return rc;
  if (!n_steps || !net_ids || !d_states) return fail(EQ_EINVAL, "null n_steps, net_ids or d_states");
  if (!(trial_fraction > 0.0f && trial_fraction <= 1.0f)) return fail(EQ_EINVAL, "trial_fraction must be in (0, 1]");
  const size_t count = b->nets.size();
  std::vector<int32_t> trial(count);
  for (size_t k = 0; k < count; ++k) {
    if (n_steps[k] < 0) return fail(EQ_EINVAL, "n_steps[%zu] < 0", k);
    trial[k] = n_steps[k] ? std::max<int32_t>(1, (int32_t)std::ceil((double)n_steps[k] * trial_fraction)) : 0;
  }
  hipStream_t st = (hipStream_t)stream;
  eq_batch_desc td = *d;
  td.use_graph = 0;
  float best_ms = 0.0f;
  int best_w = 0;
  for (int w : {1, 2, 4, 8, 16}) {
    td.waves_per_block = w;
    if ((rc = eq_batch_run(b, &td, trial.data(), net_ids, d_states, d_sums, stream))) return rc;   // warm-up
    float ms = 0.0f;
    rc = time_on_stream(st, [&] { return eq_batch_run(b, &td, trial.data(), net_ids, d_states, d_sums, stream); },
                        &ms);
    if (rc) return rc;
    if (!best_w || ms < best_ms) { best_ms = ms; best_w = w; }
  }
  for (auto &t : b->tuned)
    if (t[0] == d->scheme && t[1] == d->dep_mode && t[2] == d->reps) t[3] = best_w;
  bool have = false;
  for (const auto &t : b->tuned) have |= t[0] == d->scheme && t[1] == d->dep_mode && t[2] == d->reps;
  if (!have) b->tuned.push_back({d->scheme, d->dep_mode, d->reps, best_w});
  if (best) *best = best_w;
  return eq_batch_check(b, stream);
}

int eq_batch_check(eq_batch *b, void *stream) {
  if (!b) return fail(EQ_EINVAL, "null batch");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (eq_net *n : b->nets) {
    int rc = eq_sim_check(n, stream);
    if (rc) return rc;
  }
  return EQ_OK;
}

}  // extern "C"

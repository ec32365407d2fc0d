// eq_internal.h -- types shared between the kernels and the host side of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eq {

constexpr int kRcpTabHost = 256;   // entries fp32(1/(i+1)), i = 0..255, of the sampler table
constexpr int kStateLimit = 1 << 27;   // states at or above this raise the sticky flag

// Per-station constants of one run (32 bytes, one record load per item).
struct StationParam {
  int c;        // servers m_i
  float mu;     // per-server rate mu_i
  float pdep;   // fp32(1 - exp(-mu_i dt))
  float rate;   // fp32(m_i mu_i)
  float mudt;   // fp32(mu_i dt)   (naive rule)
  float lam0;   // base external rate, 0 if not a source
  int e0, e1;   // CSR edge range of the routing row
};

// Per-station inflow ring of the sweep kernels: `depth` slots starting at slot `off`
// (backward: 2 slots, double buffer; forward: 1 + largest level gap of an edge into the
// station) and the station's lag (forward: its longest-path level; backward: 0).
struct StationRing {
  int off, depth, lag, pad;
};

// Per-station constants of the score runs (likelihood-ratio gradients).
struct ScoreParam {
  float kap;    // fp32(dt e^{-mu dt} / (1 - e^{-mu dt})), the binomial-branch score constant
  int src;      // index of the station in the source list, -1 if it has no external arrivals
};

// Constants of Binomial(., p) that depend on p alone (see binom_prep): the drawn probability
// ph = min(p, 1 - p), ph = 0 for p <= 0 or p >= 1; flip: the result is n minus the draw
// (p > 1/2); r = ph / (1 - ph); lq = ln(1 - ph).
struct BinomP {
  float ph, r, lq;
  int flip;
};

// Routing edge: the multinomial split draws Binomial(rem, q_e) with
// q_e = p_e / (p_exit + sum_{l >= e} p_l), stored as the constants of that binomial.
struct Edge {
  int col2;     // 2 * target station + flip
  float ph, r, lq;
};

struct SimArgs {
  const StationParam *sp;
  const BinomP *dep;       // [n] constants of Binomial(., pdep_i)
  const Edge *edges;
  const float *g;          // [K] integral of the arrival shape over each step
  const int *order;        // stations sorted by level (forward)
  const int *level_ptr;    // [n_levels + 1]
  const int *init;         // [n][reps] or nullptr
  const int *segidx;       // [K] staffing segment of each interval, or nullptr (constant servers)
  const int *seg_m;        // [n_seg][n] servers per segment
  const float *seg_rate;   // [n_seg][n] fp32(m mu) per segment
  int *state;              // [n][reps]
  long long *sums;         // [3][n][tiles] statistics tile sums (kStatReps replications per tile) or nullptr
  unsigned *flags;         // sticky: bit0 state limit / block budget, bit1 retry cap
  int n, K, reps, rep0, R, log2R, items, n_levels, dep_mode, tiles;
  float dt;
  uint32_t k0, k1;
};

// One network as seen by the sweep kernels: device tables, run buffers and sizes.
struct NetView {
  const StationParam *sp;
  const BinomP *dep;       // [n] constants of Binomial(., pdep_i)
  const int *heavy;        // [n] stations by decreasing m_i mu_i (task order within a launch)
  const StationRing *sp2;
  const Edge *edges;
  const float *g;          // [K]
  const int *segidx;       // [K] staffing segment of each interval, or nullptr (constant servers)
  const int *seg_m;        // [n_seg][n]
  const float *seg_rate;   // [n_seg][n]
  int *N;                  // [n][reps] state
  int *ring;               // inflow slots [sum depth][reps]
  long long *tsums;        // [3][n][stiles] statistics tile sums or nullptr
  // score runs only (nullptr otherwise)
  const ScoreParam *scp;   // [n]
  float *smu;              // [n][reps] summed departure scores in mu_i
  float *slam;             // [n_src][reps] summed arrival scores in lambda0_s
  long long *sq;           // [n][reps] sum over tau of (N_tau - m_i)^+
  // path recording (nullptr otherwise): steps rec_t0 .. rec_t0 + rec_len - 1
  int *rec_N, *rec_D;      // [rec_len][n][reps] N_tau, D_tau
  int *rec_R;              // [rec_len][nnz][reps] routed count per edge
  int rec_t0, rec_len, nnz;
  int n, K, reps, rep0, tiles, extra;   // tiles: 64-replication tasks per station; extra:
                                        // launches beyond K (forward: levels - 1)
  int stiles;              // statistics tiles, ceil(reps / kStatReps)
  uint32_t k0, k1;         // Philox key
};

struct SweepArgs {
  NetView v;
  unsigned *flags;
  int iter, dep_mode;
  float dt;
};

// Both schemes of one network in one launch per iteration (average scheme).
struct PairArgs {
  NetView vb, vf;          // backward and forward views (own state, slots, sums)
  unsigned *flags;
  int iter, dep_mode;
  float dt;
};

// Batched sweep: networks sorted by launches needed (K + extra, descending) so that the
// networks still running at a launch are a prefix; task0 is the prefix sum of n * tiles.
struct BatchNet {
  NetView v;
  long long task0;
};

struct BatchArgs {
  const BatchNet *nets;
  int count;               // networks active in this launch (a prefix)
  int iter, dep_mode;
  float dt;
  unsigned *flags;
};

constexpr int kTileReps = 64;   // replications per sweep task (one wavefront)
// Replications per statistics tile: half a wavefront, so that a run of 1024 replications
// has 32 tile means for its standard errors.
constexpr int kStatReps = 32;
__host__ __device__ constexpr int stat_tiles(int reps) { return (reps + kStatReps - 1) / kStatReps; }

hipError_t launch_sweep_init(int *N, const int *init, long long nstate, int *ring, long long nring,
                             long long *tsums, long long nsums, hipStream_t st);
// mode: 0 plain, 1 scores, 2 path recording
hipError_t launch_sweep(const SweepArgs &a, int scheme, int mode, int wpb, hipStream_t st);
hipError_t launch_sweep_finish(const SweepArgs &a, int mode, int wpb, hipStream_t st);
hipError_t launch_zero(void *p, long long words32, hipStream_t st);
hipError_t launch_prep_edges(const int *col, const float *q, Edge *edges, int nnz, hipStream_t st);
hipError_t launch_prep_dep(const StationParam *sp, BinomP *dep, int n, hipStream_t st);
hipError_t launch_cost(const double *hold, const long long *sumq, int n, int reps, int K, double *f,
                       double *mean_se, hipStream_t st);
hipError_t launch_grad(const double *f, const double *mean_se, const float *score, int reps, int n_par,
                       double *grad, double *se, hipStream_t st);
hipError_t launch_sweep_pair(const PairArgs &a, int wpb, hipStream_t st);
// Reachability-pruned gradient: reach [n_par][n] bytes, workspace of grad_reach_workspace_bytes.
size_t grad_reach_workspace_bytes(int n, int n_par, int reps);
hipError_t launch_grad_reach(const unsigned char *reach, const double *hold, const long long *sumq,
                             const float *score, int n, int n_par, int reps, int K, double *ws, double *grad,
                             double *se, hipStream_t st);

// Sojourn sampling over a recorded path (Algorithm 4).
struct SojournArgs {
  const StationParam *sp;
  const Edge *edges;
  const int *segidx, *seg_m;            // staffing, or nullptr
  const int *rec_N, *rec_D, *rec_R;     // as in NetView
  const int *i0, *tau0;                 // [n_samples]
  int *out;                             // [n_samples][reps] sojourn in intervals, -1 if censored
  int n, nnz, reps, rep0, rec_t0, rec_len, n_samples, scheme;
  uint32_t k0, k1;
};
hipError_t launch_sojourn(const SojournArgs &a, hipStream_t st);
hipError_t launch_batch_step(const BatchArgs &a, long long tasks, int scheme, int waves_per_block, hipStream_t st);
hipError_t launch_batch_finish(const BatchArgs &a, long long tasks, int waves_per_block, hipStream_t st);
hipError_t upload_sampler_tables(const float *rcp, const float *fc);

// Scratch of the allocation-free run entry point: a static device array of this many bytes
// (the sweep kernels' inflow slots).  setup_noalloc_scratch takes its address on device `dev`
// (current) once; noalloc_scratch returns it (nullptr before set-up).
constexpr long long kNoAllocScratchBytes = 64ll << 20;
hipError_t setup_noalloc_scratch(int dev);
int *noalloc_scratch(int dev);
hipError_t launch_backward(const SimArgs &a, int grid, int block, size_t lds, hipStream_t st);
hipError_t launch_forward(const SimArgs &a, int grid, int block, size_t lds, hipStream_t st);
hipError_t launch_stats(const long long *tsums, const int *state, const long long *tsums2,
                        const int *state2, const int *init, int n, int reps, int K, float dt, double *out,
                        hipStream_t st);
hipError_t launch_selftest_math(int kind, const float *x, float *y, long long count, hipStream_t st);
hipError_t launch_selftest_sample(int kind, long long count, uint32_t k0, uint32_t k1, uint32_t rep0,
                                  uint32_t station, uint32_t step0, uint32_t sub, int i0, int i1,
                                  float f0, float f1, float f2, float f3, float *out,
                                  unsigned *dflags, hipStream_t st);
hipError_t launch_selftest_score(int kind, long long count, uint32_t k0, uint32_t k1, uint32_t rep0,
                                 uint32_t station, uint32_t step0, uint32_t sub, int x, int m, float f0,
                                 float f1, float pdep, float rate, float mudt, float kap, float *val,
                                 float *score, unsigned *dflags, hipStream_t st);
hipError_t launch_valu_peak(float *out, int grid, int iters, hipStream_t st);
hipError_t launch_selftest_philox(long long count, const uint32_t *ctr, const uint32_t *key,
                                  uint32_t *out, hipStream_t st);

}  // namespace eq

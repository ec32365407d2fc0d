/*
 * eulerq.h -- C ABI of the MI355X (gfx950) Euler-approximation simulator for Markovian
 * queueing networks (Hong, Song & Wang, "Fast Discrete-Event Simulation of Markovian
 * Queueing Networks through Euler Approximation").
 *
 * Model (Section 2.2, Assumption 2): n stations; station i has m_i servers of exponential
 * rate mu_i; a customer finishing service at i moves to j with probability p_ij or leaves
 * with probability 1 - sum_j p_ij; station s in the source set receives Poisson arrivals at
 * rate lambda_s(t) = lambda0_s * shape(t).
 *
 * Method: time step h (called dt here), step tau covers ((tau-1) dt, tau dt].
 *   Backward scheme (Section 2.2, Algorithm 1): D_tau = GenerateDeparture(N_{tau-1}) at every
 *     station, departures split multinomially over the routing row, and external and internal
 *     arrivals are added at the end of the interval.
 *   Forward scheme (Section 2.2, Algorithm 2 generalised node-by-node to a DAG): arrivals of
 *     the interval are present at its start; D_tau = GenerateDeparture(N_{tau-1} + A^ex + A^in)
 *     in topological order.
 *   GenerateDeparture is the exact pure-departure sampler (Lemma 1, Algorithm 3); the naive
 *   rule of Eq. (1) is available as EQ_DEP_NAIVE.
 *
 * Randomness is counter-based (Philox4x32-10): every draw is a function of
 * (seed, net_id, replication, station, step, substream), so results do not depend on launch
 * shape, replication sharding or execution order.  Counter (replication, station, step - 1,
 * substream << 24 | block), key (low word of seed, high word of seed XOR net_id); substreams
 * 0 external arrivals, 1 departures, 2 routing, 3 sojourn sampling (counter (replication,
 * sample, 0, 3 << 24 | block)); the four output words are used in order, then the block
 * advances.
 *
 * Conventions: every function returns EQ_OK (0) or a negative EQ_E* code; the message of the
 * last failure on the calling thread is available from eq_last_error().  Arrays passed by
 * the caller are only read during the call (the library copies what it keeps).  Pointers
 * documented as "device" are HIP device allocations owned by the caller (for example torch
 * tensors' data_ptr()); the library never frees them.  "stream" is a hipStream_t (NULL =
 * default stream); asynchronous calls enqueue work and return.  A handle must not be used by
 * two threads at once; distinct handles may.  No C++ exception crosses this interface.
 */
#ifndef EULERQ_H
#define EULERQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    EQ_OK = 0,
    EQ_EINVAL = -1,    /* invalid argument (message names it) */
    EQ_ENOTDAG = -2,   /* forward scheme needs every edge i -> j to have j > i */
    EQ_ENOMEM = -3,    /* host or device allocation failed */
    EQ_EDEVICE = -4,   /* HIP runtime error or no gfx950 device */
    EQ_EOVERFLOW = -5  /* sticky device flag: a state reached 2^27, a sampler's retry cap hit, or
                          a draw outside the samplers' exact fp32 range (eq_sim_check) */
};

enum { EQ_BACKWARD = 0, EQ_FORWARD = 1 };
enum { EQ_DEP_EXACT = 0, EQ_DEP_NAIVE = 1 };
enum { EQ_SHAPE_CONST = 0, EQ_SHAPE_SINUSOID = 1, EQ_SHAPE_PIECEWISE = 2 };

/* External arrivals (Section 2.1.1: non-homogeneous Poisson, rate lambda_s(t)):
 * lambda_s(t) = lambda0[k] * shape(t) for s = src[k], with
 *   CONST      shape(t) = 1;
 *   SINUSOID   shape(t) = 1 + amp sin(2 pi t / period + phase), |amp| <= 1, period > 0;
 *   PIECEWISE  shape(t) = knot_shape[k] for knot_t[k] <= t < knot_t[k+1] (the last piece
 *              open-ended), knot_t[0] = 0 strictly increasing, knot_shape >= 0; with
 *              period > 0 the pattern repeats every `period` (all knots inside it), with
 *              period = 0 it does not.
 * A step's arrival mean is lambda0 times the fp64 integral of the shape over the step,
 * rounded to fp32 (for PIECEWISE the pieces' overlaps with the step, summed in time order).
 * src must be strictly increasing station ids; lambda0 >= 0.  Knot arrays are copied. */
typedef struct {
    int32_t n_src;
    const int32_t *src;     /* host [n_src] */
    const float *lambda0;   /* host [n_src] */
    int32_t shape_kind;
    double amp, period, phase;
    int32_t n_knots;            /* PIECEWISE only */
    const double *knot_t;       /* host [n_knots] */
    const double *knot_shape;   /* host [n_knots] */
} eq_arrivals;

typedef struct eq_net eq_net;   /* opaque, library-owned */

/* Create a network.  row_ptr [n+1], col [nnz], prob [nnz] give the routing matrix in CSR
 * form (nnz = row_ptr[n]); servers [n] >= 1; mu [n] > 0.  All host arrays, copied.
 * Errors: EQ_EINVAL for n <= 0, non-monotone row_ptr, col out of range, negative or
 * non-finite prob, a row summing above 1 + 1e-6, servers < 1, mu <= 0, bad arrivals.
 * Builds the host tables (Section 3 quantities: exit probabilities, routing conditionals,
 * topological levels); needs no GPU.  Device copies are made on first use. */
int eq_net_create(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
                  const int32_t *servers, const float *mu, const eq_arrivals *arrivals,
                  eq_net **out);
/* Frees the handle and its device tables and workspace, after a device synchronisation (runs
 * still queued with the handle finish first).  NULL is ignored. */
void eq_net_destroy(eq_net *net);

/* Time-varying staffing (Section 2.1: servers change at chosen times, placed on interval
 * boundaries, constant within an interval; a customer whose server is withdrawn rejoins the
 * queue, so only min(N, m) changes).  Segment k starts at interval index seg_start[k]
 * (0-based tau - 1; seg_start[0] = 0, strictly increasing) and gives station i the servers
 * servers[k * n + i] >= 1; with period > 0 the schedule repeats every `period` intervals
 * (every start < period).  Departures of interval tau use its servers and fp32(m mu); the
 * statistic (N_tau - m)^+ uses the servers of the interval that ends at tau h.  n_seg = 0
 * restores the constant servers.  Copies its inputs; the next run rebuilds the device
 * tables (after a device synchronisation).  EQ_EINVAL on a malformed schedule. */
int eq_net_set_staffing(eq_net *net, int32_t n_seg, const int32_t *seg_start, const int32_t *servers,
                        int32_t period);

/* The model's parameters (Section 2.2: per-server service rates, external arrival rates).
 * Replace the service rates mu [n] (> 0) and/or the base arrival rates lambda0 [n_src] (>= 0,
 * in the order of the arrivals' src list); NULL leaves that set unchanged.  For finite
 * differences and parameter updates without rebuilding the network.  Copies its inputs; the
 * next run rebuilds the device tables (after a device synchronisation).  EQ_EINVAL on an
 * invalid value (nothing is changed then). */
int eq_net_set_params(eq_net *net, const float *mu, const float *lambda0);

/* Host copies of the per-run tables for step dt and K steps (no GPU needed):
 * q [nnz]  conditional routing probabilities p_e / (p_exit + sum_{l >= e} p_l), fp32;
 * pdep [n] 1 - exp(-mu_i dt); rate [n] m_i mu_i; mudt [n] mu_i dt;
 * kap [n]  dt exp(-mu_i dt) / (1 - exp(-mu_i dt)) (score constant of the binomial branch);
 * g [K]    integral of shape(t) over step tau (index tau-1).  Any output may be NULL. */
int eq_net_tables(const eq_net *net, float dt, int32_t K, float *q, float *pdep, float *rate,
                  float *mudt, float *kap, float *g);

/* Longest-path level of every station (level [n], may be NULL); returns the number of levels
 * (>= 1), or EQ_ENOTDAG if some edge does not go to a higher station index. */
int eq_net_levels(const eq_net *net, int32_t *level);

/* One simulation run. */
enum { EQ_KERNEL_AUTO = 0, EQ_KERNEL_TILE = 1, EQ_KERNEL_SWEEP = 2 };

typedef struct {
    int32_t scheme;      /* EQ_BACKWARD or EQ_FORWARD */
    int32_t dep_mode;    /* EQ_DEP_EXACT (Algorithm 3) or EQ_DEP_NAIVE (Eq. (1)) */
    float dt;            /* step h > 0 */
    int32_t n_steps;     /* K >= 0 (horizon T = K dt) */
    uint64_t seed;
    uint32_t net_id;     /* mixed into the Philox key: distinct networks, distinct streams */
    int32_t rep0;        /* global id of the first replication (for sharding) >= 0 */
    int32_t reps;        /* number of replications >= 1 */
    int32_t kernel;      /* EQ_KERNEL_AUTO, _TILE (workgroup-resident state in LDS, one launch;
                            small networks) or _SWEEP (station-coherent wavefronts, state in
                            HBM, one launch per step; any size).  Results do not depend on it. */
    int32_t tile_reps;   /* TILE kernel: 0 = automatic, else replications per workgroup
                            (power of two <= 64) */
    int32_t block;       /* threads per workgroup, 0 = automatic.  TILE kernel: a multiple of 64,
                            <= 1024.  SWEEP kernel: 64 (the automatic choice), 128, 192 or 256;
                            other values are ignored when SWEEP is chosen automatically */
} eq_run_desc;

/* Device bytes of the workspace a run needs (the SWEEP kernel's inflow slots: 2 n reps int32
 * for the backward scheme, sum_j D_j reps int32 for the forward scheme).  The handle owns and
 * reuses this workspace; it grows to the largest run made with the handle (a growth
 * synchronises the device first).  Runs on one handle therefore share it: enqueue them on
 * one stream, or synchronise between runs made on different streams. */
size_t eq_sim_workspace_bytes(const eq_net *net, const eq_run_desc *desc);

/* Replications per statistics tile of the d_sums outputs: tiles = ceil(reps / EQ_STAT_TILE_REPS). */
#define EQ_STAT_TILE_REPS 32

/* Run the scheme on the GPU (asynchronous on `stream`).
 * d_init  device int32 [n][reps] initial state N_0, or NULL for an empty system
 *         (Assumption 1: initially idle).  Must not alias d_state.
 * d_state device int32 [n][reps] (replication index fastest): receives N_K.
 * d_sums  device int64 [3][n][tiles], tiles = ceil(reps / EQ_STAT_TILE_REPS), or NULL: for
 *         every station and tile of 32 consecutive replications of this run (the last tile may
 *         be short), the sums over those replications and over tau = 1..K of N_tau,
 *         (N_tau - m_i)^+ and D_tau.
 * The first call on a network for a given (dt, K) uploads its tables (synchronously).
 * Errors: EQ_EINVAL, EQ_ENOTDAG (forward scheme on a non index-ordered DAG), EQ_ENOMEM,
 * EQ_EDEVICE. */
int eq_sim_run(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state,
               int64_t *d_sums, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): eq_sim_run with the same arguments, results and
 * stream semantics, making no allocation.  The SWEEP kernel's inflow slots live in a static
 * device array of EQ_NOALLOC_SCRATCH_BYTES (64 MiB) that each device holds from the library's
 * first call on it until the process ends; a run needing more (2 n reps int32 for the
 * backward scheme, sum_j D_j reps int32 for the forward scheme; see eq_sim_workspace_bytes)
 * returns EQ_EINVAL.  The TILE kernel needs no scratch.  The network's device tables must
 * already exist for this device, dt and n_steps (one eq_sim_run with the same dt and n_steps
 * builds them), else EQ_EINVAL.  Every call on a device shares that device's array and keeps
 * what the last call left there (each run clears its slots first): calls that overlap on one
 * device, on any streams, race. */
#define EQ_NOALLOC_SCRATCH_BYTES (64ll << 20)
int eq_sim_run_noalloc(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state,
                       int64_t *d_sums, void *stream);

/* The scheme of eq_sim_run (Section 2.2, Algorithms 1-2; Algorithm 3 departures) with the
 * statistics of eq_stats_reduce, as one synchronous call on host buffers.  It allocates the
 * device buffers, runs (eq_sim_run on the default stream), reduces the statistics
 * (eq_stats_reduce), checks the device flags (eq_sim_check) and copies back.  init host int32 [n][reps] or NULL (empty start);
 * final_state host int32 [n][reps] or NULL; stats host double [6][n] (as eq_stats_reduce) or
 * NULL.  For callers without their own device memory; the outputs are those of the
 * asynchronous path.  Errors as eq_sim_run, plus EQ_EOVERFLOW from the flag check. */
int eq_sim_run_host(eq_net *net, const eq_run_desc *desc, const int32_t *init, int32_t *final_state,
                    double *stats);

/* Per-station statistics from a run's outputs (asynchronous, fp64, deterministic order).
 * d_out device double [6][n]: mean N, standard error of mean N, mean queue length (N-m)^+,
 * its standard error, throughput (departures per unit time) and mean waiting time in queue
 * by Little's law, sum (N-m)^+ dt / (number of arrivals), arrivals = N_K - N_0 + sum D.
 * Standard errors treat the 32-replication tiles' time averages as independent samples
 * (weighted by tile size; 0 when the run has a single tile).  With n_steps = 0 the means,
 * standard errors and throughput are 0; the waiting time is 0 where no customer arrived.
 * d_init may be NULL (empty start). */
int eq_stats_reduce(const eq_net *net, const eq_run_desc *desc, const int64_t *d_sums,
                    const int32_t *d_state, const int32_t *d_init, double *d_out, void *stream);

/* Autotuner for one network and run shape: times every candidate launch shape -- the LDS tile
 * kernel at 1, 2, 4, ..., 64 replications per workgroup (those whose tile fits in LDS), and the
 * sweep kernel at 64, 128 and 256 threads per workgroup -- on the first min(n_steps,
 * trial_steps) steps with HIP events on `stream`, and writes the fastest into *best (desc with
 * kernel, tile_reps and block set).  The launch shape never changes results.  d_state device int32
 * [n][reps] is scratch (overwritten).  Synchronous; errors as eq_sim_run. */
int eq_sim_tune(eq_net *net, const eq_run_desc *desc, int32_t trial_steps, int32_t *d_state, void *stream,
                eq_run_desc *best);

/* ---- sample paths and sojourn times (Section 6, Algorithm 4, Lemma 3) ----------------------
 * A recording run is eq_sim_run (same draws, states and statistics; sweep kernel) that also
 * stores, for the steps tau = rec_t0 .. rec_t0 + rec_len - 1 (1 <= rec_t0), the end-of-interval
 * state N_tau, the departures D_tau and the routed count R_{tau,e} of every edge (CSR order):
 *   d_rec_N, d_rec_D  device int32 [rec_len][n][reps],  d_rec_R  device int32 [rec_len][nnz][reps]
 * (caller-owned, overwritten; steps beyond n_steps read 0; d_rec_R may be NULL if nnz = 0). */
int eq_sim_run_record(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state,
                      int64_t *d_sums, int32_t rec_t0, int32_t rec_len, int32_t *d_rec_N, int32_t *d_rec_D,
                      int32_t *d_rec_R, void *stream);

/* Sojourn times of tagged customers over a recorded path (Algorithm 4): sample k is a customer
 * entering node i0[k] during interval tau0[k] (host arrays of n_samples), walked through the
 * record of every replication.  It is the last of the N_tau present at tau h and waits while its
 * position exceeds the servers; in service, interval tau+1 keeps it with the probability of
 * Lemma 3 for the departure base x (N_tau for the backward scheme, N_{tau+1} + D_{tau+1} for the
 * forward; at least 1) and the interval's departures d; on leaving it goes to node j with
 * probability R_{tau+1,i,j} / D_{tau+1,i}, else exits.  Its uniforms are Philox substream 3 of
 * (replication, k).  desc: the recording run's descriptor (scheme, dt, n_steps, seed, net_id,
 * rep0, reps; the record lies within n_steps).  d_out device int32 [n_samples][reps]: the
 * sojourn in intervals, -1 where the walk needs a step outside the record.  Synchronous. */
int eq_sojourn(eq_net *net, const eq_run_desc *desc, int32_t rec_t0, int32_t rec_len, const int32_t *d_rec_N,
               const int32_t *d_rec_D, const int32_t *d_rec_R, int32_t n_samples, const int32_t *i0,
               const int32_t *tau0, int32_t *d_out, void *stream);

/* The average scheme (Section 7: the customer counts of the backward and the forward scheme,
 * run with common random numbers, averaged): both schemes of one network advance in the same
 * launch per step, each with its own state and statistics buffers, exactly as two eq_sim_run
 * calls with desc->scheme = EQ_BACKWARD and EQ_FORWARD would (same seed, hence the same
 * draws).  desc->scheme and desc->kernel are ignored; desc->block 64..256 sets the workgroup
 * size.  The forward scheme needs an index-ordered DAG (EQ_ENOTDAG).  d_sums_b / d_sums_f:
 * both or neither.  Asynchronous on `stream`. */
int eq_sim_run_pair(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state_b,
                    int32_t *d_state_f, int64_t *d_sums_b, int64_t *d_sums_f, void *stream);

/* Statistics of the average scheme from a pair run: as eq_stats_reduce, with each station's
 * sums pooled over both schemes (means over 2K station-steps per replication, standard errors
 * from the pooled tile means, throughput and Little's-law waiting time from pooled departures
 * and arrivals).  d_out device fp64 [6][n]. */
int eq_stats_reduce_pair(const eq_net *net, const eq_run_desc *desc, const int64_t *d_sums_b,
                         const int64_t *d_sums_f, const int32_t *d_state_b, const int32_t *d_state_f,
                         const int32_t *d_init, double *d_out, void *stream);

/* Synchronise `stream`, then read and clear the network's sticky device flags.
 * Returns EQ_OK, EQ_EOVERFLOW (since the last check: a state reached 2^27 -- the statistics
 * partials' headroom --, a stream used 2^24 Philox blocks, a sampler hit its retry cap, or a
 * draw's values passed what fp32 represents exactly: a binomial mode or a Poisson mean of 2^24
 * or more; the run still completes, identically on every path) or EQ_EDEVICE.  States are exact integers throughout;
 * the samplers convert x to fp32, exactly below 2^24 and with identical rounding above it. */
int eq_sim_check(eq_net *net, void *stream);

/* ---- likelihood-ratio gradients ------------------------------------------------------------
 * A score run is eq_sim_run (same draws, same states, same statistics) that also sums, per
 * replication r and in step order, the likelihood-ratio score of every draw it takes: the
 * derivative of the draw's log-density with respect to the parameter that drives it.
 *   arrivals A ~ Poisson(lambda0_s g[tau-1]) (Section 2.1.1):  A / lambda0_s - g[tau-1];
 *   departures, GenerateDeparture (Lemma 1, Algorithm 3), in mu_i:
 *     x <= m: D ~ Binomial(x, 1 - e^{-mu dt}):  D kap - (x - D) dt;
 *     x >  m: the Erlang(x - m, m mu) time T:  (x - m) / mu - m T, and if T <= dt the
 *             completions D' ~ Binomial(m, p2), p2 = 1 - e^{-mu (dt - T)}, add
 *             -(m - D') (dt - T) + D' (dt - T) (1 - p2) / p2  (the split when T > dt is
 *             free of mu);
 *     naive rule, Eq. (1): S / mu - min(x, m) dt for the Poisson draw S.
 *   Routing draws do not depend on mu or lambda0.  Sums are fp32, one add per draw.
 * Buffers (device, caller-owned, overwritten; any contents on entry):
 *   d_sumq      int64 [n][reps]     sum over tau = 1..K of (N_tau,i - m_i)^+
 *   d_score_mu  fp32  [n][reps]     summed departure scores of station i
 *   d_score_lam fp32  [n_src][reps] summed arrival scores of source s (NULL if n_src = 0)
 * Score runs always use the sweep kernel (desc->kernel AUTO or SWEEP).  Other arguments and
 * errors as eq_sim_run. */
int eq_sim_run_scores(eq_net *net, const eq_run_desc *desc, const int32_t *d_init, int32_t *d_state,
                      int64_t *d_sums, int64_t *d_sumq, float *d_score_mu, float *d_score_lam,
                      void *stream);

/* Waiting cost per replication f_r = (sum_i hold_i d_sumq[i][r]) / n_steps (device fp64 [reps]
 * into d_f), and d_mean_se[0] = mean of f, d_mean_se[1] = its standard error (device fp64
 * [2]).  d_hold device fp64 [n].  Fixed summation order.  Asynchronous on `stream`. */
int eq_cost_reduce(int32_t n, int32_t reps, int32_t n_steps, const double *d_hold,
                   const int64_t *d_sumq, double *d_f, double *d_mean_se, void *stream);

/* Likelihood-ratio gradient of E[f]: for each of the n_par score rows j (device fp32
 * [n_par][reps], e.g. the mu rows followed by the lambda0 rows in one buffer),
 * d_grad[j] = sum_r (f_r - mean f) score[j][r] / (reps - 1) and d_se[j] its standard error
 * (sample deviation of the products / sqrt(reps) * reps / (reps - 1)), fp64 in a fixed order.
 * d_f and d_mean_se as written by eq_cost_reduce.  reps >= 2.  Asynchronous on `stream`. */
int eq_grad_reduce(int32_t n_par, int32_t reps, const double *d_f, const double *d_mean_se,
                   const float *d_score, double *d_grad, double *d_se, void *stream);

/* The same gradient with each parameter's score correlated only with the waiting cost of the
 * stations that parameter can influence: for mu_j, station j and every station reachable
 * from it along routing edges; for lambda0 of source s, the source station and the stations
 * reachable from it.  A station outside that set evolves with draws whose laws do not involve
 * the parameter, so dropping its cost leaves the estimate unbiased and removes its noise:
 *   g_j = sum_r (f_{j,r} - mean_r f_{j,r}) S[j][r] / (R - 1),
 *   f_{j,r} = sum_{i reachable from j} hold_i Q[i][r] / K,
 * with its standard error as for eq_grad_reduce, fp64 in a fixed order.  d_hold device double
 * [n], d_sumq device int64 [n][reps], d_score device float [n + n_src][reps] (both as written
 * by eq_sim_run_scores), n_steps = K >= 1, reps >= 2; d_grad, d_se device double
 * [n + n_src].  The network's tables must live on the current device (its score run made
 * them).  The first call builds the reach table on the host and uploads it; the reduction's
 * workspace (about 8 n (n + n_src) + 16 (n + n_src) reps / 64 bytes) is owned by the network
 * and grows as needed.  Asynchronous on `stream`. */
/* The reach table the pruned gradient uses: reach[j][i] = 1 when station i is reachable from
 * parameter j's station along routing edges, itself included (row j < n: station j, the
 * parameter mu_j; row n + s: source s's station, the parameter lambda0_s), else 0.  reach is a
 * host array of (n + n_src) n bytes, or NULL to ask for the row count.  Returns n + n_src, or a
 * negative error code. */
int eq_net_reach(eq_net *net, uint8_t *reach);

int eq_grad_reduce_reach(eq_net *net, int32_t reps, int32_t n_steps, const double *d_hold,
                         const int64_t *d_sumq, const float *d_score, double *d_grad, double *d_se,
                         void *stream);

/* ---- batches of networks ------------------------------------------------------------------
 * Many independent networks of uneven size simulated together: one launch per step covers the
 * station-coherent tasks of every network still running (networks are ordered longest-first so
 * the running ones form a prefix), optionally replayed as a captured hipGraph of the whole step
 * loop.  Network k uses Philox network id net_ids[k], so its results equal those of
 * eq_sim_run on that network alone with the same seed and net_id. */
typedef struct eq_batch eq_batch;   /* opaque; references (does not own) its networks */

/* A batch of `count` distinct network handles (EQ_EINVAL for a null or repeated handle: a
 * network holds device tables for one (h, K) at a time). */
int eq_batch_create(int32_t count, eq_net *const *nets, eq_batch **out);
/* Frees the batch (graph, descriptors, workspace) after a device synchronisation; its
 * networks stay valid.  NULL is ignored. */
void eq_batch_destroy(eq_batch *batch);

typedef struct {
    int32_t scheme, dep_mode;
    float dt;                  /* common step h > 0 */
    uint64_t seed;
    int32_t reps;              /* replications of every network */
    int32_t waves_per_block;   /* 0 = the value eq_batch_tune picked (else 1), or 1, 2, 4, 8, 16 */
    int32_t use_graph;         /* 1: capture the step loop in a hipGraph and replay it (the graph is
                                  cached in the batch and reused while the run shape and buffers
                                  stay the same) */
} eq_batch_desc;

/* Offsets (in elements) of network k's outputs in the concatenated buffers: state_off[k] into
 * int32 [n_k][reps] blocks, sums_off[k] into int64 [3][n_k][tiles] blocks; count + 1 entries
 * each (the last is the total).  Either may be NULL. */
int eq_batch_layout(const eq_batch *batch, int32_t reps, int64_t *state_off, int64_t *sums_off);

/* Run network k for n_steps[k] steps (host arrays of count entries).  d_states (device int32,
 * total from eq_batch_layout) receives every N_K; d_sums (device int64, or NULL) the tile sums.
 * Asynchronous on `stream`.  A run that does not replay the cached graph first waits for the
 * device (an earlier run of the batch, on any stream, may still read the descriptors it
 * replaces); runs of one batch share its workspace, so they must not overlap (the same stream,
 * or a synchronisation between them).  Errors as eq_sim_run. */
int eq_batch_run(eq_batch *batch, const eq_batch_desc *desc, const int32_t *n_steps,
                 const uint32_t *net_ids, int32_t *d_states, int64_t *d_sums, void *stream);

/* Autotuner for the batch: runs it (without a graph) with 1, 2, 4, 8 and 16 wavefronts per
 * workgroup on a shortened horizon -- network k runs ceil(n_steps[k] * trial_fraction) steps,
 * which keeps the mix of long and short networks -- timing each with HIP events, and returns
 * the fastest in *best (may be NULL).  The batch remembers it: later eq_batch_run calls with
 * waves_per_block = 0 and the same scheme, dep_mode and reps use it (untuned default: 1).
 * d_states / d_sums as for eq_batch_run, overwritten.  Synchronous. */
int eq_batch_tune(eq_batch *batch, const eq_batch_desc *desc, const int32_t *n_steps,
                  const uint32_t *net_ids, float trial_fraction, int32_t *d_states, int64_t *d_sums,
                  void *stream, int32_t *best);

/* Synchronise `stream` and read and clear the sticky flags of every network of the batch. */
int eq_batch_check(eq_batch *batch, void *stream);

/* ---- diagnostics: the device building blocks, for parity tests against a reference ---- */

/* y[i] = f(x[i]) with the library's device fp32 function: kind 0 log, 1 log1p, 2 exp,
 * 3 expm1, 4 the uniform (2 (b >> 9) + 1) 2^-24 of the 32-bit word b with the bits of x[i]
 * (the samplers' map from a Philox output word to (0, 1)).  x, y device float [count]. */
int eq_selftest_math(int32_t kind, const float *d_x, float *d_y, int64_t count, void *stream);

/* Draw count samples; sample s uses the uniform stream (rep0 + s, station, step0, sub) with
 * key (seed, net_id = 0).  kind 0 Poisson(f0), 1 Binomial(i0, f0), 2 Gamma(i0) (integer
 * shape), 3 GenerateDeparture(x=i0, m=i1, mu=f0, dt=f1, pdep=f2, rate=f3),
 * 4 naive departures (x=i0, m=i1, mu dt=f0).  d_out device float [count]. */
int eq_selftest_sample(int32_t kind, int64_t count, uint64_t seed, uint32_t rep0,
                       uint32_t station, uint32_t step0, uint32_t sub, int32_t i0, int32_t i1,
                       float f0, float f1, float f2, float f3, float *d_out, void *stream);

/* Draws with their scores, sample s on the stream (rep0 + s, station, step0, sub), key
 * (seed, 0): kind 0 A ~ Poisson(f0 f1), score in lambda0 = f0 (f1 = g); kind 3
 * GenerateDeparture(x, m, mu = f0, dt = f1), kind 4 naive departures (same arguments), score
 * in mu, with the constants pdep, m mu, mu dt and kap made as eq_net_tables makes them.
 * d_value, d_score device float [count]. */
int eq_selftest_score(int32_t kind, int64_t count, uint64_t seed, uint32_t rep0, uint32_t station,
                      uint32_t step0, uint32_t sub, int32_t x, int32_t m, float f0, float f1,
                      float *d_value, float *d_score, void *stream);

/* VALU throughput probe: `grid` workgroups of 256 threads, each thread `iters` x 128
 * independent non-packed fp32 FMAs (8 chains), one float written per thread to d_out
 * (device float [grid * 256]).  Time it with events on `stream`; lane-FMAs = grid * 256 *
 * iters * 128.  Asynchronous. */
int eq_selftest_valu_peak(int32_t grid, int32_t iters, float *d_out, void *stream);

/* Philox4x32-10 blocks: ctr device uint32 [count][4], key device uint32 [count][2],
 * out device uint32 [count][4]. */
int eq_selftest_philox(int64_t count, const uint32_t *d_ctr, const uint32_t *d_key,
                       uint32_t *d_out, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *eq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EULERQ_H */

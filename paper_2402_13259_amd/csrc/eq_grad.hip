// eq_grad.hip -- fp64 reductions of the likelihood-ratio gradient.
//
// A score run leaves, per replication r, the int64 sums Q[i][r] = sum_tau (N_tau,i - m_i)^+
// and the fp32 score sums S[j][r] (j over mu_1..mu_n, then lambda0 of each source).  With
// the waiting cost f_r = sum_i hold_i Q[i][r] / K, the estimate of d E[f] / d theta_j is
// the covariance  g_j = sum_r (f_r - mean f) S[j][r] / (R - 1); every sum here is fp64 in a
// fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include "eq_internal.h"

namespace eq {

constexpr int kRedThreads = 256;

// fixed-order tree sum of one value per thread; every thread gets the total
__device__ double block_sum(double v, double *lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (t < w) lds[t] += lds[t + w];
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

// f_r = (sum_i hold_i Q[i][r]) / K, one thread per replication (rows of Q are read
// coalesced across replications).
__global__ __launch_bounds__(kRedThreads) void k_cost(const double *hold, const long long *sumq, int n, int reps,
                                                       int K, double *f) {
  const int r = blockIdx.x * kRedThreads + threadIdx.x;
  if (r >= reps) return;
  double acc = 0.0;
  for (int i = 0; i < n; ++i) acc += hold[i] * (double)sumq[(long long)i * reps + r];
  f[r] = acc / (double)K;
}

// mean and standard error of f (one workgroup)
__global__ __launch_bounds__(kRedThreads) void k_mean_se(const double *f, int reps, double *mean_se) {
  __shared__ double lds[kRedThreads];
  double a = 0.0;
  for (int r = threadIdx.x; r < reps; r += kRedThreads) a += f[r];
  const double mean = block_sum(a, lds) / (double)reps;
  double b = 0.0;
  for (int r = threadIdx.x; r < reps; r += kRedThreads) {
    const double d = f[r] - mean;
    b += d * d;
  }
  const double ss = block_sum(b, lds);
  if (threadIdx.x == 0) {
    mean_se[0] = mean;
    mean_se[1] = reps > 1 ? sqrt(ss / (double)(reps - 1) / (double)reps) : 0.0;
  }
}

// One workgroup per parameter j: g_j = sum_r p_r / (R - 1) with p_r = (f_r - mean) S[j][r],
// and its standard error sqrt(var(p) / R) * R / (R - 1).
__global__ __launch_bounds__(kRedThreads) void k_grad(const double *f, const double *mean_se, const float *score,
                                                       int reps, double *grad, double *se) {
  __shared__ double lds[kRedThreads];
  const int j = blockIdx.x;
  const double mean = mean_se[0];
  const float *row = score + (long long)j * reps;
  double a = 0.0, b = 0.0;
  for (int r = threadIdx.x; r < reps; r += kRedThreads) {
    const double pr = (f[r] - mean) * (double)row[r];
    a += pr;
    b += pr * pr;
  }
  const double sa = block_sum(a, lds);
  const double sb = block_sum(b, lds);
  if (threadIdx.x == 0) {
    const double R = (double)reps;
    grad[j] = sa / (R - 1.0);
    const double var = (sb - sa * sa / R) / (R - 1.0);
    se[j] = sqrt(var > 0.0 ? var : 0.0) / sqrt(R) * R / (R - 1.0);
  }
}

// ---- reachability-pruned estimator ------------------------------------------------------------
// Parameter j (mu_j for j < n, then lambda0 of each source) is correlated only with the cost of
// the stations it can reach: f_{j,r} = sum_i M[j][i] Q[i][r], M[j][i] = hold_i / K if station i
// is reachable from j (itself included), else 0.  Then p_{j,r} = (f_{j,r} - mean_r f_{j,r}) S[j][r],
// g_j = sum_r p / (R - 1), and its standard error as in k_grad.  mean_r f_{j,r} = sum_i M[j][i]
// mean_r Q[i][r] by linearity.  The contraction over stations is the dense part (n_par x n x R
// multiply-adds): LDS tiles of 64 parameters x 64 replications, 16 stations per stage, 4 x 4
// outputs per thread; per tile, the sums of p and p^2 over its 64 replications go to a buffer
// that a second kernel adds in replication order, so results do not depend on scheduling.
constexpr int kGT = 64;     // parameters and replications per tile
constexpr int kGI = 16;     // stations per LDS stage

__global__ __launch_bounds__(kRedThreads) void k_qmean(const long long *sumq, int reps, double *qmean) {
  __shared__ double lds[kRedThreads];
  const int i = blockIdx.x;
  double a = 0.0;
  for (int r = threadIdx.x; r < reps; r += kRedThreads) a += (double)sumq[(long long)i * reps + r];
  const double t = block_sum(a, lds);
  if (threadIdx.x == 0) qmean[i] = t / (double)reps;
}

// M[j][i] and fbar_j = sum_i M[j][i] qmean_i, one workgroup per parameter
__global__ __launch_bounds__(kRedThreads) void k_reach_weights(const unsigned char *reach, const double *hold,
                                                                const double *qmean, int n, int K, double *M,
                                                                double *fbar) {
  __shared__ double lds[kRedThreads];
  const int j = blockIdx.x;
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += kRedThreads) {
    const double w = reach[(long long)j * n + i] ? hold[i] / (double)K : 0.0;
    M[(long long)j * n + i] = w;
    a += w * qmean[i];
  }
  const double t = block_sum(a, lds);
  if (threadIdx.x == 0) fbar[j] = t;
}

__global__ __launch_bounds__(kRedThreads) void k_grad_reach_tiles(const double *M, const long long *sumq,
                                                                   const float *score, const double *fbar, int n,
                                                                   int n_par, int reps, double *part) {
  __shared__ double Ms[kGI][kGT];          // [station][parameter]
  __shared__ double Qs[kGI][kGT];          // [station][replication]
  __shared__ double red[2][kGT][kGT / 4];  // [sum, sum of squares][parameter][replication group]
  const int tid = threadIdx.x;
  const int tj = tid / 16, tr = tid % 16;  // outputs: parameters 4 tj .. 4 tj + 3, replications 4 tr .. 4 tr + 3
  const int j0 = blockIdx.x * kGT, r0 = blockIdx.y * kGT;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int i0 = 0; i0 < n; i0 += kGI) {
    // stage M[j0..j0+63][i0..i0+15] (transposed) and Q[i0..i0+15][r0..r0+63]: 1024 values each
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = tid + k * kRedThreads;
      const int mi = e % kGI, mj = e / kGI;            // consecutive threads read consecutive stations
      const int gj = j0 + mj, gi = i0 + mi;
      Ms[mi][mj] = (gj < n_par && gi < n) ? M[(long long)gj * n + gi] : 0.0;
      const int qi = e / kGT, qr = e % kGT;            // consecutive threads read consecutive replications
      const int hi = i0 + qi, hr = r0 + qr;
      Qs[qi][qr] = (hi < n && hr < reps) ? (double)sumq[(long long)hi * reps + hr] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int i = 0; i < kGI; ++i) {
      double mv[4], qv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) mv[a] = Ms[i][4 * tj + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) qv[b] = Qs[i][4 * tr + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_fma(mv[a], qv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int j = j0 + 4 * tj + a;
    double s1 = 0.0, s2 = 0.0;
    if (j < n_par) {
      const double fb = fbar[j];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int r = r0 + 4 * tr + b;
        if (r < reps) {
          const double pr = (acc[a][b] - fb) * (double)score[(long long)j * reps + r];
          s1 += pr;
          s2 += pr * pr;
        }
      }
    }
    red[0][4 * tj + a][tr] = s1;
    red[1][4 * tj + a][tr] = s2;
  }
  __syncthreads();
  if (tid < kGT) {
    const int j = j0 + tid;
    double s1 = 0.0, s2 = 0.0;
    for (int g = 0; g < kGT / 4; ++g) {
      s1 += red[0][tid][g];
      s2 += red[1][tid][g];
    }
    if (j < n_par) {
      const long long at = ((long long)j * gridDim.y + blockIdx.y) * 2;
      part[at] = s1;
      part[at + 1] = s2;
    }
  }
}

// one thread per parameter: the tile partials in replication order
__global__ __launch_bounds__(kRedThreads) void k_grad_reach_finish(const double *part, int n_par, int rtiles,
                                                                    int reps, double *grad, double *se) {
  const int j = blockIdx.x * kRedThreads + threadIdx.x;
  if (j >= n_par) return;
  double sa = 0.0, sb = 0.0;
  for (int t = 0; t < rtiles; ++t) {
    sa += part[((long long)j * rtiles + t) * 2];
    sb += part[((long long)j * rtiles + t) * 2 + 1];
  }
  const double R = (double)reps;
  grad[j] = sa / (R - 1.0);
  const double var = (sb - sa * sa / R) / (R - 1.0);
  se[j] = sqrt(var > 0.0 ? var : 0.0) / sqrt(R) * R / (R - 1.0);
}

size_t grad_reach_workspace_bytes(int n, int n_par, int reps) {
  const long long rtiles = (reps + kGT - 1) / kGT;
  return sizeof(double) * ((size_t)n + (size_t)n_par * n + (size_t)n_par + (size_t)n_par * rtiles * 2);
}

hipError_t launch_grad_reach(const unsigned char *reach, const double *hold, const long long *sumq,
                             const float *score, int n, int n_par, int reps, int K, double *ws, double *grad,
                             double *se, hipStream_t st) {
  if (n_par <= 0) return hipSuccess;
  const int rtiles = (reps + kGT - 1) / kGT;
  double *qmean = ws, *M = qmean + n, *fbar = M + (long long)n_par * n, *part = fbar + n_par;
  hipLaunchKernelGGL(k_qmean, dim3(n), dim3(kRedThreads), 0, st, sumq, reps, qmean);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reach_weights, dim3(n_par), dim3(kRedThreads), 0, st, reach, hold, qmean, n, K, M, fbar);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_reach_tiles, dim3((n_par + kGT - 1) / kGT, rtiles), dim3(kRedThreads), 0, st, M, sumq,
                     score, fbar, n, n_par, reps, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_reach_finish, dim3((n_par + kRedThreads - 1) / kRedThreads), dim3(kRedThreads), 0, st,
                     part, n_par, rtiles, reps, grad, se);
  return hipGetLastError();
}

hipError_t launch_cost(const double *hold, const long long *sumq, int n, int reps, int K, double *f,
                       double *mean_se, hipStream_t st) {
  hipLaunchKernelGGL(k_cost, dim3((reps + kRedThreads - 1) / kRedThreads), dim3(kRedThreads), 0, st, hold, sumq,
                     n, reps, K, f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mean_se, dim3(1), dim3(kRedThreads), 0, st, f, reps, mean_se);
  return hipGetLastError();
}

hipError_t launch_grad(const double *f, const double *mean_se, const float *score, int reps, int n_par,
                       double *grad, double *se, hipStream_t st) {
  if (n_par <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad, dim3(n_par), dim3(kRedThreads), 0, st, f, mean_se, score, reps, grad, se);
  return hipGetLastError();
}

}  // namespace eq

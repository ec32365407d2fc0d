// probes.hip -- one kernel per building block of the samplers, for counting the VALU
// instructions the gfx950 build spends on each (tests/isa/op_costs.py).  Compiled to assembly
// only, never launched.  Each block sits between two inline-asm comment markers that also pin
// its inputs and outputs (values in VGPRs are per-lane, values in SGPRs wave-uniform, as in the
// sweep kernel), and __builtin_assume selects one branch of a block that has several.
#include "eq_device.h"

namespace eq {
__constant__ float4 c_rcp4[kRcpTab / 4];
__constant__ float c_fc[10];
}  // namespace eq

using namespace eq;

#define BEGIN(...) asm volatile("; probe begin" : __VA_ARGS__)
#define END(...) asm volatile("; probe end" ::__VA_ARGS__)

__global__ void probe_philox(uint32_t *o, uint32_t station, uint32_t step0, uint32_t k0, uint32_t k1) {
  uint32_t rep = threadIdx.x, blk = threadIdx.x >> 2;
  BEGIN("+v"(rep), "+v"(blk), "+s"(station), "+s"(step0), "+s"(k0), "+s"(k1));
  const U4 r = philox10(U4{rep, station, step0, (2u << 24) | blk}, k0, k1);
  END("v"(r.x), "v"(r.y), "v"(r.z), "v"(r.w));
  o[threadIdx.x] = r.x;
}

__global__ void probe_unit(float *o) {
  uint32_t x = threadIdx.x * 2654435761u;
  BEGIN("+v"(x));
  const float u = to_unit(x);
  END("v"(u));
  o[threadIdx.x] = u;
}

__global__ void probe_ln(float *o) {
  float x = (float)threadIdx.x + 1.5f;
  BEGIN("+v"(x));
  __builtin_assume(x > 0.0f);
  const float y = ln(x);
  END("v"(y));
  o[threadIdx.x] = y;
}

// ln1p's two branches: |x| < 1/4 evaluates the series directly; otherwise it rounds 1 + x,
// recovers the rounding error and takes ln_corr of it (probed here; the few operations before
// it are added in op_costs.py)
__global__ void probe_ln1p_small(float *o) {
  float x = (float)threadIdx.x * 1e-3f;
  BEGIN("+v"(x));
  const float y = ln1p_small(x, 0.0f);
  END("v"(y));
  o[threadIdx.x] = y;
}

__global__ void probe_ln_corr(float *o) {
  float u = (float)threadIdx.x + 1.5f, c = (float)threadIdx.x * 1e-9f;
  BEGIN("+v"(u), "+v"(c));
  const float y = ln_corr(u, c);
  END("v"(y));
  o[threadIdx.x] = y;
}

__global__ void probe_ex(float *o) {
  float x = -(float)threadIdx.x * 0.1f;
  BEGIN("+v"(x));
  __builtin_assume(x >= -86.0f && x <= 88.0f);
  const float y = ex(x);
  END("v"(y));
  o[threadIdx.x] = y;
}

// exm1's general branch (|x| >= ln2 / 2): reduction by ln 2 around expm1_small (probed here;
// the reduction is added in op_costs.py)
__global__ void probe_expm1_small(float *o) {
  float r = -(float)threadIdx.x * 0.001f;
  BEGIN("+v"(r));
  const float y = expm1_small(r);
  END("v"(y));
  o[threadIdx.x] = y;
}

__global__ void probe_div(float *o) {
  float a = (float)threadIdx.x + 1.0f, b = (float)threadIdx.x + 3.0f;
  BEGIN("+v"(a), "+v"(b));
  const float y = a / b;
  END("v"(y));
  o[threadIdx.x] = y;
}

__global__ void probe_sqrt(float *o) {
  float a = (float)threadIdx.x + 1.0f;
  BEGIN("+v"(a));
  __builtin_assume(a >= 0.0f);
  const float y = __builtin_sqrtf(a);
  END("v"(y));
  o[threadIdx.x] = y;
}

__global__ void probe_floor(float *o) {
  float a = (float)threadIdx.x * 0.37f;
  BEGIN("+v"(a));
  const float y = __builtin_floorf(a);
  END("v"(y));
  o[threadIdx.x] = y;
}

__global__ void probe_stirling_series(float *o) {
  int j = (int)threadIdx.x + 10;
  BEGIN("+v"(j));
  __builtin_assume(j >= 10);
  const float y = stirling_tail(j);
  END("v"(y));
  o[threadIdx.x] = y;
}

// (float) of an fp64 fma of an fp32 and two exact integers, as the binomial sampler's log-ratios use
__global__ void probe_fma64(float *o) {
  float r = (float)threadIdx.x * 0.01f;
  int n = (int)threadIdx.x + 1000, k = (int)threadIdx.x;
  BEGIN("+v"(r), "+v"(n), "+v"(k));
  const float y = (float)__builtin_fma((double)r, (double)(n - k + 1), -(double)(k + 1));
  END("v"(y));
  o[threadIdx.x] = y;
}

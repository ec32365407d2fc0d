// CPU emulation of the part of HIP that the simulator library uses, for running the library's
// own sources (host code and kernels) on the host under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Test infrastructure: it is put on the include path only by the
// sanitizer tests, never by the product build.
//
// Execution model.  A kernel launch runs its workgroups on a pool of host threads; within a
// workgroup every GPU thread is a fiber with its own stack.  Fibers switch only at the points
// where GPU threads synchronise: a wavefront operation (__shfl_xor, readfirstlane) completes
// once every lane of the 64-lane wavefront has reached it, __syncthreads once every thread of
// the workgroup has.  A wavefront operation reached by part of a wavefront while the rest has
// left the kernel, and a workgroup whose threads wait on one another forever, are reported as
// errors and abort the process.  Ballots see only the calling lane (the library uses a ballot
// only to learn whether any lane needs an optional test, which every lane may also evaluate
// alone).  Device allocations are separate host heap blocks, so the sanitizer's red zones
// guard every buffer; launches run to completion before the call returns, except on a stream
// under graph capture, where they are recorded and replayed by hipGraphLaunch.
#pragma once
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <functional>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __constant__
#define __align__(n) __attribute__((aligned(n)))
// a workgroup runs on one host thread, so a thread-local static is shared by exactly its
// GPU threads (and, like LDS, holds stale contents when the next workgroup starts)
#define __shared__ static thread_local
#define HIP_SYMBOL(x) ((const void *)&(x))

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct alignas(16) float4 {
  float x, y, z, w;
};

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidDevice = 101,
  hipErrorInvalidSymbol = 13,
  hipErrorNotSupported = 801,
  hipErrorStreamCaptureUnsupported = 900,
  hipErrorUnknown = 999
} hipError_t;

typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
} hipStreamCaptureMode;

#define hipStreamNonBlocking 0x01

typedef struct emu_stream *hipStream_t;
typedef struct emu_event *hipEvent_t;
typedef struct emu_graph *hipGraph_t;
typedef struct emu_graph *hipGraphExec_t;
typedef struct hipGraphNode *hipGraphNode_t;

typedef struct hipDeviceProp_t {
  char name[256];
  char gcnArchName[256];
  int multiProcessorCount;
  size_t totalGlobalMem;
} hipDeviceProp_t;

namespace emu {
const dim3 &thread_idx();
const dim3 &block_idx();
const dim3 &block_dim();
const dim3 &grid_dim();
void *dyn_lds();
uint64_t wave_exchange(int kind, uint64_t value, int arg);   // kind 0: xor shuffle, 1: first lane
void syncthreads();
void launch(dim3 grid, dim3 block, size_t shmem, hipStream_t stream, std::function<void()> body);
}  // namespace emu

#define threadIdx (::emu::thread_idx())
#define blockIdx (::emu::block_idx())
#define blockDim (::emu::block_dim())
#define gridDim (::emu::grid_dim())

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  ::emu::launch(dim3(grid), dim3(block), (size_t)(shmem), (stream), [=]() { kernel(__VA_ARGS__); })

inline void __syncthreads() { ::emu::syncthreads(); }

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  static_assert(sizeof(T) <= 8, "shuffle of at most 8 bytes");
  (void)width;
  uint64_t bits = 0;
  memcpy(&bits, &v, sizeof(T));
  bits = ::emu::wave_exchange(0, bits, mask);
  T out;
  memcpy(&out, &bits, sizeof(T));
  return out;
}

inline uint32_t emu_readfirstlane(uint32_t v) { return (uint32_t)::emu::wave_exchange(1, v, 0); }
inline uint64_t emu_ballot(bool pred) { return pred ? 1ull << (threadIdx.x & 63) : 0ull; }
#define __builtin_amdgcn_readfirstlane(v) emu_readfirstlane((uint32_t)(v))
#define __builtin_amdgcn_ballot_w64(p) emu_ballot((bool)(p))

// gfx950's three-input bitwise operation: bit i of the truth table is the result for the
// input bits (a, b, c) = (i >> 2 & 1, i >> 1 & 1, i & 1).
inline uint32_t emu_bitop3(uint32_t a, uint32_t b, uint32_t c, unsigned table) {
  uint32_t out = 0;
  for (unsigned i = 0; i < 8; ++i)
    if (table >> i & 1u) out |= ((i & 4u) ? a : ~a) & ((i & 2u) ? b : ~b) & ((i & 1u) ? c : ~c);
  return out;
}
#define __builtin_amdgcn_bitop3_b32(a, b, c, t) emu_bitop3((uint32_t)(a), (uint32_t)(b), (uint32_t)(c), (unsigned)(t))

// HIP's integer min / max of device code
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }

inline uint32_t __float_as_uint(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}
inline float __uint_as_float(uint32_t u) {
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// Workgroups of one launch run concurrently on several host threads, so the device atomics
// are host atomics.
inline int atomicAdd(int *p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) {
  return __atomic_fetch_add(p, v, __ATOMIC_RELAXED);
}
inline unsigned atomicOr(unsigned *p, unsigned v) { return __atomic_fetch_or(p, v, __ATOMIC_RELAXED); }

hipError_t hipMalloc(void **p, size_t bytes);
template <typename T>
inline hipError_t hipMalloc(T **p, size_t bytes) {
  return hipMalloc(reinterpret_cast<void **>(p), bytes);
}
hipError_t hipFree(void *p);
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipMemset(void *dst, int value, size_t bytes);
hipError_t hipMemsetAsync(void *dst, int value, size_t bytes, hipStream_t s);
hipError_t hipMemcpyToSymbol(const void *symbol, const void *src, size_t bytes, size_t offset = 0,
                             hipMemcpyKind kind = hipMemcpyHostToDevice);
hipError_t hipGetSymbolAddress(void **ptr, const void *symbol);
hipError_t hipDeviceSynchronize();
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipGetDevice(int *dev);
hipError_t hipSetDevice(int dev);
hipError_t hipGetDeviceCount(int *count);
hipError_t hipGetDeviceProperties(hipDeviceProp_t *prop, int dev);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *err_node, char *log,
                               size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);

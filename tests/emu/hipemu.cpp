// hipemu.cpp -- the host runtime behind tests/emu/hip/hip_runtime.h (see there for the model).
//
// Fibers: every GPU thread of a running workgroup has its own stack and is switched by a small
// x86-64 routine (callee-saved registers, SSE and x87 control words, stack pointer), so a
// switch costs no system call; AddressSanitizer is told about every switch.  The scheduler of
// a workgroup resumes each ready fiber until it yields at a synchronisation point or returns,
// then completes every wavefront operation whose lanes have all arrived and, when nothing else
// can move, every barrier that all remaining threads have reached.
#include <atomic>
#include <chrono>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include <sys/mman.h>

#include "hip/hip_runtime.h"

#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
#define EMU_ASAN 1
#endif

extern "C" void emu_ctx_switch(void **save_sp, void *load_sp);
extern "C" void emu_fiber_trampoline();
extern "C" void emu_fiber_main();

// emu_ctx_switch(save, load): push the callee-saved registers and the MXCSR / x87 control
// words on the current stack, store the stack pointer in *save, continue on the stack `load`
// (popping the same frame); a fresh fiber's frame returns into emu_fiber_trampoline.
asm(R"(
  .text
  .globl emu_ctx_switch
  .type emu_ctx_switch,@function
emu_ctx_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  subq $8, %rsp
  stmxcsr (%rsp)
  fnstcw 4(%rsp)
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  ldmxcsr (%rsp)
  fldcw 4(%rsp)
  addq $8, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
  .size emu_ctx_switch,.-emu_ctx_switch

  .globl emu_fiber_trampoline
  .type emu_fiber_trampoline,@function
emu_fiber_trampoline:
  call emu_fiber_main
  ud2
  .size emu_fiber_trampoline,.-emu_fiber_trampoline
)");

namespace emu {
namespace {

[[noreturn]] void fatal(const char *what) {
  std::fprintf(stderr, "hipemu: %s\n", what);
  std::fflush(stderr);
  std::abort();
}

enum State { READY, WAIT_WAVE, WAIT_BAR, DONE };

constexpr size_t kStack = 256 * 1024;
constexpr int kMaxThreads = 1024;

struct Fiber {
  void *sp = nullptr;
  char *stack = nullptr;
  State state = DONE;
  dim3 tid;
  int kind = 0, arg = 0;
  uint64_t value = 0, result = 0;
  long long seq = 0;
  void *asan_fake = nullptr;
};

struct Worker {
  std::vector<Fiber> fibers;
  Fiber *cur = nullptr;
  void *sched_sp = nullptr;
  const void *sched_bottom = nullptr;
  size_t sched_size = 0;
  dim3 bidx, bdim, gdim;
  void *lds = nullptr;
  const std::function<void()> *body = nullptr;
};

thread_local Worker *tw = nullptr;
std::atomic<long long> g_nonuniform{0};

void ensure_fibers(Worker *w, int nt) {
  while ((int)w->fibers.size() < nt) {
    Fiber f;
    void *m = mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (m == MAP_FAILED) fatal("cannot map a fiber stack");
    f.stack = (char *)m;
    w->fibers.push_back(f);
  }
}

void init_fiber(Fiber *f) {
  uintptr_t top = ((uintptr_t)(f->stack + kStack)) & ~(uintptr_t)15;
  uint64_t *sp = (uint64_t *)top;
  *--sp = (uint64_t)(uintptr_t)&emu_fiber_trampoline;   // return address
  for (int r = 0; r < 6; ++r) *--sp = 0;                  // rbp rbx r12 r13 r14 r15
  *--sp = ((uint64_t)0x037F << 32) | 0x1F80;              // MXCSR, x87 control word
  f->sp = sp;
}

void resume(Worker *w, Fiber *f) {
  w->cur = f;
#ifdef EMU_ASAN
  void *fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, f->stack, kStack);
#endif
  emu_ctx_switch(&w->sched_sp, f->sp);
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
  w->cur = nullptr;
}

void yield_to_scheduler() {
  Worker *w = tw;
  Fiber *f = w->cur;
#ifdef EMU_ASAN
  __sanitizer_start_switch_fiber(&f->asan_fake, w->sched_bottom, w->sched_size);
#endif
  emu_ctx_switch(&f->sp, w->sched_sp);
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(f->asan_fake, &w->sched_bottom, &w->sched_size);
#endif
}

Fiber *current() {
  if (!tw || !tw->cur) fatal("a device operation was called outside a kernel");
  return tw->cur;
}

void run_block(Worker *w) {
  if (w->bdim.y != 1 || w->bdim.z != 1) fatal("only one-dimensional workgroups are emulated");
  const int nt = (int)w->bdim.x;
  if (nt < 1 || nt > kMaxThreads) fatal("workgroup size out of range");
  ensure_fibers(w, nt);
  for (int t = 0; t < nt; ++t) {
    Fiber &f = w->fibers[t];
    f.state = READY;
    f.tid = dim3((unsigned)t);
    f.seq = 0;
    init_fiber(&f);
  }
  for (;;) {
    for (int t = 0; t < nt; ++t)
      if (w->fibers[t].state == READY) resume(w, &w->fibers[t]);
    int done = 0, bar = 0;
    for (int t = 0; t < nt; ++t) {
      done += w->fibers[t].state == DONE;
      bar += w->fibers[t].state == WAIT_BAR;
    }
    if (done == nt) return;
    bool released = false;
    for (int w0 = 0; w0 < nt; w0 += 64) {
      const int w1 = w0 + 64 < nt ? w0 + 64 : nt;
      int waiting = 0;
      for (int t = w0; t < w1; ++t) waiting += w->fibers[t].state == WAIT_WAVE;
      if (!waiting) continue;
      if (waiting != w1 - w0) fatal("a wavefront operation was reached by only part of a wavefront");
      const Fiber &l0 = w->fibers[w0];
      for (int t = w0; t < w1; ++t) {
        const Fiber &f = w->fibers[t];
        if (f.kind != l0.kind || f.seq != l0.seq || f.arg != l0.arg)
          fatal("lanes of a wavefront are at different wavefront operations");
      }
      for (int t = w0; t < w1; ++t) {
        Fiber &f = w->fibers[t];
        if (f.kind == 0) {
          const int src = w0 + (((t - w0) ^ f.arg) & 63);
          if (src >= w1) fatal("shuffle from a lane beyond the workgroup");
          f.result = w->fibers[src].value;
        } else {
          f.result = l0.value;
          if (f.value != l0.value) g_nonuniform.fetch_add(1, std::memory_order_relaxed);
        }
      }
      for (int t = w0; t < w1; ++t) w->fibers[t].state = READY;
      released = true;
    }
    if (released) continue;
    if (bar > 0 && bar + done == nt) {
      for (int t = 0; t < nt; ++t)
        if (w->fibers[t].state == WAIT_BAR) w->fibers[t].state = READY;
      continue;
    }
    fatal("the threads of a workgroup wait on one another forever");
  }
}

std::vector<std::unique_ptr<Worker>> g_workers;
std::mutex g_workers_mu;

int worker_count() {
  static int n = [] {
    const char *e = std::getenv("HIPEMU_THREADS");
    int v = e ? std::atoi(e) : (int)std::thread::hardware_concurrency();
    return v < 1 ? 1 : (v > 64 ? 64 : v);
  }();
  return n;
}

void execute(dim3 grid, dim3 block, size_t shmem, const std::function<void()> &body) {
  if (grid.z != 1) fatal("only one- and two-dimensional grids are emulated");
  const long long blocks = (long long)grid.x * grid.y;
  if (blocks <= 0) return;
  const int nw = (int)std::min<long long>(worker_count(), blocks);
  {
    std::lock_guard<std::mutex> lk(g_workers_mu);
    while ((int)g_workers.size() < nw) g_workers.emplace_back(new Worker());
  }
  std::atomic<long long> next{0};
  auto work = [&](Worker *w) {
    Worker *saved = tw;
    tw = w;
    for (;;) {
      const long long b = next.fetch_add(1);
      if (b >= blocks) break;
      w->bidx = dim3((unsigned)(b % grid.x), (unsigned)(b / grid.x));
      w->bdim = block;
      w->gdim = grid;
      w->lds = shmem ? std::malloc(shmem) : nullptr;
      w->body = &body;
      run_block(w);
      std::free(w->lds);
      w->lds = nullptr;
    }
    tw = saved;
  };
  std::vector<std::thread> th;
  for (int i = 1; i < nw; ++i) th.emplace_back(work, g_workers[i].get());
  work(g_workers[0].get());
  for (auto &t : th) t.join();
}

}  // namespace

extern "C" void emu_fiber_main() {
  Worker *w = tw;
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(nullptr, &w->sched_bottom, &w->sched_size);
#endif
  (*w->body)();
  Fiber *f = w->cur;
  f->state = DONE;
#ifdef EMU_ASAN
  __sanitizer_start_switch_fiber(nullptr, w->sched_bottom, w->sched_size);
#endif
  void *dead = nullptr;
  emu_ctx_switch(&dead, w->sched_sp);
  __builtin_unreachable();
}

const dim3 &thread_idx() { return current()->tid; }
const dim3 &block_idx() {
  current();
  return tw->bidx;
}
const dim3 &block_dim() {
  current();
  return tw->bdim;
}
const dim3 &grid_dim() {
  current();
  return tw->gdim;
}
void *dyn_lds() {
  current();
  return tw->lds;
}

uint64_t wave_exchange(int kind, uint64_t value, int arg) {
  Fiber *f = current();
  f->kind = kind;
  f->value = value;
  f->arg = arg;
  f->seq += 1;
  f->state = WAIT_WAVE;
  yield_to_scheduler();
  return f->result;
}

void syncthreads() {
  Fiber *f = current();
  f->state = WAIT_BAR;
  yield_to_scheduler();
}

long long nonuniform_readfirstlane() { return g_nonuniform.load(); }

}  // namespace emu

// ---- streams, graphs, events -------------------------------------------------------------
struct emu_stream {
  bool capturing = false;
  std::vector<std::function<void()>> ops;
};
struct emu_graph {
  std::vector<std::function<void()>> ops;
};
struct emu_event {
  double t = 0.0;
};

namespace emu {
void launch(dim3 grid, dim3 block, size_t shmem, hipStream_t s, std::function<void()> body) {
  if (s && s->capturing) {
    s->ops.push_back([grid, block, shmem, body]() { execute(grid, block, shmem, body); });
    return;
  }
  execute(grid, block, shmem, body);
}
}  // namespace emu

namespace {
bool record_op(hipStream_t s, std::function<void()> op) {
  if (s && s->capturing) {
    s->ops.push_back(std::move(op));
    return true;
  }
  return false;
}
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
int g_device = 0;
}  // namespace

extern "C" long long hipemu_nonuniform_readfirstlane() { return emu::nonuniform_readfirstlane(); }

hipError_t hipMalloc(void **p, size_t bytes) {
  if (!p) return hipErrorInvalidValue;
  *p = std::malloc(bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind) {
  if (bytes) std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  if (record_op(s, [dst, src, bytes]() {
        if (bytes) std::memcpy(dst, src, bytes);
      }))
    return hipSuccess;
  if (bytes) std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemset(void *dst, int value, size_t bytes) {
  if (bytes) std::memset(dst, value, bytes);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void *dst, int value, size_t bytes, hipStream_t s) {
  if (record_op(s, [dst, value, bytes]() {
        if (bytes) std::memset(dst, value, bytes);
      }))
    return hipSuccess;
  if (bytes) std::memset(dst, value, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyToSymbol(const void *symbol, const void *src, size_t bytes, size_t offset, hipMemcpyKind) {
  if (!symbol) return hipErrorInvalidSymbol;
  std::memcpy((char *)symbol + offset, src, bytes);
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **ptr, const void *symbol) {
  if (!ptr || !symbol) return hipErrorInvalidSymbol;
  *ptr = const_cast<void *>(symbol);
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }
hipError_t hipGetDevice(int *dev) {
  *dev = g_device;
  return hipSuccess;
}
hipError_t hipSetDevice(int dev) {
  if (dev != 0) return hipErrorInvalidDevice;
  g_device = dev;
  return hipSuccess;
}
hipError_t hipGetDeviceCount(int *count) {
  *count = 1;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t *prop, int dev) {
  if (dev != 0) return hipErrorInvalidDevice;
  std::memset(prop, 0, sizeof *prop);
  std::strcpy(prop->name, "host emulation");
  std::strcpy(prop->gcnArchName, "gfx950");
  prop->multiProcessorCount = 256;
  prop->totalGlobalMem = (size_t)1 << 34;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = new emu_stream();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s || s->capturing) return hipErrorStreamCaptureUnsupported;
  s->capturing = true;
  s->ops.clear();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
  if (!s || !s->capturing) return hipErrorStreamCaptureUnsupported;
  *g = new emu_graph{std::move(s->ops)};
  s->ops.clear();
  s->capturing = false;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
  *exec = new emu_graph(*g);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s) {
  if (record_op(s, [exec]() {
        for (auto &op : exec->ops) op();
      }))
    return hipSuccess;
  for (auto &op : exec->ops) op();
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
  delete exec;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
  *e = new emu_event();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  e->t = now_s();
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)((b->t - a->t) * 1e3);
  return hipSuccess;
}

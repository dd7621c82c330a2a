// Runtime of the host emulation of the HIP kernels (see hip/hip_runtime.h here).  The threads of a
// block are user-level fibers on one OS thread: each runs until it blocks at a
// barrier (or finishes), in thread order, so an emulated run is deterministic.
// A fiber that reads shared state after a barrier sees everything the lower-
// numbered fibers did before their next barrier, which exposes missing
// barriers (a deadlock with a state dump) instead of hiding them.
#include <hip/hip_runtime.h>
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>

// minimal x86-64 context switch: callee-saved registers + stack pointer
extern "C" void simt_swap(void **save_sp, void *load_sp);
asm(R"(
.text
.globl simt_swap
.type simt_swap,@function
simt_swap:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
.size simt_swap, .-simt_swap
)");

#include <string>

namespace simt {
thread_local Ctx ctx;

[[noreturn]] void die(const char *msg) {
  fprintf(stderr, "SIMT FATAL: %s\n", msg);
  fflush(stderr);
  abort();
}

static std::string g_kernel;
constexpr size_t STACK = 512 * 1024;

enum { READY = 0, BLOCKED = 1, DONE = 2 };
struct Fiber {
  void *sp = nullptr;
  char *stack = nullptr;
  int state = DONE;
  int where = 0;   // 1 block barrier, 10 + lg group barrier
  Ctx c;
};
static Fiber g_fib[1024];
static void *g_sched_sp = nullptr;
static const void *g_main_bottom = nullptr;
static size_t g_main_size = 0;
static int g_cur = -1, g_n = 0;
static const std::function<void()> *g_body = nullptr;

struct Bar {
  int n = 0, count = 0;
  int waiters[1024];
  int nw = 0;
};
static Bar g_block;
static Bar g_groups[7][1024];
static uint64_t g_slots[1024 * 8];
static void *g_dyn = nullptr;

static void to_sched() {
  void *fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, g_main_bottom, g_main_size);
  simt_swap(&g_fib[g_cur].sp, g_sched_sp);
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
}

static void bar_wait(Bar &b, int where) {
  if (++b.count == b.n) {
    b.count = 0;
    for (int i = 0; i < b.nw; ++i) g_fib[b.waiters[i]].state = READY;
    b.nw = 0;
    return;   // the last to arrive continues
  }
  b.waiters[b.nw++] = g_cur;
  g_fib[g_cur].state = BLOCKED;
  g_fib[g_cur].where = where;
  to_sched();
  g_fib[g_cur].where = 0;
}

void block_sync() { bar_wait(g_block, 1); }
void group_sync(int size) {
  int lg = 0;
  while ((1 << lg) < size) ++lg;
  if ((1 << lg) != size || lg > 6) die("group size");
  bar_wait(g_groups[lg][ctx.flat >> lg], 10 + lg);
}
uint64_t *slots() { return g_slots; }
void *dyn_lds() { return g_dyn; }

static void fiber_entry() {
  __sanitizer_finish_switch_fiber(nullptr, &g_main_bottom, &g_main_size);
  (*g_body)();
  g_fib[g_cur].state = DONE;
  __sanitizer_start_switch_fiber(nullptr, g_main_bottom, g_main_size);
  simt_swap(&g_fib[g_cur].sp, g_sched_sp);
  die("finished fiber resumed");
}

static void dump_states() {
  int cnt[32] = {0}, ex[32];
  for (int i = 0; i < 32; ++i) ex[i] = -1;
  for (int t = 0; t < g_n; ++t) {
    const int w = g_fib[t].state == DONE ? 31 : g_fib[t].where;
    cnt[w] += 1;
    if (ex[w] < 0) ex[w] = t;
  }
  for (int i = 0; i < 32; ++i)
    if (cnt[i]) fprintf(stderr, "   %s %d: %d threads (e.g. thread %d)\n", i == 31 ? "finished" : "waiting at", i, cnt[i], ex[i]);
}

static void run_block(dim3 b, dim3 g, dim3 bd) {
  const int n = (int)(bd.x * bd.y * bd.z);
  g_n = n;
  for (int t = 0; t < n; ++t) {
    Fiber &f = g_fib[t];
    if (!f.stack) f.stack = (char *)malloc(STACK);
    // initial frame: 6 callee-saved registers, then the entry address for `ret`
    uintptr_t top = ((uintptr_t)(f.stack + STACK)) & ~(uintptr_t)15;
    void **sp = (void **)top;
    *--sp = nullptr;                          // fake return address of fiber_entry
    *--sp = (void *)&fiber_entry;
    for (int r = 0; r < 6; ++r) *--sp = nullptr;
    f.sp = sp;
    f.state = READY;
    f.where = 0;
    f.c.bid = b;
    f.c.gdim = g;
    f.c.bdim = bd;
    f.c.flat = t;
    f.c.tid = dim3(t % bd.x, (t / bd.x) % bd.y, t / (bd.x * bd.y));
  }
  for (;;) {
    bool any = false, all_done = true;
    for (int t = 0; t < n; ++t) {
      if (g_fib[t].state != DONE) all_done = false;
      if (g_fib[t].state != READY) continue;
      any = true;
      g_cur = t;
      ctx = g_fib[t].c;
      void *fake = nullptr;
      __sanitizer_start_switch_fiber(&fake, g_fib[t].stack, STACK);
      simt_swap(&g_sched_sp, g_fib[t].sp);
      __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
      g_fib[t].c = ctx;
    }
    if (all_done) break;
    if (!any) {
      fprintf(stderr, "SIMT: deadlock in %s, block (%u, %u)\n", g_kernel.c_str(), b.x, b.y);
      dump_states();
      die("deadlock");
    }
  }
  for (int t = 0; t < n; ++t) ASAN_UNPOISON_MEMORY_REGION(g_fib[t].stack, STACK);
}

long long g_launches = 0;

void launch_exec(const char *name, dim3 grid, dim3 block, size_t lds, const std::function<void()> &body) {
  const int n = (int)(block.x * block.y * block.z);
  if (n < 1 || n > 1024 || (n % 64) != 0) die("block size");
  g_kernel = name;
  g_block.n = n;
  g_block.count = 0;
  g_block.nw = 0;
  for (int lg = 0; lg <= 6; ++lg)
    for (int gi = 0; gi < n >> lg; ++gi) {
      g_groups[lg][gi].n = 1 << lg;
      g_groups[lg][gi].count = 0;
      g_groups[lg][gi].nw = 0;
    }
  void *dyn = malloc(lds ? lds : 1);
  g_dyn = dyn;
  g_body = &body;
  for (unsigned by = 0; by < grid.y; ++by)
    for (unsigned bx = 0; bx < grid.x; ++bx) run_block(dim3(bx, by, 0), grid, block);
  free(dyn);
  g_dyn = nullptr;
  ++g_launches;
}
}  // namespace simt

// ---------------------------------------------------------------- streams, events, graphs
struct Op {
  std::string name;
  dim3 grid, block;
  size_t lds = 0;
  std::function<void()> body;   // a kernel body, or (lds == (size_t)-1) a host-side copy/fill
};
struct ihipGraph {
  std::vector<Op> ops;
  std::vector<ihipStream_t *> joined;
};
struct ihipGraphExec {
  std::vector<Op> ops;
};
struct ihipStream_t {
  bool capturing = false;
  ihipGraph *g = nullptr;
};
struct ihipEvent_t {
  ihipGraph *g = nullptr;
};

static void run_op(const Op &o) {
  if (o.lds == (size_t)-1) o.body();
  else simt::launch_exec(o.name.c_str(), o.grid, o.block, o.lds, o.body);
}

namespace simt {
void launch_impl(const char *name, dim3 grid, dim3 block, size_t lds, void *stream, std::function<void()> body) {
  ihipStream_t *s = (ihipStream_t *)stream;
  Op o{name, grid, block, lds, std::move(body)};
  if (s && s->capturing) s->g->ops.push_back(std::move(o));
  else run_op(o);
}
}  // namespace simt

static void host_op(hipStream_t s, std::function<void()> f) {
  Op o{"host", dim3(), dim3(), (size_t)-1, std::move(f)};
  if (s && s->capturing) s->g->ops.push_back(std::move(o));
  else run_op(o);
}

hipError_t hipMalloc(void **p, size_t n) {
  void *q = nullptr;
  if (posix_memalign(&q, 256, n ? n : 1)) return hipErrorOutOfMemory;
  memset(q, 0xA5, n);   // device memory starts with garbage
  *p = q;
  return hipSuccess;
}
hipError_t hipFree(void *p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t st) {
  host_op(st, [=] { memcpy(d, s, n); });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t st) {
  host_op(st, [=] { memset(d, v, n); });
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = new ihipStream_t();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  e->g = (s && s->capturing) ? s->g : nullptr;
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  if (e->g && s && !s->capturing) {
    s->capturing = true;
    s->g = e->g;
    e->g->joined.push_back(s);
  }
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? 4 : 163840;
  return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void *, hipFuncAttribute, int v) { return v <= 163840 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s || s->capturing) return hipErrorInvalidValue;
  s->capturing = true;
  s->g = new ihipGraph();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
  if (!s || !s->capturing) return hipErrorInvalidValue;
  *g = s->g;
  for (ihipStream_t *j : s->g->joined) {
    j->capturing = false;
    j->g = nullptr;
  }
  s->capturing = false;
  s->g = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, void *, char *, size_t) {
  *x = new ihipGraphExec{g->ops};
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) {
  for (const Op &o : x->ops) run_op(o);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;
  return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "emulated"; }

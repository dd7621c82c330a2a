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

#include <algorithm>
#include <deque>
#include <random>
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
constexpr int MAXB = 64;   // resident blocks of a launch whose workgroups run together

enum { READY = 0, BLOCKED = 1, DONE = 2 };
struct Fiber {
  void *sp = nullptr;
  char *stack = nullptr;
  int state = DONE;
  int where = 0;   // 1 block barrier, 10 + lg group barrier
  Ctx c;
};
static Fiber g_fib[MAXB * 512];   // a sequential launch uses up to 1024 of them
static int g_fib_blk[MAXB * 512];
static void *g_sched_sp = nullptr;
static const void *g_main_bottom = nullptr;
static size_t g_main_size = 0;
static int g_cur = -1, g_n = 0;
static const std::function<void()> *g_body = nullptr;

struct Bar {
  int n = 0, count = 0;
  std::vector<int> waiters;
};
// per resident block: barriers, exchange slots, dynamic LDS
struct BlockState {
  Bar block;
  Bar groups[7][1024];
  uint64_t slots[1024 * 8];
  void *dyn = nullptr;       // dynamic LDS: 8 bytes past a 16-byte boundary, the weakest
  void *dyn_raw = nullptr;   // alignment the device gives an `extern __shared__ double[]`
};
static BlockState *g_bs[MAXB];
static int g_cur_blk = 0;

static void to_sched() {
  void *fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, g_main_bottom, g_main_size);
  simt_swap(&g_fib[g_cur].sp, g_sched_sp);
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
}

static void bar_wait(Bar &b, int where) {
  if (++b.count == b.n) {
    b.count = 0;
    for (int w : b.waiters) g_fib[w].state = READY;
    b.waiters.clear();
    return;   // the last to arrive continues
  }
  b.waiters.push_back(g_cur);
  g_fib[g_cur].state = BLOCKED;
  g_fib[g_cur].where = where;
  to_sched();
  g_fib[g_cur].where = 0;
}

void block_sync() { bar_wait(g_bs[g_cur_blk]->block, 1); }
void group_sync(int size) {
  int lg = 0;
  while ((1 << lg) < size) ++lg;
  if ((1 << lg) != size || lg > 6) die("group size");
  bar_wait(g_bs[g_cur_blk]->groups[lg][ctx.flat >> lg], 10 + lg);
}
uint64_t *slots() { return g_bs[g_cur_blk]->slots; }
void *dyn_lds() { return g_bs[g_cur_blk]->dyn; }
int block_linear() { return g_cur_blk; }
// a spin-wait iteration: let every other fiber run before this one continues
void yield() {
  g_fib[g_cur].state = READY;
  g_fib[g_cur].where = 2;
  to_sched();
  g_fib[g_cur].where = 0;
}

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

// run the blocks listed in `blocks` as one set of fibers (concurrently when
// there are several: a launch whose workgroups wait on each other)
static void run_blocks(const std::vector<dim3> &blocks, dim3 g, dim3 bd, size_t lds) {
  const int per = (int)(bd.x * bd.y * bd.z);
  const int nb = (int)blocks.size();
  if (nb > MAXB || (nb > 1 && per > 512)) die("too many resident blocks");
  for (int bi = 0; bi < nb; ++bi) {
    if (!g_bs[bi]) g_bs[bi] = new BlockState();
    BlockState &B = *g_bs[bi];
    B.block.n = per;
    B.block.count = 0;
    B.block.waiters.clear();
    for (int lg = 0; lg <= 6; ++lg)
      for (int gi = 0; gi < per >> lg; ++gi) {
        B.groups[lg][gi].n = 1 << lg;
        B.groups[lg][gi].count = 0;
        B.groups[lg][gi].waiters.clear();
      }
    B.dyn_raw = aligned_alloc(16, ((lds + 8) + 15) & ~(size_t)15);
    B.dyn = (char *)B.dyn_raw + 8;
    // the bytes past the launch's size are poisoned, so the bound stays exact
    ASAN_POISON_MEMORY_REGION((char *)B.dyn + lds, (((lds + 8) + 15) & ~(size_t)15) - 8 - lds);
  }
  const int n = nb * per;
  g_n = n;
  for (int f = 0; f < n; ++f) {
    const int bi = f / per, t = f % per;
    Fiber &fb = g_fib[f];
    if (!fb.stack) fb.stack = (char *)malloc(STACK);
    uintptr_t top = ((uintptr_t)(fb.stack + STACK)) & ~(uintptr_t)15;
    void **sp = (void **)top;
    *--sp = nullptr;                          // fake return address of fiber_entry
    *--sp = (void *)&fiber_entry;
    for (int r = 0; r < 6; ++r) *--sp = nullptr;
    fb.sp = sp;
    fb.state = READY;
    fb.where = 0;
    fb.c.bid = blocks[bi];
    fb.c.gdim = g;
    fb.c.bdim = bd;
    fb.c.flat = t;
    fb.c.tid = dim3(t % bd.x, (t / bd.x) % bd.y, t / (bd.x * bd.y));
    g_fib_blk[f] = bi;
  }
  for (;;) {
    bool any = false, all_done = true;
    for (int f = 0; f < n; ++f) {
      if (g_fib[f].state != DONE) all_done = false;
      if (g_fib[f].state != READY) continue;
      any = true;
      g_cur = f;
      g_cur_blk = g_fib_blk[f];
      ctx = g_fib[f].c;
      void *fake = nullptr;
      __sanitizer_start_switch_fiber(&fake, g_fib[f].stack, STACK);
      simt_swap(&g_sched_sp, g_fib[f].sp);
      __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
      g_fib[f].c = ctx;
    }
    if (all_done) break;
    if (!any) {
      fprintf(stderr, "SIMT: deadlock in %s, block (%u, %u)\n", g_kernel.c_str(), blocks[0].x, blocks[0].y);
      dump_states();
      die("deadlock");
    }
  }
  for (int f = 0; f < n; ++f) ASAN_UNPOISON_MEMORY_REGION(g_fib[f].stack, STACK);
  for (int bi = 0; bi < nb; ++bi) {
    const size_t tot = ((lds + 8) + 15) & ~(size_t)15;
    ASAN_UNPOISON_MEMORY_REGION(g_bs[bi]->dyn_raw, tot);
    free(g_bs[bi]->dyn_raw);
    g_bs[bi]->dyn_raw = g_bs[bi]->dyn = nullptr;
  }
  g_cur_blk = 0;
}

long long g_launches = 0;
long long g_resident_launches = 0;   // launches run with all blocks resident together

void launch_exec(const char *name, dim3 grid, dim3 block, size_t lds, const std::function<void()> &body) {
  const int n = (int)(block.x * block.y * block.z);
  if (n < 1 || n > 1024 || (n % 64) != 0) die("block size");
  g_kernel = name;
  g_body = &body;
  // workgroups that wait on each other run as one set of fibers
  const bool together = strstr(name, "k_cpqr_persist") != nullptr || strstr(name, "k_rowid_reg") != nullptr;
  if (together) {
    std::vector<dim3> all;
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) all.push_back(dim3(bx, by, 0));
    run_blocks(all, grid, block, lds);
    ++g_resident_launches;
  } else {
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) run_blocks({dim3(bx, by, 0)}, grid, block, lds);
  }
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
// A queued stream item: an operation, or a wait for another stream to have
// completed `pos` items (hipStreamWaitEvent).
struct Item {
  bool wait = false;
  Op op;
  ihipStream_t *src = nullptr;
  long long pos = 0;
};
struct ihipStream_t {
  bool capturing = false;
  ihipGraph *g = nullptr;
  int id = 0;
  std::deque<Item> q;
  long long issued = 0, done = 0;
};
struct ihipEvent_t {
  ihipGraph *g = nullptr;
  ihipStream_t *src = nullptr;   // deferred streams: the stream and item count it marks
  long long pos = 0;
};

static void run_op(const Op &o) {
  if (o.lds == (size_t)-1) o.body();
  else simt::launch_exec(o.name.c_str(), o.grid, o.block, o.lds, o.body);
}

// Streams run operations as they are enqueued, in host issue order, unless
// SIMT_STREAMS=defer:<order>: then every stream queues its work (waits on
// events included) and the queues advance only when the host synchronises,
// one item at a time from a stream chosen among those whose front item can
// run: order 0 the stream created first, 1 the one created last, any other
// value a seeded random choice.  Work on different streams that is not
// ordered by events then runs in different interleavings, and a race between
// streams changes the results.
static int g_defer = -1;
static long long g_order = 0;
static std::mt19937_64 g_rng;
static std::vector<ihipStream_t *> g_streams;
static ihipStream_t g_null_stream;
static int g_stream_ids = 0;

static long long g_items = 0, g_choices = 0, g_switches = 0;   // deferred streams: items run, steps with a
static ihipStream_t *g_last = nullptr;                          // choice of stream, changes of stream
static void report() {
  fprintf(stderr, "SIMT streams: %lld items, %lld with a choice of stream, %lld stream changes\n", g_items, g_choices,
          g_switches);
}

static bool deferred() {
  if (g_defer < 0) {
    const char *e = getenv("SIMT_STREAMS");
    g_defer = (e && strncmp(e, "defer", 5) == 0) ? 1 : 0;
    if (g_defer && e[5] == ':') g_order = atoll(e + 6);
    g_rng.seed((uint64_t)g_order);
    g_streams.push_back(&g_null_stream);
    if (g_defer) atexit(report);
  }
  return g_defer == 1;
}
static ihipStream_t *stream_of(hipStream_t s) { return s ? s : &g_null_stream; }

static bool front_ready(const ihipStream_t *x) {
  if (x->q.empty()) return false;
  const Item &f = x->q.front();
  return !f.wait || f.src->done >= f.pos;
}

static void drain(const std::function<bool()> &satisfied) {
  while (!satisfied()) {
    std::vector<ihipStream_t *> r;
    for (ihipStream_t *x : g_streams)
      if (front_ready(x)) r.push_back(x);
    if (r.empty()) simt::die("streams deadlocked (a wait that no queued work satisfies)");
    ihipStream_t *x = g_order == 0 ? r.front() : g_order == 1 ? r.back() : r[g_rng() % r.size()];
    g_items += 1;
    if (r.size() > 1) g_choices += 1;
    if (x != g_last) g_switches += 1;
    g_last = x;
    Item it = std::move(x->q.front());
    x->q.pop_front();
    if (!it.wait) run_op(it.op);
    x->done += 1;
  }
}
static void drain_all() {
  drain([] {
    for (ihipStream_t *x : g_streams)
      if (!x->q.empty()) return false;
    return true;
  });
}
namespace simt {
void sync_all() {
  if (deferred()) drain_all();
}
}  // namespace simt

static void submit(hipStream_t st, Op o) {
  ihipStream_t *s = st;
  if (s && s->capturing) {
    s->g->ops.push_back(std::move(o));
    return;
  }
  if (!deferred()) {
    run_op(o);
    return;
  }
  ihipStream_t *x = stream_of(st);
  Item it;
  it.op = std::move(o);
  x->q.push_back(std::move(it));
  x->issued += 1;
}

namespace simt {
void launch_impl(const char *name, dim3 grid, dim3 block, size_t lds, void *stream, std::function<void()> body) {
  submit((hipStream_t)stream, Op{name, grid, block, lds, std::move(body)});
}
}  // namespace simt

static void host_op(hipStream_t s, std::function<void()> f) {
  submit(s, Op{"host", dim3(), dim3(), (size_t)-1, std::move(f)});
}

hipError_t hipMalloc(void **p, size_t n) {
  void *q = nullptr;
  if (posix_memalign(&q, 256, n ? n : 1)) return hipErrorOutOfMemory;
  memset(q, 0xA5, n);   // device memory starts with garbage
  *p = q;
  return hipSuccess;
}
hipError_t hipFree(void *p) {
  simt::sync_all();   // hipFree waits for the device
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
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (deferred()) {
    ihipStream_t *x = stream_of(s);
    drain([x] { return x->q.empty(); });
  }
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() {
  simt::sync_all();
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  deferred();
  *s = new ihipStream_t();
  (*s)->id = ++g_stream_ids;
  g_streams.push_back(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (deferred()) drain([s] { return s->q.empty(); });
  g_streams.erase(std::remove(g_streams.begin(), g_streams.end(), s), g_streams.end());
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
  e->src = nullptr;
  if (!e->g && deferred()) {
    e->src = stream_of(s);
    e->pos = e->src->issued;
  }
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (deferred() && e->src) {
    ihipStream_t *x = e->src;
    const long long pos = e->pos;
    drain([x, pos] { return x->done >= pos; });
  }
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  if (e->g && s && !s->capturing) {
    s->capturing = true;
    s->g = e->g;
    e->g->joined.push_back(s);
  } else if (deferred() && e->src && !(s && s->capturing)) {
    ihipStream_t *x = stream_of(s);
    Item it;
    it.wait = true;
    it.src = e->src;
    it.pos = e->pos;
    x->q.push_back(std::move(it));
    x->issued += 1;
  }
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int) {
  const char *cu = getenv("SIMT_CU");
  *v = a == hipDeviceAttributeMultiprocessorCount ? (cu ? atoi(cu) : 4) : 163840;
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
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  for (const Op &o : x->ops) submit(s, o);
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

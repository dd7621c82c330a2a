// B^T = A^T Q (the one full pass of Alg. 2) for callers that cannot allocate
// device memory: code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc.  Same kernels, same launch plan and so the same
// bytes as dsk_project; the plan's workspace (the packed Q and, when the pass
// is split over the rows of A, the per-split partial outputs) lives in a
// static device array instead of the handle's arena.
//
// The array is part of the code object: each device the library runs on holds
// its own copy, of NOALLOC_BYTES, from the module's load until the process
// ends.  Its device address is taken once per device, in dsk_create with that
// device current, and kept per device; on the host the array's name is not a
// device address, so it is never passed to a kernel or a copy.  All calls on a
// device use the same array (calls that overlap on one device race).  Nothing
// in it must start at zero: the kernels write every byte they later read.
#include <mutex>

#include "dsk_internal.h"

namespace {

constexpr size_t NOALLOC_BYTES = (size_t)32 << 20;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_mu;
void *g_scratch[MAX_DEVICES];   // device address of `scratch` on each device, set at dsk_create

}  // namespace

int noalloc_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return DSK_ERR_BASE + (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return 0;
  void *ptr = nullptr;
  DSK_TRY(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
  g_scratch[device] = ptr;
  return 0;
}

int dsk_project_noalloc(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                        const void *Q, int32_t ell, void *Bt, int32_t mode) {
  if (const int bad = project_args(h, A, dtype, m, n, lda, Q, ell, Bt, mode)) return bad;
  DSK_TRY(hipSetDevice(h->device));
  void *ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (h->device >= 0 && h->device < MAX_DEVICES) ws = g_scratch[h->device];
  }
  if (!ws) return DSK_ERR_SCRATCH;
  if (stream_scratch_bytes(dtype, m, n, ell, mode, h->cu_count) > NOALLOC_BYTES) return DSK_ERR_SCRATCH;
  hipEvent_t e0, e1;
  timing_slot(h, &e0, &e1);
  return launch_stream(h->stream, A, dtype, m, n, lda, Q, dtype == DSK_F64, ell, Bt, ell, mode, ws, h->cu_count, e0,
                       e1);
}

// Host emulation of the HIP subset used by libdsketch's kernels (CPU checking only).
// Every GPU thread of a block is a fiber (see simt_rt.cpp); blocks of a launch run one after
// another.  __shared__ arrays become static storage (one block at a time),
// dynamic LDS is a heap buffer of exactly the launch's size, wave operations
// exchange values through per-group barriers.  Built with AddressSanitizer this
// reports out-of-bounds accesses to device buffers and LDS.
#pragma once
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <math.h>
#include <stdlib.h>
#include <stdio.h>
#include <algorithm>
#include <atomic>
#include <functional>
#include <vector>
#include <utility>
#include <tuple>

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace simt {
struct Ctx {
  dim3 tid, bid, bdim, gdim;
  int flat;
};
extern thread_local Ctx ctx;
void block_sync();
void group_sync(int size);                 // barrier among the aligned group of `size` lanes of this thread
uint64_t *slots();                          // per-block exchange slots: 1024 threads x 8 words
void *dyn_lds();
int block_linear();                         // resident-block index of this thread (per-block static LDS)
void yield();                               // a spin-wait iteration: let the other threads run
void sync_all();                            // deferred streams: run every queued item
[[noreturn]] void die(const char *msg);
void launch_impl(const char *name, dim3 grid, dim3 block, size_t lds, void *stream, std::function<void()> body);
template <typename T>
inline void put(int w, T v) {
  static_assert(sizeof(T) <= 8, "slot");
  uint64_t u = 0;
  memcpy(&u, &v, sizeof(T));
  slots()[ctx.flat * 8 + w] = u;
}
template <typename T>
inline T get(int t, int w) {
  T v;
  uint64_t u = slots()[t * 8 + w];
  memcpy(&v, &u, sizeof(T));
  return v;
}
}  // namespace simt

#define threadIdx (simt::ctx.tid)
#define blockIdx (simt::ctx.bid)
#define blockDim (simt::ctx.bdim)
#define gridDim (simt::ctx.gdim)
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))

inline void __syncthreads() { simt::block_sync(); }
inline void __threadfence() { __atomic_thread_fence(__ATOMIC_SEQ_CST); }

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  const int lane = simt::ctx.flat & 63, base = simt::ctx.flat - (lane % width);
  simt::put(0, v);
  simt::group_sync(width);
  const T r = simt::get<T>(base + ((lane % width) ^ mask), 0);
  simt::group_sync(width);
  return r;
}
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  const int lane = simt::ctx.flat & 63, base = simt::ctx.flat - (lane % width);
  simt::put(0, v);
  simt::group_sync(width);
  const T r = simt::get<T>(base + (src % width), 0);
  simt::group_sync(width);
  return r;
}
inline int __builtin_amdgcn_readlane(int v, int l) {
  const int base = simt::ctx.flat & ~63;
  simt::put(0, v);
  simt::group_sync(64);
  const int r = simt::get<int>(base + l, 0);
  simt::group_sync(64);
  return r;
}
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int rm, int bm, bool bc) {
  (void)old; (void)rm; (void)bm; (void)bc;
  const int t = simt::ctx.flat, lane = t & 63;
  int s, gsz;   // source lane, and the lane group the pattern stays within
  if (ctrl < 0x100) { s = (lane & ~3) + ((ctrl >> (2 * (lane & 3))) & 3); gsz = 4; }
  else if (ctrl == 0x140) { s = (lane & ~15) + 15 - (lane & 15); gsz = 16; }
  else if (ctrl == 0x141) { s = (lane & ~7) + 7 - (lane & 7); gsz = 8; }
  else if (ctrl >= 0x150 && ctrl <= 0x15F) { s = (lane & ~15) + (ctrl & 15); gsz = 16; }   // row_newbcast
  else { simt::die("unsupported dpp control"); }
  simt::put(0, src);
  simt::group_sync(gsz);
  const int r = simt::get<int>((t & ~63) + s, 0);
  simt::group_sync(gsz);
  return r;
}
#define __builtin_amdgcn_wave_barrier() simt::group_sync(64)
#define __builtin_amdgcn_fence(order, scope) __atomic_thread_fence(order)
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)
#define __builtin_amdgcn_s_sleep(x) simt::yield()
inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }
inline float __builtin_amdgcn_rcpf(float x) { return 1.0f / x; }
inline double __builtin_amdgcn_rsq(double x) { return 1.0 / sqrt(x); }

typedef double simt_d4 __attribute__((ext_vector_type(4)));
typedef float simt_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 simt_bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 simt_h8 __attribute__((ext_vector_type(8)));

// D(i, j) of the f64 16x16x4 MFMA sits in lane j + 16 (i mod 4), register i / 4;
// A(i, k) in lane i + 16 k, B(k, j) in lane j + 16 k.
inline simt_d4 __builtin_amdgcn_mfma_f64_16x16x4f64(double a, double b, simt_d4 c, int, int, int) {
  const int t = simt::ctx.flat, l = t & 63, base = t & ~63;
  simt::put(0, a);
  simt::put(1, b);
  simt::group_sync(64);
  simt_d4 d;
  for (int v = 0; v < 4; ++v) {
    const int i = (l >> 4) + 4 * v, j = l & 15;
    double s = c[v];
    for (int k = 0; k < 4; ++k) s += simt::get<double>(base + i + 16 * k, 0) * simt::get<double>(base + j + 16 * k, 1);
    d[v] = s;
  }
  simt::group_sync(64);
  return d;
}
// f32-output MFMAs: D(i, j) in lane j + 16 (i / 4), register i mod 4.
inline simt_f4 __builtin_amdgcn_mfma_f32_16x16x4f32(float a, float b, simt_f4 c, int, int, int) {
  const int t = simt::ctx.flat, l = t & 63, base = t & ~63;
  simt::put(0, a);
  simt::put(1, b);
  simt::group_sync(64);
  simt_f4 d;
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * (l >> 4) + r, j = l & 15;
    float s = c[r];
    for (int k = 0; k < 4; ++k) s += simt::get<float>(base + i + 16 * k, 0) * simt::get<float>(base + j + 16 * k, 1);
    d[r] = s;
  }
  simt::group_sync(64);
  return d;
}
template <typename V>
inline simt_f4 simt_mfma_k32(V a, V b, simt_f4 c) {
  const int t = simt::ctx.flat, l = t & 63, base = t & ~63;
  uint64_t wa[2], wb[2];
  memcpy(wa, &a, 16);
  memcpy(wb, &b, 16);
  for (int w = 0; w < 2; ++w) {
    simt::slots()[t * 8 + w] = wa[w];
    simt::slots()[t * 8 + 2 + w] = wb[w];
  }
  simt::group_sync(64);
  simt_f4 d;
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * (l >> 4) + r, j = l & 15;
    float s = c[r];
    for (int k = 0; k < 32; ++k) {
      V va, vb;
      memcpy(&va, &simt::slots()[(base + i + 16 * (k / 8)) * 8], 16);
      memcpy(&vb, &simt::slots()[(base + j + 16 * (k / 8)) * 8 + 2], 16);
      s += (float)va[k % 8] * (float)vb[k % 8];
    }
    d[r] = s;
  }
  simt::group_sync(64);
  return d;
}
typedef short simt_i16x4 __attribute__((ext_vector_type(4)));
// ds_read_b64_tr_b16: in each aligned group of 16 lanes, lane i points at 4
// consecutive 16-bit values (row i / 4, columns 4 (i % 4) .. + 3 of a 4 x 16
// block); lane j receives column j of the block, rows 0 .. 3.
inline simt_i16x4 __builtin_amdgcn_ds_read_tr16_b64_v4i16(const void *p) {
  const int t = simt::ctx.flat, lane = t & 63, base = t - (lane & 15), j = lane & 15;
  simt::put(0, p);
  simt::group_sync(16);
  simt_i16x4 r;
  for (int y = 0; y < 4; ++y) r[y] = static_cast<const short *>(simt::get<const void *>(base + 4 * y + (j >> 2), 0))[j & 3];
  simt::group_sync(16);
  return r;
}
inline simt_f4 __builtin_amdgcn_mfma_f32_16x16x32_bf16(simt_bf8 a, simt_bf8 b, simt_f4 c, int, int, int) {
  return simt_mfma_k32(a, b, c);
}
inline simt_f4 __builtin_amdgcn_mfma_f32_16x16x32_f16(simt_h8 a, simt_h8 b, simt_f4 c, int, int, int) {
  return simt_mfma_k32(a, b, c);
}

// atomics (device and workgroup scopes collapse to the host's)
#define __HIP_MEMORY_SCOPE_WAVEFRONT 1
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __HIP_MEMORY_SCOPE_SYSTEM 4
template <typename T>
inline T simt_atomic_load(const T *p) {
  T r;
  __atomic_load(p, &r, __ATOMIC_SEQ_CST);
  return r;
}
template <typename T, typename V>
inline void simt_atomic_store(T *p, V v) {
  T x = (T)v;
  __atomic_store(p, &x, __ATOMIC_SEQ_CST);
}
#define __hip_atomic_load(p, order, scope) simt_atomic_load(p)
#define __hip_atomic_store(p, v, order, scope) simt_atomic_store(p, v)
#define __hip_atomic_fetch_add(p, v, order, scope) __atomic_fetch_add(p, v, order)
template <typename A, typename B>
inline auto min(A a, B b) -> decltype(a < b ? a : b) { return a < b ? a : b; }
template <typename A, typename B>
inline auto max(A a, B b) -> decltype(a < b ? a : b) { return a < b ? b : a; }
inline int atomicOr(int *p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicOr(unsigned *p, unsigned v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline int atomicAdd(int *p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicAdd(unsigned *p, unsigned v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicExch(unsigned *p, unsigned v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }
inline int atomicExch(int *p, int v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }
template <typename T>
inline T simt_atomic_min(T *p, T v) {
  T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (v < cur && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return cur;
}
template <typename T>
inline T simt_atomic_max(T *p, T v) {
  T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (v > cur && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return cur;
}
inline int atomicMin(int *p, int v) { return simt_atomic_min(p, v); }
inline unsigned long long atomicMin(unsigned long long *p, unsigned long long v) { return simt_atomic_min(p, v); }
inline int atomicMax(int *p, int v) { return simt_atomic_max(p, v); }

inline long long __double_as_longlong(double d) { long long r; memcpy(&r, &d, 8); return r; }
inline double __longlong_as_double(long long l) { double r; memcpy(&r, &l, 8); return r; }
inline float __uint_as_float(unsigned u) { float r; memcpy(&r, &u, 4); return r; }
inline unsigned __float_as_uint(float f) { unsigned r; memcpy(&r, &f, 4); return r; }

// HIP's vector types are aligned to their size; so are these, and their
// copies and assignments go member by member, so that the alignment sanitizer
// reports every load or store through a misaligned vector pointer (as a
// 16-byte LDS access at an 8-byte boundary would be on the device)
#define SIMT_VEC4(T, E, A)                                                             \
  struct alignas(A) T {                                                                \
    E x, y, z, w;                                                                      \
    T() = default;                                                                     \
    constexpr T(E a, E b, E c, E d) : x(a), y(b), z(c), w(d) {}                        \
    T(const T &o) : x(o.x), y(o.y), z(o.z), w(o.w) {}                                  \
    T &operator=(const T &o) {                                                         \
      x = o.x;                                                                         \
      y = o.y;                                                                         \
      z = o.z;                                                                         \
      w = o.w;                                                                         \
      return *this;                                                                    \
    }                                                                                  \
  };
#define SIMT_VEC2(T, E, A)                                                             \
  struct alignas(A) T {                                                                \
    E x, y;                                                                            \
    T() = default;                                                                     \
    constexpr T(E a, E b) : x(a), y(b) {}                                              \
    T(const T &o) : x(o.x), y(o.y) {}                                                  \
    T &operator=(const T &o) {                                                         \
      x = o.x;                                                                         \
      y = o.y;                                                                         \
      return *this;                                                                    \
    }                                                                                  \
  };
// bit casts through memcpy (the vector types above are not trivially copyable)
template <class To, class From>
inline To simt_bit_cast(const From &f) {
  static_assert(sizeof(To) == sizeof(From), "bit cast between types of different sizes");
  To t;
  memcpy((void *)&t, (const void *)&f, sizeof(To));
  return t;
}
#define __builtin_bit_cast(T, v) simt_bit_cast<T>(v)
SIMT_VEC4(uint4, unsigned, 16)
SIMT_VEC4(float4, float, 16)
SIMT_VEC2(double2, double, 16)
SIMT_VEC2(uint2, unsigned, 8)
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return uint4{a, b, c, d}; }
inline float4 make_float4(float a, float b, float c, float d) { return float4{a, b, c, d}; }
inline double2 make_double2(double a, double b) { return double2{a, b}; }
template <typename T, unsigned N> using HIP_vector_type = T;

// ---------------------------------------------------------------- runtime API
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorInvalidDevice = 101,
       hipErrorLaunchFailure = 719 };
struct ihipStream_t;
struct ihipEvent_t;
struct ihipGraph;
struct ihipGraphExec;
typedef ihipStream_t *hipStream_t;
typedef ihipEvent_t *hipEvent_t;
typedef ihipGraph *hipGraph_t;
typedef ihipGraphExec *hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount, hipDeviceAttributeMaxSharedMemoryPerBlock };

hipError_t hipMalloc(void **p, size_t n);
template <typename T>
inline hipError_t hipMalloc(T **p, size_t n) { return hipMalloc(reinterpret_cast<void **>(p), n); }
hipError_t hipFree(void *p);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t st);
hipError_t hipStreamSynchronize(hipStream_t st);
hipError_t hipDeviceSynchronize();
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned f);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned f);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned f);
hipError_t hipSetDevice(int d);
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int d);
hipError_t hipFuncSetAttribute(const void *f, hipFuncAttribute a, int v);
hipError_t hipGetLastError();
// device globals are host globals here: the symbol's address is the array's
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) {
  *p = const_cast<void *>(sym);
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, void *, char *, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t x);
const char *hipGetErrorString(hipError_t e);

namespace simt {
template <typename K, typename... A>
void launch(const char *name, K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st, A... args) {
  launch_impl(name, grid, block, lds, (void *)st, [=]() { kernel(args...); });
}
}  // namespace simt
#define hipLaunchKernelGGL(k, g, b, l, s, ...) simt::launch(#k, k, g, b, l, s, __VA_ARGS__)

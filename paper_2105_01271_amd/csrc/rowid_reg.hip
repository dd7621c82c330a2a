// Row ID pivot steps in one launch with the rows of W held in registers
// (paper Sec. 4, row ID; TPC-ID, Alg. 4): rank-k column-pivoted QR of W^T,
// W m x s row-major, taken in its left-looking (pivoted Cholesky) form so that
// no residual is ever stored or exchanged.
//
// With c_{i,l} = q_l . w_i (the entries R[l, i] of the pivoted QR) and
// nu_i = ||residual_i||^2, step j with pivot p computes, for every unselected i,
//
//   R_jj = sqrt(nu_p),   c_{i,j} = (w_i . w_p - sum_{l<j} c_{p,l} c_{i,l}) / R_jj,
//   nu_i <- nu_i - c_{i,j}^2,
//
// which is the Gram-Schmidt recurrence with q_j = (w_p - sum_l c_{p,l} q_l) / R_jj
// written without q: only the original rows (read-only) and the coefficients
// are needed.  The pivot rule is that of the other ID kernels (largest nu, nu
// truncated to 34 mantissa bits, ties to the lowest index), on downdated norms:
// nu_i carries a relative error of about u (nu_0 / nu_i)^(3/2) (the
// subtraction and the coefficients' own rounding), which stays below 1e-8 of
// a pivot gap while the pivot's norm^2 is above 1e-5 of the first pivot's.
// Past that point the launch stops (every workgroup takes the same decision)
// and the one-workgroup kernel after it redoes the factorization with
// recomputed norms.  Products are FP64; W is read as FP32 only when its
// values are FP32 numbers exactly.
//
// Launch: G = ceil(m / RPW) workgroups of NT threads, at most one per compute
// unit (the rows of a workgroup fill its registers), all resident at once.
// Thread t holds entries t + NT u (u < EPT) of each of its workgroup's rows.
// Each step has one exchange: a workgroup stores the norms of its rows and
// its coefficient column (into R), then its word (step in the top bits, then
// pivot rank, then the inverted index) in its own slot; thread g of every
// workgroup waits for slot g to carry the step and the maximum over the slots
// names the pivot, whose norm and coefficients are read back from where its
// owner stored them.  Exchanges use device-coherent relaxed atomic stores and
// loads, a writer's data stores complete before its word (devsync.h), and the
// slots alternate by step parity (a workgroup is at most one step ahead of any
// other).  Every wait is
// bounded: past the bound the workgroup raises DSK_FLAG_SYNC_TIMEOUT and sets
// the abort word, every workgroup leaves, and the one-workgroup kernel after
// it (k_rowid_rescue: right-looking Gram-Schmidt with norms recomputed from the
// residuals, as the per-step kernels) redoes the factorization from W, so the
// outputs stay valid without the host having to look.
#include <algorithm>

#include "devsync.h"
#include "dsk_internal.h"
#include "wavechol.h"

namespace {

constexpr int KMAX = 112;
constexpr int TAGW = 32;                   // one word per 256-byte line
constexpr long long SPIN_LIMIT = 1LL << 22;
constexpr double DOWNDATE_MIN = 1e-5;      // smallest pivot norm^2 / first pivot norm^2 taken here

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// pivot order: nu truncated to 34 mantissa bits (+1); selected / NaN -> 0
__device__ __forceinline__ unsigned long long nu_rank(double v) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFull;
  return (v >= 0.0) ? (bits >> 18) + 1ull : 0ull;
}

// step (7 bits) at 57.., pivot rank (46 bits) at 11.., inverted index (11 bits)
// at 0..10: the maximum over a step's words is its pivot (largest rank, then
// lowest index), and any word of a later step exceeds every word of this one
__device__ __forceinline__ unsigned long long pack_word(int step, unsigned long long rank, long long idx) {
  return ((unsigned long long)step << 57) | (rank << 11) | (unsigned long long)(~idx & 0x7FF);
}

// bounded wait for slot wp to carry step `step`; false on timeout or abort
__device__ __forceinline__ bool wait_word(const unsigned long long *wp, int step, int *abort_flag,
                                          unsigned long long &word) {
  long long spins = 0;
  for (;;) {
    word = (unsigned long long)ds::ld_dev(reinterpret_cast<const long long *>(wp));
    if ((int)(word >> 57) == step) break;
    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || ++spins > SPIN_LIMIT) {
      atomicOr(abort_flag, 1);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  ds::after_flag();
  return true;
}

template <typename T>
__device__ __forceinline__ double to_f64(T v) { return (double)v; }
__device__ __forceinline__ double to_f64(__bf16 v) { return (double)(float)v; }
__device__ __forceinline__ double to_f64(_Float16 v) { return (double)(float)v; }

// 16 bytes of T as a native vector (a struct copy from global memory would
// become a memcpy that keeps the values out of registers)
template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<__bf16> { typedef __bf16 type __attribute__((ext_vector_type(8))); };
template <> struct Vec16<_Float16> { typedef _Float16 type __attribute__((ext_vector_type(8))); };

// The EPT elements of row i that thread t holds: runs of VE = 16 / sizeof(T)
// consecutive columns, VE t + NT VE q + v (q < EPT / VE), fetched with 16-byte
// loads when rows start 16-byte aligned (vec); else one element per load.
template <typename T, int NT, int EPT>
__device__ __forceinline__ void load_row(const T *__restrict__ W, int64_t m, int64_t s, int64_t i, bool vec,
                                         T (&dst)[EPT]) {
  constexpr int VE = 16 / (int)sizeof(T);
  static_assert(EPT % VE == 0, "whole 16-byte runs per thread");
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < EPT / VE; ++q) {
    const int64_t e0 = (int64_t)VE * t + (int64_t)NT * VE * q;
    if (vec && i < m && e0 + VE <= s) {
      const typename Vec16<T>::type x = *reinterpret_cast<const typename Vec16<T>::type *>(W + i * s + e0);
#pragma unroll
      for (int v = 0; v < VE; ++v) dst[q * VE + v] = x[v];
    } else {
#pragma unroll
      for (int v = 0; v < VE; ++v) dst[q * VE + v] = (i < m && e0 + v < s) ? W[i * s + e0 + v] : T(0);
    }
  }
}

// Sum over the wave in lane 0: DPP sums within each row of 16 lanes, then the
// four row sums in row order (no LDS round trips).
__device__ __forceinline__ double wave_total(double v) {
  v = wc::row16_sum(v);
  return (wc::readlane_f64(v, 0) + wc::readlane_f64(v, 16)) + (wc::readlane_f64(v, 32) + wc::readlane_f64(v, 48));
}

// Sum over the workgroup of v[r] for each r < R (wave sums, then waves in a
// fixed order); thread r < R receives the total of v[r].  One barrier; the
// caller keeps a barrier between this call and the next (red is reused).
template <int NW, int R>
__device__ __forceinline__ double block_sums(double (&v)[R], double (*red)[R]) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double a = wave_total(v[r]);
    if (lane == 0) red[wave][r] = a;
  }
  __syncthreads();
  double a = 0.0;
  if (t < R)
    for (int w = 0; w < NW; ++w) a += red[w][t];
  return a;
}

template <typename T, int NT, int RPW, int EPT>
__global__ void __launch_bounds__(NT) k_rowid_reg(const T *__restrict__ W, int64_t m, int64_t s, int k, int vec,
                                                  unsigned long long *words, double *nuG, int *abort_flag, double *__restrict__ nu_final, double *Rk,
                                                  int64_t *__restrict__ piv, int *__restrict__ dflags) {
  constexpr int NW = NT / 64;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int G = gridDim.x, gid = blockIdx.x;
  __shared__ double red[NW][RPW];
  __shared__ unsigned long long bk[NW];
  __shared__ double nu_sh[RPW];
  __shared__ int live_sh[RPW];
  __shared__ double cl[RPW][KMAX];     // c_{i,l} of this workgroup's rows
  __shared__ double cp[KMAX];          // c_{p,l} of the pivot
  __shared__ unsigned long long key_sh;
  __shared__ double rjj_sh;
  __shared__ double nu_first;
  __shared__ int stop_sh;   // written by thread 0 before the barrier that precedes every read
  __shared__ int down_sh;   // likewise, in the pivot phase

  const int64_t row0 = (int64_t)gid * RPW;
  T w[RPW][EPT];
#pragma unroll
  for (int r = 0; r < RPW; ++r) load_row<T, NT, EPT>(W, m, s, row0 + r, vec != 0, w[r]);
  {
    double v[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      double a = 0.0;
#pragma unroll
      for (int u = 0; u < EPT; ++u) a = fma(to_f64(w[r][u]), to_f64(w[r][u]), a);
      v[r] = a;
    }
    const double a = block_sums<NW, RPW>(v, red);
    if (t < RPW) nu_sh[t] = a;
  }
  if (t < RPW) {
    live_sh[t] = (row0 + t < m) ? 1 : 0;
    if (live_sh[t] && !isfinite(nu_sh[t])) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
  }
  if (t == 0) {
    stop_sh = 0;
    down_sh = 0;
  }
  __syncthreads();

  for (int j = 0; j < k; ++j) {
    const int par = j & 1;
    // ---- publish: norms of this workgroup's rows (selected: -1), then the word
    if (t < RPW && row0 + t < m) ds::st_dev(&nuG[(int64_t)par * m + row0 + t], live_sh[t] ? nu_sh[t] : -1.0);
    ds::stores_done();
    __syncthreads();
    if (t == 0) {
      unsigned long long brank = 0;
      long long bidx = m;
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        if (!live_sh[r]) continue;
        const unsigned long long rk = nu_rank(nu_sh[r]);
        if (rk > brank) { brank = rk; bidx = row0 + r; }   // ascending rows: ties keep the lower index
      }
      ds::st_dev(reinterpret_cast<long long *>(&words[((int64_t)par * G + gid) * TAGW]),
                 (long long)pack_word(j + 1, brank, bidx));
    }
    // ---- every slot of the step; maximum of (rank, inverted index)
    unsigned long long best = 0;
    for (int g = t; g < G; g += NT) {
      unsigned long long wd;
      if (!wait_word(&words[((int64_t)par * G + g) * TAGW], j + 1, abort_flag, wd)) {
        stop_sh = 1;
        break;
      }
      best = max(best, wd);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = max(best, (unsigned long long)__shfl_xor((long long)best, o, 64));
    if (lane == 0) bk[wave] = best;
    __syncthreads();
    if (t == 0) {
      unsigned long long b = bk[0];
      for (int w2 = 1; w2 < NW; ++w2) b = max(b, bk[w2]);
      key_sh = b;
    }
    __syncthreads();
    if (stop_sh) break;
    const unsigned long long key = key_sh;
    const int64_t p = ((key >> 11) & ((1ull << 46) - 1)) ? (int64_t)(~key & 0x7FF) : m;
    // ---- the pivot: its row from W, its norm and coefficients from where its owner
    // stored them, all requested at once (one round trip)
    T wp[EPT];
    load_row<T, NT, EPT>(W, m, s, p, vec != 0, wp);
    if (t == 0) {
      const double nup = (p < m) ? ds::ld_dev(&nuG[(int64_t)par * m + p]) : 0.0;
      rjj_sh = nup > 0.0 ? sqrt(nup) : 0.0;
      if (j == 0) nu_first = nup;
      // downdated norms no longer resolve 1e-8 pivot gaps: leave to the exact rescue
      if (nup < DOWNDATE_MIN * nu_first && nup > 0.0) down_sh = 1;
    }
    if (t < j) cp[t] = (p < m) ? ds::ld_dev(&Rk[(int64_t)t * m + p]) : 0.0;
    __syncthreads();
    if (down_sh) break;
    const double rjj = rjj_sh;
    if (gid == 0 && t == 0) {
      piv[j] = p;
      if (p < m) ds::st_dev(&Rk[(int64_t)j * m + p], rjj);
      if (!(rjj > 0.0)) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_RANK_DEFICIENT);
    }
    // ---- w_i . w_p - sum_{l<j} c_{p,l} c_{i,l} for this workgroup's rows.  The rows
    // are marked as rewritten each step so that their FP64 conversions are not
    // hoisted out of the loop (that would double the registers they take).
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
      for (int u = 0; u < EPT; ++u) asm volatile("" : "+v"(w[r][u]));
    double v[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      double a = 0.0;
#pragma unroll
      for (int u = 0; u < EPT; ++u) a = fma(to_f64(w[r][u]), to_f64(wp[u]), a);
      if (t < j) a = fma(-cp[t], cl[r][t], a);
      v[r] = a;
    }
    const double num = block_sums<NW, RPW>(v, red);
    if (t < RPW) {
      const int64_t i = row0 + t;
      if (i == p) live_sh[t] = 0;
      if (live_sh[t]) {
        const double c = rjj > 0.0 ? num / rjj : 0.0;
        cl[t][j] = c;
        ds::st_dev(&Rk[(int64_t)j * m + i], c);
        const double nn = nu_sh[t] - c * c;
        nu_sh[t] = nn > 0.0 ? nn : 0.0;
      }
    }
    __syncthreads();
  }
  if (stop_sh || down_sh) {
    if (t == 0) {
      atomicOr(&dflags[FLAGW_BITS], stop_sh ? DSK_FLAG_SYNC_TIMEOUT : DSK_FLAG_FALLBACK);
      if (!stop_sh) atomicOr(abort_flag, 1);
    }
    return;
  }
  if (t < RPW && row0 + t < m) nu_final[row0 + t] = live_sh[t] ? nu_sh[t] : -1.0;
}

// Leaves at once unless the one-launch kernel gave up (a wait timed out, or the
// downdated norms ran out of accuracy); then one workgroup redoes the whole
// factorization as the per-step kernels do: right-looking modified
// Gram-Schmidt on an FP64 copy Wr of W, norms recomputed from the residuals
// every step, the same pivot rule.  Slow for wide W, but only taken then.
template <typename T>
__global__ void __launch_bounds__(1024) k_rowid_rescue(const T *__restrict__ W, int64_t m, int64_t s, int k,
                                                       const int *abort_flag, double *__restrict__ Wr,
                                                       double *__restrict__ nuR, double *__restrict__ nu_final,
                                                       double *__restrict__ Rk, int64_t *__restrict__ piv,
                                                       int *__restrict__ dflags) {
  if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  constexpr int WV = 16;
  __shared__ unsigned long long bk[WV];
  __shared__ int64_t p_sh;
  __shared__ double rjj_sh;
  for (int64_t x = t; x < m * s; x += 1024) Wr[x] = to_f64(W[x]);
  __syncthreads();
  for (int64_t i = wave; i < m; i += WV) {
    double a = 0.0;
    for (int64_t e = lane; e < s; e += 64) a = fma(Wr[i * s + e], Wr[i * s + e], a);
    a = wsum(a);
    if (lane == 0) nuR[i] = a;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    unsigned long long best = 0;
    for (int64_t i = t; i < m; i += 1024) {
      const unsigned long long key = (nu_rank(nuR[i]) << 11) | (unsigned long long)(~i & 0x7FF);
      best = max(best, key);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = max(best, (unsigned long long)__shfl_xor((long long)best, o, 64));
    if (lane == 0) bk[wave] = best;
    __syncthreads();
    if (t == 0) {
      unsigned long long b = bk[0];
      for (int w2 = 1; w2 < WV; ++w2) b = max(b, bk[w2]);
      const int64_t p = (b >> 11) ? (int64_t)(~b & 0x7FF) : m;
      const double nup = p < m ? nuR[p] : 0.0;
      p_sh = p;
      rjj_sh = nup > 0.0 ? sqrt(nup) : 0.0;
      piv[j] = p;
      if (p < m) {
        Rk[(int64_t)j * m + p] = rjj_sh;
        nuR[p] = -1.0;
      }
      if (!(rjj_sh > 0.0)) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_RANK_DEFICIENT);
    }
    __syncthreads();
    const int64_t p = p_sh;
    const double qs = rjj_sh > 0.0 ? 1.0 / rjj_sh : 0.0;
    for (int64_t i = wave; i < m; i += WV) {
      if (!(nuR[i] >= 0.0) || p >= m) continue;
      double a = 0.0;
      for (int64_t e = lane; e < s; e += 64) a = fma(Wr[p * s + e] * qs, Wr[i * s + e], a);
      a = wsum(a);
      double nn = 0.0;
      for (int64_t e = lane; e < s; e += 64) {
        const double v = fma(-a, Wr[p * s + e] * qs, Wr[i * s + e]);
        Wr[i * s + e] = v;
        nn = fma(v, v, nn);
      }
      nn = wsum(nn);
      if (lane == 0) {
        Rk[(int64_t)j * m + i] = a;
        nuR[i] = nn;
      }
    }
    __syncthreads();
  }
  for (int64_t i = t; i < m; i += 1024) nu_final[i] = nuR[i] >= 0.0 ? nuR[i] : -1.0;
}

__global__ void k_rowid_reset(unsigned long long *words, int nslots, int *abort_flag, int64_t *piv, int k) {
  for (int i = threadIdx.x; i < nslots; i += blockDim.x) words[(int64_t)i * TAGW] = 0;
  if (threadIdx.x == 0) *abort_flag = 0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) piv[i] = -1;
}

struct Plan {
  int nt, rpw, ept, g;
};

// Workgroup size, rows per workgroup and entries per thread, or rpw = 0 when
// the shape does not fit (more than one workgroup per compute unit, rows wider
// than 8192, more than 2048 candidates, or more than 128 registers of row
// data per thread).
Plan plan_of(int64_t m, int64_t s, int k, int esize, int cu_count) {
  Plan pl{0, 0, 0, 0};
  if (m < 1 || s < 1 || k < 1 || k > KMAX || m > 2048 || s > 8192) return pl;
  const int nt = 512;
  // (at least one 16-byte run per thread)
  const int ept = std::max(s <= 2048 ? 4 : (s <= 4096 ? 8 : 16), 16 / esize);
  for (int rpw : {4, 8}) {
    const int64_t g = (m + rpw - 1) / rpw;
    if (g > cu_count) continue;
    if (rpw * ept * esize / 4 > 128) continue;
    pl.nt = nt;
    pl.rpw = rpw;
    pl.ept = ept;
    pl.g = (int)g;
    return pl;
  }
  return pl;
}

template <typename T>
int launch_typed(hipStream_t st, const T *W, int64_t m, int64_t s, int k, double *nu_final, double *Rk, int64_t *piv,
                 char *ws, const Plan &pl, int *dflags) {
  unsigned long long *words = reinterpret_cast<unsigned long long *>(ws);           // 2 G slots, one line each
  double *nuG = reinterpret_cast<double *>(ws + (size_t)2 * pl.g * TAGW * 8);
  double *nuR = nuG + 2 * m;
  double *Wr = nuR + m;                          // the rescue's FP64 residuals, m x s
  int *abort_flag = reinterpret_cast<int *>(Wr + (size_t)m * s);
  hipLaunchKernelGGL(k_rowid_reset, dim3(1), dim3(256), 0, st, words, 2 * pl.g, abort_flag, piv, k);
  DSK_TRY(hipGetLastError());
  // 16-byte runs need aligned row starts
  const int vec = ((s * (int64_t)sizeof(T)) % 16 == 0 && (reinterpret_cast<uintptr_t>(W) & 15) == 0) ? 1 : 0;
#define DSK_RREG(NT_, R_, E_)                                                                                   \
  if constexpr (E_ % (16 / (int)sizeof(T)) == 0 && R_ * E_ * (int)sizeof(T) / 4 <= 128)                       \
    if (pl.nt == NT_ && pl.rpw == R_ && pl.ept == E_)                                                           \
      hipLaunchKernelGGL((k_rowid_reg<T, NT_, R_, E_>), dim3(pl.g), dim3(NT_), 0, st, W, m, s, k, vec, words, nuG, \
                         abort_flag, nu_final, Rk, piv, dflags);
  DSK_RREG(512, 4, 4) DSK_RREG(512, 8, 4) DSK_RREG(512, 4, 8) DSK_RREG(512, 8, 8) DSK_RREG(512, 4, 16)
  DSK_RREG(512, 8, 16)
#undef DSK_RREG
  DSK_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_rowid_rescue<T>, dim3(1), dim3(1024), 0, st, W, m, s, k, abort_flag, Wr, nuR, nu_final, Rk,
                     piv, dflags);
  DSK_TRY(hipGetLastError());
  return 0;
}

}  // namespace

static int wsize(int wdt) { return wdt == DSK_F64 ? 8 : (wdt == DSK_F32 ? 4 : 2); }

size_t rowid_reg_ws_bytes(int64_t m, int64_t s, int k, int wdt, int cu_count) {
  const Plan pl = plan_of(m, s, k, wsize(wdt), cu_count);
  if (!pl.rpw) return 0;
  return (size_t)2 * pl.g * TAGW * 8 + (size_t)3 * m * 8 + (size_t)m * s * 8 + 256;
}

int launch_rowid_reg(hipStream_t st, const void *W, int wdt, int64_t m, int64_t s, int k, double *nu_final,
                     double *Rk, int64_t *piv, void *ws, int cu_count, int *dflags) {
  const Plan pl = plan_of(m, s, k, wsize(wdt), cu_count);
  if (!pl.rpw) return -1;
  char *w = reinterpret_cast<char *>(ws);
  switch (wdt) {
    case DSK_F64: return launch_typed<double>(st, (const double *)W, m, s, k, nu_final, Rk, piv, w, pl, dflags);
    case DSK_F32: return launch_typed<float>(st, (const float *)W, m, s, k, nu_final, Rk, piv, w, pl, dflags);
    case DSK_BF16: return launch_typed<__bf16>(st, (const __bf16 *)W, m, s, k, nu_final, Rk, piv, w, pl, dflags);
    default: return launch_typed<_Float16>(st, (const _Float16 *)W, m, s, k, nu_final, Rk, piv, w, pl, dflags);
  }
}

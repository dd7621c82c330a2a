// Small dense factorizations of the sketch pipeline.
//
//  * Orthonormalisation of tall-skinny blocks (the QR steps of Alg. 2 and
//    Alg. 7): CholeskyQR2 with an FP64 Gram, FP64 Cholesky and FP64 R^{-1}.
//    If the first Cholesky meets a non-positive or negligible pivot, the same
//    kernel retries with the shift 11 (rows*ell + ell(ell+1)) u ||Y||_F^2 and
//    raises DSK_FLAG_FALLBACK; a third (conditional) pass then restores
//    orthonormality (shifted CholeskyQR3, Fukaya et al. 2020).
//  * Single-workgroup Householder QR with explicit Q (FP64 path, where blocks
//    may be numerically rank deficient).
//  * Skinny products out = X M diag(scale) and the sign normalisation of U.
// All reductions use fixed orders, so repeated runs give identical bytes.
#include <algorithm>

#include "dsk_internal.h"

namespace {

constexpr int ELL_MAX = 112;
constexpr double U64 = 1.1102230246251565e-16;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum in a fixed order (per-wave shuffles, then waves in order).
template <int NT>
__device__ double block_sum(double v, double *scratch /* >= NT/64 + 1 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += scratch[w];
    scratch[NT / 64] = s;
  }
  __syncthreads();
  return scratch[NT / 64];
}

// ---------------------------------------------------------------- Gram partials
// Each thread owns up to three 4x4 blocks (bi <= bj) of the ellp x ellp Gram,
// block ids threadIdx.x, threadIdx.x + 256, threadIdx.x + 512; three separate
// statically indexed accumulators keep everything in registers.
struct GramAcc {
  double a0[16], a1[16], a2[16];
};

__device__ __forceinline__ void gram_zero(GramAcc &g) {
#pragma unroll
  for (int e = 0; e < 16; ++e) { g.a0[e] = 0.0; g.a1[e] = 0.0; g.a2[e] = 0.0; }
}

__device__ __forceinline__ void pair_of(int pid, int nb, int &bi, int &bj) {
  int r = 0, rem = pid;
  while (rem >= nb - r) { rem -= nb - r; ++r; }
  bi = r;
  bj = r + rem;
}

__device__ __forceinline__ void gram_chunk_u(const double *sh, int CH, int ellp, int bi, int bj, bool on,
                                             double (&acc)[16]) {
  if (!on) return;
  for (int r = 0; r < CH; ++r) {
    const double *row = sh + r * ellp;
    double xs[4], ys[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) { xs[a] = row[4 * bi + a]; ys[a] = row[4 * bj + a]; }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a * 4 + b] = fma(xs[a], ys[b], acc[a * 4 + b]);
  }
}

struct GramSlots {
  int bi[3], bj[3];
  bool on[3];
};

__device__ __forceinline__ GramSlots gram_slots(int ellp) {
  GramSlots s;
  const int nb = ellp / 4, npairs = nb * (nb + 1) / 2;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int pid = threadIdx.x + 256 * u;
    s.on[u] = pid < npairs;
    s.bi[u] = s.bj[u] = 0;
    if (s.on[u]) pair_of(pid, nb, s.bi[u], s.bj[u]);
  }
  return s;
}

__device__ __forceinline__ void gram_chunk(const double *sh, int CH, int ellp, const GramSlots &s, GramAcc &g) {
  gram_chunk_u(sh, CH, ellp, s.bi[0], s.bj[0], s.on[0], g.a0);
  gram_chunk_u(sh, CH, ellp, s.bi[1], s.bj[1], s.on[1], g.a1);
  gram_chunk_u(sh, CH, ellp, s.bi[2], s.bj[2], s.on[2], g.a2);
}

__device__ __forceinline__ void gram_store_u(const double (&acc)[16], int bi, int bj, bool on, int ell,
                                             double *part) {
  if (!on) return;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = 4 * bi + a, c = 4 * bj + b;
      if (r < ell && c < ell) {
        part[r * ell + c] = acc[a * 4 + b];
        part[c * ell + r] = acc[a * 4 + b];
      }
    }
}

__device__ __forceinline__ void gram_store(const GramAcc &g, const GramSlots &s, int ell, double *part) {
  gram_store_u(g.a0, s.bi[0], s.bj[0], s.on[0], ell, part);
  gram_store_u(g.a1, s.bi[1], s.bj[1], s.on[1], ell, part);
  gram_store_u(g.a2, s.bi[2], s.bj[2], s.on[2], ell, part);
}

constexpr int GCH = 32;

template <typename T>
__global__ void __launch_bounds__(256) k_gram_part(const T *__restrict__ X, int64_t rows, int ell, int64_t ldx,
                                                   int64_t rows_per_blk, double *__restrict__ part,
                                                   const int *__restrict__ dflags, int cond) {
  if (cond && !(dflags[FLAGW_BITS] & DSK_FLAG_FALLBACK)) return;
  __shared__ double sh[GCH * ELL_MAX];
  const int ellp = (ell + 3) & ~3;
  const GramSlots slots = gram_slots(ellp);
  GramAcc g;
  gram_zero(g);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(rows, r0 + rows_per_blk);
  for (int64_t c0 = r0; c0 < r1; c0 += GCH) {
    for (int e = threadIdx.x; e < GCH * ellp; e += 256) {
      const int rr = e / ellp, c = e - rr * ellp;
      const int64_t r = c0 + rr;
      sh[e] = (r < r1 && c < ell) ? (double)X[r * ldx + c] : 0.0;
    }
    __syncthreads();
    gram_chunk(sh, GCH, ellp, slots, g);
    __syncthreads();
  }
  gram_store(g, slots, ell, part + (int64_t)blockIdx.x * ell * ell);
}

// Gram partials of a long block (ell <= 64): every thread owns one 4x4 block of
// the Gram for one of RG = 256 / npairs row groups (rows r = rg mod RG of each
// 32-row chunk), so all threads work; the next chunk is prefetched into
// registers while the current one is consumed from LDS.  Row groups are
// combined in a fixed order at the end.
template <typename T>
__global__ void __launch_bounds__(256) k_gram_rows(const T *__restrict__ X, int64_t rows, int ell, int64_t ldx,
                                                   int64_t rows_per_blk, double *__restrict__ part) {
  constexpr int PF = GCH * 64 / 256;
  __shared__ double sh[GCH * 64];
  __shared__ double comb[256 * 16];
  const int ellp = (ell + 3) & ~3, nb = ellp / 4, npairs = nb * (nb + 1) / 2;
  const int RG = 256 / npairs;
  const int t = threadIdx.x, rg = t / npairs, pid = t - rg * npairs;
  const bool on = rg < RG;
  int bi = 0, bj = 0;
  if (on) pair_of(pid, nb, bi, bj);
  double acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(rows, r0 + rows_per_blk);
  const int tot = GCH * ellp;
  T pf[PF];
  auto fetch = [&](int64_t c0) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = t + 256 * u;
      const int rr = e / ellp, c = e - rr * ellp;
      const int64_t r = c0 + rr;
      pf[u] = (e < tot && r < r1 && c < ell) ? X[r * ldx + c] : T(0);
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t c0 = r0; c0 < r1; c0 += GCH) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = t + 256 * u;
      if (e < tot) sh[e] = (double)pf[u];
    }
    __syncthreads();
    if (c0 + GCH < r1) fetch(c0 + GCH);
    if (on) {
      for (int r = rg; r < GCH; r += RG) {
        const double *row = sh + r * ellp;
        double xs[4], ys[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) { xs[a] = row[4 * bi + a]; ys[a] = row[4 * bj + a]; }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a * 4 + b] = fma(xs[a], ys[b], acc[a * 4 + b]);
      }
    }
    __syncthreads();
  }
  if (on && rg > 0) {
#pragma unroll
    for (int e = 0; e < 16; ++e) comb[((rg - 1) * npairs + pid) * 16 + e] = acc[e];
  }
  __syncthreads();
  if (on && rg == 0) {
    for (int g = 1; g < RG; ++g)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e] += comb[((g - 1) * npairs + pid) * 16 + e];
    gram_store_u(acc, bi, bj, true, ell, part + (int64_t)blockIdx.x * ell * ell);
  }
}

// G = sum of nparts partials (n2 entries each).  A 256-thread workgroup covers
// 16 consecutive entries x 16 part groups; part group g adds parts g, g + 16, ...
// in order, then the 16 group sums are combined in a fixed order.
__global__ void __launch_bounds__(256) k_gram_reduce(const double *__restrict__ part, int nparts, int n2,
                                                     double *__restrict__ G) {
  __shared__ double red[16][17];
  const int t = threadIdx.x, eo = t & 15, g = t >> 4;
  const int e = blockIdx.x * 16 + eo;
  double s = 0.0;
  if (e < n2) {
    int p = g;
    double s1 = 0.0;
    for (; p + 16 < nparts; p += 32) {
      s += part[(int64_t)p * n2 + e];
      s1 += part[(int64_t)(p + 16) * n2 + e];
    }
    if (p < nparts) s += part[(int64_t)p * n2 + e];
    s += s1;
  }
  red[g][eo] = s;
  __syncthreads();
  if (t < 16 && blockIdx.x * 16 + t < n2) {
    double tot = 0.0;
    for (int i = 0; i < 16; ++i) tot += red[i][t];
    G[blockIdx.x * 16 + t] = tot;
  }
}

// G (LDS) = sum of the nparts (<= 32) Gram partials, n2 entries each, added in
// part order.  The partials were just written by other workgroups (other
// XCDs' L2), so every load is a long round trip: each thread keeps two entries
// x 16 parts of loads in flight per batch (256-thread workgroup).
__device__ void sum_parts_lds(const double *__restrict__ part, int nparts, int n2, double *G) {
  const int t = threadIdx.x;
  for (int e0 = t; e0 < n2; e0 += 2 * 256) {
    const int e1 = e0 + 256;
    double a = 0.0, b = 0.0;
    for (int p0 = 0; p0 < nparts; p0 += 16) {
      double va[16], vb[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int p = p0 + u;
        va[u] = (p < nparts) ? part[(int64_t)p * n2 + e0] : 0.0;
        vb[u] = (p < nparts && e1 < n2) ? part[(int64_t)p * n2 + e1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        a += va[u];
        b += vb[u];
      }
    }
    G[e0] = a;
    if (e1 < n2) G[e1] = b;
  }
}

// ---------------------------------------------------------------- Cholesky + inverse (one block)
// Sums the Gram partials in a fixed order, factors G = L L^T (retrying once with
// a shift on breakdown), inverts L in place and writes R = L^T, Rinv = L^{-T}.
// Thread t works on rows j + 1 + t/4 (+64) and on every 4th column (t % 4).
// Runs on one 256-thread workgroup; dyn must hold ell*ell + ell doubles.
__device__ void chol_body(const double *__restrict__ part, int nparts, int ell, int64_t rows,
                          double *__restrict__ R, double *__restrict__ Rinv, int *__restrict__ dflags,
                          double *dyn) {
  double *G = dyn;                 // ell x ell
  double *tmp = dyn + ell * ell;   // ell
  __shared__ double red[8];
  __shared__ int bad;
  __shared__ double pivinv;
  const int t = threadIdx.x;
  const int tr4 = t >> 2, tc4 = t & 3;
  const int n2 = ell * ell;
  for (int attempt = 0; attempt < 2; ++attempt) {
    sum_parts_lds(part, nparts, n2, G);
    __syncthreads();
    double trc = 0.0;
    for (int i = t; i < ell; i += 256) trc += G[i * ell + i];
    trc = block_sum<256>(trc, red);
    if (attempt == 1) {
      const double shift = 11.0 * ((double)rows * ell + (double)ell * (ell + 1)) * U64 * trc;
      for (int i = t; i < ell; i += 256) G[i * ell + i] += shift;
    }
    if (t == 0) bad = !(trc > 0.0) || !isfinite(trc);
    __syncthreads();
    const double thr = 1e-15 * trc;
    for (int j = 0; j < ell; ++j) {
      if (t == 0 && !bad) {
        const double d = G[j * ell + j];
        if (!(d > thr) || !isfinite(d)) {
          bad = 1;
        } else {
          G[j * ell + j] = sqrt(d);
          pivinv = 1.0 / d;
        }
      }
      __syncthreads();
      if (bad) break;
      // scale the column of the previous step (no thread reads it in this step)
      if (j > 0) {
        const double inv_prev = 1.0 / G[(j - 1) * ell + (j - 1)];
        for (int i = j + t; i < ell; i += 256) G[i * ell + (j - 1)] *= inv_prev;
      }
      // trailing update with the unscaled column j: G_ic -= G_ij G_cj / d
      const double pinv = pivinv;
      for (int i = j + 1 + tr4; i < ell; i += 64) {
        const double gij = G[i * ell + j] * pinv;
        for (int c = j + 1 + tc4; c <= i; c += 4) G[i * ell + c] -= gij * G[c * ell + j];
      }
      __syncthreads();
    }
    if (!bad) break;   // (the last column has nothing below its diagonal to scale)
    if (t == 0) atomicOr(&dflags[FLAGW_BITS], attempt == 0 ? DSK_FLAG_FALLBACK : DSK_FLAG_RANK_DEFICIENT);
    __syncthreads();
    if (attempt == 1) {
      // still failing (non-finite input): identity factors keep the pipeline finite
      for (int i = t >> 6; i < ell; i += 4)
        for (int c = t & 63; c < ell; c += 64) {
          R[i * ell + c] = (i == c) ? 1.0 : 0.0;
          Rinv[i * ell + c] = (i == c) ? 1.0 : 0.0;
        }
      if (t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
      return;
    }
    if (t == 0) bad = 0;
    __syncthreads();
  }
  // R = L^T
  for (int i = t >> 6; i < ell; i += 4)
    for (int c = t & 63; c < ell; c += 64) R[i * ell + c] = (c >= i) ? G[c * ell + i] : 0.0;
  __syncthreads();
  // in-place inverse of the lower-triangular L, column j from the inverted trailing block
  for (int j = ell - 1; j >= 0; --j) {
    if (t == 0) G[j * ell + j] = 1.0 / G[j * ell + j];
    for (int i = j + 1 + t; i < ell; i += 256) tmp[i] = G[i * ell + j];
    __syncthreads();
    const double ajj = -G[j * ell + j];
    for (int ib = j + 1; ib < ell; ib += 64) {
      const int i = ib + tr4;
      double s = 0.0;
      if (i < ell)
        for (int c = j + 1 + tc4; c <= i; c += 4) s += G[i * ell + c] * tmp[c];
      s += __shfl_xor(s, 1, 4);
      s += __shfl_xor(s, 2, 4);
      if (i < ell && tc4 == 0) G[i * ell + j] = ajj * s;
    }
    __syncthreads();
  }
  for (int i = t >> 6; i < ell; i += 4)
    for (int c = t & 63; c < ell; c += 64) Rinv[i * ell + c] = (c >= i) ? G[c * ell + i] : 0.0;
}

__global__ void __launch_bounds__(256) k_chol(const double *__restrict__ part, int nparts, int ell, int64_t rows,
                                              double *__restrict__ R, double *__restrict__ Rinv,
                                              int *__restrict__ dflags, int cond) {
  if (cond && !(dflags[FLAGW_BITS] & DSK_FLAG_FALLBACK)) return;
  extern __shared__ double dyn[];
  chol_body(part, nparts, ell, rows, R, Rinv, dflags, dyn);
}

// True in exactly one workgroup of the grid: the last one to publish its
// partial.  Release fence before the ticket, acquire fence after it (device
// scope), so the elected workgroup sees every partial.  The ticket counter is
// reset for the next launch by the elected workgroup.
__device__ bool last_block_done(unsigned *counter) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1) ? 1 : 0;
    if (last) atomicExch(counter, 0u);
  }
  __syncthreads();
  if (last) __threadfence();
  return last != 0;
}

// Gram partials of X; with a counter, the last workgroup also reduces them and
// factors (Cholesky + inverse), writing R and Rinv.
template <typename T>
__global__ void __launch_bounds__(256) k_gram_chol(const T *__restrict__ X, int64_t rows, int ell, int64_t ldx,
                                                   int64_t rows_per_blk, double *__restrict__ part,
                                                   unsigned *__restrict__ counter, double *__restrict__ R,
                                                   double *__restrict__ Rinv, int *__restrict__ dflags) {
  extern __shared__ double dyn[];
  double *sh = dyn;   // GCH x ellp (reused by the factorization afterwards)
  const int ellp = (ell + 3) & ~3;
  const GramSlots slots = gram_slots(ellp);
  GramAcc g;
  gram_zero(g);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(rows, r0 + rows_per_blk);
  for (int64_t c0 = r0; c0 < r1; c0 += GCH) {
    for (int e = threadIdx.x; e < GCH * ellp; e += 256) {
      const int rr = e / ellp, c = e - rr * ellp;
      const int64_t r = c0 + rr;
      sh[e] = (r < r1 && c < ell) ? (double)X[r * ldx + c] : 0.0;
    }
    __syncthreads();
    gram_chunk(sh, GCH, ellp, slots, g);
    __syncthreads();
  }
  gram_store(g, slots, ell, part + (int64_t)blockIdx.x * ell * ell);
  if (last_block_done(counter)) chol_body(part, gridDim.x, ell, rows, R, Rinv, dflags, dyn);
}

// ---------------------------------------------------------------- Q = Y Rinv (+ Gram partials of Q)
// Thread t owns output column c = t % CW and rows t/CW + (256/CW) u of each
// 32-row chunk; every Rinv entry is read once per chunk and reused across rows.
// cond = 1: run only after a shifted first pass.  With part != nullptr the
// workgroup also accumulates the Gram of the rounded output, and with a counter
// the last workgroup factors it into R, Rinv (all other workgroups have finished
// reading Rinv by then).  gram_cond = 1: the Gram/factorization only after a
// shifted first pass.
template <typename T, int CW>
__global__ void __launch_bounds__(256) k_apply(const T *__restrict__ Y, int64_t rows, int ell, int64_t ldy,
                                               double *__restrict__ Rinv, T *__restrict__ Q, int64_t ldq,
                                               int64_t rows_per_blk, double *__restrict__ part,
                                               int *__restrict__ dflags, int cond, unsigned *__restrict__ counter,
                                               double *__restrict__ R, int gram_cond) {
  const bool fallback = (dflags[FLAGW_BITS] & DSK_FLAG_FALLBACK) != 0;
  if (cond && !fallback) return;
  if (gram_cond && !fallback) {
    part = nullptr;
    counter = nullptr;
  }
  constexpr int RG = 256 / CW;            // row groups
  constexpr int RPT = GCH / RG;           // rows per thread per chunk
  extern __shared__ double dyn[];
  const int ellp = (ell + 3) & ~3;
  double *Rs = dyn;                       // ell x ell
  double *sh = dyn + ell * ell;           // GCH x ellp
  for (int e = threadIdx.x; e < ell * ell; e += 256) Rs[e] = Rinv[e];
  const GramSlots slots = gram_slots(ellp);
  GramAcc g;
  gram_zero(g);
  const int c = threadIdx.x % CW, rg = threadIdx.x / CW;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(rows, r0 + rows_per_blk);
  for (int64_t c0 = r0; c0 < r1; c0 += GCH) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int rr = rg + RG * u;
      const int64_t r = c0 + rr;
      for (int cc = c; cc < ellp; cc += CW) sh[rr * ellp + cc] = (r < r1 && cc < ell) ? (double)Y[r * ldy + cc] : 0.0;
    }
    __syncthreads();
    double acc[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) acc[u] = 0.0;
    if (c < ell) {
      for (int q = 0; q <= c; ++q) {
        const double rv = Rs[q * ell + c];
#pragma unroll
        for (int u = 0; u < RPT; ++u) acc[u] = fma(sh[(rg + RG * u) * ellp + q], rv, acc[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int rr = rg + RG * u;
      const int64_t r = c0 + rr;
      const T v = (T)acc[u];
      const bool ok = r < r1 && c < ell;
      if (c < ellp) sh[rr * ellp + c] = ok ? (double)v : 0.0;
      if (ok) Q[r * ldq + c] = v;
    }
    __syncthreads();
    if (part) gram_chunk(sh, GCH, ellp, slots, g);
  }
  if (part) gram_store(g, slots, ell, part + (int64_t)blockIdx.x * ell * ell);
  if (part && counter) {
    __syncthreads();   // LDS (Rs, sh) is reused by the factorization
    if (last_block_done(counter)) chol_body(part, gridDim.x, ell, rows, R, Rinv, dflags, dyn);
  }
}

// ---------------------------------------------------------------- Householder QR (one block)
// X: rows x ell (row-major, ld = ell), overwritten; Q: rows x ell explicit; R: ell x ell.
__global__ void __launch_bounds__(1024) k_hhqr(double *__restrict__ X, int64_t rows, int ell,
                                               double *__restrict__ Q, double *__restrict__ R,
                                               int *__restrict__ dflags) {
  __shared__ double tau[ELL_MAX];
  __shared__ double wv[ELL_MAX];
  __shared__ double red[17];
  const int t = threadIdx.x;
  const int grp = t >> 4, gl = t & 15;   // 64 groups of 16
  for (int j = 0; j < ell; ++j) {
    double s = 0.0;
    for (int64_t i = j + t; i < rows; i += 1024) {
      const double v = X[i * ell + j];
      s += v * v;
    }
    s = block_sum<1024>(s, red);
    const double x0 = X[(int64_t)j * ell + j];
    const double alpha = sqrt(s);
    double beta = 0.0, tj = 0.0, scale = 0.0;
    if (alpha > 0.0 && (int64_t)j < rows) {
      beta = (x0 >= 0.0) ? -alpha : alpha;
      tj = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    __syncthreads();
    for (int64_t i = j + 1 + t; i < rows; i += 1024) X[i * ell + j] *= scale;
    if (t == 0) {
      tau[j] = tj;
      R[j * ell + j] = beta;
      if (alpha == 0.0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_RANK_DEFICIENT);
    }
    __syncthreads();
    for (int c = j + 1 + grp; c < ell; c += 64) {
      double p = 0.0;
      for (int64_t i = j + 1 + gl; i < rows; i += 16) p += X[i * ell + j] * X[i * ell + c];
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) p += __shfl_xor(p, o, 16);
      if (gl == 0) wv[c] = p + X[(int64_t)j * ell + c];
    }
    __syncthreads();
    const int nc = ell - j - 1;
    if (nc > 0) {
      for (int64_t e = t; e < (rows - j) * nc; e += 1024) {
        const int64_t i = j + e / nc;
        const int c = j + 1 + (int)(e % nc);
        const double vi = (i == j) ? 1.0 : X[i * ell + j];
        X[i * ell + c] -= tj * vi * wv[c];
      }
    }
    __syncthreads();
  }
  for (int e = t; e < ell * ell; e += 1024) {
    const int i = e / ell, c = e % ell;
    if (c > i) R[e] = X[(int64_t)i * ell + c];
    else if (c < i) R[e] = 0.0;
  }
  for (int64_t e = t; e < rows * ell; e += 1024) {
    const int64_t i = e / ell;
    const int c = (int)(e % ell);
    Q[e] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = ell - 1; j >= 0; --j) {
    const double tj = tau[j];
    for (int c = j + grp; c < ell; c += 64) {
      double p = 0.0;
      for (int64_t i = j + 1 + gl; i < rows; i += 16) p += X[i * ell + j] * Q[i * ell + c];
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) p += __shfl_xor(p, o, 16);
      if (gl == 0) wv[c] = p + Q[(int64_t)j * ell + c];
    }
    __syncthreads();
    const int nc = ell - j;
    for (int64_t e = t; e < (rows - j) * nc; e += 1024) {
      const int64_t i = j + e / nc;
      const int c = j + (int)(e % nc);
      const double vi = (i == j) ? 1.0 : X[i * ell + j];
      Q[i * ell + c] -= tj * vi * wv[c];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- skinny product out = X M diag(scale)
// X rows x ell (ldx), M ell x kout (ldm, f64), out rows x kout (ldo).  TS_ROWS rows
// per block (large inputs: 128 for f32, 64 for f64; short inputs: 32); thread
// (row, part) accumulates KH outputs in registers, every M row is a broadcast
// LDS read reused for all of them.
template <typename T>
constexpr int ts_rows() { return sizeof(T) == 8 ? 64 : 128; }

template <typename T, int KB, int TS_ROWS>
__global__ void __launch_bounds__(256) k_tsmm(const T *__restrict__ X, int64_t rows, int ell, int64_t ldx,
                                              const double *__restrict__ M, int ldm, int kout,
                                              const double *__restrict__ scale, T *__restrict__ out,
                                              int64_t ldo) {
  constexpr int TPR = 256 / TS_ROWS;
  constexpr int KH = KB / TPR;
  extern __shared__ double dyn[];
  T *Ms = reinterpret_cast<T *>(dyn);                    // ell x KB (zero padded)
  T *Xs = Ms + ell * KB;                                 // TS_ROWS x (ell + 1)
  const int ldxs = ell + 1;
  for (int e = threadIdx.x; e < ell * KB; e += 256) {
    const int i = e / KB, c = e - (e / KB) * KB;
    Ms[e] = (c < kout) ? (T)(M[i * ldm + c] * (scale ? scale[c] : 1.0)) : T(0);
  }
  const int64_t r0 = (int64_t)blockIdx.x * TS_ROWS;
  for (int rr = threadIdx.x >> 6; rr < TS_ROWS; rr += 4) {
    const int64_t r = r0 + rr;
    for (int c = threadIdx.x & 63; c < ell; c += 64) Xs[rr * ldxs + c] = r < rows ? X[r * ldx + c] : T(0);
  }
  __syncthreads();
  const int rr = threadIdx.x / TPR, half = threadIdx.x % TPR;
  const int64_t r = r0 + rr;
  T acc[KH];
#pragma unroll
  for (int u = 0; u < KH; ++u) acc[u] = 0;
  const T *mrow = Ms + half * KH;
  for (int q = 0; q < ell; ++q) {
    const T xv = Xs[rr * ldxs + q];
#pragma unroll
    for (int u = 0; u < KH; ++u) acc[u] = fma(xv, mrow[q * KB + u], acc[u]);
  }
  if (r >= rows) return;
#pragma unroll
  for (int u = 0; u < KH; ++u) {
    const int c = half * KH + u;
    if (c < kout) out[r * ldo + c] = acc[u];
  }
}

// ---------------------------------------------------------------- sign normalisation of U
template <typename T>
__global__ void __launch_bounds__(256) k_sign_fix(T *__restrict__ U, int64_t m, int k, double *__restrict__ sign) {
  const int j = blockIdx.x;
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  double best = -1.0;
  int64_t idx = 0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const double v = fabs((double)U[i * k + j]);
    if (v > best) { best = v; idx = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double ov = bv[threadIdx.x + w];
      const int64_t oi = bi[threadIdx.x + w];
      if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = ov;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const double sg = ((double)U[bi[0] * k + j] < 0.0) ? -1.0 : 1.0;
  __syncthreads();
  if (threadIdx.x == 0) sign[j] = sg;
  if (sg < 0.0)
    for (int64_t i = threadIdx.x; i < m; i += 256) U[i * k + j] = -U[i * k + j];
}

int gram_parts(int64_t rows) { return (int)std::min<int64_t>(std::max<int64_t>(1, (rows + 127) / 128), 16); }

template <typename T, int CW>
void launch_apply(hipStream_t st, int nparts, size_t lds, const T *Y, int64_t rows, int ell, double *Rinv, T *Q,
                  int64_t rpb, double *part, int *dflags, int cond, unsigned *counter, double *R, int gram_cond) {
  allow_lds(k_apply<T, CW>, lds);
  hipLaunchKernelGGL((k_apply<T, CW>), dim3(nparts), dim3(256), lds, st, Y, rows, ell, (int64_t)ell, Rinv, Q,
                     (int64_t)ell, rpb, part, dflags, cond, counter, R, gram_cond);
}

// CholeskyQR2 in 3 launches (+1 after a shifted first pass):
//   [Gram(Y) -> chol]  [Q1 = Y R1^-1, Gram(Q1) -> chol]  [Q = Q1 R2^-1 (, Gram(Q) -> chol)]  [(Q = Q R3^-1)]
// The factorizations run in the workgroup that finishes its Gram partial last.
// Blocks at most 64 wide take the MFMA path of cholqr64.hip; wider blocks
// multiply by an explicit inverse.
template <typename T>
int cholqr2_typed(hipStream_t st, const T *Y, int64_t rows, int ell, T *Q, void *ws, int *dflags, int passes) {
  if (ell <= 64) return launch_cholqr64(st, Y, sizeof(T) == 8, rows, ell, Q, ws, dflags, passes);
  // ws layout: part (nparts*ell*ell f64) | R (ell^2) | Rinv (ell^2) | Q1 (rows*ell T)
  const int nparts = gram_parts(rows);
  const int64_t rpb = ((rows + nparts - 1) / nparts + GCH - 1) / GCH * GCH;
  double *part = reinterpret_cast<double *>(ws);
  double *R = part + (size_t)nparts * ell * ell;
  double *Rinv = R + ell * ell;
  T *Q1 = reinterpret_cast<T *>(Rinv + ell * ell);
  unsigned *counter = reinterpret_cast<unsigned *>(dflags + FLAGW_TICKET);
  const int ellp = (ell + 3) & ~3;
  const size_t chol_lds = (size_t)(ell * ell + ell) * sizeof(double);
  const size_t gram_lds = std::max<size_t>(chol_lds, (size_t)GCH * ellp * sizeof(double));
  const size_t apply_lds = std::max<size_t>(chol_lds, (size_t)(ell * ell + GCH * ellp) * sizeof(double));
  auto apply = [&](const T *src, T *dst, double *prt, int cond, unsigned *ctr, int gcond) {
    launch_apply<T, 128>(st, nparts, apply_lds, src, rows, ell, Rinv, dst, rpb, prt, dflags, cond, ctr, R, gcond);
  };
  allow_lds(k_gram_chol<T>, gram_lds);
  hipLaunchKernelGGL(k_gram_chol<T>, dim3(nparts), dim3(256), gram_lds, st, Y, rows, ell, (int64_t)ell, rpb, part,
                     counter, R, Rinv, dflags);
  if (passes == 1) {
    launch_apply<T, 128>(st, nparts, apply_lds, Y, rows, ell, Rinv, Q, rpb, nullptr, dflags, 0, nullptr, R, 0);
    DSK_TRY(hipGetLastError());
    return 0;
  }
  apply(Y, Q1, part, 0, counter, 0);
  apply(Q1, Q, part, 0, counter, 1);     // third factorization only after a shifted first pass
  apply(Q, Q, nullptr, 1, nullptr, 0);   // third application only after a shifted first pass
  DSK_TRY(hipGetLastError());
  return 0;
}

}  // namespace

size_t cholqr2_ws_bytes(int64_t rows, int ell) {
  if (ell <= 64) return cholqr64_ws_bytes(rows, ell);
  const int nparts = gram_parts(rows);
  return ((size_t)nparts * ell * ell + 2 * (size_t)ell * ell) * sizeof(double) + (size_t)rows * ell * sizeof(double) +
         1024;
}

int launch_cholqr2(hipStream_t st, const void *Y, int f64, int64_t rows, int ell, void *Q, void *ws, int *dflags,
                   double *Rout, int passes) {
  (void)Rout;
  if (ell < 1 || ell > ELL_MAX || passes < 1 || passes > 2) return -1;
  if (f64) return cholqr2_typed<double>(st, (const double *)Y, rows, ell, (double *)Q, ws, dflags, passes);
  return cholqr2_typed<float>(st, (const float *)Y, rows, ell, (float *)Q, ws, dflags, passes);
}

int launch_hhqr(hipStream_t st, double *X, int64_t rows, int ell, double *Q, double *R, int *dflags) {
  if (ell < 1 || ell > ELL_MAX) return -1;
  hipLaunchKernelGGL(k_hhqr, dim3(1), dim3(1024), 0, st, X, rows, ell, Q, R, dflags);
  DSK_TRY(hipGetLastError());
  return 0;
}

// G = X^T X (ell x ell, FP64) for a rows x ell block: partials over at most
// nparts row ranges, then a fixed-order reduction.  part: nparts * ell^2 doubles.
template <typename T>
void gram_parts_launch(hipStream_t st, const T *X, int64_t rows, int ell, int64_t rpb, int nblk, double *part) {
  if (ell <= 64)
    hipLaunchKernelGGL(k_gram_rows<T>, dim3(nblk), dim3(256), 0, st, X, rows, ell, (int64_t)ell, rpb, part);
  else
    hipLaunchKernelGGL(k_gram_part<T>, dim3(nblk), dim3(256), 0, st, X, rows, ell, (int64_t)ell, rpb, part,
                       (const int *)nullptr, 0);
}

int launch_gram(hipStream_t st, const void *X, int f64, int64_t rows, int ell, double *G, double *part, int nparts) {
  if (ell < 1 || ell > ELL_MAX || nparts < 1 || rows < 1) return -1;
  const int64_t rpb = ((rows + nparts - 1) / nparts + GCH - 1) / GCH * GCH;
  const int nblk = (int)((rows + rpb - 1) / rpb);
  if (f64) gram_parts_launch<double>(st, (const double *)X, rows, ell, rpb, nblk, part);
  else gram_parts_launch<float>(st, (const float *)X, rows, ell, rpb, nblk, part);
  const int n2 = ell * ell;
  hipLaunchKernelGGL(k_gram_reduce, dim3((n2 + 15) / 16), dim3(256), 0, st, (const double *)part, nblk, n2, G);
  DSK_TRY(hipGetLastError());
  return 0;
}

template <typename T, int KB, int TS_ROWS>
void tsmm_r(hipStream_t st, const T *X, int64_t rows, int ell, int64_t ldx, const double *M, int ldm, int kout,
            const double *colscale, T *out, int64_t ldo) {
  const unsigned blocks = (unsigned)((rows + TS_ROWS - 1) / TS_ROWS);
  const size_t lds = ((size_t)ell * KB + (size_t)TS_ROWS * (ell + 1)) * sizeof(T);
  allow_lds(k_tsmm<T, KB, TS_ROWS>, lds);
  hipLaunchKernelGGL((k_tsmm<T, KB, TS_ROWS>), dim3(blocks), dim3(256), lds, st, X, rows, ell, ldx, M, ldm, kout,
                     colscale, out, ldo);
}

template <typename T, int KB>
void tsmm_t(hipStream_t st, const T *X, int64_t rows, int ell, int64_t ldx, const double *M, int ldm, int kout,
            const double *colscale, T *out, int64_t ldo) {
  // short inputs: 32-row blocks so that more workgroups share the work
  if (rows < 64 * 256) tsmm_r<T, KB, 32>(st, X, rows, ell, ldx, M, ldm, kout, colscale, out, ldo);
  else tsmm_r<T, KB, ts_rows<T>()>(st, X, rows, ell, ldx, M, ldm, kout, colscale, out, ldo);
}

template <typename T>
int tsmm_any(hipStream_t st, const T *X, int64_t rows, int ell, int64_t ldx, const double *M, int ldm, int kout,
             const double *colscale, T *out, int64_t ldo) {
  if (kout <= 16) tsmm_t<T, 16>(st, X, rows, ell, ldx, M, ldm, kout, colscale, out, ldo);
  else if (kout <= 32) tsmm_t<T, 32>(st, X, rows, ell, ldx, M, ldm, kout, colscale, out, ldo);
  else if (kout <= 64) tsmm_t<T, 64>(st, X, rows, ell, ldx, M, ldm, kout, colscale, out, ldo);
  else if (kout <= 128) tsmm_t<T, 128>(st, X, rows, ell, ldx, M, ldm, kout, colscale, out, ldo);
  else return -1;
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_tsmm(hipStream_t st, const void *X, int f64, int64_t rows, int ell, int64_t ldx, const double *M, int ldm,
                int kout, const double *colscale, void *out, int64_t ldo) {
  if (f64) return tsmm_any<double>(st, (const double *)X, rows, ell, ldx, M, ldm, kout, colscale, (double *)out, ldo);
  return tsmm_any<float>(st, (const float *)X, rows, ell, ldx, M, ldm, kout, colscale, (float *)out, ldo);
}

int launch_sign_fix(hipStream_t st, void *U, int f64, int64_t m, int k, double *sign) {
  if (f64)
    hipLaunchKernelGGL(k_sign_fix<double>, dim3(k), dim3(256), 0, st, (double *)U, m, k, sign);
  else
    hipLaunchKernelGGL(k_sign_fix<float>, dim3(k), dim3(256), 0, st, (float *)U, m, k, sign);
  DSK_TRY(hipGetLastError());
  return 0;
}

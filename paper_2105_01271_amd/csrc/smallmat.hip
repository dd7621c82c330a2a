// Small dense factorizations of the sketch pipeline.
//
//  * Orthonormalisation of tall-skinny blocks (the QR steps of Alg. 2 and
//    Alg. 7): CholeskyQR2 with an FP64 Gram and FP64 Cholesky, dispatched to
//    cholqr64.hip (ell <= 64) and cholqr128.hip (wider).  If the first
//    Cholesky meets a non-positive or negligible pivot, it is retried with the
//    shift 11 (rows*ell + ell(ell+1)) u ||Y||_F^2 and DSK_FLAG_FALLBACK is
//    raised; a third (conditional) pass then restores orthonormality (shifted
//    CholeskyQR3, Fukaya et al. 2020).
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

__device__ __forceinline__ void pair_of(int pid, int nb, int &bi, int &bj) {
  int r = 0, rem = pid;
  while (rem >= nb - r) { rem -= nb - r; ++r; }
  bi = r;
  bj = r + rem;
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

constexpr int GCH = 32;

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
  // eight loads in flight per thread, compared in ascending row order
  int64_t i = threadIdx.x;
  for (; i + 7 * 256 < m; i += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = fabs((double)U[(i + 256 * u) * k + j]);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (v[u] > best) { best = v[u]; idx = i + 256 * u; }
  }
  for (; i < m; i += 256) {
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

template <typename T>
int cholqr2_typed(hipStream_t st, const T *Y, int64_t rows, int ell, T *Q, void *ws, int *dflags, int passes) {
  if (ell <= 64) return launch_cholqr64(st, Y, sizeof(T) == 8, rows, ell, Q, ws, dflags, passes);
  return launch_cholqr128(st, Y, sizeof(T) == 8, rows, ell, Q, ws, dflags, passes);
}

}  // namespace

size_t cholqr2_ws_bytes(int64_t rows, int ell) {
  if (ell <= 64) return cholqr64_ws_bytes(rows, ell);
  return cholqr128_ws_bytes(rows, ell);
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
  hipLaunchKernelGGL(k_gram_rows<T>, dim3(nblk), dim3(256), 0, st, X, rows, ell, (int64_t)ell, rpb, part);
}

int launch_gram(hipStream_t st, const void *X, int f64, int64_t rows, int ell, double *G, double *part, int nparts) {
  if (ell < 1 || ell > ELL_MAX || nparts < 1 || rows < 1) return -1;
  if (ell > 16) return launch_gram_mfma(st, X, f64, rows, ell, G, part, nparts);
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
  // short inputs: 8-, 16- or 32-row blocks so that more workgroups share the work
  if constexpr (KB >= 32) {
    if (rows < 8 * 256) {
      tsmm_r<T, KB, 8>(st, X, rows, ell, ldx, M, ldm, kout, colscale, out, ldo);
      return;
    }
  }
  if (rows < 16 * 256 && KB >= 16) tsmm_r<T, KB, 16>(st, X, rows, ell, ldx, M, ldm, kout, colscale, out, ldo);
  else if (rows < 64 * 256) tsmm_r<T, KB, 32>(st, X, rows, ell, ldx, M, ldm, kout, colscale, out, ldo);
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

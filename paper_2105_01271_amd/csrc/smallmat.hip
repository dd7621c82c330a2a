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
//  * Two-sided cyclic Jacobi eigen-solver of an ell x ell FP64 Gram (core of
//    SVD(B) through B B^T), one-sided Jacobi SVD of an ell x ell triangular
//    factor (core of SVD(B) from a QR of B^T without squaring), round-robin
//    ordering, everything resident in LDS.
//  * Skinny products out = X M diag(scale) and the sign normalisation of U.
// All reductions use fixed orders, so repeated runs give identical bytes.
#include <algorithm>

#include "dsk_internal.h"

namespace {

constexpr int ELL_MAX = 112;   // LDS budget: packed Gram + eigenvectors in 160 KB
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
  // enumerate (bi <= bj) row-major over the upper triangle of an nb x nb block grid
  int r = 0, rem = pid;
  while (rem >= nb - r) { rem -= nb - r; ++r; }
  bi = r;
  bj = r + rem;
}

template <int U>
__device__ __forceinline__ void gram_chunk_u(const double *sh, int CH, int ellp, double (&acc)[16]) {
  const int nb = ellp / 4, npairs = nb * (nb + 1) / 2;
  const int pid = threadIdx.x + 256 * U;
  if (pid >= npairs) return;
  int bi, bj;
  pair_of(pid, nb, bi, bj);
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

// sh: CH x ellp chunk (row-major, zero padded)
__device__ __forceinline__ void gram_chunk(const double *sh, int CH, int ellp, GramAcc &g) {
  gram_chunk_u<0>(sh, CH, ellp, g.a0);
  gram_chunk_u<1>(sh, CH, ellp, g.a1);
  gram_chunk_u<2>(sh, CH, ellp, g.a2);
}

template <int U>
__device__ __forceinline__ void gram_store_u(const double (&acc)[16], int ell, int ellp, double *part) {
  const int nb = ellp / 4, npairs = nb * (nb + 1) / 2;
  const int pid = threadIdx.x + 256 * U;
  if (pid >= npairs) return;
  int bi, bj;
  pair_of(pid, nb, bi, bj);
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

__device__ __forceinline__ void gram_store(const GramAcc &g, int ell, int ellp, double *part) {
  gram_store_u<0>(g.a0, ell, ellp, part);
  gram_store_u<1>(g.a1, ell, ellp, part);
  gram_store_u<2>(g.a2, ell, ellp, part);
}

constexpr int GCH = 32;

template <typename T>
__global__ void __launch_bounds__(256) k_gram_part(const T *__restrict__ X, int64_t rows, int ell, int64_t ldx,
                                                   int64_t rows_per_blk, double *__restrict__ part,
                                                   const int *__restrict__ dflags, int cond) {
  if (cond && !(dflags[FLAGW_BITS] & DSK_FLAG_FALLBACK)) return;
  __shared__ double sh[GCH * ELL_MAX];
  const int ellp = (ell + 3) & ~3;
  GramAcc g;
  gram_zero(g);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(rows, r0 + rows_per_blk);
  for (int64_t c0 = r0; c0 < r1; c0 += GCH) {
    for (int e = threadIdx.x; e < GCH * ellp; e += 256) {
      const int rr = e / ellp, c = e % ellp;
      const int64_t r = c0 + rr;
      sh[e] = (r < r1 && c < ell) ? (double)X[r * ldx + c] : 0.0;
    }
    __syncthreads();
    gram_chunk(sh, GCH, ellp, g);
    __syncthreads();
  }
  gram_store(g, ell, ellp, part + (int64_t)blockIdx.x * ell * ell);
}

// ---------------------------------------------------------------- Cholesky + inverse (one block)
// Sums the Gram partials in a fixed order, factors G = L L^T (retrying once with
// a shift on breakdown), inverts L in place and writes R = L^T, Rinv = L^{-T}.
__global__ void __launch_bounds__(256) k_chol(const double *__restrict__ part, int nparts, int ell, int64_t rows,
                                              double *__restrict__ R, double *__restrict__ Rinv,
                                              int *__restrict__ dflags, int cond) {
  if (cond && !(dflags[FLAGW_BITS] & DSK_FLAG_FALLBACK)) return;
  extern __shared__ double dyn[];
  double *G = dyn;                 // ell x ell
  double *tmp = dyn + ell * ell;   // ell
  __shared__ double red[8];
  __shared__ int bad;
  const int t = threadIdx.x;
  const int n2 = ell * ell;
  double shift = 0.0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    for (int e = t; e < n2; e += 256) {
      double s = 0.0;
      for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * n2 + e];
      G[e] = s;
    }
    __syncthreads();
    double tr = 0.0;
    for (int i = t; i < ell; i += 256) tr += G[i * ell + i];
    tr = block_sum<256>(tr, red);
    if (attempt == 1) {
      shift = 11.0 * ((double)rows * ell + (double)ell * (ell + 1)) * U64 * tr;
      for (int i = t; i < ell; i += 256) G[i * ell + i] += shift;
    }
    if (t == 0) bad = !(tr > 0.0) || !isfinite(tr);
    __syncthreads();
    const double thr = 1e-15 * tr;
    for (int j = 0; j < ell && !bad; ++j) {
      if (t == 0) {
        const double d = G[j * ell + j];
        if (!(d > thr) || !isfinite(d)) bad = 1;
        else G[j * ell + j] = sqrt(d);
      }
      __syncthreads();
      if (bad) break;
      const double dj = G[j * ell + j];
      for (int i = j + 1 + t; i < ell; i += 256) G[i * ell + j] /= dj;
      __syncthreads();
      const int m = ell - j - 1;
      for (int e = t; e < m * m; e += 256) {
        const int i = j + 1 + e / m, c = j + 1 + e % m;
        if (c <= i) G[i * ell + c] -= G[i * ell + j] * G[c * ell + j];
      }
      __syncthreads();
    }
    __syncthreads();
    if (!bad) break;
    if (t == 0) atomicOr(&dflags[FLAGW_BITS], attempt == 0 ? DSK_FLAG_FALLBACK : DSK_FLAG_RANK_DEFICIENT);
    __syncthreads();
    if (attempt == 1) {
      // still failing (non-finite input): identity factors keep the pipeline finite
      for (int e = t; e < n2; e += 256) {
        const int i = e / ell, c = e % ell;
        R[e] = (i == c) ? 1.0 : 0.0;
        Rinv[e] = (i == c) ? 1.0 : 0.0;
      }
      if (t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
      return;
    }
    if (t == 0) bad = 0;
    __syncthreads();
  }
  // R = L^T
  for (int e = t; e < n2; e += 256) {
    const int i = e / ell, c = e % ell;
    R[e] = (c >= i) ? G[c * ell + i] : 0.0;
  }
  __syncthreads();
  // in-place inverse of lower-triangular L (column j from the already inverted trailing block)
  for (int j = ell - 1; j >= 0; --j) {
    if (t == 0) G[j * ell + j] = 1.0 / G[j * ell + j];
    for (int i = j + 1 + t; i < ell; i += 256) tmp[i] = G[i * ell + j];
    __syncthreads();
    const double ajj = -G[j * ell + j];
    for (int i = j + 1 + t; i < ell; i += 256) {
      double s = 0.0;
      for (int c = j + 1; c <= i; ++c) s += G[i * ell + c] * tmp[c];
      G[i * ell + j] = ajj * s;
    }
    __syncthreads();
  }
  for (int e = t; e < n2; e += 256) {
    const int i = e / ell, c = e % ell;
    Rinv[e] = (c >= i) ? G[c * ell + i] : 0.0;
  }
}

// ---------------------------------------------------------------- Q = Y Rinv (+ Gram partials of Q)
template <typename T>
__global__ void __launch_bounds__(256) k_apply(const T *__restrict__ Y, int64_t rows, int ell, int64_t ldy,
                                               const double *__restrict__ Rinv, T *__restrict__ Q, int64_t ldq,
                                               int64_t rows_per_blk, double *__restrict__ part,
                                               const int *__restrict__ dflags, int cond) {
  if (cond && !(dflags[FLAGW_BITS] & DSK_FLAG_FALLBACK)) return;
  extern __shared__ double dyn[];
  const int ellp = (ell + 3) & ~3;
  double *Rs = dyn;                   // ell x ell
  double *sh = dyn + ell * ell;       // GCH x ellp
  for (int e = threadIdx.x; e < ell * ell; e += 256) Rs[e] = Rinv[e];
  GramAcc g;
  gram_zero(g);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(rows, r0 + rows_per_blk);
  for (int64_t c0 = r0; c0 < r1; c0 += GCH) {
    __syncthreads();
    for (int e = threadIdx.x; e < GCH * ellp; e += 256) {
      const int rr = e / ellp, c = e % ellp;
      const int64_t r = c0 + rr;
      sh[e] = (r < r1 && c < ell) ? (double)Y[r * ldy + c] : 0.0;
    }
    __syncthreads();
    constexpr int NU = (GCH * ELL_MAX + 255) / 256;
    double outv[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = threadIdx.x + 256 * u;
      double s = 0.0;
      if (e < GCH * ellp) {
        const int rr = e / ellp, c = e % ellp;
        if (c < ell)
          for (int q = 0; q <= c; ++q) s = fma(sh[rr * ellp + q], Rs[q * ell + c], s);
      }
      outv[u] = s;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < GCH * ellp) {
        const int rr = e / ellp, c = e % ellp;
        const int64_t r = c0 + rr;
        const T v = (T)outv[u];
        sh[e] = (r < r1 && c < ell) ? (double)v : 0.0;
        if (r < r1 && c < ell) Q[r * ldq + c] = v;
      }
    }
    __syncthreads();
    if (part) gram_chunk(sh, GCH, ellp, g);
  }
  if (part) gram_store(g, ell, ellp, part + (int64_t)blockIdx.x * ell * ell);
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
    // w_c = x_jc + sum_{i>j} v_i x_ic for trailing columns
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
  // explicit Q = H_0 ... H_{ell-1} [I; 0]
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

// ---------------------------------------------------------------- round-robin pairing
// Circle method on n (even) players: player 0 fixed, others rotate; pair i of
// round r joins positions i and n-1-i.
__device__ __forceinline__ int rr_player(int pos, int r, int n) {
  return pos == 0 ? 0 : ((pos - 1 + r) % (n - 1)) + 1;
}

__device__ __forceinline__ int pk(int a, int b, int n) {   // packed upper index, a <= b
  return a * n - (a * (a - 1)) / 2 + (b - a);
}

// ---------------------------------------------------------------- two-sided Jacobi eigen
// G (ell x ell, symmetric) given as nparts partial sums.  Outputs eigenvalues in
// descending order and the matching eigenvectors as columns of V (ell x ell).
__global__ void __launch_bounds__(1024) k_jacobi_eig(const double *__restrict__ part, int nparts, int ell,
                                                     double *__restrict__ lam, double *__restrict__ Vout,
                                                     int *__restrict__ dflags) {
  extern __shared__ double dyn[];
  const int n = (ell + 1) & ~1;            // even number of players (one zero pad if odd)
  const int npk = n * (n + 1) / 2;
  double *Gp = dyn;                        // packed upper, n x n
  double *V = dyn + npk;                   // n x n row-major
  __shared__ double rc[ELL_MAX / 2 + 1], rs[ELL_MAX / 2 + 1];
  __shared__ int pp[ELL_MAX / 2 + 1], pq[ELL_MAX / 2 + 1];
  __shared__ double red[17];
  __shared__ int rank_of[ELL_MAX + 2];
  const int t = threadIdx.x;
  const int np = n / 2;
  for (int e = t; e < npk; e += 1024) Gp[e] = 0.0;
  __syncthreads();
  double fro = 0.0;
  for (int e = t; e < ell * ell; e += 1024) {
    const int a = e / ell, b = e % ell;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * ell * ell + e];
    if (a <= b) Gp[pk(a, b, n)] = s;
    fro += s * s;
  }
  for (int e = t; e < n * n; e += 1024) V[e] = (e / n == e % n) ? 1.0 : 0.0;
  fro = block_sum<1024>(fro, red);
  if (!isfinite(fro) && t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
  const double tol2 = 1e-30 * fro;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int e = t; e < npk; e += 1024) {
      // off-diagonal mass (each strictly-upper entry counted twice)
      int a = 0, rem = e;
      while (rem >= n - a) { rem -= n - a; ++a; }
      const int b = a + rem;
      if (b > a) off += 2.0 * Gp[e] * Gp[e];
    }
    off = block_sum<1024>(off, red);
    if (!(off > tol2)) break;
    for (int r = 0; r < n - 1; ++r) {
      if (t < np) {
        int p = rr_player(t, r, n), q = rr_player(n - 1 - t, r, n);
        if (p > q) { const int x = p; p = q; q = x; }
        const double gpp = Gp[pk(p, p, n)], gqq = Gp[pk(q, q, n)], gpq = Gp[pk(p, q, n)];
        double c = 1.0, s = 0.0;
        if (gpq != 0.0 && fabs(gpq) > 1e-300) {
          const double theta = (gqq - gpp) / (2.0 * gpq);
          const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        rc[t] = c; rs[t] = s; pp[t] = p; pq[t] = q;
      }
      __syncthreads();
      // G <- J^T G J over 2x2 blocks (P1 <= P2)
      const int nblk = np * (np + 1) / 2;
      for (int e = t; e < nblk; e += 1024) {
        int P1 = 0, rem = e;
        while (rem >= np - P1) { rem -= np - P1; ++P1; }
        const int P2 = P1 + rem;
        const int p1 = pp[P1], q1 = pq[P1], p2 = pp[P2], q2 = pq[P2];
        const double c1 = rc[P1], s1 = rs[P1], c2 = rc[P2], s2 = rs[P2];
        if (P1 == P2) {
          const double gpp = Gp[pk(p1, p1, n)], gqq = Gp[pk(q1, q1, n)], gpq = Gp[pk(p1, q1, n)];
          Gp[pk(p1, p1, n)] = c1 * c1 * gpp - 2.0 * c1 * s1 * gpq + s1 * s1 * gqq;
          Gp[pk(q1, q1, n)] = s1 * s1 * gpp + 2.0 * c1 * s1 * gpq + c1 * c1 * gqq;
          Gp[pk(p1, q1, n)] = 0.0;
        } else {
          const int i_pp = pk(min(p1, p2), max(p1, p2), n), i_pq = pk(min(p1, q2), max(p1, q2), n);
          const int i_qp = pk(min(q1, p2), max(q1, p2), n), i_qq = pk(min(q1, q2), max(q1, q2), n);
          const double bpp = Gp[i_pp], bpq = Gp[i_pq], bqp = Gp[i_qp], bqq = Gp[i_qq];
          // rows: p' = c1 p - s1 q ; q' = s1 p + c1 q
          const double rpp = c1 * bpp - s1 * bqp, rpq = c1 * bpq - s1 * bqq;
          const double rqp = s1 * bpp + c1 * bqp, rqq = s1 * bpq + c1 * bqq;
          // cols: p' = c2 p - s2 q ; q' = s2 p + c2 q
          Gp[i_pp] = c2 * rpp - s2 * rpq;
          Gp[i_pq] = s2 * rpp + c2 * rpq;
          Gp[i_qp] = c2 * rqp - s2 * rqq;
          Gp[i_qq] = s2 * rqp + c2 * rqq;
        }
      }
      // V <- V J
      for (int e = t; e < n * np; e += 1024) {
        const int a = e / np, P = e % np;
        const int p = pp[P], q = pq[P];
        const double c = rc[P], s = rs[P];
        const double vp = V[a * n + p], vq = V[a * n + q];
        V[a * n + p] = c * vp - s * vq;
        V[a * n + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // sort eigenvalues (descending, ties by index) among the ell real players
  for (int a = t; a < ell; a += 1024) {
    const double da = Gp[pk(a, a, n)];
    int rnk = 0;
    for (int b = 0; b < ell; ++b) {
      const double db = Gp[pk(b, b, n)];
      if (db > da || (db == da && b < a)) ++rnk;
    }
    rank_of[a] = rnk;
  }
  __syncthreads();
  for (int a = t; a < ell; a += 1024) lam[rank_of[a]] = Gp[pk(a, a, n)];
  for (int e = t; e < ell * ell; e += 1024) {
    const int i = e / ell, a = e % ell;
    Vout[i * ell + rank_of[a]] = V[i * n + a];
  }
}

// ---------------------------------------------------------------- one-sided Jacobi SVD
// Rm (ell x ell, row-major).  W = Rm V with orthogonal columns; sig_j = ||w_j||.
// Outputs (descending): sig, Vr (ell x ell, columns = right vectors V),
// Ur (ell x ell, columns = w_j / sig_j, 0 where sig_j = 0).
__global__ void __launch_bounds__(1024) k_jacobi_svd(const double *__restrict__ Rm, int ell,
                                                     double *__restrict__ sig, double *__restrict__ Vr,
                                                     double *__restrict__ Ur, int *__restrict__ dflags) {
  extern __shared__ double dyn[];
  const int n = (ell + 1) & ~1;
  double *W = dyn;               // column-major n cols x ell rows: W[col*ell + row]
  double *V = dyn + n * ell;     // column-major n x n
  __shared__ int rank_of[ELL_MAX + 2];
  __shared__ double nrm[ELL_MAX + 2];
  __shared__ int rotated;
  const int t = threadIdx.x;
  const int np = n / 2;
  for (int e = t; e < n * ell; e += 1024) {
    const int col = e / ell, row = e % ell;
    W[e] = (col < ell) ? Rm[row * ell + col] : 0.0;
  }
  for (int e = t; e < n * n; e += 1024) V[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  const int gs = 16;   // threads per pair
  const int grp = t / gs, gl = t % gs;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < n - 1; ++r) {
      for (int P = grp; P < np; P += 1024 / gs) {
        int p = rr_player(P, r, n), q = rr_player(n - 1 - P, r, n);
        if (p > q) { const int x = p; p = q; q = x; }
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = gl; i < ell; i += gs) {
          const double wp = W[p * ell + i], wq = W[q * ell + i];
          al += wp * wp; be += wq * wq; ga += wp * wq;
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, 16);
          be += __shfl_xor(be, o, 16);
          ga += __shfl_xor(ga, o, 16);
        }
        if (ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + tt * tt), s = tt * c;
          for (int i = gl; i < ell; i += gs) {
            const double wp = W[p * ell + i], wq = W[q * ell + i];
            W[p * ell + i] = c * wp - s * wq;
            W[q * ell + i] = s * wp + c * wq;
          }
          for (int i = gl; i < n; i += gs) {
            const double vp = V[p * n + i], vq = V[q * n + i];
            V[p * n + i] = c * vp - s * vq;
            V[q * n + i] = s * vp + c * vq;
          }
          if (gl == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
  }
  for (int col = t; col < ell; col += 1024) {
    double s = 0.0;
    for (int i = 0; i < ell; ++i) s += W[col * ell + i] * W[col * ell + i];
    nrm[col] = sqrt(s);
  }
  __syncthreads();
  for (int a = t; a < ell; a += 1024) {
    int rnk = 0;
    for (int b = 0; b < ell; ++b)
      if (nrm[b] > nrm[a] || (nrm[b] == nrm[a] && b < a)) ++rnk;
    rank_of[a] = rnk;
    if (!isfinite(nrm[a])) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
  }
  __syncthreads();
  for (int a = t; a < ell; a += 1024) sig[rank_of[a]] = nrm[a];
  for (int e = t; e < ell * ell; e += 1024) {
    const int i = e / ell, a = e % ell;
    Vr[i * ell + rank_of[a]] = V[a * n + i];
    Ur[i * ell + rank_of[a]] = nrm[a] > 0.0 ? W[a * ell + i] / nrm[a] : 0.0;
  }
}

// ---------------------------------------------------------------- skinny product out = X M diag(scale)
// X rows x ell (ldx), M ell x kout (ldm, f64), out rows x kout (ldo).  32 rows per
// block, 8 threads per row.
template <typename T>
__global__ void __launch_bounds__(256) k_tsmm(const T *__restrict__ X, int64_t rows, int ell, int64_t ldx,
                                              const double *__restrict__ M, int ldm, int kout,
                                              const double *__restrict__ scale, T *__restrict__ out,
                                              int64_t ldo) {
  extern __shared__ double dyn[];
  T *Ms = reinterpret_cast<T *>(dyn);                              // ell x kout
  T *Xs = Ms + ((ell * kout + 1) & ~1);                            // 32 x ell
  for (int e = threadIdx.x; e < ell * kout; e += 256) {
    const int i = e / kout, c = e % kout;
    Ms[e] = (T)(M[i * ldm + c] * (scale ? scale[c] : 1.0));
  }
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  for (int e = threadIdx.x; e < 32 * ell; e += 256) {
    const int rr = e / ell, c = e % ell;
    const int64_t r = r0 + rr;
    Xs[e] = r < rows ? X[r * ldx + c] : T(0);
  }
  __syncthreads();
  const int rr = threadIdx.x >> 3, cl = threadIdx.x & 7;
  const int64_t r = r0 + rr;
  if (r >= rows) return;
  for (int c = cl; c < kout; c += 8) {
    T s = 0;
    for (int q = 0; q < ell; ++q) s = fma(Xs[rr * ell + q], Ms[q * kout + c], s);
    out[r * ldo + c] = s;
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

template <typename T>
int cholqr2_typed(hipStream_t st, const T *Y, int64_t rows, int ell, T *Q, void *ws, int *dflags) {
  // ws layout: part (nparts*ell*ell f64) | R (ell^2) | Rinv (ell^2) | Q1 (rows*ell T)
  const int nparts = (int)std::min<int64_t>(std::max<int64_t>(1, (rows + 63) / 64), 240);
  const int64_t rpb = ((rows + nparts - 1) / nparts + GCH - 1) / GCH * GCH;
  double *part = reinterpret_cast<double *>(ws);
  double *R = part + (size_t)nparts * ell * ell;
  double *Rinv = R + ell * ell;
  T *Q1 = reinterpret_cast<T *>(Rinv + ell * ell);
  const size_t chol_lds = (size_t)(ell * ell + ell) * sizeof(double);
  const size_t apply_lds = (size_t)(ell * ell + GCH * ((ell + 3) & ~3)) * sizeof(double);
  allow_lds(k_chol, chol_lds);
  allow_lds(k_apply<T>, apply_lds);
  hipLaunchKernelGGL(k_gram_part<T>, dim3(nparts), dim3(256), 0, st, Y, rows, ell, (int64_t)ell, rpb, part,
                     dflags, 0);
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), chol_lds, st, part, nparts, ell, rows, R, Rinv, dflags, 0);
  hipLaunchKernelGGL(k_apply<T>, dim3(nparts), dim3(256), apply_lds, st, Y, rows, ell, (int64_t)ell, Rinv, Q1,
                     (int64_t)ell, rpb, part, dflags, 0);
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), chol_lds, st, part, nparts, ell, rows, R, Rinv, dflags, 0);
  hipLaunchKernelGGL(k_apply<T>, dim3(nparts), dim3(256), apply_lds, st, Q1, rows, ell, (int64_t)ell, Rinv, Q,
                     (int64_t)ell, rpb, part, dflags, 0);
  // third pass only after a shifted first pass
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), chol_lds, st, part, nparts, ell, rows, R, Rinv, dflags, 1);
  hipLaunchKernelGGL(k_apply<T>, dim3(nparts), dim3(256), apply_lds, st, Q, rows, ell, (int64_t)ell, Rinv, Q,
                     (int64_t)ell, rpb, (double *)nullptr, dflags, 1);
  DSK_TRY(hipGetLastError());
  return 0;
}

}  // namespace

size_t cholqr2_ws_bytes(int64_t rows, int ell) {
  const int nparts = (int)std::min<int64_t>(std::max<int64_t>(1, (rows + 63) / 64), 240);
  return ((size_t)nparts * ell * ell + 2 * (size_t)ell * ell) * sizeof(double) + (size_t)rows * ell * sizeof(double) +
         1024;
}

int launch_cholqr2(hipStream_t st, const void *Y, int f64, int64_t rows, int ell, void *Q, void *ws, int *dflags,
                   double *Rout) {
  (void)Rout;
  if (ell < 1 || ell > ELL_MAX) return -1;
  if (f64) return cholqr2_typed<double>(st, (const double *)Y, rows, ell, (double *)Q, ws, dflags);
  return cholqr2_typed<float>(st, (const float *)Y, rows, ell, (float *)Q, ws, dflags);
}

int launch_hhqr(hipStream_t st, double *X, int64_t rows, int ell, double *Q, double *R, int *dflags) {
  if (ell < 1 || ell > ELL_MAX) return -1;
  hipLaunchKernelGGL(k_hhqr, dim3(1), dim3(1024), 0, st, X, rows, ell, Q, R, dflags);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_gram(hipStream_t st, const void *X, int f64, int64_t rows, int ell, double *G, double *part, int nparts) {
  (void)G;
  if (ell < 1 || ell > ELL_MAX) return -1;
  const int64_t rpb = ((rows + nparts - 1) / nparts + GCH - 1) / GCH * GCH;
  if (f64)
    hipLaunchKernelGGL(k_gram_part<double>, dim3(nparts), dim3(256), 0, st, (const double *)X, rows, ell,
                       (int64_t)ell, rpb, part, (const int *)nullptr, 0);
  else
    hipLaunchKernelGGL(k_gram_part<float>, dim3(nparts), dim3(256), 0, st, (const float *)X, rows, ell,
                       (int64_t)ell, rpb, part, (const int *)nullptr, 0);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_jacobi_eig_parts(hipStream_t st, const double *part, int nparts, int ell, double *lam, double *V,
                            int *dflags) {
  if (ell < 1 || ell > ELL_MAX) return -1;
  const int n = (ell + 1) & ~1;
  const size_t lds = ((size_t)n * (n + 1) / 2 + (size_t)n * n) * sizeof(double);
  allow_lds(k_jacobi_eig, lds);
  hipLaunchKernelGGL(k_jacobi_eig, dim3(1), dim3(1024), lds, st, part, nparts, ell, lam, V, dflags);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_jacobi_eig(hipStream_t st, const double *G, int ell, double *lam, double *V, int *dflags) {
  return launch_jacobi_eig_parts(st, G, 1, ell, lam, V, dflags);
}

int launch_jacobi_svd(hipStream_t st, const double *Rm, int ell, double *sig, double *Vr, double *Ur, int *dflags) {
  if (ell < 1 || ell > 100) return -1;
  const int n = (ell + 1) & ~1;
  const size_t lds = ((size_t)n * ell + (size_t)n * n) * sizeof(double);
  allow_lds(k_jacobi_svd, lds);
  hipLaunchKernelGGL(k_jacobi_svd, dim3(1), dim3(1024), lds, st, Rm, ell, sig, Vr, Ur, dflags);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_tsmm(hipStream_t st, const void *X, int f64, int64_t rows, int ell, int64_t ldx, const double *M, int ldm,
                int kout, const double *colscale, void *out, int64_t ldo) {
  const unsigned blocks = (unsigned)((rows + 31) / 32);
  if (f64) {
    const size_t lds = ((size_t)((ell * kout + 1) & ~1) + 32 * (size_t)ell) * sizeof(double);
    allow_lds(k_tsmm<double>, lds);
    hipLaunchKernelGGL(k_tsmm<double>, dim3(blocks), dim3(256), lds, st, (const double *)X, rows, ell, ldx, M, ldm,
                       kout, colscale, (double *)out, ldo);
  } else {
    const size_t lds = ((size_t)((ell * kout + 1) & ~1) + 32 * (size_t)ell) * sizeof(float);
    allow_lds(k_tsmm<float>, lds);
    hipLaunchKernelGGL(k_tsmm<float>, dim3(blocks), dim3(256), lds, st, (const float *)X, rows, ell, ldx, M, ldm,
                       kout, colscale, (float *)out, ldo);
  }
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_sign_fix(hipStream_t st, void *U, int f64, int64_t m, int k, double *sign) {
  if (f64)
    hipLaunchKernelGGL(k_sign_fix<double>, dim3(k), dim3(256), 0, st, (double *)U, m, k, sign);
  else
    hipLaunchKernelGGL(k_sign_fix<float>, dim3(k), dim3(256), 0, st, (float *)U, m, k, sign);
  DSK_TRY(hipGetLastError());
  return 0;
}

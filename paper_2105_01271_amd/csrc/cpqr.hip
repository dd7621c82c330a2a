// Row interpolative decomposition by rank-k column-pivoted QR of W^T
// (paper Sec. 4, row ID; TPC-ID, Alg. 4).
//
// W is m x s, row-major, FP64: row i of W is column i of X = W^T, the i-th
// candidate (time step).  The factorization is right-looking modified
// Gram-Schmidt with column pivoting, FP64 throughout:
//   step t: p = argmax over unselected i of nu_i = ||residual_i||^2
//           (exact ties -> lowest index), q = residual_p / ||residual_p||,
//           for every unselected i:  R[t, i] = q . residual_i,
//           residual_i -= R[t, i] q,  nu_i = ||residual_i||^2 recomputed from
//           the updated residual (no norm downdating).
// In exact arithmetic this is the Householder CPQR of X (same pivots, same R
// up to row signs); the residual norms are recomputed every step so pivot
// decisions keep full FP64 relative accuracy.
//
// One launch per step.  Every workgroup computes the same argmax from the
// previous step's nu (double-buffered, so no workgroup reads a value written in
// the same launch); the pivot row is never written during the step that reads
// it.  Selected candidates carry nu = -1.
#include <algorithm>

#include "dsk_internal.h"

namespace {

constexpr int CPB = 4;     // candidates per workgroup
constexpr int NT = 256;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// zero fill by a kernel (keeps the sequence capturable in a graph)
__global__ void k_fill0(double *__restrict__ x, int64_t count) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
    x[t] = 0.0;
}

__global__ void __launch_bounds__(NT) k_cpqr_norms(const double *__restrict__ W, int64_t m, int64_t s,
                                                   double *__restrict__ nu) {
  const int64_t i = blockIdx.x;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < s; e += NT) {
    const double v = W[i * s + e];
    acc += v * v;
  }
  __shared__ double red[NT / 64];
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    nu[i] = t;
  }
}

__global__ void __launch_bounds__(NT) k_cpqr_step(double *__restrict__ W, int64_t m, int64_t s, int step,
                                                  const double *__restrict__ nu_in, double *__restrict__ nu_out,
                                                  double *__restrict__ Rk, int64_t *__restrict__ piv,
                                                  int *__restrict__ dflags) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  __shared__ double bv[NT / 64];
  __shared__ int64_t bi[NT / 64];
  __shared__ int64_t p_sh;
  __shared__ double red[NT / 64][CPB];
  __shared__ double coef[CPB];

  // ---- argmax of nu_in over unselected candidates (ties -> lowest index)
  double best = -1.0;
  int64_t bidx = m;
  for (int64_t i = t; i < m; i += NT) {
    const double v = nu_in[i];
    if (v > best) { best = v; bidx = i; }   // ascending i: strict '>' keeps the lowest index
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(best, o, 64);
    const int64_t oi = __shfl_xor(bidx, o, 64);
    if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
  }
  if (lane == 0) { bv[wave] = best; bi[wave] = bidx; }
  __syncthreads();
  if (t == 0) {
    double b = bv[0];
    int64_t ix = bi[0];
    for (int w = 1; w < NT / 64; ++w)
      if (bv[w] > b || (bv[w] == b && bi[w] < ix)) { b = bv[w]; ix = bi[w]; }
    p_sh = ix;
  }
  __syncthreads();
  const int64_t p = p_sh;
  const double nup = (p < m) ? nu_in[p] : 0.0;
  const double rpp = nup > 0.0 ? sqrt(nup) : 0.0;
  const double qscale = rpp > 0.0 ? 1.0 / rpp : 0.0;
  if (blockIdx.x == 0 && t == 0) {
    piv[step] = p;
    if (p < m) Rk[(int64_t)step * m + p] = rpp;
    if (!(rpp > 0.0)) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_RANK_DEFICIENT);
  }
  const double *qrow = W + p * s;   // residual of the pivot (not written this step)

  // ---- my candidates
  int64_t cand[CPB];
  bool live[CPB];
#pragma unroll
  for (int c = 0; c < CPB; ++c) {
    cand[c] = (int64_t)blockIdx.x * CPB + c;
    const bool inr = cand[c] < m;
    const double v = inr ? nu_in[cand[c]] : -1.0;
    live[c] = inr && v >= 0.0 && cand[c] != p;
    if (inr && !live[c] && t == 0) nu_out[cand[c]] = -1.0;   // selected (now or before)
  }
  // dots with q
  double d[CPB];
#pragma unroll
  for (int c = 0; c < CPB; ++c) d[c] = 0.0;
  if (p < m) {
    for (int64_t e = t; e < s; e += NT) {
      const double qe = qrow[e] * qscale;
#pragma unroll
      for (int c = 0; c < CPB; ++c)
        if (live[c]) d[c] = fma(qe, W[cand[c] * s + e], d[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < CPB; ++c) {
    const double v = wsum(d[c]);
    if (lane == 0) red[wave][c] = v;
  }
  __syncthreads();
  if (t < CPB) {
    double v = 0.0;
    for (int w = 0; w < NT / 64; ++w) v += red[w][t];
    coef[t] = v;
  }
  __syncthreads();
  double r[CPB];
#pragma unroll
  for (int c = 0; c < CPB; ++c) r[c] = coef[c];
  // update residuals and recompute norms
  double nn[CPB];
#pragma unroll
  for (int c = 0; c < CPB; ++c) nn[c] = 0.0;
  for (int64_t e = t; e < s; e += NT) {
    const double qe = (p < m) ? qrow[e] * qscale : 0.0;
#pragma unroll
    for (int c = 0; c < CPB; ++c) {
      if (!live[c]) continue;
      double* wp = W + cand[c] * s + e;
      const double w = fma(-r[c], qe, *wp);
      *wp = w;
      nn[c] = fma(w, w, nn[c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CPB; ++c) {
    const double v = wsum(nn[c]);
    if (lane == 0) red[wave][c] = v;
  }
  __syncthreads();
  if (t < CPB && live[t]) {
    double v = 0.0;
    for (int w = 0; w < NT / 64; ++w) v += red[w][t];
    nu_out[cand[t]] = v;
    Rk[(int64_t)step * m + cand[t]] = r[t];
    if (!isfinite(v)) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
  }
}

// C = R_1^{-1} R_2 by back substitution; P(piv[b], :) = e_b, P(i, :) = C(:, i)^T.
// One wave per block, one candidate per lane; the solution vector lives in LDS.
constexpr int KMAX = 112;

__global__ void __launch_bounds__(64) k_id_solve(const double *__restrict__ Rk, const int64_t *__restrict__ piv,
                                                 const double *__restrict__ nu_final, int64_t m, int k,
                                                 double *__restrict__ P, int *__restrict__ dflags) {
  extern __shared__ double dyn[];
  double *R1 = dyn;              // k x k upper, R1[a][b] = Rk[a, piv[b]]
  double *cs = dyn + k * k;      // k x 64 per-lane solution
  const int t = threadIdx.x;
  for (int e = t; e < k * k; e += 64) {
    const int a = e / k, b = e % k;
    const int64_t pb = piv[b];
    R1[e] = (b >= a && pb >= 0 && pb < m) ? Rk[(int64_t)a * m + pb] : 0.0;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 64 + t;
  if (i >= m) return;
  if (nu_final[i] < 0.0) {
    // a pivot: identity row
    int b = -1;
    for (int q = 0; q < k; ++q)
      if (piv[q] == i) b = q;
    for (int q = 0; q < k; ++q) P[i * k + q] = (q == b) ? 1.0 : 0.0;
    return;
  }
  const double dmax = fabs(R1[0]);
  for (int b = 0; b < k; ++b) cs[b * 64 + t] = Rk[(int64_t)b * m + i];
  for (int b = k - 1; b >= 0; --b) {
    const double dbb = R1[b * k + b];
    double x = 0.0;
    if (fabs(dbb) > 1e-14 * dmax) x = cs[b * 64 + t] / dbb;
    else if (t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_RANK_DEFICIENT);
    cs[b * 64 + t] = x;
    for (int a = 0; a < b; ++a) cs[a * 64 + t] = fma(-R1[a * k + b], x, cs[a * 64 + t]);
  }
  for (int q = 0; q < k; ++q) P[i * k + q] = cs[q * 64 + t];
}

}  // namespace

int launch_cpqr(hipStream_t st, double *W, int64_t m, int64_t s, int k, double *nu0, double *nu1, double *Rk,
                int64_t *piv, int *dflags) {
  hipLaunchKernelGGL(k_cpqr_norms, dim3((unsigned)m), dim3(NT), 0, st, (const double *)W, m, s, nu0);
  DSK_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_fill0, dim3((unsigned)std::min<int64_t>(((int64_t)k * m + 255) / 256, 4096)), dim3(256), 0, st,
                     Rk, (int64_t)k * m);
  DSK_TRY(hipGetLastError());
  const unsigned blocks = (unsigned)((m + CPB - 1) / CPB);
  for (int t = 0; t < k; ++t) {
    const double *in = (t & 1) ? nu1 : nu0;
    double *out = (t & 1) ? nu0 : nu1;
    hipLaunchKernelGGL(k_cpqr_step, dim3(blocks), dim3(NT), 0, st, W, m, s, t, in, out, Rk, piv, dflags);
    DSK_TRY(hipGetLastError());
  }
  return 0;
}

// nu_final: the nu buffer written by the last step (selected entries are -1).
int launch_id_solve(hipStream_t st, const double *Rk, const int64_t *piv, const double *nu_final, int64_t m, int k,
                    double *P, int *dflags) {
  if (k < 1 || k > KMAX) return -1;
  const size_t lds = ((size_t)k * k + (size_t)k * 64) * sizeof(double);
  allow_lds(k_id_solve, lds);
  hipLaunchKernelGGL(k_id_solve, dim3((unsigned)((m + 63) / 64)), dim3(64), lds, st, Rk, piv, nu_final, m, k, P,
                     dflags);
  DSK_TRY(hipGetLastError());
  return 0;
}

// Row interpolative decomposition by rank-k column-pivoted QR of W^T
// (paper Sec. 4, row ID; TPC-ID, Alg. 4).
//
// W is m x s, row-major, FP64: row i of W is column i of X = W^T, the i-th
// candidate (time step).  The factorization is right-looking modified
// Gram-Schmidt with column pivoting, FP64 throughout:
//   step t: p = argmax over unselected i of nu_i = ||residual_i||^2, in the
//           order of nu_rank (nu truncated to 34 mantissa bits, ties -> lowest
//           index), q = residual_p / ||residual_p||,
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
#include "wavechol.h"

namespace {

constexpr int CPB = 4;     // candidates per workgroup
constexpr int NT = 256;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Pivot order of a candidate with residual norm^2 v (larger wins): v truncated
// to 34 mantissa bits, so candidates closer than 2^-34 relative rank equal and
// the lower index wins; selected (negative) or NaN candidates rank 0 and never
// win.  The one-launch factorization (rowid_reg.hip) uses the same rule.
__device__ __forceinline__ unsigned long long nu_rank(double v) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFull;
  return (v >= 0.0) ? (bits >> 18) + 1ull : 0ull;
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
  __shared__ unsigned long long bv[NT / 64];
  __shared__ int64_t bi[NT / 64];
  __shared__ int64_t p_sh;
  __shared__ double red[NT / 64][CPB];
  __shared__ double coef[CPB];

  // ---- pivot: maximum of nu_rank over unselected candidates (ties -> lowest index)
  unsigned long long best = 0;
  int64_t bidx = m;
  for (int64_t i = t; i < m; i += NT) {
    const unsigned long long r = nu_rank(nu_in[i]);
    if (r > best) { best = r; bidx = i; }   // ascending i: strict '>' keeps the lowest index
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long ov = (unsigned long long)__shfl_xor((long long)best, o, 64);
    const int64_t oi = __shfl_xor(bidx, o, 64);
    if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
  }
  if (lane == 0) { bv[wave] = best; bi[wave] = bidx; }
  __syncthreads();
  if (t == 0) {
    unsigned long long b = bv[0];
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

// Register-resident variant for s <= 256*SPT: the workgroup's CB candidate
// rows are loaded before the argmax (they do not depend on the pivot), kept in
// registers for the dot products and the update, and written back once.
template <int SPT, int CB>
__global__ void __launch_bounds__(NT) k_cpqr_step_reg(double *__restrict__ W, int64_t m, int64_t s, int step,
                                                      const double *__restrict__ nu_in, double *__restrict__ nu_out,
                                                      double *__restrict__ Rk, int64_t *__restrict__ piv,
                                                      int *__restrict__ dflags) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  __shared__ unsigned long long bv[NT / 64];
  __shared__ int64_t bi[NT / 64];
  __shared__ int64_t p_sh;
  __shared__ double red[NT / 64][CB];
  __shared__ double coef[CB];

  int64_t cand[CB];
  bool live[CB];
  double w[CB][SPT];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    cand[c] = (int64_t)blockIdx.x * CB + c;
    const bool inr = cand[c] < m;
    live[c] = inr && nu_in[cand[c]] >= 0.0;
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int64_t e = t + (int64_t)NT * u;
      w[c][u] = (live[c] && e < s) ? W[cand[c] * s + e] : 0.0;
    }
  }

  // ---- pivot: maximum of nu_rank over unselected candidates (ties -> lowest index)
  unsigned long long best = 0;
  int64_t bidx = m;
  for (int64_t i = t; i < m; i += NT) {
    const unsigned long long r = nu_rank(nu_in[i]);
    if (r > best) { best = r; bidx = i; }   // ascending i: strict '>' keeps the lowest index
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long ov = (unsigned long long)__shfl_xor((long long)best, o, 64);
    const int64_t oi = __shfl_xor(bidx, o, 64);
    if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
  }
  if (lane == 0) { bv[wave] = best; bi[wave] = bidx; }
  __syncthreads();
  if (t == 0) {
    unsigned long long b = bv[0];
    int64_t ix = bi[0];
    for (int ww = 1; ww < NT / 64; ++ww)
      if (bv[ww] > b || (bv[ww] == b && bi[ww] < ix)) { b = bv[ww]; ix = bi[ww]; }
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
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    if (cand[c] == p) live[c] = false;                         // the pivot itself is never written
    if (cand[c] < m && !live[c] && t == 0) nu_out[cand[c]] = -1.0;
  }
  double qv[SPT];
#pragma unroll
  for (int u = 0; u < SPT; ++u) {
    const int64_t e = t + (int64_t)NT * u;
    qv[u] = (p < m && e < s) ? W[p * s + e] * qscale : 0.0;
  }
  double d[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < SPT; ++u) a = fma(qv[u], w[c][u], a);
    d[c] = wsum(a);
    if (lane == 0) red[wave][c] = d[c];
  }
  __syncthreads();
  if (t < CB) {
    double v = 0.0;
    for (int ww = 0; ww < NT / 64; ++ww) v += red[ww][t];
    coef[t] = v;
  }
  __syncthreads();
  double nn[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const double r = coef[c];
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const double x = fma(-r, qv[u], w[c][u]);
      w[c][u] = x;
      a = fma(x, x, a);
    }
    nn[c] = a;
    if (live[c]) {
#pragma unroll
      for (int u = 0; u < SPT; ++u) {
        const int64_t e = t + (int64_t)NT * u;
        if (e < s) W[cand[c] * s + e] = w[c][u];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const double v = wsum(nn[c]);
    if (lane == 0) red[wave][c] = v;
  }
  __syncthreads();
  if (t < CB && live[t]) {
    double v = 0.0;
    for (int ww = 0; ww < NT / 64; ++ww) v += red[ww][t];
    nu_out[cand[t]] = v;
    Rk[(int64_t)step * m + cand[t]] = coef[t];
    if (!isfinite(v)) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
  }
}

// C = R_1^{-1} R_2 by back substitution; P(piv[b], :) = e_b, P(i, :) = C(:, i)^T.
// One wave per candidate: lane l holds entries a = l and a = l + 64 of the
// right-hand side; each of the k substitution steps takes x_b from lane b by
// readlane (b is the same in every lane) and updates all a < b in parallel.
// R_1 is staged transposed in LDS (column b of R_1 contiguous) with the
// reciprocals of its diagonal, shared by the waves of a workgroup.
constexpr int KMAX = 112;
constexpr int SOLVE_WAVES = 4;

__global__ void __launch_bounds__(64 * SOLVE_WAVES) k_id_solve(const double *__restrict__ Rk,
                                                               const int64_t *__restrict__ piv,
                                                               const double *__restrict__ nu_final, int64_t m, int k,
                                                               double *__restrict__ P, int *__restrict__ dflags) {
  extern __shared__ double dyn[];
  double *R1t = dyn;             // R1t[b*k + a] = R_1[a][b] = Rk[a, piv[b]] (a <= b)
  double *rd = dyn + k * k;      // 1 / R_1[b][b], 0 for a negligible pivot
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // the gathered R_1 entries, eight loads in flight per thread
  constexpr int NTS = 64 * SOLVE_WAVES;
  for (int e0 = 0; e0 < k * k; e0 += 8 * NTS) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + t + NTS * u;
      double x = 0.0;
      if (e < k * k) {
        const int b = e / k, a = e - b * k;
        const int64_t pb = piv[b];
        if (a <= b && pb >= 0 && pb < m) x = Rk[(int64_t)a * m + pb];
      }
      v[u] = x;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + t + NTS * u;
      if (e < k * k) R1t[e] = v[u];
    }
  }
  __syncthreads();
  const double dmax = fabs(R1t[0]);
  for (int b = t; b < k; b += 64 * SOLVE_WAVES) {
    const double dbb = R1t[b * k + b];
    rd[b] = fabs(dbb) > 1e-14 * dmax ? 1.0 / dbb : 0.0;
  }
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * SOLVE_WAVES + wave; i < m; i += (int64_t)gridDim.x * SOLVE_WAVES) {
    if (nu_final[i] < 0.0) {
      // a pivot: identity row
      for (int q = lane; q < k; q += 64) P[i * k + q] = (piv[q] == i) ? 1.0 : 0.0;
      continue;
    }
    double c0 = (lane < k) ? Rk[(int64_t)lane * m + i] : 0.0;
    double c1 = (lane + 64 < k) ? Rk[(int64_t)(lane + 64) * m + i] : 0.0;
    bool deficient = false;
    for (int b = k - 1; b >= 64; --b) {
      const double rb = rd[b];
      const double x = wc::readlane_f64(c1, b - 64) * rb;
      deficient |= rb == 0.0;
      if (lane == b - 64) c1 = x;
      const double *col = R1t + b * k;
      c0 = fma(-col[lane], x, c0);                       // every a = lane < 64 <= b
      if (lane + 64 < b) c1 = fma(-col[lane + 64], x, c1);
    }
    for (int b = std::min(k, 64) - 1; b >= 0; --b) {
      const double rb = rd[b];
      const double x = wc::readlane_f64(c0, b) * rb;
      deficient |= rb == 0.0;
      if (lane == b) c0 = x;
      if (lane < b) c0 = fma(-R1t[b * k + lane], x, c0);
    }
    if (deficient && lane == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_RANK_DEFICIENT);
    if (lane < k) P[i * k + lane] = c0;
    if (lane + 64 < k) P[i * k + lane + 64] = c1;
  }
}

}  // namespace

int launch_cpqr(hipStream_t st, double *W, int64_t m, int64_t s, int k, double *nu0, double *nu1, double *Rk,
                int64_t *piv, int *dflags) {
  hipLaunchKernelGGL(k_fill0, dim3((unsigned)std::min<int64_t>(((int64_t)k * m + 255) / 256, 4096)), dim3(256), 0, st,
                     Rk, (int64_t)k * m);
  DSK_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_cpqr_norms, dim3((unsigned)m), dim3(NT), 0, st, (const double *)W, m, s, nu0);
  DSK_TRY(hipGetLastError());
  const unsigned blocks = (unsigned)((m + CPB - 1) / CPB);
  for (int t = 0; t < k; ++t) {
    const double *in = (t & 1) ? nu1 : nu0;
    double *out = (t & 1) ? nu0 : nu1;
    if (s <= 256 * 4)
      hipLaunchKernelGGL((k_cpqr_step_reg<4, 4>), dim3((unsigned)((m + 3) / 4)), dim3(NT), 0, st, W, m, s, t, in, out,
                         Rk, piv, dflags);
    else if (s <= 256 * 8)
      hipLaunchKernelGGL((k_cpqr_step_reg<8, 4>), dim3((unsigned)((m + 3) / 4)), dim3(NT), 0, st, W, m, s, t, in, out,
                         Rk, piv, dflags);
    else if (s <= 256 * 16)
      hipLaunchKernelGGL((k_cpqr_step_reg<16, 4>), dim3((unsigned)((m + 3) / 4)), dim3(NT), 0, st, W, m, s, t, in,
                         out, Rk, piv, dflags);
    else if (s <= 256 * 32)
      hipLaunchKernelGGL((k_cpqr_step_reg<32, 2>), dim3((unsigned)((m + 1) / 2)), dim3(NT), 0, st, W, m, s, t, in,
                         out, Rk, piv, dflags);
    else
      hipLaunchKernelGGL(k_cpqr_step, dim3(blocks), dim3(NT), 0, st, W, m, s, t, in, out, Rk, piv, dflags);
    DSK_TRY(hipGetLastError());
  }
  return 0;
}

// nu_final: the nu buffer written by the last step (selected entries are -1).
int launch_id_solve(hipStream_t st, const double *Rk, const int64_t *piv, const double *nu_final, int64_t m, int k,
                    double *P, int *dflags) {
  if (k < 1 || k > KMAX) return -1;
  const size_t lds = ((size_t)k * k + k) * sizeof(double);
  allow_lds(k_id_solve, lds);
  const unsigned blocks = (unsigned)std::min<int64_t>((m + SOLVE_WAVES - 1) / SOLVE_WAVES, 256);
  hipLaunchKernelGGL(k_id_solve, dim3(blocks), dim3(64 * SOLVE_WAVES), lds, st, Rk, piv, nu_final, m, k, P, dflags);
  DSK_TRY(hipGetLastError());
  return 0;
}

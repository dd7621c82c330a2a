// Symmetric eigensolver of the core SVD (Alg. 2, "SVD(B)" step) for the
// FP32 / 16-bit paths: all eigenpairs of the ell x ell FP64 Gram G_B = B B^T
// (ell <= 112), whose eigenvalues are sigma_j^2 and whose eigenvectors are the
// left singular vectors U_B of B.  Three launches:
//
//   1. k_tri_reduce (one workgroup): Householder tridiagonalisation
//      Q^T G Q = T in LDS; step j reflects column j below the diagonal,
//      p = tau A v (symmetric product), w = p - (tau/2)(p.v) v,
//      A -= v w^T + w v^T.  Writes T (d, e), the reflectors and the
//      Gershgorin bounds.
//   2. k_tri_vec (one workgroup per eigenvalue index): multisection on Sturm
//      counts (the signs of the LDL^T pivots of T - x I), 512 points per
//      round, to the rounding level; then the eigenvector of T by the twisted
//      factorisation T - lambda I = N_r Delta_r N_r^T at the twist index r of
//      smallest |gamma_r| (z_r = 1, the two bidiagonal solves on two waves at
//      once), normalised, and its residual ||T z - lambda z|| checked against
//      2e-9 ||T||.
//   3. k_tri_back (one workgroup): vectors of eigenvalues closer than
//      1e-9 ||T|| are re-orthogonalised in order; then U = Q Z, four threads
//      per eigenvector, the reflectors applied from the last to the first.
//
// A failed residual (or a non-finite value) sets the workspace's fail word:
// the back-transformation then writes nothing and the Jacobi core
// eigensolver, launched after it and gated on that word, computes the result.
// Absolute accuracy: eigenvalues within a few u ||G||, eigenvectors within
// about u ||G|| / gap (backward stable reduction, bisection to the rounding
// level), far inside the FP32 parity tolerances of the paths that use it.
// Output as the Jacobi core: lam descending, U row-major with column j the
// eigenvector of lam[j].
#include <algorithm>

#include "dsk_internal.h"
#include "wavechol.h"

namespace {

constexpr int TNT = 512;           // threads of the reduction kernel (two waves per SIMD)
constexpr int TMAX = 112;          // largest ell
constexpr double TU = 1.1102230246251565e-16;

// Sum over the wave, the same value in every lane: DPP sums within each row of
// 16 lanes, then the four row sums in row order.
__device__ __forceinline__ double wave_sum(double v) {
  v = wc::row16_sum(v);
  return (wc::readlane_f64(v, 0) + wc::readlane_f64(v, 16)) + (wc::readlane_f64(v, 32) + wc::readlane_f64(v, 48));
}

// Numbers of eigenvalues of T (diagonal d, squared off-diagonal e2) below
// each of P shifts x[u]: the negative pivots of the LDL^T factorisation of
// T - x I, a pivot of magnitude below pivmin replaced by -pivmin.  The P
// recurrences are interleaved so that their latencies overlap.
template <int P>
__device__ __forceinline__ void sturm_counts(const double *d, const double *e2, int n, const double *x,
                                             double pivmin, int *c) {
  double q[P];
#pragma unroll
  for (int u = 0; u < P; ++u) {
    q[u] = d[0] - x[u];
    if (fabs(q[u]) < pivmin) q[u] = -pivmin;
    c[u] = q[u] < 0.0 ? 1 : 0;
  }
  for (int i = 1; i < n; ++i) {
    const double di = d[i], ei = e2[i - 1];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      q[u] = (di - x[u]) - ei * wc::rcp_nr(q[u]);
      if (fabs(q[u]) < pivmin) q[u] = -pivmin;
      c[u] += q[u] < 0.0 ? 1 : 0;
    }
  }
}

// Point s (0 .. np - 1) of the np interior points of [a, b]; increasing in s.
__device__ __forceinline__ double msec_point(double a, double b, int s, int np) {
  return a + (b - a) * (double)(s + 1) / (double)(np + 1);
}

// LDS (dynamic): A [ell][ell + 1].  Outputs: Td = (d, e) of T, the reflectors
// (Vt, taus), bnd = (lo, hi, pivmin, ||T||) for the multisection; clears the
// fail word.
__global__ void __launch_bounds__(TNT) k_tri_reduce(const double *__restrict__ G, int ell,
                                                    double *__restrict__ Vt, double *__restrict__ taus,
                                                    double *__restrict__ Td, double *__restrict__ bnd,
                                                    int *__restrict__ fail, int *__restrict__ dflags) {
  extern __shared__ double dyn[];
  const int n = ell, ld = ell + 1;
  double *A = dyn;                          // n x ld
  __shared__ double d[TMAX], e[TMAX], tau[TMAX], vv[TMAX], pv[TMAX];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;

  for (int x = t; x < n * n; x += TNT) {
    const int r = x / n, c = x - (x / n) * n;
    A[r * ld + c] = G[x];
  }
  if (t < TMAX) tau[t] = 0.0;
  if (t == 0) *fail = 0;
  __syncthreads();

  // ---- 1. tridiagonalisation, three barriers per column: wave 0 forms the
  // reflector; p = tau A' v by columns (A' = A[j+1:, j+1:] is symmetric), four
  // threads of a quad per column, each every fourth row, summed by DPP; every
  // wave forms K = (tau/2) p.v itself, then A' -= v w^T + w v^T with
  // w = p - K v, a thread owning one column and every fourth row (row-wise LDS
  // access; v_r, p_r are broadcast reads).  Loads go out four at a time.
  const int qc = t >> 2, qh = t & 3;          // matvec: column, row phase
  const int uc = t & 127, uh = t >> 7;        // update: column, row phase
  for (int j = 0; j + 2 < n; ++j) {
    const int L = n - j - 1, o = j + 1;          // x = A[o:, j], length L
    if (wave == 0) {
      double s2 = 0.0;
      for (int i = 1 + lane; i < L; i += 64) {
        const double v = A[(o + i) * ld + j];
        s2 = fma(v, v, s2);
      }
      s2 = wave_sum(s2);
      const double alpha = A[o * ld + j];
      double beta, tj, scale;
      if (s2 == 0.0) {
        beta = alpha;
        tj = 0.0;
        scale = 0.0;
      } else {
        beta = -copysign(sqrt(fma(alpha, alpha, s2)), alpha);
        tj = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      for (int i = 1 + lane; i < L; i += 64) {
        const double v = A[(o + i) * ld + j] * scale;
        A[(o + i) * ld + j] = v;
        vv[i] = v;
      }
      wc::wave_lds_sync();                         // every lane has read alpha
      if (lane == 0) {
        A[o * ld + j] = 1.0;                       // v_0 (e[j] keeps the subdiagonal)
        vv[0] = 1.0;
        tau[j] = tj;
        e[j] = beta;
      }
    }
    __syncthreads();
    const double tj = tau[j];
    {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      if (qc < L) {
        const double *col = &A[o * ld + o + qc];
        int r = qh;
        for (; r + 12 < L; r += 16) {
          const double x0 = col[r * ld], x1 = col[(r + 4) * ld], x2 = col[(r + 8) * ld], x3 = col[(r + 12) * ld];
          const double y0 = vv[r], y1 = vv[r + 4], y2 = vv[r + 8], y3 = vv[r + 12];
          a0 = fma(x0, y0, a0);
          a1 = fma(x1, y1, a1);
          a2 = fma(x2, y2, a2);
          a3 = fma(x3, y3, a3);
        }
        for (; r < L; r += 4) a0 = fma(col[r * ld], vv[r], a0);
      }
      double a = (a0 + a1) + (a2 + a3);
      a += wc::dpp_f64<0xB1>(a);                   // quad: lanes 2i, 2i+1
      a += wc::dpp_f64<0x4E>(a);                   // quad: pairs
      if (qc < L && qh == 0) pv[qc] = tj * a;
    }
    __syncthreads();
    double sk = 0.0;
    for (int i = lane; i < L; i += 64) sk = fma(pv[i], vv[i], sk);
    const double K = 0.5 * tj * wave_sum(sk);
    if (uc < L) {
      const double vc = vv[uc];
      const double wcc = fma(-K, vc, pv[uc]);
      double *col = &A[o * ld + o + uc];
      int r = uh;
      for (; r + 12 < L; r += 16) {
        double x[4], vr[4], pr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          x[u] = col[(r + 4 * u) * ld];
          vr[u] = vv[r + 4 * u];
          pr[u] = pv[r + 4 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double wr = fma(-K, vr[u], pr[u]);
          col[(r + 4 * u) * ld] = x[u] - fma(vr[u], wcc, wr * vc);
        }
      }
      for (; r < L; r += 4) {
        const double vr = vv[r];
        const double wr = fma(-K, vr, pv[r]);
        col[r * ld] -= fma(vr, wcc, wr * vc);
      }
    }
    __syncthreads();
  }
  // diagonal, last subdiagonal; reflectors (row j of Vt: v_j at columns j+1 .. n-1)
  if (t < n) d[t] = A[t * ld + t];
  if (t == 0 && n >= 2) {
    e[n - 2] = A[(n - 1) * ld + n - 2];
    e[n - 1] = 0.0;
    tau[n - 2] = 0.0;
  }
  for (int x = t; x < n * n; x += TNT) {
    const int j = x / n, c = x - (x / n) * n;
    Vt[x] = (j + 2 < n && c > j) ? A[c * ld + j] : 0.0;
  }
  if (t < n) taus[t] = (t + 2 < n) ? tau[t] : 0.0;
  __syncthreads();

  if (t < n) {
    Td[t] = d[t];
    Td[TMAX + t] = e[t];
  }
  if (t == 0) {
    double lo = d[0], hi = d[0], tmax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
      lo = fmin(lo, d[i] - r);
      hi = fmax(hi, d[i] + r);
      tmax = fmax(tmax, fabs(d[i]) + r);
    }
    double emax = 0.0;
    for (int i = 0; i + 1 < n; ++i) emax = fmax(emax, e[i] * e[i]);
    const double pad = 2.0 * TU * tmax * n + 1e-300;
    bnd[0] = lo - pad;
    bnd[1] = hi + pad;
    bnd[2] = 1e-290 * fmax(1.0, emax);          // pivmin
    bnd[3] = tmax;
    if (!isfinite(tmax)) {
      atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
      *fail = 1;
    }
  }
}

// Eigenpair ei = blockIdx.x (ascending order) of T.  Multisection: every
// round evaluates the Sturm counts at NPV = 512 interior points of the
// current interval [a, b] (two interleaved recurrences per thread) and keeps
// [x_{s-1}, x_s] for the first point s whose count exceeds ei; the first such
// s is a workgroup minimum in LDS, one barrier per round (three slots used in
// rotation, so the slot reset for round r + 1 is one no thread still reads).
// Stops when b - a <= max(4 u max(|a|, |b|), 2 u ||T||).
__global__ void __launch_bounds__(256) k_tri_vec(const double *__restrict__ Td, const double *__restrict__ bnd,
                                                 int ell, double *__restrict__ lam, double *__restrict__ Zg,
                                                 int *__restrict__ fail, int *__restrict__ dflags) {
  constexpr int NPV = 512;
  __shared__ double d[TMAX], e[TMAX], e2[TMAX], dp[TMAX], dm[TMAX], z[TMAX], red[4];
  __shared__ int smin[3];
  __shared__ unsigned long long gkey;
  __shared__ int rsh;
  const int n = ell, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int ei = blockIdx.x;
  if (t < n) {
    d[t] = Td[t];
    e[t] = Td[TMAX + t];
    e2[t] = (t + 1 < n) ? e[t] * e[t] : 0.0;
  }
  if (t < 3) smin[t] = NPV;
  if (t == 0) gkey = ~0ull;
  __syncthreads();
  const double pivmin = bnd[2], tnorm = bnd[3];
  double a = bnd[0], b = bnd[1];
  int round = 0;
  for (; round < 64; ++round) {
    if (!(b - a > 4.0 * TU * fmax(fabs(a), fabs(b)) + 1e-300 && b - a > 2.0 * TU * tnorm)) break;
    double xs[2];
    int cs[2];
    xs[0] = msec_point(a, b, 2 * t, NPV);
    xs[1] = msec_point(a, b, 2 * t + 1, NPV);
    sturm_counts<2>(d, e2, n, xs, pivmin, cs);
    const int mine = cs[0] > ei ? 2 * t : (cs[1] > ei ? 2 * t + 1 : NPV);
    const int slot = round % 3;
    if (mine < NPV) atomicMin(&smin[slot], mine);
    if (t == 0) smin[(round + 1) % 3] = NPV;
    __syncthreads();
    const int sf = smin[slot];
    const double na = sf > 0 ? msec_point(a, b, sf - 1, NPV) : a;
    const double nb = sf < NPV ? msec_point(a, b, sf, NPV) : b;
    a = na;
    b = nb;
  }
  const double lm = 0.5 * (a + b);
  // twisted factorisation: D+ top-down (wave 0), D- bottom-up (wave 1), at once
  if (t == 0) {
    double v = d[0] - lm;
    if (fabs(v) < pivmin) v = -pivmin;
    dp[0] = v;
    for (int i = 0; i + 1 < n; ++i) {
      v = (d[i + 1] - lm) - e2[i] * wc::rcp_nr(v);
      if (fabs(v) < pivmin) v = -pivmin;
      dp[i + 1] = v;
    }
  } else if (t == 64) {
    double v = d[n - 1] - lm;
    if (fabs(v) < pivmin) v = -pivmin;
    dm[n - 1] = v;
    for (int i = n - 2; i >= 0; --i) {
      v = (d[i] - lm) - e2[i] * wc::rcp_nr(v);
      if (fabs(v) < pivmin) v = -pivmin;
      dm[i] = v;
    }
  }
  __syncthreads();
  // r = argmin |gamma_i|, gamma_i = D+_i + D-_i - (d_i - lambda); ties: lowest i
  if (t < n) {
    const double g = fabs(dp[t] + dm[t] - (d[t] - lm));
    const unsigned long long key = ((unsigned long long)__double_as_longlong(g) & ~0x7Full) | (unsigned)t;
    atomicMin(&gkey, key);
  }
  __syncthreads();
  const int r = (int)(gkey & 0x7F);
  // z_r = 1; up: z_i = -(e_i / D+_i) z_{i+1} (wave 0); down: z_{i+1} = -(e_i / D-_{i+1}) z_i (wave 1)
  if (t == 0) {
    double v = 1.0;
    z[r] = 1.0;
    for (int i = r - 1; i >= 0; --i) {
      v = -(e[i] * wc::rcp_nr(dp[i])) * v;
      z[i] = v;
    }
  } else if (t == 64) {
    double v = 1.0;
    for (int i = r; i + 1 < n; ++i) {
      v = -(e[i] * wc::rcp_nr(dm[i + 1])) * v;
      z[i + 1] = v;
    }
  }
  __syncthreads();
  // ||z||^2 in a fixed order: per wave, then the waves in order
  double s2 = 0.0;
  if (t < n) s2 = z[t] * z[t];
  s2 = wave_sum(s2);
  if (lane == 0) red[wave] = s2;
  __syncthreads();
  const double sc = wc::rsq_nr((red[0] + red[1]) + (red[2] + red[3]));
  bool bad = false;
  if (t < n) {
    const double zi = z[t] * sc;
    double res = (d[t] - lm) * zi;
    if (t > 0) res = fma(e[t - 1], z[t - 1] * sc, res);
    if (t + 1 < n) res = fma(e[t], z[t + 1] * sc, res);
    bad = !isfinite(zi) || !(fabs(res) <= 2e-9 * tnorm);
    Zg[t * n + (n - 1 - ei)] = zi;            // column n - 1 - ei: descending order
  }
  if (bad) atomicOr(fail, 1);
  if (t == 0) {
    lam[n - 1 - ei] = lm;
    if (!isfinite(lm)) atomicOr(fail, 1);
    atomicMax(&dflags[FLAGW_SWEEPS], round);
  }
}

// Vectors of close eigenvalues (gap <= 1e-9 ||T||) re-orthogonalised in
// ascending order of eigenvalue, two passes of Gram-Schmidt against the
// earlier members of the cluster, by wave 0 on Zg in global memory (column
// n - 1 - a holds the vector of ascending index a).  Equal eigenvalues give
// equal twisted vectors; a member that keeps less than half its norm is
// replaced by one step of inverse iteration, (T - lambda I) y = x with the
// LDL^T factorisation of T - lambda I, from a fixed start x orthogonal to the
// earlier members (the step amplifies the cluster's eigenspace by about
// 1 / (u ||T||)), then orthogonalised again.  Then U = Q Z:
// Q = H_0 H_1 ... H_{n-3}, H_j = I - tau_j v_j v_j^T (v_j in row j of Vt,
// columns j+1 ..).  Four threads per column, rows interleaved by 4; the
// reflectors go from the last to the first.  RPT = rows per thread; the rows
// of Vt sit in LDS with stride 4 RPT, zero outside v_j's support, so the
// products need no bounds tests (a load behind a branch waits on its own).
template <int RPT>
__global__ void __launch_bounds__(512) k_tri_back(const double *__restrict__ Vt, const double *__restrict__ taus,
                                                  double *__restrict__ Zg, const double *__restrict__ lam,
                                                  const double *__restrict__ Td, const double *__restrict__ bnd,
                                                  int ell, const int *__restrict__ fail, double *__restrict__ U) {
  extern __shared__ double vlds[];         // ell rows of 4 RPT
  __shared__ double tls[TMAX], lsh[TMAX];
  if (*fail) return;                       // the gated Jacobi core writes U
  constexpr int NP = 4 * RPT;
  const int n = ell, t = threadIdx.x;
  if (t < 64) {
    const int lane = t;
    const double gtol = 1e-9 * fmax(bnd[3], 1e-300), pivmin = bnd[2];
    auto col = [&](int asc) { return n - 1 - asc; };
    // x <- x - sum over the members s0 .. c-1 of (x . z_s) z_s, twice; returns ||x||^2
    auto mgs = [&](int s0, int c) {
      for (int pass = 0; pass < 2; ++pass) {
        for (int sv = s0; sv < c; ++sv) {
          double dot = 0.0;
          for (int i = lane; i < n; i += 64) dot = fma(Zg[i * n + col(sv)], Zg[i * n + col(c)], dot);
          dot = wave_sum(dot);
          for (int i = lane; i < n; i += 64) Zg[i * n + col(c)] = fma(-dot, Zg[i * n + col(sv)], Zg[i * n + col(c)]);
        }
      }
      double nn = 0.0;
      for (int i = lane; i < n; i += 64) nn = fma(Zg[i * n + col(c)], Zg[i * n + col(c)], nn);
      return wave_sum(nn);
    };
    auto scale = [&](int c, double f) {
      for (int i = lane; i < n; i += 64) Zg[i * n + col(c)] *= f;
    };
    for (int c = 1; c < n; ++c) {
      if (lam[col(c)] - lam[col(c - 1)] > gtol) continue;   // ascending gap
      int s0 = c - 1;
      while (s0 > 0 && lam[col(s0)] - lam[col(s0 - 1)] <= gtol) --s0;
      double nn = mgs(s0, c);
      if (!(nn >= 0.25)) {
        // fixed start: entries in (-1/2, 1/2) from a multiplicative hash of (i, c)
        for (int i = lane; i < n; i += 64)
          Zg[i * n + col(c)] = (double)((unsigned)(i * 2654435761u + c * 40503u) >> 8) * 0x1p-24 - 0.5;
        nn = mgs(s0, c);
        scale(c, nn > 0.0 ? wc::rsq_nr(nn) : 0.0);
        // lane 0 reads every row: the wave's stores come first
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
          // (T - lambda I) y = x: T - lambda I = L D L^T, L unit lower bidiagonal (l_i = e_i / D_i)
          const double lm = lam[col(c)];
          const double *dT = Td, *eT = Td + TMAX;
          double Dp = dT[0] - lm;
          if (fabs(Dp) < pivmin) Dp = -pivmin;
          double w = Zg[col(c)];
          Zg[col(c)] = w / Dp;                     // v_0 = w_0 / D_0; l_0 kept implicit
          for (int i = 0; i + 1 < n; ++i) {
            const double li = eT[i] / Dp;
            double Dn = (dT[i + 1] - lm) - li * eT[i];
            if (fabs(Dn) < pivmin) Dn = -pivmin;
            w = Zg[(i + 1) * n + col(c)] - li * w;  // forward: w_{i+1} = x_{i+1} - l_i w_i
            Zg[(i + 1) * n + col(c)] = w / Dn;
            Dp = Dn;
          }
          // backward: y_i = v_i - l_i y_{i+1}, with l_i recomputed from the same pivots
          double Dq = dT[0] - lm;
          if (fabs(Dq) < pivmin) Dq = -pivmin;
          double *ls = lsh;
          for (int i = 0; i + 1 < n; ++i) {
            ls[i] = eT[i] / Dq;
            double Dn = (dT[i + 1] - lm) - ls[i] * eT[i];
            if (fabs(Dn) < pivmin) Dn = -pivmin;
            Dq = Dn;
          }
          double y = Zg[(n - 1) * n + col(c)], ymax = fabs(y);
          for (int i = n - 2; i >= 0; --i) {
            y = Zg[i * n + col(c)] - ls[i] * y;
            Zg[i * n + col(c)] = y;
            ymax = fmax(ymax, fabs(y));
          }
          const double f = (ymax > 0.0 && isfinite(ymax)) ? 1.0 / ymax : 0.0;
          for (int i = 0; i < n; ++i) Zg[i * n + col(c)] *= f;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        nn = mgs(s0, c);
      }
      scale(c, nn > 0.0 ? wc::rsq_nr(nn) : 0.0);
    }
  }
  __syncthreads();
  for (int x = t; x < n * NP; x += 512) {
    const int j = x / NP, c = x - (x / NP) * NP;
    vlds[x] = c < n ? Vt[j * n + c] : 0.0;
  }
  if (t < n) tls[t] = taus[t];
  __syncthreads();
  const int c = t >> 2, g = t & 3;
  const bool act = c < n;
  double z[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int r = g + 4 * u;
    z[u] = (act && r < n) ? Zg[r * n + c] : 0.0;
  }
  for (int j = n - 3; j >= 0; --j) {
    const double tj = tls[j];
    const double *v = &vlds[j * NP + g];
    double vr[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) vr[u] = v[4 * u];
    double w0 = 0.0, w1 = 0.0;
#pragma unroll
    for (int u = 0; u < RPT; u += 2) {
      w0 = fma(vr[u], z[u], w0);
      w1 = fma(vr[u + 1], z[u + 1], w1);
    }
    double w = w0 + w1;
    w += wc::dpp_f64<0xB1>(w);
    w += wc::dpp_f64<0x4E>(w);
    const double tw = tj * w;
#pragma unroll
    for (int u = 0; u < RPT; ++u) z[u] = fma(-tw, vr[u], z[u]);
  }
  if (act)
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int r = g + 4 * u;
      if (r < n) U[r * n + c] = z[u];
    }
}

}  // namespace

size_t core_eig_tri_ws_bytes(int ell) {
  return ((size_t)2 * ell * ell + ell + 2 * TMAX + 4 + 8) * sizeof(double);
}

int launch_core_eig_tri(hipStream_t st, const double *G, int ell, double *lam, double *U, double *ws, int *dflags) {
  if (ell < 3 || ell > TMAX) return launch_core_eig(st, G, ell, lam, U, dflags);
  double *Vt = ws;
  double *Zg = Vt + (size_t)ell * ell;
  double *taus = Zg + (size_t)ell * ell;
  double *Td = taus + ell;
  double *bnd = Td + 2 * TMAX;
  int *fail = reinterpret_cast<int *>(bnd + 4);
  const size_t lds1 = (size_t)ell * (ell + 1) * sizeof(double);
  allow_lds(k_tri_reduce, lds1);
  hipLaunchKernelGGL(k_tri_reduce, dim3(1), dim3(TNT), lds1, st, G, ell, Vt, taus, Td, bnd, fail, dflags);
  DSK_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_tri_vec, dim3(ell), dim3(256), 0, st, (const double *)Td, (const double *)bnd, ell, lam, Zg,
                     fail, dflags);
  DSK_TRY(hipGetLastError());
  if (ell <= 64) {
    const size_t lds2 = (size_t)ell * 64 * sizeof(double);
    allow_lds(k_tri_back<16>, lds2);
    hipLaunchKernelGGL(k_tri_back<16>, dim3(1), dim3(512), lds2, st, Vt, taus, Zg, (const double *)lam,
                       (const double *)Td, (const double *)bnd, ell, fail, U);
  } else {
    const size_t lds2 = (size_t)ell * 112 * sizeof(double);
    allow_lds(k_tri_back<28>, lds2);
    hipLaunchKernelGGL(k_tri_back<28>, dim3(1), dim3(512), lds2, st, Vt, taus, Zg, (const double *)lam,
                       (const double *)Td, (const double *)bnd, ell, fail, U);
  }
  DSK_TRY(hipGetLastError());
  // fallback: the Jacobi core, which leaves at once unless the fail word is set
  return launch_core_eig_gated(st, G, ell, lam, U, dflags, fail, 1);
}

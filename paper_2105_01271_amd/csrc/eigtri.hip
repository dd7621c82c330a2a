// Symmetric eigensolver of the core SVD (Alg. 2, "SVD(B)" step) for the
// FP32 / 16-bit paths: all eigenpairs of the ell x ell FP64 Gram G_B = B B^T
// (ell <= 112), whose eigenvalues are sigma_j^2 and whose eigenvectors are the
// left singular vectors U_B of B.
//
//   1. Householder tridiagonalisation Q^T G Q = T (G in LDS, one workgroup of
//      four waves): step j reflects column j below the diagonal, p = tau A v
//      (symmetric product), w = p - (tau/2)(p.v) v, A -= v w^T + w v^T.
//   2. Eigenvalues of T by multisection: every eigenvalue index owns a group
//      of threads, each round evaluates Sturm counts (the signs of the LDL^T
//      pivots of T - x I) at the group's interior points (four per thread,
//      interleaved) and keeps the sub-interval that holds the index.
//   3. Eigenvectors of T by the twisted factorisation at each eigenvalue:
//      T - lambda I = N_r Delta_r N_r^T with the twist index r where |gamma_r|
//      is smallest; z_r = 1 and the two bidiagonal solves give z.  Vectors of
//      eigenvalues closer than 1e-9 ||T|| are re-orthogonalised in order.
//      Every vector's residual ||T z - lambda z|| is checked against 2e-9 ||T||;
//      a failure (or a non-finite value) sets the workspace's fail word, the
//      back-transformation then writes nothing and the Jacobi core eigensolver,
//      launched after it and gated on that word, computes the result instead.
//   4. Back-transformation U = Q Z (second kernel): four threads per
//      eigenvector, the reflectors applied from the last to the first.
//
// Absolute accuracy: eigenvalues within a few u ||G||, eigenvectors within
// about u ||G|| / gap (backward stable reduction, bisection to the rounding
// level), far inside the FP32 parity tolerances of the paths that use it.
// Output as the Jacobi core: lam descending, U row-major with column j the
// eigenvector of lam[j].
#include <algorithm>

#include "dsk_internal.h"
#include "wavechol.h"

namespace {

constexpr int TNT = 512;           // threads of the reduction / eigenvalue kernel (two waves per SIMD)
constexpr int TMAX = 112;          // largest ell
constexpr int NPT = 4;             // Sturm counts per thread and multisection round
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

// LDS (dynamic): A [ell][ell + 1] (the matrix, later Z), then small arrays.
__global__ void __launch_bounds__(TNT) k_tri_eig(const double *__restrict__ G, int ell, double *__restrict__ lam,
                                                 double *__restrict__ Vt, double *__restrict__ taus,
                                                 double *__restrict__ Zg, int *__restrict__ fail,
                                                 int *__restrict__ dflags) {
  extern __shared__ double dyn[];
  const int n = ell, ld = ell + 1;
  double *A = dyn;                          // n x ld
  __shared__ double d[TMAX], e[TMAX], e2[TMAX], tau[TMAX], vv[TMAX], pv[TMAX], lo_sh[TMAX], hi_sh[TMAX],
      lamu[TMAX];
  __shared__ int cnt_sh[TNT * NPT];
  __shared__ double red[TNT / 64];
  __shared__ double bcast[4];
  __shared__ int clus_sh;
  __shared__ int bad_sh;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;

  for (int x = t; x < n * n; x += TNT) {
    const int r = x / n, c = x - (x / n) * n;
    A[r * ld + c] = G[x];
  }
  if (t < TMAX) tau[t] = 0.0;
  if (t == 0) bad_sh = 0;
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
    tau[n - 2] = 0.0;
  }
  for (int x = t; x < n * n; x += TNT) {
    const int j = x / n, c = x - (x / n) * n;
    Vt[x] = (j + 2 < n && c > j) ? A[c * ld + j] : 0.0;
  }
  if (t < n) taus[t] = (t + 2 < n) ? tau[t] : 0.0;
  __syncthreads();

  // ---- 2. eigenvalues: multisection on Sturm counts
  if (t < n) e2[t] = (t + 1 < n) ? e[t] * e[t] : 0.0;
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
    bcast[0] = lo - pad;
    bcast[1] = hi + pad;
    bcast[2] = 1e-290 * fmax(1.0, emax);          // pivmin
    bcast[3] = tmax;
    if (!isfinite(tmax)) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
  }
  __syncthreads();
  const double pivmin = bcast[2], tnorm = bcast[3];
  if (t < n) {
    lo_sh[t] = bcast[0];
    hi_sh[t] = bcast[1];
  }
  const int ns = TNT / n;                         // threads per eigenvalue (>= 4)
  const int np = ns * NPT;                        // points per eigenvalue and round
  const int ei = t / ns, si = t - (t / ns) * ns;
  int rounds = 0;
  for (; rounds < 128; ++rounds) {
    __syncthreads();
    if (t == 0) clus_sh = 0;
    __syncthreads();
    double a = 0.0, b = 0.0;
    if (ei < n) {
      a = lo_sh[ei];
      b = hi_sh[ei];
      if (b - a > 4.0 * TU * fmax(fabs(a), fabs(b)) + 1e-300 && b - a > 2.0 * TU * tnorm) clus_sh = 1;
    }
    __syncthreads();
    if (!clus_sh) break;
    if (ei < n) {
      double xs[NPT];
      int cs[NPT];
#pragma unroll
      for (int u = 0; u < NPT; ++u) xs[u] = msec_point(a, b, si * NPT + u, np);
      sturm_counts<NPT>(d, e2, n, xs, pivmin, cs);
#pragma unroll
      for (int u = 0; u < NPT; ++u) cnt_sh[t * NPT + u] = cs[u];
    }
    __syncthreads();
    if (ei < n && si == 0) {
      // points x_s increase with s; keep [last x with count <= ei, first x with count > ei]
      double na = a, nb = b;
      for (int s = 0; s < np; ++s) {
        const double x = msec_point(a, b, s, np);
        if (cnt_sh[ei * np + s] <= ei) na = x;
        else { nb = x; break; }
      }
      lo_sh[ei] = na;
      hi_sh[ei] = nb;
    }
  }
  __syncthreads();
  if (t < n) lamu[t] = 0.5 * (lo_sh[t] + hi_sh[t]);   // ascending
  if (t == 0) dflags[FLAGW_SWEEPS] = rounds;
  __syncthreads();

  // ---- 3. eigenvectors of T: twisted factorisation, column t of Z (A reused, ld)
  double *Z = A;
  if (t < n) {
    const double lm = lamu[t];
    // top-down: D+_i into Z[i][t]
    double dp = d[0] - lm;
    if (fabs(dp) < pivmin) dp = -pivmin;
    Z[t] = dp;
    for (int i = 0; i + 1 < n; ++i) {
      dp = (d[i + 1] - lm) - e2[i] * wc::rcp_nr(dp);
      if (fabs(dp) < pivmin) dp = -pivmin;
      Z[(i + 1) * ld + t] = dp;
    }
    // bottom-up: D-_i and gamma_i = D+_i + D-_i - (d_i - lambda); r = argmin |gamma|
    double dm = d[n - 1] - lm;
    if (fabs(dm) < pivmin) dm = -pivmin;
    int r = n - 1;
    double gbest = fabs(Z[(n - 1) * ld + t]);          // gamma_{n-1} = D+_{n-1}
    for (int i = n - 2; i >= 0; --i) {
      dm = (d[i] - lm) - e2[i] * wc::rcp_nr(dm);
      if (fabs(dm) < pivmin) dm = -pivmin;
      const double g = fabs(Z[i * ld + t] + dm - (d[i] - lm));
      if (g < gbest) { gbest = g; r = i; }
    }
    // D-_i for i > r into Z[i][t]
    dm = d[n - 1] - lm;
    if (fabs(dm) < pivmin) dm = -pivmin;
    for (int i = n - 1; i > r; --i) {
      Z[i * ld + t] = dm;
      if (i - 1 > r) {
        dm = (d[i - 1] - lm) - e2[i - 1] * wc::rcp_nr(dm);
        if (fabs(dm) < pivmin) dm = -pivmin;
      }
    }
    // z_r = 1; up: z_i = -(e_i / D+_i) z_{i+1}; down: z_{i+1} = -(e_i / D-_{i+1}) z_i
    double zr = 1.0, nrm = 1.0;
    double z = zr;
    for (int i = r - 1; i >= 0; --i) {
      z = -(e[i] * wc::rcp_nr(Z[i * ld + t])) * z;
      Z[i * ld + t] = z;
      nrm = fma(z, z, nrm);
    }
    Z[r * ld + t] = zr;
    z = zr;
    for (int i = r; i + 1 < n; ++i) {
      z = -(e[i] * wc::rcp_nr(Z[(i + 1) * ld + t])) * z;
      Z[(i + 1) * ld + t] = z;
      nrm = fma(z, z, nrm);
    }
    const double sc = wc::rsq_nr(nrm);
    for (int i = 0; i < n; ++i) Z[i * ld + t] *= sc;
  }
  __syncthreads();
  // re-orthogonalise vectors of close eigenvalues (one wave, in ascending order)
  if (wave == 0) {
    const double gtol = 1e-9 * fmax(tnorm, 1e-300);
    for (int c = 1; c < n; ++c) {
      if (lamu[c] - lamu[c - 1] > gtol) continue;
      int s0 = c - 1;
      while (s0 > 0 && lamu[s0] - lamu[s0 - 1] <= gtol) --s0;
      for (int pass = 0; pass < 2; ++pass) {
        for (int sv = s0; sv < c; ++sv) {
          double dot = 0.0;
          for (int i = lane; i < n; i += 64) dot = fma(Z[i * ld + sv], Z[i * ld + c], dot);
          dot = wave_sum(dot);
          for (int i = lane; i < n; i += 64) Z[i * ld + c] = fma(-dot, Z[i * ld + sv], Z[i * ld + c]);
          wc::wave_lds_sync();
        }
      }
      double nn = 0.0;
      for (int i = lane; i < n; i += 64) nn = fma(Z[i * ld + c], Z[i * ld + c], nn);
      nn = wave_sum(nn);
      const double sc = nn > 0.0 ? wc::rsq_nr(nn) : 0.0;
      for (int i = lane; i < n; i += 64) Z[i * ld + c] *= sc;
      wc::wave_lds_sync();
    }
  }
  __syncthreads();
  // residual check of every vector
  if (t < n) {
    const double lm = lamu[t];
    double rmax = 0.0;
    bool fin = isfinite(lm);
    for (int i = 0; i < n; ++i) {
      const double zi = Z[i * ld + t];
      double r = (d[i] - lm) * zi;
      if (i > 0) r = fma(e[i - 1], Z[(i - 1) * ld + t], r);
      if (i + 1 < n) r = fma(e[i], Z[(i + 1) * ld + t], r);
      rmax = fmax(rmax, fabs(r));
      fin = fin && isfinite(zi);
    }
    if (!fin || !(rmax <= 2e-9 * tnorm)) bad_sh = 1;
  }
  __syncthreads();
  if (t == 0) *fail = bad_sh;
  // descending order out: column j of Zg = eigenvector of lamu[n - 1 - j]
  for (int x = t; x < n * n; x += TNT) {
    const int i = x / n, j = x - (x / n) * n;
    Zg[x] = Z[i * ld + (n - 1 - j)];
  }
  if (t < n) lam[t] = lamu[n - 1 - t];
}

// U = Q Z: Q = H_0 H_1 ... H_{n-3}, H_j = I - tau_j v_j v_j^T (v_j in row j of Vt,
// columns j+1 ..).  Four threads per column, rows interleaved by 4; the
// reflectors go from the last to the first.  RPT = rows per thread; the rows
// of Vt sit in LDS with stride 4 RPT, zero outside v_j's support, so the
// products need no bounds tests (a load behind a branch waits on its own).
template <int RPT>
__global__ void __launch_bounds__(512) k_tri_back(const double *__restrict__ Vt, const double *__restrict__ taus,
                                                  const double *__restrict__ Zg, int ell, const int *__restrict__ fail,
                                                  double *__restrict__ U) {
  extern __shared__ double vlds[];         // ell rows of 4 RPT
  __shared__ double tls[TMAX];
  if (*fail) return;                       // the gated Jacobi core writes U
  constexpr int NP = 4 * RPT;
  const int n = ell, t = threadIdx.x;
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

size_t core_eig_tri_ws_bytes(int ell) { return ((size_t)2 * ell * ell + ell + 64) * sizeof(double); }

int launch_core_eig_tri(hipStream_t st, const double *G, int ell, double *lam, double *U, double *ws, int *dflags) {
  if (ell < 3 || ell > TMAX) return launch_core_eig(st, G, ell, lam, U, dflags);
  double *Vt = ws;
  double *Zg = ws + (size_t)ell * ell;
  double *taus = Zg + (size_t)ell * ell;
  int *fail = reinterpret_cast<int *>(taus + ell);
  const size_t lds1 = (size_t)ell * (ell + 1) * sizeof(double);
  allow_lds(k_tri_eig, lds1);
  hipLaunchKernelGGL(k_tri_eig, dim3(1), dim3(TNT), lds1, st, G, ell, lam, Vt, taus, Zg, fail, dflags);
  DSK_TRY(hipGetLastError());
  if (ell <= 64) {
    const size_t lds2 = (size_t)ell * 64 * sizeof(double);
    allow_lds(k_tri_back<16>, lds2);
    hipLaunchKernelGGL(k_tri_back<16>, dim3(1), dim3(512), lds2, st, Vt, taus, Zg, ell, fail, U);
  } else {
    const size_t lds2 = (size_t)ell * 112 * sizeof(double);
    allow_lds(k_tri_back<28>, lds2);
    hipLaunchKernelGGL(k_tri_back<28>, dim3(1), dim3(512), lds2, st, Vt, taus, Zg, ell, fail, U);
  }
  DSK_TRY(hipGetLastError());
  // fallback: the Jacobi core, which leaves at once unless the fail word is set
  return launch_core_eig_gated(st, G, ell, lam, U, dflags, fail, 1);
}

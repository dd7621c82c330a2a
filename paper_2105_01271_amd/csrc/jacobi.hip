// Small dense eigen / SVD cores of SVD(B), B = Q^T A (Alg. 2, "SVD(B)" step):
//
//  * k_jacobi_eig: two-sided cyclic Jacobi on the ell x ell FP64 Gram
//    G_B = B B^T (F32 / BF16 / F16 paths): eigenvalues lambda_j = sigma_j^2
//    and eigenvectors U_B.  Round-robin (circle) ordering: n/2 disjoint
//    rotations per round, n-1 rounds per sweep.  Every thread owns a fixed
//    set of 2x2 blocks of G (pairs of pairs) and of (row, pair) entries of V,
//    decoded once before the sweeps, so a round is: rotation angles (n/2
//    threads) -> barrier -> in-place block updates -> barrier.  G is kept
//    packed (upper triangle) and V row-major, both in LDS (ell <= 112).
//  * k_jacobi_svd: one-sided (Hestenes) Jacobi on an ell x ell triangular
//    factor R (FP64 path, B^T = Q_B R): no squaring of the singular values.
#include <algorithm>

#include "dsk_internal.h"

namespace {

constexpr int JNT = 1024;
constexpr int JELL_MAX = 112;
constexpr int JNP_MAX = JELL_MAX / 2;
// per-thread item counts for a size class with at most NMAX rows (NMAX even)
template <int NMAX>
constexpr int gi_of() { return ((NMAX / 2) * (NMAX / 2 + 1) / 2 + JNT - 1) / JNT; }   // 2x2 blocks of G
template <int NMAX>
constexpr int vi_of() { return (NMAX * (NMAX / 2) + JNT - 1) / JNT; }                  // (row, pair) of V

__device__ __forceinline__ int rr_player(int pos, int r, int n) {
  return pos == 0 ? 0 : ((pos - 1 + r) % (n - 1)) + 1;
}

__device__ __forceinline__ int pk(int a, int b, int n) {   // packed upper index, a <= b
  return a * n - ((a * (a - 1)) >> 1) + (b - a);
}

template <int NT>
__device__ double jblock_sum(double v, double *scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
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

template <int NMAX>
__global__ void __launch_bounds__(JNT) k_jacobi_eig(const double *__restrict__ part, int nparts, int ell,
                                                    double tol2_rel, double *__restrict__ lam,
                                                    double *__restrict__ Vout, int *__restrict__ dflags) {
  extern __shared__ double dyn[];
  const int n = (ell + 1) & ~1;    // one zero row/column pads an odd size
  const int np = n / 2;
  const int npk = n * (n + 1) / 2;
  double *Gp = dyn;
  double *V = dyn + npk;           // n x n row-major
  __shared__ double rc[JNP_MAX], rs[JNP_MAX];
  __shared__ int pp[JNP_MAX], pq[JNP_MAX];
  __shared__ double red[JNT / 64 + 1];
  __shared__ int rank_of[JELL_MAX + 2];
  const int t = threadIdx.x;
  constexpr int GI = gi_of<NMAX>();
  constexpr int VI = vi_of<NMAX>();

  for (int e = t; e < npk; e += JNT) Gp[e] = 0.0;
  for (int e = t; e < n * n; e += JNT) V[e] = 0.0;
  __syncthreads();
  double fro = 0.0;
  const int nup = ell * (ell + 1) / 2;
  for (int u = t; u < nup; u += JNT) {
    int a = 0, rem = u;
    while (rem >= ell - a) { rem -= ell - a; ++a; }
    const int b = a + rem;
    const int64_t e = (int64_t)a * ell + b;
    const int64_t st = (int64_t)ell * ell;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;   // fixed association: deterministic
    int p = 0;
    for (; p + 3 < nparts; p += 4) {
      s0 += part[p * st + e];
      s1 += part[(p + 1) * st + e];
      s2 += part[(p + 2) * st + e];
      s3 += part[(p + 3) * st + e];
    }
    for (; p < nparts; ++p) s0 += part[p * st + e];
    const double s = (s0 + s1) + (s2 + s3);
    Gp[pk(a, b, n)] = s;
    fro += (a == b ? 1.0 : 2.0) * s * s;
  }
  for (int a = t; a < n; a += JNT) V[a * n + a] = 1.0;
  fro = jblock_sum<JNT>(fro, red);
  if (!isfinite(fro) && t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);

  // fixed per-thread work lists
  const int nblk = np * (np + 1) / 2;
  int gP1[GI], gP2[GI];
#pragma unroll
  for (int u = 0; u < GI; ++u) {
    const int e = t + JNT * u;
    gP1[u] = -1;
    gP2[u] = -1;
    if (e < nblk) {
      int P1 = 0, rem = e;
      while (rem >= np - P1) { rem -= np - P1; ++P1; }
      gP1[u] = P1;
      gP2[u] = P1 + rem;
    }
  }
  int va[VI], vP[VI];
#pragma unroll
  for (int u = 0; u < VI; ++u) {
    const int e = t + JNT * u;
    va[u] = -1;
    vP[u] = 0;
    if (e < n * np) {
      va[u] = e / np;
      vP[u] = e - va[u] * np;
    }
  }

  const double tol2 = tol2_rel * fro;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // off-diagonal mass over the round-0 block decomposition (covers each pair once)
    double off = 0.0;
#pragma unroll
    for (int u = 0; u < GI; ++u) {
      if (gP1[u] < 0) continue;
      int p1 = rr_player(gP1[u], 0, n), q1 = rr_player(n - 1 - gP1[u], 0, n);
      int p2 = rr_player(gP2[u], 0, n), q2 = rr_player(n - 1 - gP2[u], 0, n);
      if (gP1[u] == gP2[u]) {
        const double x = Gp[pk(min(p1, q1), max(p1, q1), n)];
        off += 2.0 * x * x;
      } else {
        const double a = Gp[pk(min(p1, p2), max(p1, p2), n)], b = Gp[pk(min(p1, q2), max(p1, q2), n)];
        const double c = Gp[pk(min(q1, p2), max(q1, p2), n)], d = Gp[pk(min(q1, q2), max(q1, q2), n)];
        off += 2.0 * (a * a + b * b + c * c + d * d);
      }
    }
    off = jblock_sum<JNT>(off, red);
    if (!(off > tol2)) break;
    for (int r = 0; r < n - 1; ++r) {
      if (t < np) {
        int p = rr_player(t, r, n), q = rr_player(n - 1 - t, r, n);
        if (p > q) { const int x = p; p = q; q = x; }
        const double gpp = Gp[pk(p, p, n)], gqq = Gp[pk(q, q, n)], gpq = Gp[pk(p, q, n)];
        double c = 1.0, s = 0.0;
        if (fabs(gpq) > 1e-300 && fabs(gpq) > 1e-18 * sqrt(fabs(gpp * gqq))) {
          const double theta = (gqq - gpp) / (2.0 * gpq);
          const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        rc[t] = c; rs[t] = s; pp[t] = p; pq[t] = q;
      }
      __syncthreads();
      // all LDS loads of this thread's items first, then the stores (items are
      // disjoint within a round, so nothing here reads what another item writes)
      int gi[GI][4];
      double gv[GI][4], gc1[GI], gs1[GI], gc2[GI], gs2[GI];
      bool gdiag[GI];
#pragma unroll
      for (int u = 0; u < GI; ++u) {
        const int P1 = gP1[u] < 0 ? 0 : gP1[u], P2 = gP2[u] < 0 ? 0 : gP2[u];
        const int p1 = pp[P1], q1 = pq[P1], p2 = pp[P2], q2 = pq[P2];
        gc1[u] = rc[P1]; gs1[u] = rs[P1]; gc2[u] = rc[P2]; gs2[u] = rs[P2];
        gdiag[u] = (P1 == P2);
        if (gdiag[u]) {
          gi[u][0] = pk(p1, p1, n); gi[u][1] = pk(q1, q1, n); gi[u][2] = pk(p1, q1, n); gi[u][3] = gi[u][2];
        } else {
          gi[u][0] = pk(min(p1, p2), max(p1, p2), n); gi[u][1] = pk(min(p1, q2), max(p1, q2), n);
          gi[u][2] = pk(min(q1, p2), max(q1, p2), n); gi[u][3] = pk(min(q1, q2), max(q1, q2), n);
        }
      }
#pragma unroll
      for (int u = 0; u < GI; ++u)
#pragma unroll
        for (int x = 0; x < 4; ++x) gv[u][x] = (gP1[u] >= 0) ? Gp[gi[u][x]] : 0.0;
      int vpi[VI], vqi[VI];
      double vcs[VI], vsn[VI], vpv[VI], vqv[VI];
#pragma unroll
      for (int u = 0; u < VI; ++u) {
        const int P = vP[u];
        const int a = va[u] < 0 ? 0 : va[u];
        vpi[u] = a * n + pp[P];
        vqi[u] = a * n + pq[P];
        vcs[u] = rc[P];
        vsn[u] = rs[P];
      }
#pragma unroll
      for (int u = 0; u < VI; ++u) {
        vpv[u] = (va[u] >= 0) ? V[vpi[u]] : 0.0;
        vqv[u] = (va[u] >= 0) ? V[vqi[u]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < GI; ++u) {
        if (gP1[u] < 0) continue;
        const double c1 = gc1[u], s1 = gs1[u], c2 = gc2[u], s2 = gs2[u];
        if (gdiag[u]) {
          const double gpp = gv[u][0], gqq = gv[u][1], gpq = gv[u][2];
          Gp[gi[u][0]] = c1 * c1 * gpp - 2.0 * c1 * s1 * gpq + s1 * s1 * gqq;
          Gp[gi[u][1]] = s1 * s1 * gpp + 2.0 * c1 * s1 * gpq + c1 * c1 * gqq;
          Gp[gi[u][2]] = 0.0;
        } else {
          const double bpp = gv[u][0], bpq = gv[u][1], bqp = gv[u][2], bqq = gv[u][3];
          const double rpp = c1 * bpp - s1 * bqp, rpq = c1 * bpq - s1 * bqq;   // rows: J^T
          const double rqp = s1 * bpp + c1 * bqp, rqq = s1 * bpq + c1 * bqq;
          Gp[gi[u][0]] = c2 * rpp - s2 * rpq;                                   // columns: J
          Gp[gi[u][1]] = s2 * rpp + c2 * rpq;
          Gp[gi[u][2]] = c2 * rqp - s2 * rqq;
          Gp[gi[u][3]] = s2 * rqp + c2 * rqq;
        }
      }
#pragma unroll
      for (int u = 0; u < VI; ++u) {
        if (va[u] < 0) continue;
        V[vpi[u]] = vcs[u] * vpv[u] - vsn[u] * vqv[u];
        V[vqi[u]] = vsn[u] * vpv[u] + vcs[u] * vqv[u];
      }
      __syncthreads();
    }
  }
  // eigenvalues in descending order (ties by index) over the ell real indices
  for (int a = t; a < ell; a += JNT) {
    const double da = Gp[pk(a, a, n)];
    int rnk = 0;
    for (int b = 0; b < ell; ++b) {
      const double db = Gp[pk(b, b, n)];
      if (db > da || (db == da && b < a)) ++rnk;
    }
    rank_of[a] = rnk;
  }
  __syncthreads();
  for (int a = t; a < ell; a += JNT) lam[rank_of[a]] = Gp[pk(a, a, n)];
  for (int e = t; e < ell * ell; e += JNT) {
    const int i = e / ell, a = e - (e / ell) * ell;
    Vout[i * ell + rank_of[a]] = V[i * n + a];
  }
}

// One-sided Jacobi SVD of a square ell x ell matrix Rm (row-major).
// W = Rm V with orthogonal columns; sig_j = ||w_j||.  Outputs (descending):
// sig, Vr (columns = right vectors), Ur (columns = w_j / sig_j, 0 where sig_j = 0).
__global__ void __launch_bounds__(1024) k_jacobi_svd(const double *__restrict__ Rm, int ell,
                                                     double *__restrict__ sig, double *__restrict__ Vr,
                                                     double *__restrict__ Ur, int *__restrict__ dflags) {
  extern __shared__ double dyn[];
  const int n = (ell + 1) & ~1;
  double *W = dyn;               // column-major: W[col*ell + row]
  double *V = dyn + n * ell;     // column-major n x n
  __shared__ int rank_of[JELL_MAX + 2];
  __shared__ double nrm[JELL_MAX + 2];
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

}  // namespace

// tol2_rel: stop when the off-diagonal Frobenius mass^2 <= tol2_rel * ||G||_F^2.
int launch_jacobi_eig_parts(hipStream_t st, const double *part, int nparts, int ell, double *lam, double *V,
                            int *dflags, double tol2_rel) {
  if (ell < 1 || ell > JELL_MAX) return -1;
  const int n = (ell + 1) & ~1;
  const size_t lds = ((size_t)n * (n + 1) / 2 + (size_t)n * n) * sizeof(double);
  if (n <= 64) {
    allow_lds(k_jacobi_eig<64>, lds);
    hipLaunchKernelGGL(k_jacobi_eig<64>, dim3(1), dim3(JNT), lds, st, part, nparts, ell, tol2_rel, lam, V, dflags);
  } else {
    allow_lds(k_jacobi_eig<JELL_MAX>, lds);
    hipLaunchKernelGGL(k_jacobi_eig<JELL_MAX>, dim3(1), dim3(JNT), lds, st, part, nparts, ell, tol2_rel, lam, V,
                       dflags);
  }
  DSK_TRY(hipGetLastError());
  return 0;
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

// Small dense eigen / SVD cores of SVD(B), B = Q^T A (Alg. 2, "SVD(B)" step):
//
//  * k_core_eig (F32 / BF16 / F16 paths): eigenpairs of the ell x ell FP64
//    Gram G_B = B B^T.  G_B + delta I (delta a few hundred ulps of tr G_B,
//    which moves no eigenvector and is subtracted from every eigenvalue at the
//    end) is factored by Cholesky, G_B + delta I = P L L^T P^T; one-sided
//    (Hestenes) Jacobi then orthogonalises the columns of L, L V = W, so the
//    left singular vectors of L -- the eigenvectors of G_B -- are the
//    normalised columns of W and no rotation is accumulated.  ell <= 64: one
//    wave factors (blocked, P = I); wider: the workgroup factors in LDS
//    with diagonal pivoting (the QR-with-column-pivoting preconditioner of
//    one-sided Jacobi, Drmac and Veselic 2008).  Pair sums use DPP
//    reductions, rotation angles refined hardware reciprocals.  The rounds
//    are bound by instruction issue, so ell <= 64 runs 4 waves (one per SIMD)
//    with 8 lanes per pair, and columns are padded in LDS so that every lane
//    loads and stores without a bounds branch.
//  * k_jacobi_svd (FP64 path): one-sided Jacobi on an ell x ell triangular
//    factor R (B^T = Q_B R): no squaring of the singular values.
// Both use round-robin (circle) ordering: n/2 disjoint pairs per round, n - 1
// rounds per sweep.
#include <algorithm>

#include "dsk_internal.h"
#include "wavechol.h"

namespace {

constexpr int JNT = 1024;
constexpr int JELL_MAX = 112;
constexpr double U64 = 1.1102230246251565e-16;

// position -> player of round r in the circle method (p in [0, n))
__device__ __forceinline__ int rr_player(int pos, int r, int n) {
  if (pos == 0) return 0;
  int x = pos - 1 + r;
  if (x >= n - 1) x -= n - 1;
  return x + 1;
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

// Sum over each aligned group of G lanes (G = 8 or 16); every lane of the group
// gets the group's sum.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G == 16) {
    return wc::row16_sum(v);
  } else {
    static_assert(G == 8, "8 or 16 lanes per pair");
    v += wc::dpp_f64<0xB1>(v);    // quad xor 1
    v += wc::dpp_f64<0x4E>(v);    // quad xor 2
    v += wc::dpp_f64<0x141>(v);   // half-row mirror: lane i + lane 7 - i
    return v;
  }
}

// Rotation (c, s) that makes columns p, q orthogonal, given alpha = |w_p|^2,
// beta = |w_q|^2, gamma = w_p . w_q (Rutishauser's formulas), with refined
// hardware reciprocals: c^2 + s^2 = 1 to working precision for any t.
__device__ __forceinline__ void jrot(double al, double be, double ga, double &c, double &s) {
  const double zeta = (be - al) * wc::rcp_nr(2.0 * ga);
  double tt;
  if (fabs(zeta) > 1e150) {
    tt = 0.5 * wc::rcp_nr(zeta);
  } else {
    const double w = fma(zeta, zeta, 1.0);
    tt = (zeta >= 0.0 ? 1.0 : -1.0) * wc::rcp_nr(fabs(zeta) + w * wc::rsq_nr(w));
  }
  c = wc::rsq_nr(fma(tt, tt, 1.0));
  s = tt * c;
}

// ell > 64: Cholesky with diagonal pivoting of G + delta I by the whole
// workgroup (G in LDS, row stride ldg; right-looking, row j of the trailing
// matrix read unscaled so that the column scaling and the update share a
// phase), then X = L column-major in place (X(r, c) at c * ldg + r; columns from
// a non-positive pivot on are zero).  perm receives the pivot order.
template <int NT>
__device__ void pivoted_chol_lds(double *G, int ell, int ldg, double delta, int *perm, int *pivsh, double *pivd) {
  const int t = threadIdx.x;
  for (int i = t; i < ell; i += NT) G[i * ldg + i] += delta;
  __syncthreads();

  int jstop = ell;
  for (int j = 0; j < ell; ++j) {
    if (t < 64) {
      double bv = -1.0;
      int bi = ell;
      for (int i = j + t; i < ell; i += 64) {
        const double v = G[i * ldg + i];
        if (v > bv) { bv = v; bi = i; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if (t == 0) { *pivsh = bi; *pivd = bv; }
    }
    __syncthreads();
    const int p = *pivsh;
    const double d = *pivd;
    if (!(d > 0.0) || !isfinite(d)) { jstop = j; break; }
    if (p != j) {
      for (int e = t; e < ell; e += NT) {
        if (e != j && e != p) {
          double a = G[j * ldg + e]; G[j * ldg + e] = G[p * ldg + e]; G[p * ldg + e] = a;
          a = G[e * ldg + j]; G[e * ldg + j] = G[e * ldg + p]; G[e * ldg + p] = a;
        }
      }
      if (t == 0) {
        const double a = G[j * ldg + j]; G[j * ldg + j] = G[p * ldg + p]; G[p * ldg + p] = a;
        const int pi = perm[j]; perm[j] = perm[p]; perm[p] = pi;
      }
      __syncthreads();
    }
    const double piv = sqrt(d), dinv = 1.0 / d, pinv = 1.0 / piv;
    for (int i = j + 1 + (t >> 5); i < ell; i += 32) {
      const double gji = G[j * ldg + i] * dinv;
      for (int c = j + 1 + (t & 31); c < ell; c += 32) G[i * ldg + c] = fma(-gji, G[j * ldg + c], G[i * ldg + c]);
    }
    for (int i = j + 1 + t; i < ell; i += NT) G[i * ldg + j] = G[j * ldg + i] * pinv;
    if (t == 0) G[j * ldg + j] = piv;
    __syncthreads();
  }
  // ---- X = L, column-major in place: X(r, c) at c * ldg + r; columns from the
  // stopping pivot on are zero
  for (int e = t; e < ell * ell; e += NT) {
    const int r = e / ell, c = e - (e / ell) * ell;
    if (r > c) {
      const double v = (c < jstop) ? G[r * ldg + c] : 0.0;
      G[c * ldg + r] = v;
      G[r * ldg + c] = 0.0;
    } else if (r == c && c >= jstop) {
      G[r * ldg + c] = 0.0;
    }
  }
  __syncthreads();
}

// G_in: ell x ell row-major FP64 Gram.  Outputs, descending: lam (ell eigenvalues,
// clipped at 0) and Uout (ell x ell row-major, column j = eigenvector j; zero
// where the factor has no column).  dflags[FLAGW_SWEEPS] = sweeps used.
// NT = 256: ell <= 64 (register Cholesky, 8 lanes x 8 entries per pair);
// NT = 1024: ell <= 112 (pivoted LDS Cholesky, 16 lanes x 7 entries per pair).
template <int NT>
constexpr int eig_ldg() { return NT == 256 ? 65 : 113; }   // LDS column stride >= lanes x entries per pair

template <int NT>
__global__ void __launch_bounds__(NT) k_core_eig(const double *__restrict__ G_in, int ell,
                                                  double *__restrict__ lam, double *__restrict__ Uout,
                                                  int *__restrict__ dflags, const int *__restrict__ gate) {
  if (gate && *gate == 0) return;   // gated: runs only where the tridiagonal eigensolver failed
  // a batch: workgroup b factors matrix b (G_in, lam, Uout advance by ell^2, ell, ell^2)
  G_in += (size_t)blockIdx.x * ell * ell;
  lam += (size_t)blockIdx.x * ell;
  Uout += (size_t)blockIdx.x * ell * ell;
  extern __shared__ double dyn[];
  constexpr int LPP = NT == 256 ? 8 : 16;     // lanes per pair
  constexpr int EPL = NT == 256 ? 8 : 7;      // entries per lane
  const int ldg = eig_ldg<NT>();              // odd stride, >= LPP * EPL: padded rows stay zero
  const int n = (ell + 1) & ~1;      // even size; an odd ell gets one zero column
  const int np = n / 2;
  double *G = dyn;                   // ell x ldg, later X column-major (n columns)
  __shared__ int perm[JELL_MAX + 2];
  __shared__ int rank_of[JELL_MAX + 2];
  __shared__ double nrm2[JELL_MAX + 2];
  __shared__ double red[JNT / 64 + 1];
  __shared__ int pivsh;
  __shared__ double pivd;
  __shared__ int rotated;
  __shared__ int bigrot;
  __shared__ int okw;
  const int t = threadIdx.x;
  const int grows = NT == 256 ? 64 : n;   // the 64-row blocked Cholesky reads padded rows
  for (int e = t; e < grows * ldg; e += NT) G[e] = 0.0;
  __syncthreads();
  for (int e = t; e < ell * ell; e += NT) {
    const int i = e / ell, c = e - (e / ell) * ell;
    G[i * ldg + c] = G_in[e];
  }
  for (int i = t; i < n; i += NT) perm[i] = i;
  __syncthreads();
  double tr = 0.0;
  for (int i = t; i < ell; i += NT) tr += G[i * ldg + i];
  tr = jblock_sum<NT>(tr, red);
  if (!isfinite(tr) && t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
  const double delta = 16.0 * (ell + 1024) * U64 * fabs(tr);
  if constexpr (NT == 256) {
    // ell <= 64, one wave: register Cholesky of G + delta I, then X = L column-major over G
    double *Lb = dyn + 64 * ldg;
    double *dinv = Lb + 64 * wc::LDL;
    for (int i = t; i < ell; i += NT) G[i * ldg + i] += delta;
    __syncthreads();
    if (t < 64) {
      const bool ok = wc::chol64_blocked(G, ell, 0.0, Lb, dinv, dinv + 64);
      if (t == 0) okw = ok ? 1 : 0;
    }
    __syncthreads();
    if (!okw && t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
  } else {
    pivoted_chol_lds<NT>(G, ell, ldg, delta, perm, &pivsh, &pivd);
  }
  const double tolj = 4.0 * ell * U64;
  const double tol2 = tolj * tolj;   // rotate when gamma^2 > tol^2 alpha beta
  int sweeps = 0;
  double *X = G;                     // columns of the factor, stride ldx
  int ldx = ldg;
  if constexpr (NT == 256) {
    // ell <= 64: X = L column-major in a 16-byte aligned static array with
    // contiguous 64-entry columns; each pair's 8 lanes move a column with four
    // 16-byte accesses, which cover every LDS bank once (no conflicts between
    // the pairs of a wave, whichever columns they hold)
    __shared__ __align__(16) double Xc[64 * 64];
    {
      const double *Lb = dyn + 64 * ldg;
      for (int e = t; e < 64 * 64; e += NT) {
        const int c = e >> 6, r = e & 63;
        Xc[e] = (okw && c < ell && r < ell && r >= c) ? Lb[r * wc::LDL + c] : 0.0;
      }
    }
    __syncthreads();
    const int pr = t >> 3, pl = t & 7;
    // Convergence is quadratic: once a sweep's rotations all have |cos| <= 1e-7
    // (gamma^2 <= 1e-14 alpha beta), the next sweep would leave every pair below
    // about 1e-14 and change nothing the outputs resolve, so it is not run.
    const double big2 = 1e-14;
    for (int sweep = 0; sweep < 40; ++sweep) {
      if (t == 0) { rotated = 0; bigrot = 0; }
      __syncthreads();
      for (int r = 0; r < n - 1; ++r) {
        if (pr < np) {
          int p = rr_player(pr, r, n), q = rr_player(n - 1 - pr, r, n);
          if (p > q) { const int x = p; p = q; q = x; }
          double2 *xp = reinterpret_cast<double2 *>(Xc + p * 64) + pl;   // entries 2 pl + 16 u, +1
          double2 *xq = reinterpret_cast<double2 *>(Xc + q * 64) + pl;
          double2 wp[4], wq[4];
          double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            wp[u] = xp[8 * u];
            wq[u] = xq[8 * u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            al = fma(wp[u].x, wp[u].x, al);
            be = fma(wq[u].x, wq[u].x, be);
            ga = fma(wp[u].x, wq[u].x, ga);
            al = fma(wp[u].y, wp[u].y, al);
            be = fma(wq[u].y, wq[u].y, be);
            ga = fma(wp[u].y, wq[u].y, ga);
          }
          al = group_sum<8>(al);
          be = group_sum<8>(be);
          ga = group_sum<8>(ga);
          if (ga != 0.0 && ga * ga > tol2 * (al * be)) {
            double c, s;
            jrot(al, be, ga, c, s);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              xp[8 * u] = make_double2(c * wp[u].x - s * wq[u].x, c * wp[u].y - s * wq[u].y);
              xq[8 * u] = make_double2(s * wp[u].x + c * wq[u].x, s * wp[u].y + c * wq[u].y);
            }
            if (pl == 0) {
              rotated = 1;
              if (ga * ga > big2 * (al * be)) bigrot = 1;
            }
          }
        }
        __syncthreads();
      }
      sweeps = sweep + 1;
      const bool stop = !rotated || !bigrot;
      __syncthreads();   // every thread has read the flags before thread 0 clears them
      if (stop) break;
    }
    X = Xc;
    ldx = 64;
  } else {
  // ---- one-sided Jacobi on the columns of X (entries past ell are zero and stay zero)
  const int pr = t / LPP, pl = t % LPP;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < n - 1; ++r) {
      if (pr < np) {
        int p = rr_player(pr, r, n), q = rr_player(n - 1 - pr, r, n);
        if (p > q) { const int x = p; p = q; q = x; }
        double *xp = G + p * ldg + pl, *xq = G + q * ldg + pl;
        double wp[EPL], wq[EPL];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int u = 0; u < EPL; ++u) {
          wp[u] = xp[LPP * u];
          wq[u] = xq[LPP * u];
        }
#pragma unroll
        for (int u = 0; u < EPL; ++u) {
          al = fma(wp[u], wp[u], al);
          be = fma(wq[u], wq[u], be);
          ga = fma(wp[u], wq[u], ga);
        }
        al = group_sum<LPP>(al);
        be = group_sum<LPP>(be);
        ga = group_sum<LPP>(ga);
        if (ga != 0.0 && ga * ga > tol2 * (al * be)) {
          double c, s;
          jrot(al, be, ga, c, s);
#pragma unroll
          for (int u = 0; u < EPL; ++u) {
            xp[LPP * u] = c * wp[u] - s * wq[u];
            xq[LPP * u] = s * wp[u] + c * wq[u];
          }
          if (pl == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    sweeps = sweep + 1;
    const bool stop = !rotated;
    __syncthreads();   // every thread has read the flag before thread 0 clears it
    if (stop) break;
  }
  }
  const int grp = t >> 4, gl = t & 15;
  // ---- eigenvalues lambda_c = |x_c|^2 - delta, eigenvectors x_c / |x_c|
  for (int c = grp; c < ell; c += NT / 16) {
    double s2 = 0.0;
    for (int i = gl; i < ell; i += 16) s2 = fma(X[c * ldx + i], X[c * ldx + i], s2);
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 16);
    if (gl == 0) nrm2[c] = s2;
  }
  __syncthreads();
  for (int a = t; a < ell; a += NT) {
    const double la = nrm2[a];
    int rnk = 0;
    for (int b = 0; b < ell; ++b) {
      const double lb = nrm2[b];
      if (lb > la || (lb == la && b < a)) ++rnk;
    }
    rank_of[a] = rnk;
    lam[rnk] = fmax(la - delta, 0.0);
    if (!isfinite(la)) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_NONFINITE);
  }
  if (t == 0) dflags[FLAGW_SWEEPS] = sweeps;
  __syncthreads();
  for (int e = t; e < ell * ell; e += NT) {
    const int c = e / ell, r = e - (e / ell) * ell;   // column c of X, row r (pivot order)
    const double nc = nrm2[c];
    Uout[perm[r] * ell + rank_of[c]] = nc > 0.0 ? X[c * ldx + r] / sqrt(nc) : 0.0;
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
    if (t == 0) dflags[FLAGW_SWEEPS] = sweep + 1;
    const bool stop = !rotated;
    __syncthreads();   // every thread has read the flag before thread 0 clears it
    if (stop) break;
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

int launch_core_eig_gated(hipStream_t st, const double *G, int ell, double *lam, double *U, int *dflags,
                          const int *gate, int count) {
  if (ell < 1 || ell > JELL_MAX || count < 1) return -1;
  const int n = (ell + 1) & ~1;
  if (ell <= 64) {
    const size_t lds = ((size_t)64 * eig_ldg<256>() + 64 * wc::LDL + 128) * sizeof(double);
    allow_lds(k_core_eig<256>, lds);
    hipLaunchKernelGGL(k_core_eig<256>, dim3(count), dim3(256), lds, st, G, ell, lam, U, dflags, gate);
  } else {
    const size_t lds = (size_t)std::max(n, ell) * eig_ldg<JNT>() * sizeof(double);
    allow_lds(k_core_eig<JNT>, lds);
    hipLaunchKernelGGL(k_core_eig<JNT>, dim3(count), dim3(JNT), lds, st, G, ell, lam, U, dflags, gate);
  }
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_core_eig_batched(hipStream_t st, const double *G, int ell, double *lam, double *U, int *dflags,
                            int count) {
  return launch_core_eig_gated(st, G, ell, lam, U, dflags, nullptr, count);
}

int launch_core_eig(hipStream_t st, const double *G, int ell, double *lam, double *U, int *dflags) {
  return launch_core_eig_gated(st, G, ell, lam, U, dflags, nullptr, 1);
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

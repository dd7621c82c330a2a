// Single-pass coarse-grid SVD (SPC-SVD, Alg. 3): the small factor that turns
// the one-pass product H = A^T Y into B^T = A^T Q for FP64 input.
//
// With Y = Q R (R upper triangular, Q orthonormal), A^T Q = H R^{-1} (the
// identity derived under Alg. 3), so the pass over A needs only Y, not Q, and
// can run while Y is being orthonormalised.  This kernel forms M = R^{-1} in
// FP64 from the Householder R of Y.  (The FP32 / 16-bit paths apply the
// CholeskyQR factor of Y to H by the blocked substitution instead.)
// Y numerically rank deficient at the precision of its data (some
// |R_jj| <= ell u_data ||Y||_F), where the single-pass formula breaks down,
// raises DSK_FLAG_RANK_DEFICIENT; a zero or non-finite diagonal entry of R
// gives a zero row of M, so the outputs stay finite.
#include "dsk_internal.h"

namespace {

constexpr int NT = 256;

// One workgroup.  LDS: one (ell + 1) x (ell + 1) array holding R in its upper
// triangle (rows 0..ell-1) and M = R^{-1} transposed strictly below the
// diagonal: M(r, c), r <= c, at row c + 1, column r.
__global__ void __launch_bounds__(NT) k_spc_rinv(const double *__restrict__ G, int ell, double u_data,
                                                 double *__restrict__ M, int *__restrict__ dflags) {
  extern __shared__ double sm[];
  const int ld = ell + 1;
  double *Rs = sm;
  auto X = [&](int r, int c) -> double & { return sm[(c + 1) * ld + r]; };
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int e = t; e < ell * ell; e += NT) {
    const int i = e / ell, c = e - (e / ell) * ell;
    Rs[i * ld + c] = G[e];
  }
  __syncthreads();
  // numerical rank at the data precision: ||Y||_F = ||R||_F
  if (t == 0) {
    double f2 = 0.0;
    for (int i = 0; i < ell; ++i)
      for (int c = i; c < ell; ++c) f2 = fma(Rs[i * ld + c], Rs[i * ld + c], f2);
    const double lim = ell * u_data * sqrt(f2);
    for (int j = 0; j < ell; ++j)
      if (!(fabs(Rs[j * ld + j]) > lim)) bad = 1;
  }
  // M = R^{-1}: thread c solves R x = e_c by back substitution (x(r) = 0 for r > c)
  if (t < ell) {
    const int c = t;
    for (int r = c; r >= 0; --r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int l = r + 1; l <= c; ++l) s = fma(-Rs[r * ld + l], X(l, c), s);
      const double d = Rs[r * ld + r];
      X(r, c) = (d != 0.0 && isfinite(d)) ? s / d : 0.0;
    }
  }
  __syncthreads();
  for (int e = t; e < ell * ell; e += NT) {
    const int i = e / ell, c = e - (e / ell) * ell;
    M[e] = i <= c ? X(i, c) : 0.0;
  }
  if (t == 0 && bad) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_RANK_DEFICIENT);
}

}  // namespace

int launch_spc_rinv(hipStream_t st, const double *G, int ell, double u_data, double *M, int *dflags) {
  if (ell < 1 || ell > 112) return -1;
  const size_t lds = (size_t)(ell + 1) * (ell + 1) * sizeof(double);
  allow_lds(k_spc_rinv, lds);
  hipLaunchKernelGGL(k_spc_rinv, dim3(1), dim3(NT), lds, st, G, ell, u_data, M, dflags);
  DSK_TRY(hipGetLastError());
  return 0;
}

// Refinement sweep of the 16-bit / FP32 SVD path (precision extension; not in
// the paper).  The assembled factors U (m x k) and V (n x k) are FP32 values:
// V = B^T U_B S^-1 divides by sigma_j, so its orthogonality loss grows like
// u_32 sigma_1 / sigma_k, and both lose orthogonality through rounding.  The
// sweep restores it in FP64 without changing the product U S V^T:
//
//   G_U = U^T U = R_U^T R_U,  G_V = V^T V = R_V^T R_V     (FP64 Grams, Cholesky)
//   M = R_U diag(S) R_V^T = U_m S' V_m^T                  (k x k SVD, one-sided Jacobi)
//   U' = U R_U^-1 U_m,  V' = V R_V^-1 V_m,  S' = singular values of M
//
// so U S V^T = U' S' V'^T with U', V' orthonormal to the rounding of their
// FP32 storage.  k <= 100; the two Cholesky factorisations and inverses run
// in LDS, one workgroup each, the k x k products in global memory.
#include <algorithm>

#include "dsk_internal.h"

namespace {

constexpr int RNT = 256;

// blockIdx.x = b: G_b (k x k, row-major) -> R_b (upper, G = R^T R) in place, then
// T_b = R_b^-1 (upper).  A non-positive pivot sets the rank flag and the pivot to 1.
// The matrix is factored in LDS (row stride k + 1), right-looking, one pivot
// per step; T by one thread per column, reading R from LDS.
constexpr int CK = 100;   // largest k
__global__ void __launch_bounds__(RNT) k_chol_inv2(double *__restrict__ G, int k, double *__restrict__ T,
                                                   int *__restrict__ dflags) {
  __shared__ double Rs[(CK + 1) * (CK + 1)];   // rows 0 .. k (row k: the last column of T)
  __shared__ double pinv_sh;
  const int ld = k + 1;
  double *R = G + (size_t)blockIdx.x * k * k;
  double *Ti = T + (size_t)blockIdx.x * k * k;
  const int t = threadIdx.x;
  for (int e = t; e < k * k; e += RNT) Rs[(e / k) * ld + e % k] = R[e];
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      double d = Rs[j * ld + j];
      if (!(d > 0.0) || !isfinite(d)) {
        atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_RANK_DEFICIENT);
        d = 1.0;
      }
      const double p = sqrt(d);
      Rs[j * ld + j] = p;
      pinv_sh = 1.0 / p;
    }
    __syncthreads();
    const double pinv = pinv_sh;
    const int rem = k - j - 1;
    // row j right of the pivot scaled; the trailing upper triangle updated from
    // the scaled row (each thread scales the two entries it reads itself)
    for (int e = t; e < rem * rem; e += RNT) {
      const int i = j + 1 + e / rem, c = j + 1 + e % rem;
      if (c >= i) Rs[i * ld + c] = fma(-(Rs[j * ld + i] * pinv), Rs[j * ld + c] * pinv, Rs[i * ld + c]);
    }
    __syncthreads();
    for (int c = j + 1 + t; c < k; c += RNT) Rs[j * ld + c] *= pinv;
    __syncthreads();
  }
  for (int e = t; e < k * k; e += RNT) {
    const int i = e / k, c = e % k;
    R[e] = i > c ? 0.0 : Rs[i * ld + c];
  }
  // T = R^-1: column c by back substitution (one thread per column), the column
  // kept in the (no longer needed) strictly lower part of Rs: T(i, c) at Rs[(c + 1) * ld + i]
  for (int c = t; c < k; c += RNT) {
    double *x = Rs + (size_t)(c + 1) * ld;   // row c + 1 of Rs, entries 0 .. c (below the diagonal of row c + 1)
    x[c] = 1.0 / Rs[c * ld + c];
    for (int i = c - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= c; ++l) s = fma(Rs[i * ld + l], x[l], s);
      x[i] = -s / Rs[i * ld + i];
    }
    for (int i = 0; i < k; ++i) Ti[i * k + c] = i <= c ? x[i] : 0.0;
  }
}

// M = R_U diag(S) R_V^T (k x k), R upper triangular.
__global__ void __launch_bounds__(RNT) k_refine_mid(const double *__restrict__ RU, const double *__restrict__ RV,
                                                    const double *__restrict__ S, int k, double *__restrict__ M) {
  for (int e = blockIdx.x * RNT + threadIdx.x; e < k * k; e += gridDim.x * RNT) {
    const int i = e / k, j = e % k;
    double s = 0.0;
    for (int l = std::max(i, j); l < k; ++l) s = fma(RU[i * k + l] * S[l], RV[j * k + l], s);
    M[e] = s;
  }
}

// F_U = T_U U_m, F_V = T_V V_m (k x k, T upper); S = sigma of M.
__global__ void __launch_bounds__(RNT) k_refine_post(const double *__restrict__ TU, const double *__restrict__ TV,
                                                     const double *__restrict__ Um, const double *__restrict__ Vm,
                                                     const double *__restrict__ sig, int k, double *__restrict__ FU,
                                                     double *__restrict__ FV, double *__restrict__ S) {
  for (int e = blockIdx.x * RNT + threadIdx.x; e < 2 * k * k; e += gridDim.x * RNT) {
    const int w = e / (k * k), f = e % (k * k);
    const int i = f / k, j = f % k;
    const double *T = w ? TV : TU;
    const double *X = w ? Vm : Um;
    double s = 0.0;
    for (int l = i; l < k; ++l) s = fma(T[i * k + l], X[l * k + j], s);
    (w ? FV : FU)[f] = s;
  }
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < k; j += RNT) S[j] = sig[j];
}

// out (k x k, FP32) = F diag(sign)
__global__ void __launch_bounds__(RNT) k_scale_cols_f32(const double *__restrict__ F, int k,
                                                        const double *__restrict__ sign, float *__restrict__ out) {
  const int e = blockIdx.x * RNT + threadIdx.x;
  if (e < k * k) out[e] = (float)(F[e] * sign[e % k]);
}

}  // namespace

size_t refine_ws_bytes(int k) { return (size_t)13 * k * k * sizeof(double) + 4 * 256 + (size_t)k * 8 + 4096; }

int launch_refine(hipStream_t st, const float *U0, int64_t m, const float *V0, int64_t n, int k, double *S,
                  float *U, float *V, double *part, int nparts, double *ws, int *dflags, int mode, void *sws,
                  int cu_count) {
  if (k < 1 || k > 100) return -1;
  const size_t k2 = (size_t)k * k;
  double *G = ws;              // G_U, G_V -> R_U, R_V
  double *T = G + 2 * k2;      // T_U, T_V
  double *M = T + 2 * k2;
  double *Um = M + k2;         // left singular vectors of M (Jacobi "Ur")
  double *Vm = Um + k2;        // right singular vectors of M (accumulated rotations)
  double *F = Vm + k2;         // F_U, F_V
  double *sig = F + 2 * k2;
  double *sign = sig + k;
  float *Fv32 = reinterpret_cast<float *>(sign + k);   // F_V diag(sign) in FP32 (k x k)
  DSK_RET(launch_gram(st, U0, 0, m, k, G, part, nparts));
  DSK_RET(launch_gram(st, V0, 0, n, k, G + k2, part, nparts));
  hipLaunchKernelGGL(k_chol_inv2, dim3(2), dim3(RNT), 0, st, G, k, T, dflags);
  const unsigned gb = (unsigned)std::min<size_t>((2 * k2 + RNT - 1) / RNT, 64);
  hipLaunchKernelGGL(k_refine_mid, dim3(gb), dim3(RNT), 0, st, G, G + k2, S, k, M);
  DSK_TRY(hipGetLastError());
  DSK_RET(launch_jacobi_svd(st, M, k, sig, Vm, Um, dflags));
  hipLaunchKernelGGL(k_refine_post, dim3(gb), dim3(RNT), 0, st, T, T + k2, Um, Vm, sig, k, F, F + k2, S);
  DSK_TRY(hipGetLastError());
  DSK_RET(launch_tsmm(st, U0, 0, m, k, k, F, k, k, nullptr, U, k));
  DSK_RET(launch_sign_fix(st, U, 0, m, k, sign));
  // V = V0 F_V diag(sign): n x k by k x k on the MFMA stream kernel (FP32 to about 2^-24)
  hipLaunchKernelGGL(k_scale_cols_f32, dim3((unsigned)((k2 + RNT - 1) / RNT)), dim3(RNT), 0, st, F + k2, k, sign,
                     Fv32);
  DSK_TRY(hipGetLastError());
  DSK_RET(launch_stream_nn(st, V0, DSK_F32, n, k, k, Fv32, k, V, k, mode, sws, cu_count));
  return 0;
}

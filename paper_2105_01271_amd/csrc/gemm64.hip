// FP64 GEMM C = alpha op(A) op(B) + beta C: the full-sketch power block of the
// row ID, W_q = (tau A_c A_c^T)^q A_c (C-PWR without re-orthonormalisation,
// Alg. 7 applied to the coarse sketch itself), and the coarse-sketch products
// of the learned restriction's loss gradient.  64x64 output tiles, 16-deep K
// tiles in LDS, 4x4 register blocking, f64 FMA on the vector units.
#include "dsk_internal.h"

namespace {

template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm64(int64_t M, int64_t N, int64_t K, double alpha,
                                                const double *__restrict__ A, int64_t lda,
                                                const double *__restrict__ B, int64_t ldb, double beta,
                                                double *__restrict__ C, int64_t ldc) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    for (int e = t; e < BM * BK; e += 256) {
      int i, kk;
      if (TA) { i = e % BM; kk = e / BM; } else { kk = e % BK; i = e / BK; }
      const int64_t gi = m0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < M && gk < K) v = TA ? A[gk * lda + gi] : A[gi * lda + gk];
      As[kk][i] = v;
    }
    for (int e = t; e < BN * BK; e += 256) {
      int j, kk;
      if (TB) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
      const int64_t gj = n0 + j, gk = k0 + kk;
      double v = 0.0;
      if (gj < N && gk < K) v = TB ? B[gj * ldb + gk] : B[gk * ldb + gj];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[kk][ty + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = Bs[kk][tx + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t i = m0 + ty + 16 * u;
    if (i >= M) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t j = n0 + tx + 16 * v;
      if (j < N) C[i * ldc + j] = alpha * acc[u][v] + (beta != 0.0 ? beta * C[i * ldc + j] : 0.0);
    }
  }
}

}  // namespace

int launch_gemm64(hipStream_t st, int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha,
                  const double *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc, double beta) {
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
  if (!transA && !transB)
    hipLaunchKernelGGL((k_gemm64<false, false>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (!transA && transB)
    hipLaunchKernelGGL((k_gemm64<false, true>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (transA && !transB)
    hipLaunchKernelGGL((k_gemm64<true, false>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else
    hipLaunchKernelGGL((k_gemm64<true, true>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  DSK_TRY(hipGetLastError());
  return 0;
}

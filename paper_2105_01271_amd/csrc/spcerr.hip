// Single-pass error estimate of SPC-ID (SPC-ID-ERR, Alg. 6) at given scales:
//   eps_hat(tau) = c lambda_max(B_f B_f^T - tau B_c B_c^T),
// B_f = the rows i of A with (i + 1) mod c == 0 (c = m / m_c), B_c = B_f D.
// The kept rows are a strided view of A (first row c - 1, row stride c lda),
// so nothing is gathered: the restriction and the row Gram read them in place.
//   * row Gram G = X X^T (r <= 112 rows, any length) in FP64: workgroups own
//     column ranges, stage 32-column tiles in LDS as FP64, and accumulate 4 x 4
//     blocks of G per thread; partials are summed in a fixed order;
//   * for every tau_i: M_i = G_f - tau_i G_c + sigma_i I with sigma_i =
//     ||G_f - tau_i G_c||_F >= |lambda_min|, a positive semidefinite matrix
//     whose largest eigenvalue is lambda_max(G_f - tau_i G_c) + sigma_i;
//   * the eigenvalues of every M_i come from the core eigensolver (one
//     workgroup per tau in one launch); eps_hat_i = c (lambda_1(M_i) - sigma_i).
#include "dsk_internal.h"

namespace {

constexpr int NT = 256;
constexpr int TW = 32;        // columns per LDS tile
constexpr int RMAX = 112;     // rows of the Gram at most

template <int DT>
__device__ __forceinline__ double ld64(const void *X, int64_t off) {
  if constexpr (DT == DSK_F64) return reinterpret_cast<const double *>(X)[off];
  if constexpr (DT == DSK_F32) return (double)reinterpret_cast<const float *>(X)[off];
  const unsigned short b = reinterpret_cast<const unsigned short *>(X)[off];
  if constexpr (DT == DSK_BF16) return (double)bf16_bits_to_f32(b);
  return (double)f16_bits_to_f32(b);
}

// Partial G over columns [c0, c1) of X (r rows, row stride ldx), written to
// part + blockIdx.x * r * r (full symmetric matrix).
template <int DT>
__global__ void __launch_bounds__(NT) k_row_gram(const void *__restrict__ X, int r, int64_t ncols, int64_t ldx,
                                                 int64_t cols_per_block, double *__restrict__ part) {
  __shared__ double Xs[RMAX][TW + 1];
  const int t = threadIdx.x;
  const int nb = (r + 3) / 4;                 // 4-row blocks
  const int npair = nb * (nb + 1) / 2;        // block pairs (I <= J); at most 28 * 29 / 2 = 406 < 2 NT
  // this thread's block pairs p = t and p = t + NT
  auto decode = [&](int p, int &I, int &J) {
    I = 0;
    int rem = p;
    while (rem >= nb - I) {
      rem -= nb - I;
      ++I;
    }
    J = I + rem;
  };
  const bool has0 = t < npair, has1 = t + NT < npair;
  int I0 = 0, J0 = 0, I1 = 0, J1 = 0;
  if (has0) decode(t, I0, J0);
  if (has1) decode(t + NT, I1, J1);
  double acc0[4][4], acc1[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc0[a][b] = 0.0;
      acc1[a][b] = 0.0;
    }
  auto tile = [&](int I, int J, double (&acc)[4][4]) {
    for (int j = 0; j < TW; ++j) {
      double xa[4], xb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        xa[a] = Xs[4 * I + a][j];
        xb[a] = Xs[4 * J + a][j];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(xa[a], xb[b], acc[a][b]);
    }
  };
  const int64_t c0 = (int64_t)blockIdx.x * cols_per_block;
  const int64_t c1 = c0 + cols_per_block < ncols ? c0 + cols_per_block : ncols;
  for (int64_t cb = c0; cb < c1; cb += TW) {
    __syncthreads();
    for (int e = t; e < RMAX * TW; e += NT) {
      const int i = e / TW, j = e - (e / TW) * TW;
      const int64_t col = cb + j;
      Xs[i][j] = (i < r && col < c1) ? ld64<DT>(X, (int64_t)i * ldx + col) : 0.0;
    }
    __syncthreads();
    if (has0) tile(I0, J0, acc0);
    if (has1) tile(I1, J1, acc1);
  }
  double *dst = part + (size_t)blockIdx.x * r * r;
  auto store = [&](int I, int J, const double (&acc)[4][4]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = 4 * I + a, j = 4 * J + b;
        if (i < r && j < r) {
          dst[(size_t)i * r + j] = acc[a][b];
          dst[(size_t)j * r + i] = acc[a][b];
        }
      }
  };
  if (has0) store(I0, J0, acc0);
  if (has1) store(I1, J1, acc1);
}

// G = sum of the nparts partials in partial order
__global__ void k_sum_partials(const double *__restrict__ part, int nparts, int n2, double *__restrict__ G) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[(size_t)p * n2 + e];
    G[e] = s;
  }
}

// block i: M_i = Gf - tau_i Gc + sigma_i I, sigma_i = ||Gf - tau_i Gc||_F
__global__ void __launch_bounds__(NT) k_eps_shift(const double *__restrict__ Gf, const double *__restrict__ Gc,
                                                  int r, const double *__restrict__ taus,
                                                  double *__restrict__ Mb, double *__restrict__ sig) {
  __shared__ double red[NT / 64];
  const int t = threadIdx.x, i = blockIdx.x;
  const double tau = taus[i];
  const int n2 = r * r;
  double s2 = 0.0;
  for (int e = t; e < n2; e += NT) {
    const double v = fma(-tau, Gc[e], Gf[e]);
    s2 = fma(v, v, s2);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
  if ((t & 63) == 0) red[t >> 6] = s2;
  __syncthreads();
  const double sigma = sqrt(((red[0] + red[1]) + red[2]) + red[3]);
  double *M = Mb + (size_t)i * n2;
  for (int e = t; e < n2; e += NT) {
    const int a = e / r, b = e - (e / r) * r;
    M[e] = fma(-tau, Gc[e], Gf[e]) + (a == b ? sigma : 0.0);
  }
  if (t == 0) sig[i] = sigma;
}

// eps_hat(tau_i) = c lambda_max(M_i); with rho, also c ||M_i||_2 = c max(lambda_max, -lambda_min)
// (the eigenvalues of M_i + sigma_i I come sorted in descending order)
__global__ void k_eps_finish(const double *__restrict__ lam, int r, const double *__restrict__ sig, int ntau,
                             double c, double *__restrict__ eps, double *__restrict__ rho) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ntau; i += gridDim.x * blockDim.x) {
    const double top = lam[(size_t)i * r] - sig[i];
    eps[i] = c * top;
    if (rho) rho[i] = c * fmax(top, sig[i] - lam[(size_t)i * r + (r - 1)]);
  }
}

template <int DT>
void row_gram_t(hipStream_t st, const void *X, int r, int64_t ncols, int64_t ldx, int64_t cpb, int nparts,
                double *part) {
  hipLaunchKernelGGL(k_row_gram<DT>, dim3(nparts), dim3(NT), 0, st, X, r, ncols, ldx, cpb, part);
}

}  // namespace

int spc_err_parts(int64_t ncols) { return (int)std::min<int64_t>(64, std::max<int64_t>(1, (ncols + 1023) / 1024)); }

int launch_row_gram(hipStream_t st, const void *X, int dtype, int r, int64_t ncols, int64_t ldx, double *part,
                    double *G) {
  if (r < 1 || r > RMAX || ncols < 1) return -1;
  const int nparts = spc_err_parts(ncols);
  const int64_t cpb = ((ncols + nparts - 1) / nparts + TW - 1) / TW * TW;
  const int nblk = (int)((ncols + cpb - 1) / cpb);
  switch (dtype) {
    case DSK_F64: row_gram_t<DSK_F64>(st, X, r, ncols, ldx, cpb, nblk, part); break;
    case DSK_F32: row_gram_t<DSK_F32>(st, X, r, ncols, ldx, cpb, nblk, part); break;
    case DSK_BF16: row_gram_t<DSK_BF16>(st, X, r, ncols, ldx, cpb, nblk, part); break;
    default: row_gram_t<DSK_F16>(st, X, r, ncols, ldx, cpb, nblk, part); break;
  }
  const int n2 = r * r;
  hipLaunchKernelGGL(k_sum_partials, dim3((n2 + 255) / 256), dim3(256), 0, st, (const double *)part, nblk, n2, G);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_eps_curve(hipStream_t st, const double *Gf, const double *Gc, int r, const double *taus, int ntau,
                     double c, double *Mb, double *sig, double *lam, double *Ub, double *eps, double *rho,
                     int *dflags) {
  if (r < 1 || r > RMAX || ntau < 1) return -1;
  hipLaunchKernelGGL(k_eps_shift, dim3(ntau), dim3(NT), 0, st, Gf, Gc, r, taus, Mb, sig);
  DSK_RET(launch_core_eig_batched(st, Mb, r, lam, Ub, dflags, ntau));
  hipLaunchKernelGGL(k_eps_finish, dim3((ntau + 255) / 256), dim3(256), 0, st, (const double *)lam, r,
                     (const double *)sig, ntau, c, eps, rho);
  DSK_TRY(hipGetLastError());
  return 0;
}

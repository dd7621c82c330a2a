// Training support of the learned linear restriction (extension; not in the
// paper).  The loss is the sketch error that Thm 3.2 bounds, measured in the
// Frobenius norm and normalised,
//
//   L = ||A - Q Q^T A||_F^2 / ||A||_F^2 = 1 - ||Q^T A||_F^2 / ||A||_F^2,
//
// with Q the ell-wide orthonormal block of the SVD path built from A_c = A D
// (start block by nested direct injection, q coarse power steps with
// re-orthonormalisation on the Gram sub-sample A_g = A(:, I) of Alg. 7, the
// direct-injection points of the conv's output grid).  L depends on Q only
// through span(Q), so every QR step X = Q R is differentiated with R held
// constant (dX = dQ R^{-T}); at the output dL/dQ = -(2 / ||A||^2) (A B^T - Q B B^T)
// with B = Q^T A.  The chain runs backwards through the power steps (A_g is
// fixed) to the start block, i.e. to dL/dA_c, and the conv backward turns it
// into weight gradients.  All coarse-sketch algebra is FP64
// (Householder QR, FP64 GEMM); the two passes over A use the projection
// kernels.  A plain Adam step updates the weights on the device.
#include <algorithm>
#include <vector>

#include "dsk_internal.h"

namespace {

constexpr int TRI_MAX = 112;

__global__ void k_fill64(double *x, int64_t count, double v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
    x[t] = v;
}

// MinvT = (R^{-1})^T for an upper-triangular ell x ell R (row-major): thread c
// solves R x = e_c by back substitution (x in LDS column c; every thread reads
// the same entry of R at a time).
__global__ void __launch_bounds__(128) k_trinv_upper_t(const double *__restrict__ R, int ell,
                                                       double *__restrict__ MinvT, int *__restrict__ dflags) {
  extern __shared__ double X[];   // ell x ell, X[r * ell + c]
  const double *Rs = R;
  const int c = threadIdx.x;
  if (c < ell) {
    bool bad = false;
    for (int r = ell - 1; r >= 0; --r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int l = r + 1; l < ell; ++l) s -= Rs[r * ell + l] * X[l * ell + c];
      const double d = Rs[r * ell + r];
      double v = 0.0;
      if (d != 0.0 && isfinite(d)) v = s / d;
      else bad = true;
      X[r * ell + c] = v;
    }
    if (bad) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_RANK_DEFICIENT);
    for (int r = 0; r < ell; ++r) MinvT[c * ell + r] = X[r * ell + c];
  }
}

// dQ = scale * (ABt - QG), scale = -2 / ||A||_F^2 read from the device
template <typename T>
__global__ void k_dq(const T *__restrict__ ABt, const double *__restrict__ QG, const double *__restrict__ nA2,
                     int64_t count, double *__restrict__ dQ) {
  const double sc = -2.0 / *nA2;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
    dQ[t] = sc * ((double)ABt[t] - QG[t]);
}

// dAc(:, j * floor(s / ell)) += dY(:, j): adjoint of the nested direct-injection start block
__global__ void k_scatter_start(double *__restrict__ dAc, const double *__restrict__ dY, int64_t m, int64_t s,
                                int ell) {
  const int64_t step = s / ell;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m * ell; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / ell;
    const int j = (int)(t - i * ell);
    dAc[i * s + j * step] += dY[t];
  }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, int64_t count, float lr, float b1, float b2, float eps, int step) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    const float gt = g[t];
    const float a = b1 * m1[t] + (1.f - b1) * gt;
    const float b = b2 * m2[t] + (1.f - b2) * gt * gt;
    m1[t] = a;
    m2[t] = b;
    p[t] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
  }
}

unsigned grid_of(int64_t count) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 4096)); }

int trinv_t(hipStream_t st, const double *R, int ell, double *MinvT, int *dflags) {
  const size_t lds = (size_t)ell * ell * sizeof(double);
  allow_lds(k_trinv_upper_t, lds);
  hipLaunchKernelGGL(k_trinv_upper_t, dim3(1), dim3(128), lds, st, R, ell, MinvT, dflags);
  DSK_TRY(hipGetLastError());
  return 0;
}

__global__ void k_zero_flags_l(int *f) {
  if (threadIdx.x < FLAGW_COUNT) f[threadIdx.x] = 0;
}

}  // namespace

extern "C" {

int dsk_conv_restrict_bwd(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                          const dsk_restriction *R, const float *gAc, float *gw1, float *gw2) {
  if (!h) return -1;
  if (!A) return -2;
  if (dtype < DSK_F64 || dtype > DSK_F16) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < n) return -6;
  if (!R || R->kind != DSK_R_LEARNED || !conv_shape_ok(n, R->ny, R->nx, R->channels) || !R->w1 || !R->w2) return -7;
  if (!gAc) return -8;
  if (!gw1) return -9;
  if (!gw2) return -10;
  DSK_TRY(hipSetDevice(h->device));
  DSK_RET(arena_reserve(h, conv_bwd_ws_bytes(m, R->ny, R->nx, R->channels)));
  const int64_t s = (int64_t)(R->ny / 4) * (R->nx / 4);
  return launch_conv_bwd(h->stream, A, dtype, m, lda, R->ny, R->nx, R->channels, R->w1, R->w2, gAc, 0, s, gw1, gw2,
                         h->arena);
}

int dsk_learned_loss_grad(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                          const dsk_restriction *R, int32_t ell, int32_t q, double *loss, float *gw1, float *gw2) {
  if (!h) return -1;
  if (!A) return -2;
  if (dtype < DSK_F64 || dtype > DSK_F16) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < n) return -6;
  if (!R || R->kind != DSK_R_LEARNED || !conv_shape_ok(n, R->ny, R->nx, R->channels) || !R->w1 || !R->w2) return -7;
  const int64_t s = (int64_t)(R->ny / 4) * (R->nx / 4);
  if (ell < 1 || ell > std::min<int64_t>(std::min<int64_t>(s, m), TRI_MAX)) return -8;
  if (q < 0 || q > 8) return -9;
  if (!loss) return -10;
  if (!gw1) return -11;
  if (!gw2) return -12;
  DSK_TRY(hipSetDevice(h->device));
  hipStream_t st = h->stream;
  const int L = ell;
  const int f64 = dtype == DSK_F64;
  const int wdt = f64 ? DSK_F64 : DSK_F32;
  const size_t we = f64 ? 8 : 4;
  const int nparts = (int)std::min<int64_t>(256, std::max<int64_t>(1, (n + 255) / 256));
  const int64_t rmax = std::max(m, s);
  Carve c{nullptr, 0, 0, true};
  for (int pass = 0; pass < 2; ++pass) {
    c.off = 0;
    double *Ac = c.take<double>((size_t)m * s);
    double *Ag = q > 0 ? c.take<double>((size_t)m * s) : nullptr;   // C-PWR's Gram sub-sample (fixed)
    double *dAc = c.take<double>((size_t)m * s);
    double *Y = c.take<double>((size_t)m * L);
    std::vector<double *> Qs(q + 1), Zs(q), Rq(q + 1), Rz(q);
    for (int i = 0; i <= q; ++i) {
      Qs[i] = c.take<double>((size_t)m * L);
      Rq[i] = c.take<double>((size_t)L * L);
    }
    for (int i = 0; i < q; ++i) {
      Zs[i] = c.take<double>((size_t)s * L);
      Rz[i] = c.take<double>((size_t)L * L);
    }
    double *tmp = c.take<double>((size_t)rmax * L);
    double *Wb = c.take<double>((size_t)rmax * L);
    char *Qw = c.take<char>((size_t)m * L * we);
    char *Bt = c.take<char>((size_t)n * L * we);
    char *ABt = c.take<char>((size_t)m * L * we);
    double *G = c.take<double>((size_t)L * L);
    double *part = c.take<double>((size_t)nparts * L * L);
    double *QG = c.take<double>((size_t)m * L);
    double *dQ = c.take<double>((size_t)m * L);
    double *dW = c.take<double>((size_t)rmax * L);
    double *dZ = c.take<double>((size_t)s * L);
    double *Minv = c.take<double>((size_t)L * L);
    char *sws = c.take<char>(std::max(stream_ws_bytes(dtype, m, n, L, DSK_MODE_DEFAULT),
                                      stream_ws_bytes(dtype, n, m, L, DSK_MODE_DEFAULT)));
    char *cws = c.take<char>(conv_bwd_ws_bytes(m, R->ny, R->nx, R->channels));
    double *fpart = c.take<double>(2048);
    double *scal = c.take<double>(4);
    if (pass == 0) {
      DSK_RET(arena_reserve(h, c.off));
      c.base = h->arena;
      c.cap = h->arena_bytes;
      c.dry = false;
      continue;
    }
    hipLaunchKernelGGL(k_zero_flags_l, dim3(1), dim3(64), 0, st, h->dflags);
    // forward: A_c (FP64), Q_0 = qr(Y), power steps
    DSK_RET(launch_restrict(st, A, dtype, m, n, lda, R, s, 1, Ac, nullptr, h->dflags));
    DSK_RET(launch_select_cols(st, Ac, 1, m, s, s, L, Y));
    DSK_RET(launch_convert(st, Y, 1, tmp, 1, m * L));
    DSK_RET(launch_hhqr(st, tmp, m, L, Qs[0], Rq[0], h->dflags));
    if (q > 0) DSK_RET(launch_gram_sample(st, A, dtype, m, n, lda, R, s, 1, Ag, h->dflags));
    for (int i = 0; i < q; ++i) {
      DSK_RET(launch_gemm64(st, 1, 0, s, L, m, 1.0, Ag, s, Qs[i], L, tmp, L));          // A_g^T Q
      DSK_RET(launch_hhqr(st, tmp, s, L, Zs[i], Rz[i], h->dflags));
      DSK_RET(launch_gemm64(st, 0, 0, m, L, s, 1.0, Ag, s, Zs[i], L, tmp, L));          // A_g Z
      DSK_RET(launch_hhqr(st, tmp, m, L, Qs[i + 1], Rq[i + 1], h->dflags));
    }
    // B^T = A^T Q, ||A||^2, ||B||^2, A B^T, B B^T
    DSK_RET(launch_convert(st, Qs[q], 1, Qw, f64, m * L));
    DSK_RET(launch_stream(st, A, dtype, m, n, lda, Qw, f64, L, Bt, L, DSK_MODE_DEFAULT, sws, h->cu_count));
    DSK_RET(launch_fro2(st, A, dtype, m, n, lda, fpart, 1024, scal + 0));
    DSK_RET(launch_fro2(st, Bt, wdt, n, L, L, fpart + 1024, 1024, scal + 1));
    DSK_RET(launch_stream_nn(st, A, dtype, m, n, lda, Bt, L, ABt, L, DSK_MODE_DEFAULT, sws, h->cu_count));
    DSK_RET(launch_gram(st, Bt, f64, n, L, G, part, nparts));
    DSK_RET(launch_tsmm(st, Qs[q], 1, m, L, L, G, L, L, nullptr, QG, L));
    if (f64)
      hipLaunchKernelGGL(k_dq<double>, dim3(grid_of(m * L)), dim3(256), 0, st, (const double *)ABt, QG, scal, m * L,
                         dQ);
    else
      hipLaunchKernelGGL(k_dq<float>, dim3(grid_of(m * L)), dim3(256), 0, st, (const float *)ABt, QG, scal, m * L,
                         dQ);
    hipLaunchKernelGGL(k_fill64, dim3(grid_of(m * s)), dim3(256), 0, st, dAc, m * s, 0.0);
    // backward through the power steps (R factors held constant; A_g does not
    // depend on the weights, so only the start block carries dA_c)
    for (int i = q - 1; i >= 0; --i) {
      DSK_RET(trinv_t(st, Rq[i + 1], L, Minv, h->dflags));
      DSK_RET(launch_tsmm(st, dQ, 1, m, L, L, Minv, L, L, nullptr, dW, L));             // dW = dQ Rq^{-T}
      DSK_RET(launch_gemm64(st, 1, 0, s, L, m, 1.0, Ag, s, dW, L, dZ, L));              // dZ = A_g^T dW
      DSK_RET(trinv_t(st, Rz[i], L, Minv, h->dflags));
      DSK_RET(launch_tsmm(st, dZ, 1, s, L, L, Minv, L, L, nullptr, Wb, L));             // dZ' = dZ Rz^{-T}
      DSK_RET(launch_gemm64(st, 0, 0, m, L, s, 1.0, Ag, s, Wb, L, dQ, L));              // dQ = A_g dZ'
    }
    DSK_RET(trinv_t(st, Rq[0], L, Minv, h->dflags));
    DSK_RET(launch_tsmm(st, dQ, 1, m, L, L, Minv, L, L, nullptr, dW, L));               // dY = dQ R0^{-T}
    hipLaunchKernelGGL(k_scatter_start, dim3(grid_of(m * L)), dim3(256), 0, st, dAc, dW, m, s, L);
    DSK_RET(launch_conv_bwd(st, A, dtype, m, lda, R->ny, R->nx, R->channels, R->w1, R->w2, dAc, 1, s, gw1, gw2,
                            cws));
    DSK_TRY(hipGetLastError());
    double nrm[2] = {0.0, 0.0};
    DSK_TRY(hipMemcpyAsync(nrm, scal, sizeof(nrm), hipMemcpyDeviceToHost, st));
    DSK_TRY(hipStreamSynchronize(st));
    *loss = nrm[0] > 0.0 ? 1.0 - nrm[1] / nrm[0] : 0.0;
    return 0;
  }
  return 0;
}

int dsk_adam_step(dsk_handle *h, float *param, const float *grad, float *m1, float *m2, int64_t count, float lr,
                  float beta1, float beta2, float eps, int32_t step) {
  if (!h) return -1;
  if (!param) return -2;
  if (!grad) return -3;
  if (!m1) return -4;
  if (!m2) return -5;
  if (count < 1) return -6;
  if (!(lr > 0.f)) return -7;
  if (!(beta1 >= 0.f && beta1 < 1.f)) return -8;
  if (!(beta2 >= 0.f && beta2 < 1.f)) return -9;
  if (!(eps > 0.f)) return -10;
  if (step < 1) return -11;
  DSK_TRY(hipSetDevice(h->device));
  hipLaunchKernelGGL(k_adam, dim3(grid_of(count)), dim3(256), 0, h->stream, param, grad, m1, m2, count, lr, beta1,
                     beta2, eps, step);
  DSK_TRY(hipGetLastError());
  return 0;
}

}  // extern "C"

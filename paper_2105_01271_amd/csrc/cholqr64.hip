// CholeskyQR for blocks at most 64 wide: the QR steps of Alg. 2 and Alg. 7
// (range finder, power-iteration bases).  Q = Y R^{-1} with R^T R = Y^T Y,
// FP64 Gram and factorization for FP32 or FP64 blocks; CholeskyQR2 for full
// orthonormality, one pass where only the span is needed.  On a non-positive
// or negligible pivot the factorization is retried with the shift
// 11 (rows ell + ell (ell + 1)) u tr(Y^T Y), DSK_FLAG_FALLBACK is raised and a
// third pass restores orthonormality (shifted CholeskyQR3).
//
// Every dependent step here is latency-bound, so the design minimises steps:
//  * Gram: each workgroup stages 64-row chunks of Y in LDS (FP64, zero padded
//    to 64 columns) and accumulates the 10 upper 16 x 16 tiles of Y^T Y with
//    v_mfma_f64_16x16x4f64 (FP32 products are exact in FP64).  The partials
//    are summed in workgroup order by the last workgroup to arrive.
//  * Factorization (that workgroup): one wave, no barriers: 16-column panels
//    in registers, trailing tiles on MFMA; then the inverses W_K of the four
//    diagonal 16 x 16 blocks of L (one wave each).
//  * Apply: Q = Y L^{-T} as a blocked forward substitution,
//    Q_J = (Y_J - sum_{K<J} Q_K L_JK^T) W_J^T, on MFMA; each wave owns 16 rows,
//    so no barrier is needed between the four block columns.  The rounded
//    output's Gram partials are accumulated in the same launch, and the last
//    workgroup factors them for the next pass.
// All sums run in fixed orders, so repeated runs give identical bytes.
#include <algorithm>

#include "devsync.h"
#include "dsk_internal.h"
#include "wavechol.h"

namespace {

using wc::d4;

constexpr int LDX = wc::LDL;           // LDS row stride (doubles) of 64-column blocks
constexpr int RPW = 64;                // rows per staged chunk
constexpr int NTILE = 10;              // 16 x 16 tiles of a triangle of a 64 x 64 matrix
constexpr int TILE = 256;
constexpr int PART = NTILE * TILE;     // doubles per Gram partial
constexpr int PMAX = 16;               // partials (workgroups of the Gram) at most
constexpr double U64 = 1.1102230246251565e-16;

// LDS pool (doubles): the factorization needs G, A, L (64 x LDX each), dinv,
// the four diagonal inverses and a reduction word; the apply needs Y and Q
// chunks, the factor tiles and per-wave 16 x 17 transposition buffers.
constexpr int FACT_LDS = 3 * 64 * LDX + 64 + 4 * TILE + 8 + 64;
constexpr int APPLY_LDS = 2 * RPW * LDX + PART + 4 * 16 * 17;
constexpr int POOL_LDS = FACT_LDS > APPLY_LDS ? FACT_LDS : APPLY_LDS;

using wc::mfma;

// upper tile t -> (I, J), I <= J: (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3)
__device__ __forceinline__ int tile_i(int t) { return t < 4 ? 0 : (t < 7 ? 1 : (t < 9 ? 2 : 3)); }
__device__ __forceinline__ int tile_j(int t) { return t < 4 ? t : (t < 7 ? t - 3 : (t < 9 ? t - 5 : 3)); }
// lower factor tile (J, K), K <= J -> index J (J + 1) / 2 + K
__device__ __forceinline__ int ltile(int J, int K) { return J * (J + 1) / 2 + K; }

// Rows [c0, c0 + RPW) of X (ld = ell): fetch issues all 16 loads of a thread
// at once (FP64 values, zero at rows >= rlim and columns >= ell); put writes
// them to Xs (RPW x LDX).  Split so that the next chunk's loads can be in
// flight while the current chunk is consumed.
constexpr int STG = RPW * 64 / 256;
template <typename T>
__device__ __forceinline__ void fetch_rows(const T *X, int64_t rlim, int ell, int64_t c0, double (&v)[STG]) {
#pragma unroll
  for (int u = 0; u < STG; ++u) {
    const int e = threadIdx.x + 256 * u, r = e >> 6, c = e & 63;
    const int64_t gr = c0 + r;
    v[u] = (gr < rlim && c < ell) ? (double)X[gr * ell + c] : 0.0;
  }
}
__device__ __forceinline__ void put_rows(const double (&v)[STG], double *Xs) {
#pragma unroll
  for (int u = 0; u < STG; ++u) {
    const int e = threadIdx.x + 256 * u;
    Xs[(e >> 6) * LDX + (e & 63)] = v[u];
  }
}

// acc[s] += tile (w + 4 s) of Xs^T Xs; wave w owns tiles w, w + 4, w + 8.
// MFMA operands: A(i, k) = Xs(k, 16 I + i) in lane i + 16 k, B(k, j) = Xs(k, 16 J + j) in lane j + 16 k.
__device__ __forceinline__ void gram_tiles(const double *Xs, d4 (&acc)[3]) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double *xa[3], *xb[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int t = w + 4 * s < NTILE ? w + 4 * s : 0;
    xa[s] = Xs + (l >> 4) * LDX + 16 * tile_i(t) + (l & 15);
    xb[s] = Xs + (l >> 4) * LDX + 16 * tile_j(t) + (l & 15);
  }
  const bool third = w + 8 < NTILE;
#pragma unroll
  for (int k4 = 0; k4 < RPW / 4; ++k4) {
    acc[0] = mfma(xa[0][4 * k4 * LDX], xb[0][4 * k4 * LDX], acc[0]);
    acc[1] = mfma(xa[1][4 * k4 * LDX], xb[1][4 * k4 * LDX], acc[1]);
    if (third) acc[2] = mfma(xa[2][4 * k4 * LDX], xb[2][4 * k4 * LDX], acc[2]);
  }
}

// D(i, j) of tile t sits in lane j + 16 (i mod 4), register i / 4.
__device__ __forceinline__ void store_tiles(const d4 (&acc)[3], double *dst) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int t = w + 4 * s;
    if (t >= NTILE) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) ds::st_dev(&dst[t * TILE + ((l >> 4) + 4 * v) * 16 + (l & 15)], acc[s][v]);
  }
}

// Sum of the P partials in partial order into the lower triangles of G and A
// (LDS, LDX; A is the working copy the factorization overwrites).
__device__ __forceinline__ void reduce_parts(const double *part, int P, double *G, double *A) {
  const int t = threadIdx.x;
  double sum[NTILE];
#pragma unroll
  for (int u = 0; u < NTILE; ++u) sum[u] = 0.0;
  for (int p0 = 0; p0 < P; p0 += 8) {
    double v[8][NTILE];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int u = 0; u < NTILE; ++u)
        v[q][u] = p0 + q < P ? ds::ld_dev(&part[(int64_t)(p0 + q) * PART + u * TILE + t]) : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int u = 0; u < NTILE; ++u) sum[u] += v[q][u];
  }
  const int i = t >> 4, j = t & 15;
#pragma unroll
  for (int u = 0; u < NTILE; ++u) {
    const int I = tile_i(u), J = tile_j(u);
    // tile (I, J) entry (i, j) is G(16 I + i, 16 J + j) = G(16 J + j, 16 I + i): keep the lower copy
    if (I < J || j >= i) {
      G[(16 * J + j) * LDX + 16 * I + i] = sum[u];
      A[(16 * J + j) * LDX + 16 * I + i] = sum[u];
    }
  }
}

// W_K = L_KK^{-1} (lower 16 x 16) for K = 0..3: wave K, lane j < 16 forms column j.
__device__ __forceinline__ void diag_inverses(const double *Lf, const double *dinv, double *W) {
  const int l = threadIdx.x & 63, K = threadIdx.x >> 6;
  if (l < 16) {
    const int j = l;
    const double *Lk = Lf + 16 * K * LDX + 16 * K;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int c = 0; c < i; ++c) s = fma(-Lk[i * LDX + c], x[c], s);
      x[i] = (i >= j) ? s * dinv[16 * K + i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) W[K * TILE + i * 16 + j] = x[i];
  }
}

// The last workgroup: reduce the partials, factor (with the shifted retry),
// invert the diagonal blocks, write the factor tiles Mf: tile (J, K), K < J, is
// L_JK and tile (J, J) is W_J = L_JJ^{-1}, each 16 x 16 row-major.
__device__ __forceinline__ void factor_last(const double *part, int P, int ell, int64_t rows, double *Mf, int *dflags, double *pool) {
  const int t = threadIdx.x;
  double *G = pool, *A = G + 64 * LDX, *Lf = A + 64 * LDX, *dinv = Lf + 64 * LDX, *W = dinv + 64, *red = W + 4 * TILE;
  double *colb = red + 8;
  reduce_parts(part, P, G, A);
  __syncthreads();
  if (t < 64) {
    double v = t < ell ? G[t * LDX + t] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (t == 0) red[0] = v;
  }
  __syncthreads();
  const double tr = red[0];
  const bool trok = tr > 0.0 && isfinite(tr);
  bool ok = false;
#pragma nounroll
  for (int attempt = 0; attempt < 2 && trok && !ok; ++attempt) {
    if (attempt) {
      const double shift = 11.0 * ((double)rows * ell + (double)ell * (ell + 1)) * U64 * tr;
      for (int e = t; e < 64 * 64; e += 256) {
        const int i = e >> 6, c = e & 63;
        if (c <= i) A[i * LDX + c] = G[i * LDX + c] + ((i == c && i < ell) ? shift : 0.0);
      }
      __syncthreads();
    }
    if (t < 64) {
      const bool okw = wc::chol64_blocked(A, ell, 1e-15 * tr, Lf, dinv, colb);
      if (t == 0) red[1] = okw ? 1.0 : 0.0;
    }
    __syncthreads();
    ok = red[1] != 0.0;
    if (!ok && attempt == 0 && t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_FALLBACK);
    __syncthreads();
  }
  if (!ok) {
    // non-finite or zero input: identity factor keeps the pipeline finite
    if (t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_FALLBACK | DSK_FLAG_RANK_DEFICIENT | DSK_FLAG_NONFINITE);
    for (int e = t; e < PART; e += 256) {
      const int r = e & (TILE - 1);
      const int tid = e / TILE;
      const bool diag = tid == 0 || tid == 2 || tid == 5 || tid == 9;
      Mf[e] = (diag && (r >> 4) == (r & 15)) ? 1.0 : 0.0;
    }
    return;
  }
  diag_inverses(Lf, dinv, W);
  __syncthreads();
  // tile u = J (J + 1) / 2 + K, entry t = (i, k)
  const int i = t >> 4, k = t & 15;
#pragma unroll
  for (int J = 0; J < 4; ++J)
#pragma unroll
    for (int K = 0; K <= J; ++K)
      Mf[ltile(J, K) * TILE + t] = (K == J) ? W[K * TILE + t] : Lf[(16 * J + i) * LDX + 16 * K + k];
}

// ---------------------------------------------------------------- launches
// Gram partials of X; the last workgroup factors them into Mf.
template <typename T>
__global__ void __launch_bounds__(256) k_cq_gram(const T *__restrict__ X, int64_t rows, int ell, int64_t rpw,
                                                 double *part, unsigned *ticket, double *Mf, int *dflags) {
  extern __shared__ double pool[];
  d4 acc[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) acc[s] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t r0 = (int64_t)blockIdx.x * rpw, r1 = std::min<int64_t>(rows, r0 + rpw);
  double v[STG];
  fetch_rows(X, r1, ell, r0, v);
  for (int64_t c0 = r0; c0 < r1; c0 += RPW) {
    __syncthreads();
    put_rows(v, pool);
    __syncthreads();
    if (c0 + RPW < r1) fetch_rows(X, r1, ell, c0 + RPW, v);
    gram_tiles(pool, acc);
  }
  store_tiles(acc, part + (int64_t)blockIdx.x * PART);
  if (ds::last_arrival(ticket)) factor_last(part, gridDim.x, ell, rows, Mf, dflags, pool);
}

// Q = Y L^{-T} for the rows of this workgroup (Q may alias Y).  With part,
// also the Gram partials of the rounded Q, factored by the last workgroup into
// Mf (every workgroup has staged Mf before it arrives).  cond = 1: only after
// a shifted pass; gram_cond = 1: the Gram and factorization only after a
// shifted pass.
template <typename T>
__global__ void __launch_bounds__(256) k_cq_apply(const T *Y, int64_t rows, int ell, double *Mf, T *Q, int64_t rpw,
                                                  double *part, unsigned *ticket, int *dflags, int cond,
                                                  int gram_cond) {
  const bool fallback = (dflags[FLAGW_BITS] & DSK_FLAG_FALLBACK) != 0;
  if (cond && !fallback) return;
  if (gram_cond && !fallback) part = nullptr;
  extern __shared__ double pool[];
  double *Ys = pool, *Qs = Ys + RPW * LDX, *Ms = Qs + RPW * LDX, *Ss = Ms + PART;
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rpw, r1 = std::min<int64_t>(rows, r0 + rpw);
  double v[STG];
  fetch_rows(Y, r1, ell, r0, v);
  {
    double m[PART / 256];
#pragma unroll
    for (int u = 0; u < PART / 256; ++u) m[u] = Mf[t + 256 * u];
#pragma unroll
    for (int u = 0; u < PART / 256; ++u) Ms[t + 256 * u] = m[u];
  }
  double *Sw = Ss + w * 16 * 17;
  d4 acc[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) acc[s] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t c0 = r0; c0 < r1; c0 += RPW) {
    __syncthreads();
    put_rows(v, Ys);
    __syncthreads();
    if (c0 + RPW < r1) fetch_rows(Y, r1, ell, c0 + RPW, v);
    // wave w: rows 16 w .. 16 w + 15 of the chunk, block columns in order
    const int rb = 16 * w;
#pragma unroll
    for (int J = 0; J < 4; ++J) {
      // S = Y_J - sum_K Q_K L_JK^T: one accumulator per K (independent MFMA chains), summed in K order
      d4 c, ck[3];
#pragma unroll
      for (int v = 0; v < 4; ++v) c[v] = Ys[(rb + (l >> 4) + 4 * v) * LDX + 16 * J + (l & 15)];
#pragma unroll
      for (int K = 0; K < 3; ++K) ck[K] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
        for (int K = 0; K < J; ++K) {
          const double a = -Qs[(rb + (l & 15)) * LDX + 16 * K + 4 * k4 + (l >> 4)];
          const double b = Ms[ltile(J, K) * TILE + (l & 15) * 16 + 4 * k4 + (l >> 4)];
          ck[K] = mfma(a, b, ck[K]);
        }
#pragma unroll
      for (int K = 0; K < J; ++K) c += ck[K];
#pragma unroll
      for (int v = 0; v < 4; ++v) Sw[((l >> 4) + 4 * v) * 17 + (l & 15)] = c[v];
      wc::wave_lds_sync();
      const double *Wt = Ms + ltile(J, J) * TILE;
      d4 q = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) q = mfma(Sw[(l & 15) * 17 + 4 * k4 + (l >> 4)], Wt[(l & 15) * 16 + 4 * k4 + (l >> 4)], q);
#pragma unroll
      for (int v = 0; v < 4; ++v) Qs[(rb + (l >> 4) + 4 * v) * LDX + 16 * J + (l & 15)] = q[v];
      wc::wave_lds_sync();
    }
    // round this wave's rows to the output type (the Gram describes the stored Q)
    for (int e = l; e < 16 * 64; e += 64) {
      double *p = &Qs[(rb + (e >> 6)) * LDX + (e & 63)];
      *p = (double)(T)(*p);
    }
    __syncthreads();
    for (int e = t; e < RPW * 64; e += 256) {
      const int r = e >> 6, c = e & 63;
      if (c0 + r < r1 && c < ell) Q[(c0 + r) * ell + c] = (T)Qs[r * LDX + c];
    }
    if (part) gram_tiles(Qs, acc);
  }
  if (!part) return;
  store_tiles(acc, part + (int64_t)blockIdx.x * PART);
  if (ticket && ds::last_arrival(ticket)) {
    __syncthreads();
    factor_last(part, gridDim.x, ell, rows, Mf, dflags, pool);
  }
}

template <typename K>
void allow_pool(K kernel) {
  allow_lds(kernel, (size_t)POOL_LDS * sizeof(double));
}

template <typename T>
int cholqr64_typed(hipStream_t st, const T *Y, int64_t rows, int ell, T *Q, void *ws, int *dflags, int passes) {
  const int64_t chunks = (rows + RPW - 1) / RPW;
  const int64_t rpw = (chunks + PMAX - 1) / PMAX * RPW;
  const int P = (int)((rows + rpw - 1) / rpw);
  double *part = reinterpret_cast<double *>(ws);
  double *Mf = part + (size_t)PMAX * PART;
  T *Q1 = reinterpret_cast<T *>(Mf + PART);
  unsigned *ticket = reinterpret_cast<unsigned *>(dflags + FLAGW_TICKET);
  const size_t lds = (size_t)POOL_LDS * sizeof(double);
  allow_pool(k_cq_gram<T>);
  allow_pool(k_cq_apply<T>);
  hipLaunchKernelGGL(k_cq_gram<T>, dim3(P), dim3(256), lds, st, Y, rows, ell, rpw, part, ticket, Mf, dflags);
  auto apply = [&](const T *src, T *dst, double *prt, int cond, int gcond) {
    hipLaunchKernelGGL(k_cq_apply<T>, dim3(P), dim3(256), lds, st, src, rows, ell, Mf, dst, rpw, prt,
                       prt ? ticket : nullptr, dflags, cond, gcond);
  };
  if (passes == 1) {
    apply(Y, Q, nullptr, 0, 0);   // span only
  } else {
    apply(Y, Q1, part, 0, 0);     // second factorization
    apply(Q1, Q, part, 0, 1);     // third factorization only after a shifted first pass
    apply(Q, Q, nullptr, 1, 0);   // third application only after a shifted first pass
  }
  DSK_TRY(hipGetLastError());
  return 0;
}

}  // namespace

int launch_cholqr64_apply(hipStream_t st, const void *X, int f64, int64_t rows, int ell, const void *ws, void *out,
                          int *dflags) {
  if (ell < 1 || ell > 64 || rows < 1) return -1;
  // the factor tiles the last factorization on ws left (after the Gram partials)
  double *Mf = const_cast<double *>(reinterpret_cast<const double *>(ws)) + (size_t)PMAX * PART;
  const unsigned grid = (unsigned)((rows + RPW - 1) / RPW);
  const size_t lds = (size_t)POOL_LDS * sizeof(double);
  if (f64) {
    allow_pool(k_cq_apply<double>);
    hipLaunchKernelGGL(k_cq_apply<double>, dim3(grid), dim3(256), lds, st, (const double *)X, rows, ell, Mf,
                       (double *)out, (int64_t)RPW, (double *)nullptr, (unsigned *)nullptr, dflags, 0, 0);
  } else {
    allow_pool(k_cq_apply<float>);
    hipLaunchKernelGGL(k_cq_apply<float>, dim3(grid), dim3(256), lds, st, (const float *)X, rows, ell, Mf,
                       (float *)out, (int64_t)RPW, (double *)nullptr, (unsigned *)nullptr, dflags, 0, 0);
  }
  DSK_TRY(hipGetLastError());
  return 0;
}

size_t cholqr64_ws_bytes(int64_t rows, int ell) {
  return ((size_t)PMAX * PART + PART) * sizeof(double) + (size_t)rows * ell * sizeof(double) + 256;
}

int launch_cholqr64(hipStream_t st, const void *Y, int f64, int64_t rows, int ell, void *Q, void *ws, int *dflags,
                    int passes) {
  if (ell < 1 || ell > 64 || rows < 1 || passes < 1 || passes > 2) return -1;
  if (f64) return cholqr64_typed<double>(st, (const double *)Y, rows, ell, (double *)Q, ws, dflags, passes);
  return cholqr64_typed<float>(st, (const float *)Y, rows, ell, (float *)Q, ws, dflags, passes);
}

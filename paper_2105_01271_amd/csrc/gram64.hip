// G = X^T X in FP64 for a tall block X (rows x ell, ell <= 128) on the FP64
// matrix cores: the Gram of B^T in the core SVD (Alg. 2, "SVD(B)" step, as
// G_B = B B^T), and the Grams of the refinement sweep and of the single-pass
// start block.  Products of FP32 values are exact in FP64, so the only rounding
// is that of the FP64 sums.
//
// k_gram_mfma: a workgroup (4 waves) takes a contiguous range of rows, stages
// 32 rows at a time in LDS as FP64, and accumulates the 16 x 16 tiles (I, J),
// I >= J, of its partial Gram with v_mfma_f64_16x16x4f64 (wave w owns tiles
// w, w + 4, ...); the partial goes to part[block] (lower tiles only), as an
// ell x ell matrix or tile-major (the 128-wide CholeskyQR).
// k_gram_fold: G(a, b) = sum over the blocks' partials in a fixed order
// (deterministic), the upper triangle mirrored.
#include <algorithm>

#include "dsk_internal.h"
#include "gramtile.h"

namespace {

constexpr int GR = 32;          // rows per LDS chunk
constexpr int GMAX = 128;       // widest block

// TILED = false: the partial is an ell x ell row-major matrix (lower tiles
// written); TILED = true: tile-major lower tiles (16 x 16 each, numbered as in
// gramtile.h), the layout the 128-wide CholeskyQR folds and factors.
template <typename T, bool TILED>
__global__ void __launch_bounds__(256) k_gram_mfma(const T *__restrict__ X, int64_t rows, int ell, int64_t ldx,
                                                   int64_t rows_per_blk, double *__restrict__ part) {
  __shared__ double sh[GR][GMAX + 2];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int nb = (ell + 15) / 16, ellp = nb * 16;
  const gt::Tiles tl = gt::tiles_of(wave, nb);
  wc::d4 acc[gt::MAXT];
  gt::zero(acc);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(rows, r0 + rows_per_blk);
  // the next chunk is loaded into registers while the current one feeds the
  // MFMAs; thread t takes column t mod 128 of rows t / 128 + 2 u (no index
  // division)
  constexpr int PF = GR * GMAX / 256;
  static_assert(GMAX == 128 && PF * 2 == GR, "two rows of 128 columns per pass of the workgroup");
  T pf[PF];
  const int fc = t & (GMAX - 1), fr = t >> 7;
  auto fetch = [&](int64_t c0) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int64_t r = c0 + fr + 2 * u;
      pf[u] = (r < r1 && fc < ell) ? X[r * ldx + fc] : T(0);
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t c0 = r0; c0 < r1; c0 += GR) {
    if (fc < ellp) {
#pragma unroll
      for (int u = 0; u < PF; ++u) sh[fr + 2 * u][fc] = (double)pf[u];
    }
    __syncthreads();
    if (c0 + GR < r1) fetch(c0 + GR);
    gt::accum<GR / 4>(&sh[0][0], GMAX + 2, tl, acc);
    __syncthreads();
  }
  if (TILED) {
    gt::store_tiles(acc, tl, wave, part + (int64_t)blockIdx.x * (nb * (nb + 1) / 2) * 256);
    return;
  }
  // D(i, j) of a tile: lane j + 16 (i mod 4), register i / 4
  double *P = part + (int64_t)blockIdx.x * ell * ell;
  const int col = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int u = 0; u < gt::MAXT; ++u) {
    if (u >= tl.n) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * tl.ti[u] + 4 * v + kk, b = 16 * tl.tj[u] + col;
      if (a < ell && b < ell) P[a * ell + b] = acc[u][v];
    }
  }
}

// Four threads (a quad) per entry: thread q sums the partials q, q + 4, ...
// in order, sixteen loads in flight before they are added (in groups of
// sixteen, each group summed in order), and the quad adds its four sums as
// (s0 + s1) + (s2 + s3): a fixed order, so repeated runs give the same bytes.
__global__ void __launch_bounds__(256) k_gram_fold(const double *__restrict__ part, int nparts, int ell,
                                                   double *__restrict__ G) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  const int e = g >> 2, q = g & 3;
  const int a = e / ell, b = e - (e / ell) * ell;
  // an upper tile is written as the mirror
  const bool live = e < ell * ell && a / 16 >= b / 16;
  const int64_t n2 = (int64_t)ell * ell;
  double s = 0.0;
  if (live) {
    int p = q;
    for (; p + 60 < nparts; p += 64) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = part[(int64_t)(p + 4 * u) * n2 + e];
      double gs = 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) gs += v[u];
      s += gs;
    }
    for (; p < nparts; p += 4) s += part[(int64_t)p * n2 + e];
  }
  s += wc::dpp_f64<0xB1>(s);   // lanes 2i, 2i + 1
  s += wc::dpp_f64<0x4E>(s);   // the two pairs of the quad
  if (live && q == 0) {
    G[e] = s;
    if (a / 16 > b / 16) G[b * ell + a] = s;
  }
}

}  // namespace

// Workgroups of the Gram: 256 rows each at least, at most two per CU of the
// MI355X (512), so that one workgroup's MFMA chain runs while the other's
// chunk is staged.
int gram_mfma_blocks(int64_t rows) {
  return (int)std::min<int64_t>(512, std::max<int64_t>(1, (rows + 255) / 256));
}

int launch_gram_mfma(hipStream_t st, const void *X, int f64, int64_t rows, int ell, double *G, double *part,
                     int nparts) {
  if (ell < 1 || ell > GMAX || rows < 1 || nparts < 1) return -1;
  const int nblk_max = std::min(nparts, gram_mfma_blocks(rows));
  const int64_t rpb = ((rows + nblk_max - 1) / nblk_max + GR - 1) / GR * GR;
  const int nblk = (int)((rows + rpb - 1) / rpb);
  if (f64)
    hipLaunchKernelGGL((k_gram_mfma<double, false>), dim3(nblk), dim3(256), 0, st, (const double *)X, rows, ell, (int64_t)ell,
                       rpb, part);
  else
    hipLaunchKernelGGL((k_gram_mfma<float, false>), dim3(nblk), dim3(256), 0, st, (const float *)X, rows, ell, (int64_t)ell,
                       rpb, part);
  DSK_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_gram_fold, dim3((4 * ell * ell + 255) / 256), dim3(256), 0, st, (const double *)part, nblk, ell, G);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_gram_tiles(hipStream_t st, const void *X, int f64, int64_t rows, int ell, int64_t rows_per_blk,
                      double *part) {
  if (ell < 1 || ell > GMAX || rows < 1 || rows_per_blk < 1 || rows_per_blk % GR) return -1;
  const int nblk = (int)((rows + rows_per_blk - 1) / rows_per_blk);
  if (f64)
    hipLaunchKernelGGL((k_gram_mfma<double, true>), dim3(nblk), dim3(256), 0, st, (const double *)X, rows, ell,
                       (int64_t)ell, rows_per_blk, part);
  else
    hipLaunchKernelGGL((k_gram_mfma<float, true>), dim3(nblk), dim3(256), 0, st, (const float *)X, rows, ell,
                       (int64_t)ell, rows_per_blk, part);
  DSK_TRY(hipGetLastError());
  return 0;
}

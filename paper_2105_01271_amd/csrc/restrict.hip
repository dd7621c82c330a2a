// Coarse restriction A_c = A D without forming D (paper Sec. 2, general sketch
// equation; direct injection, nearest-neighbour and global sketches), plus the
// small gather / conversion helpers of the pipeline.
//
// Layout: A is m x n row-major (row = snapshot) with leading dimension lda,
// stored as f64, f32, bf16 or f16.  A_c is written m x s row-major in the work
// dtype (f64 for f64 input, f32 otherwise) and, when requested, also
// transposed (s x m row-major) for the products with A_c in the power step.
//
// Memory behaviour: direct injection reads one element per coarse point, but
// on a y-major grid with x-stride sx every 128-byte line of a selected grid
// row is touched, so the physical fetch is about 1/sy of A; the algorithmic
// fetch is s/n.  The 64x64 tile keeps the A_c stores coalesced and stages the
// transposed copy through LDS.
#include <algorithm>

#include "dsk_internal.h"

namespace {

template <int DT>
__device__ __forceinline__ double load_as_f64(const void *A, int64_t off) {
  if constexpr (DT == DSK_F64) return reinterpret_cast<const double *>(A)[off];
  if constexpr (DT == DSK_F32) return (double)reinterpret_cast<const float *>(A)[off];
  if constexpr (DT == DSK_BF16) return (double)bf16_bits_to_f32(reinterpret_cast<const unsigned short *>(A)[off]);
  return (double)f16_bits_to_f32(reinterpret_cast<const unsigned short *>(A)[off]);
}

template <int DT>
__device__ __forceinline__ float load_as_f32(const void *A, int64_t off) {
  if constexpr (DT == DSK_F64) return (float)reinterpret_cast<const double *>(A)[off];
  if constexpr (DT == DSK_F32) return reinterpret_cast<const float *>(A)[off];
  if constexpr (DT == DSK_BF16) return bf16_bits_to_f32(reinterpret_cast<const unsigned short *>(A)[off]);
  return f16_bits_to_f32(reinterpret_cast<const unsigned short *>(A)[off]);
}

struct Grid2 {
  int ny, nx, sy, sx, cy, cx;
};

constexpr int KIND_DI_GRID = 100;   // internal: direct injection on the grid of a stencil / learned restriction

// Value of coarse column j of row i for each restriction kind.
// KIND 0: index gather; 1: nearest neighbour; 2: global (block mean);
// 3: direct injection on the grid (the point (sy b, sx a) itself).
template <int DT, int KIND, typename W>
__device__ __forceinline__ W coarse_value(const void *A, int64_t row_off, int64_t j,
                                          const int64_t *__restrict__ idx, Grid2 g, int64_t n, int *dflags) {
  if constexpr (KIND == 0) {
    int64_t c = idx[j];
    if (c < 0 || c >= n) {   // never read outside the row; report through the flag word
      atomicOr(dflags, DSK_FLAG_BAD_INDEX);
      c = 0;
    }
    if constexpr (sizeof(W) == 8) return load_as_f64<DT>(A, row_off + c);
    else return load_as_f32<DT>(A, row_off + c);
  } else {
    const int b = (int)(j / g.cx), a = (int)(j % g.cx);
    const int y0 = b * g.sy, x0 = a * g.sx;
    W acc = 0;
    if constexpr (KIND == 3) {
      if constexpr (sizeof(W) == 8) return load_as_f64<DT>(A, row_off + (int64_t)y0 * g.nx + x0);
      else return load_as_f32<DT>(A, row_off + (int64_t)y0 * g.nx + x0);
    } else if constexpr (KIND == 1) {
      const W w[3] = {W(0.25), W(0.5), W(0.25)};
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int y = y0 + dy;
        if (y < 0 || y >= g.ny) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int x = x0 + dx;
          if (x < 0 || x >= g.nx) continue;
          W v;
          if constexpr (sizeof(W) == 8) v = load_as_f64<DT>(A, row_off + (int64_t)y * g.nx + x);
          else v = load_as_f32<DT>(A, row_off + (int64_t)y * g.nx + x);
          acc += w[dy + 1] * w[dx + 1] * v;
        }
      }
    } else {
      const W wgt = W(1) / W(g.sy * g.sx);
      for (int dy = 0; dy < g.sy; ++dy) {
        const int y = y0 + dy;
        if (y >= g.ny) break;
        for (int dx = 0; dx < g.sx; ++dx) {
          const int x = x0 + dx;
          if (x >= g.nx) break;
          W v;
          if constexpr (sizeof(W) == 8) v = load_as_f64<DT>(A, row_off + (int64_t)y * g.nx + x);
          else v = load_as_f32<DT>(A, row_off + (int64_t)y * g.nx + x);
          acc += v;
        }
      }
      acc *= wgt;
    }
    return acc;
  }
}

constexpr int TJ = 64;   // coarse columns per tile
constexpr int TI = 64;   // rows per tile

template <int DT, int KIND, typename W>
__global__ void __launch_bounds__(256) k_restrict(const void *__restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                  int64_t s, const int64_t *__restrict__ idx, Grid2 g,
                                                  W *__restrict__ Ac, W *__restrict__ AcT, int *dflags) {
  __shared__ W tile[TI][TJ + 1];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * TJ, i0 = (int64_t)blockIdx.y * TI;
  const int64_t j = j0 + tx;
  for (int ii = ty; ii < TI; ii += 4) {
    const int64_t i = i0 + ii;
    W v = 0;
    if (i < m && j < s) {
      v = coarse_value<DT, KIND, W>(A, i * lda, j, idx, g, n, dflags);
      if (Ac) Ac[i * s + j] = v;
    }
    tile[ii][tx] = v;
  }
  if (!AcT) return;
  __syncthreads();
  for (int jj = ty; jj < TJ; jj += 4) {
    const int64_t jc = j0 + jj, i = i0 + tx;
    if (jc < s && i < m) AcT[jc * m + i] = tile[tx][jj];
  }
}

template <int DT, int KIND>
int restrict_typed(hipStream_t st, const void *A, int64_t m, int64_t n, int64_t lda, int64_t s,
                   const int64_t *idx, Grid2 g, int work_f64, void *Ac, void *AcT, int *dflags) {
  dim3 grid((unsigned)((s + TJ - 1) / TJ), (unsigned)((m + TI - 1) / TI));
  if (work_f64)
    hipLaunchKernelGGL((k_restrict<DT, KIND, double>), grid, dim3(256), 0, st, A, m, n, lda, s, idx, g,
                       (double *)Ac, (double *)AcT, dflags);
  else
    hipLaunchKernelGGL((k_restrict<DT, KIND, float>), grid, dim3(256), 0, st, A, m, n, lda, s, idx, g,
                       (float *)Ac, (float *)AcT, dflags);
  DSK_TRY(hipGetLastError());
  return 0;
}

template <int DT>
int restrict_dt(hipStream_t st, int kind, const void *A, int64_t m, int64_t n, int64_t lda, int64_t s,
                const int64_t *idx, Grid2 g, int work_f64, void *Ac, void *AcT, int *dflags) {
  if (kind == DSK_R_INDEX) return restrict_typed<DT, 0>(st, A, m, n, lda, s, idx, g, work_f64, Ac, AcT, dflags);
  if (kind == DSK_R_NN) return restrict_typed<DT, 1>(st, A, m, n, lda, s, idx, g, work_f64, Ac, AcT, dflags);
  if (kind == KIND_DI_GRID) return restrict_typed<DT, 3>(st, A, m, n, lda, s, idx, g, work_f64, Ac, AcT, dflags);
  return restrict_typed<DT, 2>(st, A, m, n, lda, s, idx, g, work_f64, Ac, AcT, dflags);
}

// Y(:, c) = Ac(:, c * floor(s / ell)): the nested direct-injection start block.
template <typename W>
__global__ void k_select_cols(const W *__restrict__ Ac, int64_t m, int64_t s, int64_t ldc, int ell,
                              W *__restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * ell) return;
  const int64_t i = t / ell;
  const int c = (int)(t % ell);
  const int64_t step = s / ell;
  Y[t] = Ac[i * ldc + (int64_t)c * step];
}

template <typename T>
__global__ void k_gather_rows(const T *__restrict__ A, int64_t m, int64_t n, int64_t lda,
                              const int64_t *__restrict__ rows, T *__restrict__ out) {
  const int r = blockIdx.y;
  const int64_t row = rows[r];
  const bool ok = row >= 0 && row < m;
  const int64_t src = ok ? row * lda : 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
    out[(int64_t)r * n + c] = ok ? A[src + c] : T(0);
}

// The same copy in 16-byte pieces when every row start (of A and of out) is
// 16-byte aligned: nb16 pieces per row.
typedef unsigned u32x4g __attribute__((ext_vector_type(4)));
__global__ void k_gather_rows16(const u32x4g *__restrict__ A, int64_t m, int64_t lda16, int64_t nb16,
                                const int64_t *__restrict__ rows, u32x4g *__restrict__ out) {
  const int r = blockIdx.y;
  const int64_t row = rows[r];
  const bool ok = row >= 0 && row < m;
  const int64_t src = ok ? row * lda16 : 0;
  const u32x4g z = {0u, 0u, 0u, 0u};
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nb16; c += (int64_t)gridDim.x * blockDim.x)
    out[(int64_t)r * nb16 + c] = ok ? A[src + c] : z;
}

// out[i, c] = A[i, idx[c]] for 16-bit storage, the bits copied unchanged
__global__ void __launch_bounds__(256) k_gather_cols16(const unsigned short *__restrict__ A, int64_t m, int64_t lda,
                                                       const int64_t *__restrict__ idx, int64_t s,
                                                       unsigned short *__restrict__ out) {
  const int64_t i = blockIdx.y;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < s; c += (int64_t)gridDim.x * 256)
    out[i * s + c] = A[i * lda + idx[c]];
}

template <typename S, typename D>
__global__ void k_convert(const S *__restrict__ src, D *__restrict__ dst, int64_t count) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = (D)src[t];
}

template <typename T>
__global__ void __launch_bounds__(256) k_transpose(const T *__restrict__ src, int64_t rows, int64_t cols,
                                                   T *__restrict__ dst) {
  __shared__ T tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * 64, r0 = (int64_t)blockIdx.y * 64;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr, c = c0 + tx;
    tile[rr][tx] = (r < rows && c < cols) ? src[r * cols + c] : T(0);
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t c = c0 + cc, r = r0 + tx;
    if (c < cols && r < rows) dst[c * rows + r] = tile[tx][cc];
  }
}

template <int DT>
__global__ void __launch_bounds__(256) k_fro2_part(const void *__restrict__ A, int64_t m, int64_t n,
                                                   int64_t lda, double *__restrict__ part) {
  double acc = 0.0;
  const int64_t total = m * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / n, j = t - i * n;
    const double v = load_as_f64<DT>(A, i * lda + j);
    acc += v * v;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_parts(const double *__restrict__ part, int nparts, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += part[i];   // fixed order: deterministic
    out[0] = s;
  }
}

}  // namespace

int launch_restrict(hipStream_t st, const void *A, int dtype, int64_t m, int64_t n, int64_t lda,
                    const dsk_restriction *R, int64_t s, int work_f64, void *Ac, void *AcT, int *dflags) {
  if (R->kind == DSK_R_LEARNED) {
    if (AcT) return -1;
    return launch_conv_fwd(st, A, dtype, m, lda, R->ny, R->nx, R->channels, R->w1, R->w2, work_f64, Ac, s,
                           conv_filter_ws(dflags));
  }
  Grid2 g{};
  if (R->kind == DSK_R_NN || R->kind == DSK_R_GLOBAL) {
    g.ny = R->ny; g.nx = R->nx; g.sy = R->sy; g.sx = R->sx;
    g.cy = (R->ny + R->sy - 1) / R->sy;
    g.cx = (R->nx + R->sx - 1) / R->sx;
  }
  const int64_t *idx = R->kind == DSK_R_INDEX ? R->index : nullptr;
  switch (dtype) {
    case DSK_F64: return restrict_dt<DSK_F64>(st, R->kind, A, m, n, lda, s, idx, g, work_f64, Ac, AcT, dflags);
    case DSK_F32: return restrict_dt<DSK_F32>(st, R->kind, A, m, n, lda, s, idx, g, work_f64, Ac, AcT, dflags);
    case DSK_BF16: return restrict_dt<DSK_BF16>(st, R->kind, A, m, n, lda, s, idx, g, work_f64, Ac, AcT, dflags);
    default: return restrict_dt<DSK_F16>(st, R->kind, A, m, n, lda, s, idx, g, work_f64, Ac, AcT, dflags);
  }
}

// The Gram sub-sample A_g = A(:, I) of C-PWR (Alg. 7).  An index restriction
// is its own I; a stencil restriction uses the direct-injection points of its
// grid and factor, the learned conv those of its stride-4 output grid.  The
// sub-sample has as many columns as the restriction (s).
int launch_gram_sample(hipStream_t st, const void *A, int dtype, int64_t m, int64_t n, int64_t lda,
                       const dsk_restriction *R, int64_t s, int work_f64, void *Ag, int *dflags) {
  if (R->kind == DSK_R_INDEX) return launch_restrict(st, A, dtype, m, n, lda, R, s, work_f64, Ag, nullptr, dflags);
  Grid2 g{};
  g.ny = R->ny; g.nx = R->nx;
  g.sy = R->kind == DSK_R_LEARNED ? 4 : R->sy;
  g.sx = R->kind == DSK_R_LEARNED ? 4 : R->sx;
  g.cy = (g.ny + g.sy - 1) / g.sy;
  g.cx = (g.nx + g.sx - 1) / g.sx;
  if ((int64_t)g.cy * g.cx != s) return -1;
  switch (dtype) {
    case DSK_F64: return restrict_dt<DSK_F64>(st, KIND_DI_GRID, A, m, n, lda, s, nullptr, g, work_f64, Ag, nullptr, dflags);
    case DSK_F32: return restrict_dt<DSK_F32>(st, KIND_DI_GRID, A, m, n, lda, s, nullptr, g, work_f64, Ag, nullptr, dflags);
    case DSK_BF16: return restrict_dt<DSK_BF16>(st, KIND_DI_GRID, A, m, n, lda, s, nullptr, g, work_f64, Ag, nullptr, dflags);
    default: return restrict_dt<DSK_F16>(st, KIND_DI_GRID, A, m, n, lda, s, nullptr, g, work_f64, Ag, nullptr, dflags);
  }
}

int launch_select_cols(hipStream_t st, const void *Ac, int work_f64, int64_t m, int64_t s, int64_t ldc,
                       int ell, void *Y) {
  const int64_t total = m * ell;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (work_f64)
    hipLaunchKernelGGL(k_select_cols<double>, dim3(blocks), dim3(256), 0, st, (const double *)Ac, m, s, ldc,
                       ell, (double *)Y);
  else
    hipLaunchKernelGGL(k_select_cols<float>, dim3(blocks), dim3(256), 0, st, (const float *)Ac, m, s, ldc,
                       ell, (float *)Y);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_gather_rows(hipStream_t st, const void *A, int dtype, int64_t m, int64_t n, int64_t lda,
                       const int64_t *rows, int k, void *out) {
  const int64_t es = dtype == DSK_F64 ? 8 : dtype == DSK_F32 ? 4 : 2;
  if ((n * es) % 16 == 0 && (lda * es) % 16 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
      reinterpret_cast<uintptr_t>(out) % 16 == 0) {
    const int64_t nb16 = n * es / 16;
    const unsigned bx16 = (unsigned)std::min<int64_t>((nb16 + 255) / 256, 256);
    hipLaunchKernelGGL(k_gather_rows16, dim3(bx16, (unsigned)k), dim3(256), 0, st, (const u32x4g *)A, m,
                       lda * es / 16, nb16, rows, (u32x4g *)out);
    DSK_TRY(hipGetLastError());
    return 0;
  }
  const unsigned bx = (unsigned)std::min<int64_t>((n + 255) / 256, 256);
  dim3 grid(bx, (unsigned)k);
  if (dtype == DSK_F64)
    hipLaunchKernelGGL(k_gather_rows<double>, grid, dim3(256), 0, st, (const double *)A, m, n, lda, rows,
                       (double *)out);
  else if (dtype == DSK_F32)
    hipLaunchKernelGGL(k_gather_rows<float>, grid, dim3(256), 0, st, (const float *)A, m, n, lda, rows,
                       (float *)out);
  else
    hipLaunchKernelGGL(k_gather_rows<unsigned short>, grid, dim3(256), 0, st, (const unsigned short *)A, m, n,
                       lda, rows, (unsigned short *)out);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_convert(hipStream_t st, const void *src, int src_f64, void *dst, int dst_f64, int64_t count) {
  const unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 4096);
  if (src_f64 && !dst_f64)
    hipLaunchKernelGGL((k_convert<double, float>), dim3(blocks), dim3(256), 0, st, (const double *)src,
                       (float *)dst, count);
  else if (!src_f64 && dst_f64)
    hipLaunchKernelGGL((k_convert<float, double>), dim3(blocks), dim3(256), 0, st, (const float *)src,
                       (double *)dst, count);
  else if (src_f64)
    hipLaunchKernelGGL((k_convert<double, double>), dim3(blocks), dim3(256), 0, st, (const double *)src,
                       (double *)dst, count);
  else
    hipLaunchKernelGGL((k_convert<float, float>), dim3(blocks), dim3(256), 0, st, (const float *)src,
                       (float *)dst, count);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_transpose(hipStream_t st, const void *src, int f64, int64_t rows, int64_t cols, void *dst) {
  dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
  if (f64)
    hipLaunchKernelGGL(k_transpose<double>, grid, dim3(256), 0, st, (const double *)src, rows, cols,
                       (double *)dst);
  else
    hipLaunchKernelGGL(k_transpose<float>, grid, dim3(256), 0, st, (const float *)src, rows, cols,
                       (float *)dst);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_fro2(hipStream_t st, const void *A, int dtype, int64_t m, int64_t n, int64_t lda, double *part,
                int nparts, double *out) {
  switch (dtype) {
    case DSK_F64:
      hipLaunchKernelGGL(k_fro2_part<DSK_F64>, dim3(nparts), dim3(256), 0, st, A, m, n, lda, part);
      break;
    case DSK_F32:
      hipLaunchKernelGGL(k_fro2_part<DSK_F32>, dim3(nparts), dim3(256), 0, st, A, m, n, lda, part);
      break;
    case DSK_BF16:
      hipLaunchKernelGGL(k_fro2_part<DSK_BF16>, dim3(nparts), dim3(256), 0, st, A, m, n, lda, part);
      break;
    default:
      hipLaunchKernelGGL(k_fro2_part<DSK_F16>, dim3(nparts), dim3(256), 0, st, A, m, n, lda, part);
  }
  DSK_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, part, nparts, out);
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_gather_cols16(hipStream_t st, const void *A, int64_t m, int64_t n, int64_t lda, const dsk_restriction *R,
                         int64_t s, void *out) {
  if (R->kind != DSK_R_INDEX || !R->index || m < 1 || s < 1 || n < 1 || m > 65535) return -1;
  const unsigned gx = (unsigned)std::min<int64_t>((s + 255) / 256, 64);
  hipLaunchKernelGGL(k_gather_cols16, dim3(gx, (unsigned)m), dim3(256), 0, st, (const unsigned short *)A, m, lda,
                     R->index, s, (unsigned short *)out);
  DSK_TRY(hipGetLastError());
  return 0;
}

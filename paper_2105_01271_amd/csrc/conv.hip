// Learned linear restriction (extension; not in the paper): A_c = A D with D
// two strided linear convolutions of every snapshot row, viewed as an
// ny x nx image (row-major, y-major flattening as everywhere in the library):
//
//   h[c, hy, hx] = sum_{ky,kx} w1[c, ky, kx] x[2 hy - 2 + ky, 2 hx - 2 + kx]     (ny/2 x nx/2, C channels)
//   y[oy, ox]    = sum_{c,ky,kx} w2[c, ky, kx] h[c, 2 oy - 2 + ky, 2 ox - 2 + kx]  (ny/4 x nx/4)
//
// 5x5 taps, stride 2, zero padding 2 on both layers, no bias, no activation,
// so the map stays linear and A_c = A D holds for the D it defines (Sec. 2).
//
// Forward: one workgroup per 16x16 tile of coarse outputs of one row.  The
// 73x73 input patch goes to LDS once; every thread keeps its 13x5 input
// window in registers and produces 5 hidden values per channel, channel by
// channel through a 35x35 LDS plane, so the hidden layer never leaves the CU.
// Backward (weight gradients of <gAc, conv(A)>): the same tiling recomputes
// the hidden plane, forms the hidden gradient of the tile's own outputs, and
// reduces both weight gradients inside the workgroup; per-workgroup partials
// are then summed in a fixed order in FP64.  FP32 arithmetic throughout.
#include <algorithm>

#include "dsk_internal.h"

namespace {

constexpr int KS = 5;
constexpr int TO = 16;               // coarse outputs per tile side
constexpr int TH = 2 * TO + 3;       // 35 hidden values per tile side
constexpr int TX = 2 * TH + 3;       // 73 input values per tile side
constexpr int CMAX = 32;
constexpr int NPART = 10;            // partial sums per tap in the backward reduction

template <typename T>
__device__ __forceinline__ float ld_in(const T *p) {
  if constexpr (sizeof(T) == 2) {
    const unsigned short b = *reinterpret_cast<const unsigned short *>(p);
    return bf16_bits_to_f32(b);
  } else {
    return (float)*p;
  }
}

template <typename T>
__device__ __forceinline__ float ld_in_f16(const T *p) {
  const unsigned short b = *reinterpret_cast<const unsigned short *>(p);
  return f16_bits_to_f32(b);
}

struct Tile {
  int cy, cx;           // coarse grid
  int hy, hx;           // hidden grid
  int oy0, ox0;         // tile origin (coarse)
};

__device__ __forceinline__ Tile tile_of(int ny, int nx) {
  Tile t;
  t.cy = ny / 4;
  t.cx = nx / 4;
  t.hy = ny / 2;
  t.hx = nx / 2;
  const int tiles_x = (t.cx + TO - 1) / TO;
  t.oy0 = (int)(blockIdx.x / tiles_x) * TO;
  t.ox0 = (int)(blockIdx.x % tiles_x) * TO;
  return t;
}

// 73x73 input patch with origin (4 oy0 - 6, 4 ox0 - 6), zero outside the grid
template <typename T, bool F16>
__device__ __forceinline__ void load_patch(const T *__restrict__ a, int ny, int nx, const Tile &tl, float *xs) {
  const int gy0 = 4 * tl.oy0 - 6, gx0 = 4 * tl.ox0 - 6;
  for (int e = threadIdx.x; e < TX * TX; e += 256) {
    const int r = e / TX, c = e - (e / TX) * TX;
    const int gy = gy0 + r, gx = gx0 + c;
    float v = 0.f;
    if (gy >= 0 && gy < ny && gx >= 0 && gx < nx) {
      const T *p = a + (int64_t)gy * nx + gx;
      v = F16 ? ld_in_f16(p) : ld_in(p);
    }
    xs[e] = v;
  }
}

// hidden plane of channel c for this thread's 5 positions (rows 5g..5g+4 of
// column j of the 35x35 tile plane); zero where the hidden position is padding
__device__ __forceinline__ void hidden5(const float (&xw)[13][5], const float *__restrict__ w1c, bool (&valid)[5],
                                        float (&h)[5]) {
  float w[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) w[k] = w1c[k];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float s = 0.f;
#pragma unroll
    for (int ky = 0; ky < KS; ++ky)
#pragma unroll
      for (int kx = 0; kx < KS; ++kx) s = fmaf(w[ky * KS + kx], xw[2 * i + ky][kx], s);
    h[i] = valid[i] ? s : 0.f;
  }
}

template <typename T, bool F16, typename TOUT>
__global__ void __launch_bounds__(256) k_conv_fwd(const T *__restrict__ A, int64_t lda, int ny, int nx, int C,
                                                  const float *__restrict__ w1, const float *__restrict__ w2,
                                                  TOUT *__restrict__ Ac, int64_t ldc) {
  __shared__ float xs[TX * TX];
  __shared__ float hs[TH * TH];
  const Tile tl = tile_of(ny, nx);
  const int t = threadIdx.x;
  load_patch<T, F16>(A + (int64_t)blockIdx.y * lda, ny, nx, tl, xs);
  __syncthreads();
  const bool act1 = t < 7 * TH;
  const int j = t % TH, g = t / TH;
  float xw[13][5];
  bool valid[5];
#pragma unroll
  for (int r = 0; r < 13; ++r)
#pragma unroll
    for (int c = 0; c < 5; ++c) xw[r][c] = act1 ? xs[(10 * g + r) * TX + 2 * j + c] : 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const int hy = 2 * tl.oy0 - 2 + 5 * g + i, hx = 2 * tl.ox0 - 2 + j;
    valid[i] = act1 && hy >= 0 && hy < tl.hy && hx >= 0 && hx < tl.hx;
  }
  const int oyl = t / TO, oxl = t % TO;
  float acc = 0.f;
  for (int c = 0; c < C; ++c) {
    float h[5];
    hidden5(xw, w1 + c * 25, valid, h);
    if (act1) {
#pragma unroll
      for (int i = 0; i < 5; ++i) hs[(5 * g + i) * TH + j] = h[i];
    }
    __syncthreads();
    const float *w2c = w2 + c * 25;
#pragma unroll
    for (int ky = 0; ky < KS; ++ky)
#pragma unroll
      for (int kx = 0; kx < KS; ++kx) acc = fmaf(w2c[ky * KS + kx], hs[(2 * oyl + ky) * TH + 2 * oxl + kx], acc);
    __syncthreads();
  }
  const int oy = tl.oy0 + oyl, ox = tl.ox0 + oxl;
  if (oy < tl.cy && ox < tl.cx) Ac[(int64_t)blockIdx.y * ldc + (int64_t)oy * tl.cx + ox] = (TOUT)acc;
}

// Weight gradients of <gAc, conv(A)>: per-workgroup partials (2 C 25 doubles:
// gw1 then gw2, channel-major).
template <typename T, bool F16, typename TG>
__global__ void __launch_bounds__(256) k_conv_bwd(const T *__restrict__ A, int64_t lda, int ny, int nx, int C,
                                                  const float *__restrict__ w1, const float *__restrict__ w2,
                                                  const TG *__restrict__ gAc, int64_t ldg,
                                                  double *__restrict__ part) {
  __shared__ float xs[TX * TX];
  __shared__ float hs[TH * TH];
  __shared__ float ghs[TH * TH];
  __shared__ float gys[TO * TO];
  __shared__ float red1[NPART][25], red2[NPART][25];
  __shared__ float acc1[CMAX * 25], acc2[CMAX * 25];
  const Tile tl = tile_of(ny, nx);
  const int t = threadIdx.x;
  load_patch<T, F16>(A + (int64_t)blockIdx.y * lda, ny, nx, tl, xs);
  {
    const int oyl = t / TO, oxl = t % TO, oy = tl.oy0 + oyl, ox = tl.ox0 + oxl;
    gys[t] = (oy < tl.cy && ox < tl.cx) ? (float)gAc[(int64_t)blockIdx.y * ldg + (int64_t)oy * tl.cx + ox] : 0.f;
  }
  for (int e = t; e < CMAX * 25; e += 256) {
    acc1[e] = 0.f;
    acc2[e] = 0.f;
  }
  __syncthreads();
  const bool act1 = t < 7 * TH;
  const int j = t % TH, g = t / TH;
  float xw[13][5];
  bool valid[5];
#pragma unroll
  for (int r = 0; r < 13; ++r)
#pragma unroll
    for (int c = 0; c < 5; ++c) xw[r][c] = act1 ? xs[(10 * g + r) * TX + 2 * j + c] : 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const int hy = 2 * tl.oy0 - 2 + 5 * g + i, hx = 2 * tl.ox0 - 2 + j;
    valid[i] = act1 && hy >= 0 && hy < tl.hy && hx >= 0 && hx < tl.hx;
  }
  const int k = t % 25, prt = t / 25;
  const int ky = k / KS, kx = k - (k / KS) * KS;
  for (int c = 0; c < C; ++c) {
    float h[5];
    hidden5(xw, w1 + c * 25, valid, h);
    const float *w2c = w2 + c * 25;
    if (act1) {
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        // hidden gradient of this tile's outputs: outputs o with 2 o + k = p
        const int py = 5 * g + i, px = j;
        float gh = 0.f;
#pragma unroll
        for (int a = 0; a < KS; ++a) {
          const int dy = py - a;
          if (dy < 0 || (dy & 1) || (dy >> 1) >= TO) continue;
#pragma unroll
          for (int b = 0; b < KS; ++b) {
            const int dx = px - b;
            if (dx < 0 || (dx & 1) || (dx >> 1) >= TO) continue;
            gh = fmaf(w2c[a * KS + b], gys[(dy >> 1) * TO + (dx >> 1)], gh);
          }
        }
        hs[py * TH + px] = h[i];
        ghs[py * TH + px] = valid[i] ? gh : 0.f;
      }
    }
    __syncthreads();
    if (prt < NPART) {
      float s2 = 0.f, s1 = 0.f;
      for (int o = prt; o < TO * TO; o += NPART)
        s2 = fmaf(gys[o], hs[(2 * (o / TO) + ky) * TH + 2 * (o % TO) + kx], s2);
      for (int p = prt; p < TH * TH; p += NPART)
        s1 = fmaf(ghs[p], xs[(2 * (p / TH) + ky) * TX + 2 * (p % TH) + kx], s1);
      red1[prt][k] = s1;
      red2[prt][k] = s2;
    }
    __syncthreads();
    if (t < 25) {
      float a1 = 0.f, a2 = 0.f;
      for (int q = 0; q < NPART; ++q) {
        a1 += red1[q][t];
        a2 += red2[q][t];
      }
      acc1[c * 25 + t] += a1;
      acc2[c * 25 + t] += a2;
    }
  }
  __syncthreads();
  double *pp = part + (int64_t)(blockIdx.y * gridDim.x + blockIdx.x) * (2 * C * 25);
  for (int e = t; e < C * 25; e += 256) {
    pp[e] = acc1[e];
    pp[C * 25 + e] = acc2[e];
  }
}

// gw[e] = sum over nblk partials (fixed order): one workgroup per weight.
__global__ void __launch_bounds__(256) k_conv_wreduce(const double *__restrict__ part, int64_t nblk, int nw,
                                                      float *__restrict__ gw1, float *__restrict__ gw2, int C) {
  __shared__ double red[256];
  const int e = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int64_t b = t; b < nblk; b += 256) s += part[b * nw + e];
  red[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) {
    if (e < C * 25) gw1[e] = (float)red[0];
    else gw2[e - C * 25] = (float)red[0];
  }
}

template <typename TOUT>
int conv_fwd_out(hipStream_t st, const void *A, int dtype, int64_t m, int64_t lda, int ny, int nx, int C,
                 const float *w1, const float *w2, TOUT *Ac, int64_t ldc) {
  const int cy = ny / 4, cx = nx / 4;
  dim3 grid((unsigned)(((cy + TO - 1) / TO) * ((cx + TO - 1) / TO)), (unsigned)m);
  switch (dtype) {
    case DSK_F64:
      hipLaunchKernelGGL((k_conv_fwd<double, false, TOUT>), grid, dim3(256), 0, st, (const double *)A, lda, ny, nx,
                         C, w1, w2, Ac, ldc);
      break;
    case DSK_F32:
      hipLaunchKernelGGL((k_conv_fwd<float, false, TOUT>), grid, dim3(256), 0, st, (const float *)A, lda, ny, nx,
                         C, w1, w2, Ac, ldc);
      break;
    case DSK_BF16:
      hipLaunchKernelGGL((k_conv_fwd<unsigned short, false, TOUT>), grid, dim3(256), 0, st,
                         (const unsigned short *)A, lda, ny, nx, C, w1, w2, Ac, ldc);
      break;
    default:
      hipLaunchKernelGGL((k_conv_fwd<unsigned short, true, TOUT>), grid, dim3(256), 0, st,
                         (const unsigned short *)A, lda, ny, nx, C, w1, w2, Ac, ldc);
      break;
  }
  DSK_TRY(hipGetLastError());
  return 0;
}

template <typename TG>
int conv_bwd_g(hipStream_t st, const void *A, int dtype, int64_t m, int64_t lda, int ny, int nx, int C,
               const float *w1, const float *w2, const TG *gAc, int64_t ldg, double *part) {
  const int cy = ny / 4, cx = nx / 4;
  dim3 grid((unsigned)(((cy + TO - 1) / TO) * ((cx + TO - 1) / TO)), (unsigned)m);
  switch (dtype) {
    case DSK_F64:
      hipLaunchKernelGGL((k_conv_bwd<double, false, TG>), grid, dim3(256), 0, st, (const double *)A, lda, ny, nx, C,
                         w1, w2, gAc, ldg, part);
      break;
    case DSK_F32:
      hipLaunchKernelGGL((k_conv_bwd<float, false, TG>), grid, dim3(256), 0, st, (const float *)A, lda, ny, nx, C,
                         w1, w2, gAc, ldg, part);
      break;
    case DSK_BF16:
      hipLaunchKernelGGL((k_conv_bwd<unsigned short, false, TG>), grid, dim3(256), 0, st,
                         (const unsigned short *)A, lda, ny, nx, C, w1, w2, gAc, ldg, part);
      break;
    default:
      hipLaunchKernelGGL((k_conv_bwd<unsigned short, true, TG>), grid, dim3(256), 0, st,
                         (const unsigned short *)A, lda, ny, nx, C, w1, w2, gAc, ldg, part);
      break;
  }
  DSK_TRY(hipGetLastError());
  return 0;
}

}  // namespace

int conv_shape_ok(int64_t n, int ny, int nx, int C) {
  return ny >= 4 && nx >= 4 && (ny % 4) == 0 && (nx % 4) == 0 && (int64_t)ny * nx == n && C >= 1 && C <= CMAX;
}

int launch_conv_fwd(hipStream_t st, const void *A, int dtype, int64_t m, int64_t lda, int ny, int nx, int C,
                    const float *w1, const float *w2, int out_f64, void *Ac, int64_t ldc) {
  if (out_f64) return conv_fwd_out<double>(st, A, dtype, m, lda, ny, nx, C, w1, w2, (double *)Ac, ldc);
  return conv_fwd_out<float>(st, A, dtype, m, lda, ny, nx, C, w1, w2, (float *)Ac, ldc);
}

size_t conv_bwd_ws_bytes(int64_t m, int ny, int nx, int C) {
  const int cy = ny / 4, cx = nx / 4;
  const int64_t nblk = (int64_t)((cy + TO - 1) / TO) * ((cx + TO - 1) / TO) * m;
  return (size_t)nblk * 2 * C * 25 * sizeof(double);
}

int launch_conv_bwd(hipStream_t st, const void *A, int dtype, int64_t m, int64_t lda, int ny, int nx, int C,
                    const float *w1, const float *w2, const void *gAc, int g_f64, int64_t ldg, float *gw1,
                    float *gw2, void *ws) {
  double *part = reinterpret_cast<double *>(ws);
  if (g_f64) DSK_RET(conv_bwd_g<double>(st, A, dtype, m, lda, ny, nx, C, w1, w2, (const double *)gAc, ldg, part));
  else DSK_RET(conv_bwd_g<float>(st, A, dtype, m, lda, ny, nx, C, w1, w2, (const float *)gAc, ldg, part));
  const int cy = ny / 4, cx = nx / 4;
  const int64_t nblk = (int64_t)((cy + TO - 1) / TO) * ((cx + TO - 1) / TO) * m;
  hipLaunchKernelGGL(k_conv_wreduce, dim3(2 * C * 25), dim3(256), 0, st, (const double *)part, nblk, 2 * C * 25,
                     gw1, gw2, C);
  DSK_TRY(hipGetLastError());
  return 0;
}

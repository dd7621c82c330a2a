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
// Forward: the two layers composed into one 13x13 stride-4 filter per border
// class (below), applied from an LDS tile of the input.
// Backward (weight gradients of <gAc, conv(A)>): one workgroup per 16x16 tile
// of coarse outputs of one row; the 73x73 input patch goes to LDS once, every
// thread keeps its 13x5 input window in registers and recomputes 5 hidden
// values per channel, channel by channel through a 35x35 LDS plane (the hidden
// layer never leaves the CU), forms the hidden gradient of the tile's own outputs, and
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


// Weight gradients of <gAc, conv(A)>: per-workgroup partials (2 C 25 doubles:
// gw1 then gw2, channel-major).
// ---- forward by the composed filter.  Both layers are linear, so
//   y[oy, ox] = sum_{dy, dx < 13} F[dy, dx] x[4 oy - 6 + dy, 4 ox - 6 + dx],
//   F[dy, dx] = sum_c sum_{2a + b = dy, 2a' + b' = dx} w2[c, a, a'] w1[c, b, b'],
// (a = second-layer tap, b = first-layer tap), except that the hidden layer's
// zero padding removes the second-layer taps whose hidden position lies
// outside the hidden grid: a < 2 for oy = 0, a = 4 for oy = cy - 1 (likewise
// in x).  Each output takes the filter of its border class (y class: bit 0
// first row, bit 1 last row; x likewise), 16 filters of 13 x 13 composed in
// FP64 once per call.  169 multiply-adds per output instead of the layers'
// 25 C + 25 per hidden value times 25 hidden values: the pass reads A once and
// is bound by HBM, not by the vector units.
constexpr int FK = 13;               // composed filter side
constexpr int FN = FK * FK;
constexpr int NCLS = 16;
constexpr int EY = 8;                // coarse rows per tile (two per thread)
constexpr int EX = 64;               // coarse columns per tile (one per lane)
constexpr int PRW = 4 * EY + 9;      // 41 patch rows
constexpr int PCL = 4 * EX + 12;     // 268 patch columns, origin 4 ox0 - 8 (a multiple of 4)
constexpr int PPL = PCL / 4 + 1;     // entries per column-phase plane

__global__ void __launch_bounds__(256) k_conv_compose(const float *__restrict__ w1, const float *__restrict__ w2,
                                                      int C, float *__restrict__ F) {
  __shared__ float ws1[CMAX * 25], ws2[CMAX * 25];
  for (int e = threadIdx.x; e < C * 25; e += 256) {
    ws1[e] = w1[e];
    ws2[e] = w2[e];
  }
  __syncthreads();
  const int cls = blockIdx.x;
  const int cly = cls >> 2, clx = cls & 3;
  const int ay0 = (cly & 1) ? 2 : 0, ay1 = (cly & 2) ? 3 : 4;
  const int ax0 = (clx & 1) ? 2 : 0, ax1 = (clx & 2) ? 3 : 4;
  for (int e = threadIdx.x; e < FN; e += 256) {
    const int dy = e / FK, dx = e - (e / FK) * FK;
    double acc = 0.0;
    for (int a = ay0; a <= ay1; ++a) {
      const int b = dy - 2 * a;
      if (b < 0 || b >= KS) continue;
      for (int a2 = ax0; a2 <= ax1; ++a2) {
        const int b2 = dx - 2 * a2;
        if (b2 < 0 || b2 >= KS) continue;
        const int o2 = a * KS + a2, o1 = b * KS + b2;
        for (int c = 0; c < C; ++c) acc += (double)ws2[c * 25 + o2] * (double)ws1[c * 25 + o1];
      }
    }
    F[cls * FN + e] = (float)acc;
  }
}

// One workgroup per 8 x 64 tile of coarse outputs of one row of A.  The 41 x 268
// input patch goes to LDS split into four column-phase planes (patch column c
// at plane c & 3, entry c >> 2), so that the 64 lanes, one coarse column each,
// read consecutive LDS words for every tap despite the stride-4 filter.  Each
// thread produces two vertically adjacent outputs (their 13-row windows share
// 9 rows).
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef double f64x4v __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4v __attribute__((ext_vector_type(4)));
template <typename T>
struct Vec4 { using type = f32x4v; };
template <> struct Vec4<double> { using type = f64x4v; };
template <> struct Vec4<unsigned short> { using type = u16x4v; };

template <typename T, bool F16>
__device__ __forceinline__ float cvt_in(T v) {
  if constexpr (sizeof(T) == 2) return F16 ? f16_bits_to_f32(v) : bf16_bits_to_f32(v);
  else return (float)v;
}

// The patch in groups of four columns (group g = columns 4g..4g+3, one per
// phase plane): nx and the patch origin are multiples of 4, so a group is all
// inside the grid or all outside.  Addresses are clamped into the grid and
// outside groups zeroed, so the loads are unconditional and independent.
// VEC: one 4-element vector load per group (row starts aligned to 4 elements).
constexpr int PGR = PCL / 4;                       // 67 groups per patch row
constexpr int NGRP = PRW * PGR;                    // groups per patch
constexpr int GPT = (NGRP + 255) / 256;            // groups per thread
template <typename T, bool F16, typename TOUT, bool VEC>
__global__ void __launch_bounds__(256) k_conv_eff(const T *__restrict__ A, int64_t lda, int ny, int nx,
                                                  const float *__restrict__ F, TOUT *__restrict__ Ac, int64_t ldc) {
  __shared__ float xs[PRW * 4 * PPL];
  __shared__ float fs[NCLS * FN];
  const int t = threadIdx.x;
  const int cy = ny / 4, cx = nx / 4;
  const int tiles_x = (cx + EX - 1) / EX;
  const int oy0 = (int)(blockIdx.x / tiles_x) * EY, ox0 = (int)(blockIdx.x % tiles_x) * EX;
  const T *a = A + (int64_t)blockIdx.y * lda;
  const int gy0 = 4 * oy0 - 6, gx0 = 4 * ox0 - 8;
  float v[GPT][4];
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const int g = t + 256 * i;
    const int r = g / PGR, q = g - (g / PGR) * PGR;
    const int gy = gy0 + r, gx = gx0 + 4 * q;
    const bool ok = g < NGRP && gy >= 0 && gy < ny && gx >= 0 && gx < nx;
    const int gyc = min(max(gy, 0), ny - 1), gxc = min(max(gx, 0), nx - 4);
    const T *p = a + (int64_t)gyc * nx + gxc;
    if constexpr (VEC) {
      const typename Vec4<T>::type u = *reinterpret_cast<const typename Vec4<T>::type *>(p);
#pragma unroll
      for (int k = 0; k < 4; ++k) v[i][k] = cvt_in<T, F16>(u[k]);
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) v[i][u] = cvt_in<T, F16>(p[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) v[i][u] = ok ? v[i][u] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const int g = t + 256 * i;
    if (g < NGRP) {
      const int r = g / PGR, q = g - (g / PGR) * PGR;
#pragma unroll
      for (int u = 0; u < 4; ++u) xs[(r * 4 + u) * PPL + q] = v[i][u];
    }
  }
  for (int e = t; e < NCLS * FN; e += 256) fs[e] = F[e];
  __syncthreads();
  const int lane = t & 63, w = t >> 6;
  const int ox = ox0 + lane;
  const int clx = (ox == 0 ? 1 : 0) | (ox == cx - 1 ? 2 : 0);
  int fo[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int oy = oy0 + 2 * w + j;
    const int cly = (oy == 0 ? 1 : 0) | (oy == cy - 1 ? 2 : 0);
    fo[j] = (cly * 4 + clx) * FN;
  }
  float acc0 = 0.f, acc1 = 0.f;
  // output row 2w + j, tap dy: patch row 8w + r with r = 4j + dy (the branches
  // on r are uniform; the row loop stays rolled to keep the registers few)
#pragma unroll 1
  for (int r = 0; r < 4 + FK; ++r) {
    const float *xr = xs + (8 * w + r) * 4 * PPL + lane;
    float xv[FK];
#pragma unroll
    for (int dx = 0; dx < FK; ++dx) {
      const int c = 2 + dx;   // patch column 4 lane + 2 + dx
      xv[dx] = xr[(c & 3) * PPL + (c >> 2)];
    }
    if (r < FK) {
      const float *wr = fs + fo[0] + r * FK;
#pragma unroll
      for (int dx = 0; dx < FK; ++dx) acc0 = fmaf(wr[dx], xv[dx], acc0);
    }
    if (r >= 4) {
      const float *wr = fs + fo[1] + (r - 4) * FK;
#pragma unroll
      for (int dx = 0; dx < FK; ++dx) acc1 = fmaf(wr[dx], xv[dx], acc1);
    }
  }
  const float acc[2] = {acc0, acc1};
  if (ox < cx) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int oy = oy0 + 2 * w + j;
      if (oy < cy) Ac[(int64_t)blockIdx.y * ldc + (int64_t)oy * cx + ox] = (TOUT)acc[j];
    }
  }
}

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

template <typename T, bool F16, typename TOUT>
void conv_eff_launch(hipStream_t st, dim3 grid, const void *A, int64_t lda, int ny, int nx, const float *F, TOUT *Ac,
                     int64_t ldc) {
  const bool vec = (lda % 4) == 0 && (reinterpret_cast<uintptr_t>(A) % (4 * sizeof(T))) == 0;
  if (vec)
    hipLaunchKernelGGL((k_conv_eff<T, F16, TOUT, true>), grid, dim3(256), 0, st, (const T *)A, lda, ny, nx, F, Ac,
                       ldc);
  else
    hipLaunchKernelGGL((k_conv_eff<T, F16, TOUT, false>), grid, dim3(256), 0, st, (const T *)A, lda, ny, nx, F, Ac,
                       ldc);
}

template <typename TOUT>
int conv_fwd_out(hipStream_t st, const void *A, int dtype, int64_t m, int64_t lda, int ny, int nx, int C,
                 const float *w1, const float *w2, TOUT *Ac, int64_t ldc, float *F) {
  hipLaunchKernelGGL(k_conv_compose, dim3(NCLS), dim3(256), 0, st, w1, w2, C, F);
  const int cy = ny / 4, cx = nx / 4;
  dim3 grid((unsigned)(((cy + EY - 1) / EY) * ((cx + EX - 1) / EX)), (unsigned)m);
  switch (dtype) {
    case DSK_F64: conv_eff_launch<double, false, TOUT>(st, grid, A, lda, ny, nx, F, Ac, ldc); break;
    case DSK_F32: conv_eff_launch<float, false, TOUT>(st, grid, A, lda, ny, nx, F, Ac, ldc); break;
    case DSK_BF16: conv_eff_launch<unsigned short, false, TOUT>(st, grid, A, lda, ny, nx, F, Ac, ldc); break;
    default: conv_eff_launch<unsigned short, true, TOUT>(st, grid, A, lda, ny, nx, F, Ac, ldc);
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
                    const float *w1, const float *w2, int out_f64, void *Ac, int64_t ldc, float *filt_ws) {
  static_assert(NCLS * FN * sizeof(float) <= CONV_FILTER_BYTES, "composed filters exceed their workspace");
  if (m > 65535) return -1;
  if (out_f64) return conv_fwd_out<double>(st, A, dtype, m, lda, ny, nx, C, w1, w2, (double *)Ac, ldc, filt_ws);
  return conv_fwd_out<float>(st, A, dtype, m, lda, ny, nx, C, w1, w2, (float *)Ac, ldc, filt_ws);
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

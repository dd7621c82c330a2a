// Tall-skinny products of the sketch pipeline:
//   TN form  out (N x ell) = X^T Y,  X is K x N row-major  (B^T = A^T Q, Eq. for B in
//            Sec. 3.1 / Alg. 2; Z = A_c^T Q of Alg. 7)
//   NN form  out (M x ell) = X Y,    X is M x K row-major  (A_c Z of Alg. 7; A_c S)
// Y is K x ell row-major.  The TN form with X = A is the single full pass over
// the snapshot matrix and dominates the memory traffic of the method (its
// leading mnn_c cost, Sec. 5 complexity table).
//
// MFMA path (f32 / bf16 / f16 storage of X):
//   * A wave owns JT 16-wide column tiles of the output rows (j) and all
//     NCT 16-wide tiles of ell (c).  D[c][j] += Y^T[c][k] X[k][j] on the
//     16x16 MFMA shapes; lane l handles k = k0 + 8*(l/16) + e, e = 0..7, for
//     both operands, so the K order inside one instruction is the same for A
//     and B and the lane layout of K never matters.
//   * Y is packed once per call into that lane order (NV x uint4 per lane per
//     (32-row block, c tile)) so each wave reads it with 16-byte loads.
//   * SPLIT6 mode (default for f32): every f32 value is split exactly into
//     three bf16 pieces x = x1 + x2 + x3 (RNE, each remainder exact in f32);
//     the product keeps the six terms y_i x_j with i + j <= 4, each exact on
//     the bf16 MFMA pipe, so the dropped terms are ~2^-24 relative: f32
//     rounding level with f32 accumulation.
//   * SPLIT3 mode: two pieces, Yhi*Xhi + Yhi*Xlo + Ylo*Xhi (dropped terms
//     ~2^-16 relative).  F32 mode uses the f32 MFMA (16x16x4) directly.
//     Stored bf16/f16 X needs no split: Yhi*X + Ylo*X.
//   * The 4 waves of a workgroup share the same output tile and take every
//     4th 32-row block of the K range; their accumulators are reduced in LDS
//     in a fixed order (deterministic).  Small N is split over K across
//     workgroups (grid.y) and summed by a second kernel in a fixed order.
//   * TN form with 16-bit X (the BF16 / F16 snapshots, B^T = A^T Q): a
//     workgroup owns W = 128 output rows j and sweeps K in 32-row chunks.  A
//     chunk (32 x W values) arrives by row-contiguous 16-byte loads
//     (prefetched three chunks ahead), goes to a double-buffered,
//     bank-swizzled LDS tile (one barrier per chunk) and is
//     read back k-contiguous by the transposing LDS read ds_read_b64_tr_b16
//     (two per 32 x 16 operand); wave w owns the ell tiles
//     (w + blockIdx) mod 4 + 4 i and all W / 16 j tiles, so each packed Y
//     operand is read once per workgroup and chunk.
// FP64 path: VALU kernel with LDS tiles (f64 FMA), same TN/NN forms.
#include <algorithm>
#include <type_traits>

#include <map>
#include <tuple>

#include "dsk_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MODE_SPLIT3 = 1;
constexpr int MODE_F32 = 2;
constexpr int MODE_BF16X = 3;   // X stored bf16, Y split hi/lo
constexpr int MODE_F16X = 4;    // X stored f16, Y split hi/lo (f16)
constexpr int MODE_SPLIT6 = 5;  // f32 X and Y in three bf16 pieces each

template <int MODE>
constexpr int nv_of() { return MODE == MODE_SPLIT6 ? 3 : 2; }

// ---------------------------------------------------------------- Y packing
// Yp[((kb*nct + ct)*NV + v)*64 + lane] : uint4
//   SPLIT6:       v=0,1,2 -> 8 bf16 pieces y1, y2, y3
//   SPLIT3/BF16X: v=0 -> 8 bf16 hi, v=1 -> 8 bf16 lo
//   F16X:         v=0 -> 8 f16 hi,  v=1 -> 8 f16 lo
//   F32:          v=0 -> floats e=0..3, v=1 -> floats e=4..7
// with element e of lane l holding Y[kb*32 + 8*(l/16) + e][ct*16 + l%16] (0 outside).
template <int MODE, typename TY>
__global__ void __launch_bounds__(64) k_pack_y(const TY *__restrict__ Y, int64_t K, int ell,
                                               int64_t ldy, int nct, uint4 *__restrict__ Yp) {
  const int kb = blockIdx.x, ct = blockIdx.y, l = threadIdx.x;
  const int c = ct * 16 + (l & 15);
  float v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t k = (int64_t)kb * 32 + 8 * (l >> 4) + e;
    v[e] = (k < K && c < ell) ? (float)Y[k * ldy + c] : 0.0f;
  }
  constexpr int NV = nv_of<MODE>();
  uint4 *dst = Yp + ((int64_t)(kb * nct + ct) * NV) * 64 + l;
  if constexpr (MODE == MODE_SPLIT6) {
    bf16x8 p1, p2, p3;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const __bf16 a1 = (__bf16)v[e];
      const float r1 = v[e] - (float)a1;
      const __bf16 a2 = (__bf16)r1;
      const float r2 = r1 - (float)a2;
      p1[e] = a1;
      p2[e] = a2;
      p3[e] = (__bf16)r2;
    }
    dst[0] = __builtin_bit_cast(uint4, p1);
    dst[64] = __builtin_bit_cast(uint4, p2);
    dst[128] = __builtin_bit_cast(uint4, p3);
  } else if constexpr (MODE == MODE_F32) {
    dst[0] = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]), __float_as_uint(v[3]));
    dst[64] = make_uint4(__float_as_uint(v[4]), __float_as_uint(v[5]), __float_as_uint(v[6]), __float_as_uint(v[7]));
  } else if constexpr (MODE == MODE_F16X) {
    f16x8 hi, lo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const _Float16 h = (_Float16)v[e];
      hi[e] = h;
      lo[e] = (_Float16)(v[e] - (float)h);
    }
    dst[0] = __builtin_bit_cast(uint4, hi);
    dst[64] = __builtin_bit_cast(uint4, lo);
  } else {
    bf16x8 hi, lo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const __bf16 h = (__bf16)v[e];
      hi[e] = h;
      lo[e] = (__bf16)(v[e] - (float)h);
    }
    dst[0] = __builtin_bit_cast(uint4, hi);
    dst[64] = __builtin_bit_cast(uint4, lo);
  }
}

// ---------------------------------------------------------------- X fragment loads
// Raw 8 K-values of one output column j for this lane, as 32-bit floats or
// 16-bit patterns.  TN: X[k][j] (k strided by ldx).  NN: X[j][k] (contiguous).
template <bool NN>
__device__ __forceinline__ void load_x_f32(const float *__restrict__ X, int64_t K, int64_t N, int64_t ldx,
                                           int64_t kbase, int64_t j, float (&x)[8]) {
  if (j >= N) {
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = 0.0f;
    return;
  }
  if constexpr (NN) {
    const float *p = X + j * ldx + kbase;
    if (kbase + 8 <= K && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
      const float4 a = *reinterpret_cast<const float4 *>(p);
      const float4 b = *reinterpret_cast<const float4 *>(p + 4);
      x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
      x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (kbase + e < K) ? p[e] : 0.0f;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = (kbase + e < K) ? X[(kbase + e) * ldx + j] : 0.0f;
  }
}

template <bool NN>
__device__ __forceinline__ void load_x_u16(const unsigned short *__restrict__ X, int64_t K, int64_t N,
                                           int64_t ldx, int64_t kbase, int64_t j, unsigned short (&x)[8]) {
  if (j >= N) {
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = 0;
    return;
  }
  if constexpr (NN) {
    const unsigned short *p = X + j * ldx + kbase;
    if (kbase + 8 <= K && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
      const uint4 a = *reinterpret_cast<const uint4 *>(p);
      const unsigned w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        x[2 * e] = (unsigned short)(w[e] & 0xffffu);
        x[2 * e + 1] = (unsigned short)(w[e] >> 16);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (kbase + e < K) ? p[e] : (unsigned short)0;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = (kbase + e < K) ? X[(kbase + e) * ldx + j] : (unsigned short)0;
  }
}

__device__ __forceinline__ f32x4 mfma_bf16(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                 c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f16(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                0, 0, 0);
}

// ---------------------------------------------------------------- TN kernel for 16-bit X
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// ds_read_b64_tr_b16: in each aligned group of 16 lanes, lane i points at 4
// consecutive 16-bit values (row i / 4, columns 4 (i % 4) .. + 3 of a 4 x 16
// block); lane j receives column j of the block, rows 0 .. 3.
__device__ __forceinline__ uint2 lds_read_tr16(const unsigned short *p) {
  const i16x4 r = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) i16x4 *)p);
  return __builtin_bit_cast(uint2, r);
}

// Output rows (columns of X) per workgroup.  (256 would halve the packed-Y
// traffic per byte of X, but its 2 x 16 accumulator tiles per wave leave one
// wave per SIMD, too few loads in flight.)
constexpr int TN16_W = 128;

// LDS tile of a chunk: 32 rows of W 16-bit values, no padding; the 16-byte
// unit u of row r sits at unit u ^ swz(r).  A transposing read of a 16-lane
// group touches rows r0 .. r0 + 3 (units 2 jt, 2 jt + 1), the other group of
// its half-wave rows r0 + 8 .. r0 + 11: with swz(r) = 2 ((r & 3) | ((r >> 3 & 1) << 2))
// those 16 units land on 16 different 4-bank slots, so every read is free of
// bank conflicts; a 16-byte store stays contiguous.
__device__ __forceinline__ int tn16_swz(int r) { return 2 * ((r & 3) | (((r >> 3) & 1) << 2)); }

// VEC: X 16-byte aligned, ldx and N multiples of 8 (every 8-column group of a
// row is one 16-byte load, wholly inside or wholly outside [0, N)).  Loads are
// issued unconditionally (rows past K read row K - 1, groups past N read
// columns 0 .. 7, prefetches past the range re-read the last chunk, an L2
// hit), so the number of loads in flight is the same on every path and the
// waits on them stay partial.
template <int MODE, int NCT, bool VEC, int W>
__global__ void __launch_bounds__(256) k_stream_tn16(const unsigned short *__restrict__ X, int64_t K, int64_t N,
                                                     int64_t ldx, const uint4 *__restrict__ Yp, int ell,
                                                     float *__restrict__ out, int64_t ldo, int kb_per_split) {
  constexpr int UPR = W / 8;                   // 16-byte units per row
  constexpr int RPS = 256 / UPR;               // rows one pass of the 256 threads covers
  constexpr int NL = 32 / RPS;                 // 16-byte loads per thread and chunk
  constexpr int NJT = W / 16;                  // j tiles
  constexpr int NCW = (NCT + 3) / 4;           // ell tiles per wave
  constexpr int XD = W == 128 ? 3 : 2;         // chunks fetched ahead
  __shared__ __attribute__((aligned(16))) unsigned short xs[2][32][W];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4, i = lane & 15;
  const int nkb = (int)((K + 31) / 32);
  const int kb_begin = blockIdx.y * kb_per_split;
  const int kb_end = min(nkb, kb_begin + kb_per_split);
  const int64_t j0 = (int64_t)blockIdx.x * W;
  const int wsh = (wave + (int)blockIdx.x) & 3;   // rotates the lighter wave over the SIMDs
  // loads: thread t fetches rows t / UPR + RPS q of the chunk, columns 8 (t % UPR) .. + 7
  const int lr = t / UPR, lu = t % UPR;
  const int64_t gj = j0 + 8 * lu;
  const int64_t gjc = gj < N ? gj : 0;              // VEC: the whole 8-column group is inside or outside
  // (16-byte values as a native vector type: a struct copy from global memory
  // would become a memcpy that keeps the prefetch slots out of registers)
  auto gload = [&](int kb, u32x4 (&v)[NL]) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int64_t r = (int64_t)kb * 32 + lr + RPS * q;
      if constexpr (VEC) {
        v[q] = *reinterpret_cast<const u32x4 *>(X + (r < K ? r : K - 1) * ldx + gjc);
      } else {
        unsigned e[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) e[c] = (r < K && gj + c < N) ? X[r * ldx + gj + c] : 0u;
        v[q] = u32x4{e[0] | (e[1] << 16), e[2] | (e[3] << 16), e[4] | (e[5] << 16), e[6] | (e[7] << 16)};
      }
    }
  };
  // (a wave with one ell tile also loads a second, clamped one, unused: loads stay unconditional)
  auto yload = [&](int kb, uint4 (&ya)[NCW], uint4 (&yb)[NCW]) {
#pragma unroll
    for (int cw = 0; cw < NCW; ++cw) {
      const int ct = min(wsh + 4 * cw, NCT - 1);
      const uint4 *src = Yp + ((int64_t)(kb * NCT + ct) * 2) * 64 + lane;
      ya[cw] = src[0];
      yb[cw] = src[64];
    }
  };
  f32x4 acc[NCW][NJT];
#pragma unroll
  for (int cw = 0; cw < NCW; ++cw)
#pragma unroll
    for (int jt = 0; jt < NJT; ++jt) acc[cw][jt] = f32x4{0.f, 0.f, 0.f, 0.f};
  // X chunks are fetched XD chunks ahead and the packed Y one chunk ahead; Y's
  // loads go out before X's, so that waiting for Y (loads complete in issue
  // order) leaves the later X fetches in flight
  u32x4 v[XD][NL];
  uint4 ya[2][NCW], yb[2][NCW];
  if (kb_begin >= kb_end) return;
  const int kb_last = kb_end - 1;
  yload(kb_begin, ya[0], yb[0]);
#pragma unroll
  for (int s = 0; s < XD; ++s) gload(min(kb_begin + s, kb_last), v[s]);
  int buf = 0;
  // one chunk; S (a compile-time constant) picks the X slot S mod XD and the Y slot S mod 2
  auto step = [&](int kb, auto SC) {
    constexpr int S = decltype(SC)::value, sx = S % XD, sy = S & 1;
    // LDS copy of the fetched chunk.  VEC stores what it read: a row past K (a
    // copy of row K - 1) meets packed-Y rows that are zero, a group past N (a
    // copy of columns 0 .. 7) feeds output rows that are never stored.
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int r = lr + RPS * q;
      *reinterpret_cast<u32x4 *>(&xs[buf][r][8 * (lu ^ tn16_swz(r))]) = v[sx][q];
    }
    __syncthreads();   // (also: every wave is done with this buffer's previous chunk)
    yload(min(kb + 1, kb_last), ya[sy ^ 1], yb[sy ^ 1]);
    gload(min(kb + XD, kb_last), v[sx]);
#pragma unroll
    for (int jt = 0; jt < NJT; ++jt) {
      // rows 8 g .. 8 g + 7 of column 16 jt + i: two 4 x 16 blocks, lane i of the group
      // at row r = 8 g + i / 4 (+ 4), columns 16 jt + 4 (i % 4): unit 2 jt + (i % 4) / 2
      const int r0 = 8 * g + (i >> 2), r1 = r0 + 4, u = 2 * jt + ((i & 3) >> 1), h = 4 * (i & 1);
      const uint2 lo = lds_read_tr16(&xs[buf][r0][8 * (u ^ tn16_swz(r0)) + h]);
      const uint2 hi = lds_read_tr16(&xs[buf][r1][8 * (u ^ tn16_swz(r1)) + h]);
      const uint4 xop = make_uint4(lo.x, lo.y, hi.x, hi.y);
#pragma unroll
      for (int cw = 0; cw < NCW; ++cw) {
        if (wsh + 4 * cw >= NCT) continue;
        if constexpr (MODE == MODE_BF16X) {
          acc[cw][jt] = mfma_bf16(ya[sy][cw], xop, acc[cw][jt]);
          acc[cw][jt] = mfma_bf16(yb[sy][cw], xop, acc[cw][jt]);
        } else {
          acc[cw][jt] = mfma_f16(ya[sy][cw], xop, acc[cw][jt]);
          acc[cw][jt] = mfma_f16(yb[sy][cw], xop, acc[cw][jt]);
        }
      }
    }
    buf ^= 1;
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  using I4 = std::integral_constant<int, 4>;
  using I5 = std::integral_constant<int, 5>;
  static_assert(6 % XD == 0, "six steps cover the X and Y slot cycles");
  int kb = kb_begin;
  for (; kb + 6 <= kb_end; kb += 6) {
    step(kb, I0{});
    step(kb + 1, I1{});
    step(kb + 2, I2{});
    step(kb + 3, I3{});
    step(kb + 4, I4{});
    step(kb + 5, I5{});
  }
  if (kb < kb_end) step(kb, I0{});
  if (kb + 1 < kb_end) step(kb + 1, I1{});
  if (kb + 2 < kb_end) step(kb + 2, I2{});
  if (kb + 3 < kb_end) step(kb + 3, I3{});
  if (kb + 4 < kb_end) step(kb + 4, I4{});
  float *dst = out + (int64_t)blockIdx.y * N * ldo;
#pragma unroll
  for (int cw = 0; cw < NCW; ++cw) {
    const int ct = wsh + 4 * cw;
    if (ct >= NCT) continue;
    const int c0 = ct * 16 + 4 * g;
#pragma unroll
    for (int jt = 0; jt < NJT; ++jt) {
      const int64_t j = j0 + 16 * jt + i;
      if (j >= N) continue;
      const f32x4 a = acc[cw][jt];
      float *p = dst + j * ldo + c0;
      if (c0 + 3 < ell && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
        *reinterpret_cast<float4 *>(p) = make_float4(a[0], a[1], a[2], a[3]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (c0 + r < ell) p[r] = a[r];
      }
    }
  }
}

// ---------------------------------------------------------------- MFMA stream kernel
// grid: x = ceil(N / (16*JT)) column groups, y = K splits.  block: 256 (4 waves).
// Split y covers 32-row blocks [y*kb_per_split, min(nkb, (y+1)*kb_per_split)).
// Output: out[j*ldo + c] (+ split*N*ldo when nsplit > 1, written to `out` as partials).
template <int MODE, bool NN, int NCT, int JT>
__global__ void __launch_bounds__(256) k_stream_mfma(const void *__restrict__ Xv, int64_t K, int64_t N,
                                                     int64_t ldx, const uint4 *__restrict__ Yp, int ell,
                                                     float *__restrict__ out, int64_t ldo, int kb_per_split) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, col = lane & 15;
  const int nkb = (int)((K + 31) / 32);
  const int kb_begin = blockIdx.y * kb_per_split;
  const int kb_end = min(nkb, kb_begin + kb_per_split);
  const int64_t j0 = (int64_t)blockIdx.x * (16 * JT);

  f32x4 acc[NCT][JT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) acc[ct][jt] = f32x4{0.f, 0.f, 0.f, 0.f};

  constexpr int NV = nv_of<MODE>();
  constexpr bool XF32 = MODE == MODE_SPLIT3 || MODE == MODE_F32 || MODE == MODE_SPLIT6;
  // software pipeline: the X fragment of the next k-block this wave handles is
  // loaded into registers before the current one is consumed
  float xn32[XF32 ? JT : 1][8];
  unsigned short xn16[XF32 ? 1 : JT][8];
  auto fetch = [&](int kb) {
    const int64_t kb0 = (int64_t)kb * 32 + 8 * g;
    if constexpr (XF32) {
#pragma unroll
      for (int jt = 0; jt < JT; ++jt)
        load_x_f32<NN>(reinterpret_cast<const float *>(Xv), K, N, ldx, kb0, j0 + 16 * jt + col, xn32[jt]);
    } else {
#pragma unroll
      for (int jt = 0; jt < JT; ++jt)
        load_x_u16<NN>(reinterpret_cast<const unsigned short *>(Xv), K, N, ldx, kb0, j0 + 16 * jt + col, xn16[jt]);
    }
  };
  if (kb_begin + wave < kb_end) fetch(kb_begin + wave);
  for (int kb = kb_begin + wave; kb < kb_end; kb += 4) {
    uint4 ya[NCT], yb[NCT], yc[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const uint4 *src = Yp + ((int64_t)(kb * NCT + ct) * NV) * 64 + lane;
      ya[ct] = src[0];
      yb[ct] = src[64];
      if constexpr (NV == 3) yc[ct] = src[128];
    }
    if constexpr (XF32) {
      float xv[JT][8];
#pragma unroll
      for (int jt = 0; jt < JT; ++jt)
#pragma unroll
        for (int e = 0; e < 8; ++e) xv[jt][e] = xn32[jt][e];
      if (kb + 4 < kb_end) fetch(kb + 4);
      if constexpr (MODE == MODE_SPLIT6) {
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) {
          bf16x8 p1, p2, p3;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const __bf16 a1 = (__bf16)xv[jt][e];
            const float r1 = xv[jt][e] - (float)a1;
            const __bf16 a2 = (__bf16)r1;
            p1[e] = a1;
            p2[e] = a2;
            p3[e] = (__bf16)(r1 - (float)a2);
          }
          const uint4 x1 = __builtin_bit_cast(uint4, p1), x2 = __builtin_bit_cast(uint4, p2),
                      x3 = __builtin_bit_cast(uint4, p3);
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            // smallest terms first into the running sum: (1,3),(3,1),(2,2),(1,2),(2,1),(1,1)
            acc[ct][jt] = mfma_bf16(ya[ct], x3, acc[ct][jt]);
            acc[ct][jt] = mfma_bf16(yc[ct], x1, acc[ct][jt]);
            acc[ct][jt] = mfma_bf16(yb[ct], x2, acc[ct][jt]);
            acc[ct][jt] = mfma_bf16(ya[ct], x2, acc[ct][jt]);
            acc[ct][jt] = mfma_bf16(yb[ct], x1, acc[ct][jt]);
            acc[ct][jt] = mfma_bf16(ya[ct], x1, acc[ct][jt]);
          }
        }
      } else if constexpr (MODE == MODE_SPLIT3) {
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) {
          bf16x8 hi, lo;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const __bf16 h = (__bf16)xv[jt][e];
            hi[e] = h;
            lo[e] = (__bf16)(xv[jt][e] - (float)h);
          }
          const uint4 xh = __builtin_bit_cast(uint4, hi), xl = __builtin_bit_cast(uint4, lo);
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            acc[ct][jt] = mfma_bf16(ya[ct], xh, acc[ct][jt]);
            acc[ct][jt] = mfma_bf16(ya[ct], xl, acc[ct][jt]);
            acc[ct][jt] = mfma_bf16(yb[ct], xh, acc[ct][jt]);
          }
        }
      } else {
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const float yv[8] = {__uint_as_float(ya[ct].x), __uint_as_float(ya[ct].y), __uint_as_float(ya[ct].z),
                               __uint_as_float(ya[ct].w), __uint_as_float(yb[ct].x), __uint_as_float(yb[ct].y),
                               __uint_as_float(yb[ct].z), __uint_as_float(yb[ct].w)};
#pragma unroll
          for (int jt = 0; jt < JT; ++jt)
#pragma unroll
            for (int e = 0; e < 8; ++e)
              acc[ct][jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(yv[e], xv[jt][e], acc[ct][jt], 0, 0, 0);
        }
      }
    } else {
      unsigned short xc[JT][8];
#pragma unroll
      for (int jt = 0; jt < JT; ++jt)
#pragma unroll
        for (int e = 0; e < 8; ++e) xc[jt][e] = xn16[jt][e];
      if (kb + 4 < kb_end) fetch(kb + 4);
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
        const unsigned short *xs = xc[jt];
        const uint4 xp = make_uint4((unsigned)xs[0] | ((unsigned)xs[1] << 16), (unsigned)xs[2] | ((unsigned)xs[3] << 16),
                                    (unsigned)xs[4] | ((unsigned)xs[5] << 16), (unsigned)xs[6] | ((unsigned)xs[7] << 16));
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          if constexpr (MODE == MODE_BF16X) {
            acc[ct][jt] = mfma_bf16(ya[ct], xp, acc[ct][jt]);
            acc[ct][jt] = mfma_bf16(yb[ct], xp, acc[ct][jt]);
          } else {
            acc[ct][jt] = mfma_f16(ya[ct], xp, acc[ct][jt]);
            acc[ct][jt] = mfma_f16(yb[ct], xp, acc[ct][jt]);
          }
        }
      }
    }
  }

  // fixed-order reduction of the 4 waves' partial tiles: ((w2+w0)+(w3+w1)), then (w1'+w0')
  __shared__ f32x4 red[2][NCT * JT][64];
  if (wave >= 2) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) red[wave - 2][ct * JT + jt][lane] = acc[ct][jt];
  }
  __syncthreads();
  if (wave < 2) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) acc[ct][jt] += red[wave][ct * JT + jt][lane];
  }
  __syncthreads();
  if (wave == 1) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) red[0][ct * JT + jt][lane] = acc[ct][jt];
  }
  __syncthreads();
  if (wave != 0) return;
  float *dst = out + (int64_t)blockIdx.y * N * ldo;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    const int c0 = ct * 16 + 4 * g;
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) {
      const f32x4 v = acc[ct][jt] + red[0][ct * JT + jt][lane];
      const int64_t j = j0 + 16 * jt + col;
      if (j >= N) continue;
      float *p = dst + j * ldo + c0;
      if (c0 + 3 < ell && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (c0 + r < ell) p[r] = v[r];
      }
    }
  }
}

// ---------------------------------------------------------------- FP64 VALU stream kernel
// Block 256 threads computes a 64 (j) x ELLP (c) tile; thread t owns columns
// j = 4*(t%16)+0..3 and c = (t/16) + 16*u, u < ELLP/16.
template <bool NN, int ELLP>
__global__ void __launch_bounds__(256) k_stream_f64(const double *__restrict__ X, int64_t K, int64_t N,
                                                    int64_t ldx, const double *__restrict__ Y, int ell,
                                                    double *__restrict__ out, int64_t ldo, int kb_per_split) {
  constexpr int KT = 16;
  constexpr int CU = ELLP / 16;
  __shared__ double xs[KT][64 + 1];
  __shared__ double ys[KT][ELLP + 1];
  const int t = threadIdx.x;
  const int tj = t & 15, tc = t >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  const int64_t kbeg = (int64_t)blockIdx.y * kb_per_split * KT;
  const int64_t kend = std::min<int64_t>(K, kbeg + (int64_t)kb_per_split * KT);
  double acc[4][CU];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int u = 0; u < CU; ++u) acc[a][u] = 0.0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += KT) {
    // X tile: xs[kk][jj]
    for (int e = t; e < KT * 64; e += 256) {
      int kk, jj;
      if constexpr (NN) { jj = e / KT; kk = e % KT; } else { kk = e / 64; jj = e % 64; }
      const int64_t k = k0 + kk, j = j0 + jj;
      double v = 0.0;
      if (k < kend && j < N) v = NN ? X[j * ldx + k] : X[k * ldx + j];
      xs[kk][jj] = v;
    }
    for (int e = t; e < KT * ELLP; e += 256) {
      const int kk = e / ELLP, c = e % ELLP;
      const int64_t k = k0 + kk;
      ys[kk][c] = (k < kend && c < ell) ? Y[k * ell + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KT; ++kk) {
      double xv[4], yv[CU];
#pragma unroll
      for (int a = 0; a < 4; ++a) xv[a] = xs[kk][4 * tj + a];
#pragma unroll
      for (int u = 0; u < CU; ++u) yv[u] = ys[kk][tc + 16 * u];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int u = 0; u < CU; ++u) acc[a][u] = fma(xv[a], yv[u], acc[a][u]);
    }
    __syncthreads();
  }
  double *dst = out + (int64_t)blockIdx.y * N * ldo;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t j = j0 + 4 * tj + a;
    if (j >= N) continue;
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      const int c = tc + 16 * u;
      if (c < ell) dst[j * ldo + c] = acc[a][u];
    }
  }
}

template <typename T>
__global__ void k_split_reduce(const T *__restrict__ part, int nsplit, int64_t N, int ell, int64_t ldp,
                               T *__restrict__ out, int64_t ldo) {
  const int64_t total = N * ell;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / ell;
    const int c = (int)(t % ell);
    T s = 0;
    for (int p = 0; p < nsplit; ++p) s += part[(int64_t)p * N * ldp + j * ldp + c];   // fixed order
    out[j * ldo + c] = s;
  }
}

// ---------------------------------------------------------------- dispatch helpers
// Process-wide table of autotuned K-splits of the MFMA stream kernels, keyed by
// (mode, NN, K, N, ell); filled by stream_autotune, read by every launch.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int64_t, int64_t, int>, int> g_tune;

int tuned_ns(int md, bool nn, int64_t K, int64_t N, int ell) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(std::make_tuple(md, (int)nn, K, N, ell));
  return it == g_tune.end() ? 0 : it->second;
}

void set_tuned_ns(int md, bool nn, int64_t K, int64_t N, int ell, int ns) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[std::make_tuple(md, (int)nn, K, N, ell)] = ns;
}

struct Plan {
  int nsplit;
  int kb_per_split;
  unsigned gx;
};

Plan plan_split(int64_t K, int64_t N, int cols_per_block, int kblk, int cu_count, int min_kb_per_split) {
  Plan p{};
  const int64_t nkb = (K + kblk - 1) / kblk;
  p.gx = (unsigned)((N + cols_per_block - 1) / cols_per_block);
  const int64_t target = 2LL * std::max(cu_count, 1);
  int64_t ns = 1;
  if ((int64_t)p.gx < target) ns = (target + p.gx - 1) / p.gx;
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, nkb / min_kb_per_split));
  ns = std::max<int64_t>(ns, 1);
  p.kb_per_split = (int)((nkb + ns - 1) / ns);
  p.nsplit = (int)((nkb + p.kb_per_split - 1) / p.kb_per_split);
  if (p.nsplit < 1) p.nsplit = 1;
  return p;
}

template <int MODE, bool NN, int NCT, int JT>
void launch_mfma_t(hipStream_t st, dim3 grid, const void *X, int64_t K, int64_t N, int64_t ldx, const uint4 *Yp,
                   int ell, float *out, int64_t ldo, int kbps) {
  hipLaunchKernelGGL((k_stream_mfma<MODE, NN, NCT, JT>), grid, dim3(256), 0, st, X, K, N, ldx, Yp, ell, out, ldo,
                     kbps);
}

template <int MODE, bool NN>
int launch_mfma_nct(hipStream_t st, int nct, dim3 grid, const void *X, int64_t K, int64_t N, int64_t ldx,
                    const uint4 *Yp, int ell, float *out, int64_t ldo, int kbps) {
  switch (nct) {
    case 1: launch_mfma_t<MODE, NN, 1, 4>(st, grid, X, K, N, ldx, Yp, ell, out, ldo, kbps); break;
    case 2: launch_mfma_t<MODE, NN, 2, 4>(st, grid, X, K, N, ldx, Yp, ell, out, ldo, kbps); break;
    case 3: launch_mfma_t<MODE, NN, 3, 4>(st, grid, X, K, N, ldx, Yp, ell, out, ldo, kbps); break;
    case 4: launch_mfma_t<MODE, NN, 4, 4>(st, grid, X, K, N, ldx, Yp, ell, out, ldo, kbps); break;
    case 5: launch_mfma_t<MODE, NN, 5, 2>(st, grid, X, K, N, ldx, Yp, ell, out, ldo, kbps); break;
    case 6: launch_mfma_t<MODE, NN, 6, 2>(st, grid, X, K, N, ldx, Yp, ell, out, ldo, kbps); break;
    case 7: launch_mfma_t<MODE, NN, 7, 2>(st, grid, X, K, N, ldx, Yp, ell, out, ldo, kbps); break;
    case 8: launch_mfma_t<MODE, NN, 8, 2>(st, grid, X, K, N, ldx, Yp, ell, out, ldo, kbps); break;
    default: return -1;
  }
  DSK_TRY(hipGetLastError());
  return 0;
}

template <bool NN>
int launch_f64_t(hipStream_t st, dim3 grid, int ellp, const double *X, int64_t K, int64_t N, int64_t ldx,
                 const double *Y, int ell, double *out, int64_t ldo, int kbps) {
  switch (ellp) {
    case 16: hipLaunchKernelGGL((k_stream_f64<NN, 16>), grid, dim3(256), 0, st, X, K, N, ldx, Y, ell, out, ldo, kbps); break;
    case 32: hipLaunchKernelGGL((k_stream_f64<NN, 32>), grid, dim3(256), 0, st, X, K, N, ldx, Y, ell, out, ldo, kbps); break;
    case 64: hipLaunchKernelGGL((k_stream_f64<NN, 64>), grid, dim3(256), 0, st, X, K, N, ldx, Y, ell, out, ldo, kbps); break;
    case 128: hipLaunchKernelGGL((k_stream_f64<NN, 128>), grid, dim3(256), 0, st, X, K, N, ldx, Y, ell, out, ldo, kbps); break;
    default: return -1;
  }
  DSK_TRY(hipGetLastError());
  return 0;
}

int mode_of(int dtype, int mode) {
  if (dtype == DSK_BF16) return MODE_BF16X;
  if (dtype == DSK_F16) return MODE_F16X;
  if (mode == DSK_MODE_F32) return MODE_F32;
  if (mode == DSK_MODE_SPLIT3) return MODE_SPLIT3;
  return MODE_SPLIT6;
}

// The split of a launch over K and the workspace it uses: the packed Y (16-bit
// and F32 inputs) and, when K is split, the per-split partial outputs.
// The TN form with 16-bit X runs on k_stream_tn16.
bool use_tn16(bool nn, int md) { return !nn && (md == MODE_BF16X || md == MODE_F16X); }

template <int MODE, bool VEC, int W>
int launch_tn16_v(hipStream_t st, int nct, dim3 grid, const unsigned short *x, int64_t K, int64_t N, int64_t ldx,
                  const uint4 *Yp, int ell, float *out, int64_t ldo, int kbps) {
#define DSK_TN16(NC)                                                                                         \
  case NC:                                                                                                   \
    hipLaunchKernelGGL((k_stream_tn16<MODE, NC, VEC, W>), grid, dim3(256), 0, st, x, K, N, ldx, Yp, ell, out, ldo, \
                       kbps);                                                                                \
    break;
  switch (nct) {
    DSK_TN16(1) DSK_TN16(2) DSK_TN16(3) DSK_TN16(4) DSK_TN16(5) DSK_TN16(6) DSK_TN16(7) DSK_TN16(8)
    default: return -1;
  }
#undef DSK_TN16
  DSK_TRY(hipGetLastError());
  return 0;
}

template <int MODE>
int launch_tn16(hipStream_t st, int nct, dim3 grid, const void *X, int64_t K, int64_t N, int64_t ldx,
                const uint4 *Yp, int ell, float *out, int64_t ldo, int kbps) {
  const unsigned short *x = reinterpret_cast<const unsigned short *>(X);
  const bool vec = (N & 7) == 0 && (ldx & 7) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  return vec ? launch_tn16_v<MODE, true, TN16_W>(st, nct, grid, x, K, N, ldx, Yp, ell, out, ldo, kbps)
             : launch_tn16_v<MODE, false, TN16_W>(st, nct, grid, x, K, N, ldx, Yp, ell, out, ldo, kbps);
}

struct StreamPlan {
  Plan p;
  size_t yp_bytes, part_bytes;
};

StreamPlan stream_plan(bool nn, int dtype, int64_t K, int64_t N, int ell, int mode, int cu_count) {
  StreamPlan sp{};
  if (dtype == DSK_F64) {
    sp.p = plan_split(K, N, 64, 16, cu_count, 2);
    sp.part_bytes = sp.p.nsplit > 1 ? (size_t)sp.p.nsplit * N * ell * sizeof(double) : 0;
    return sp;
  }
  const int md = mode_of(dtype, mode);
  const int nct = (ell + 15) / 16;
  const int jt = nct <= 4 ? 4 : 2;
  const int64_t nkb = (K + 31) / 32;
  sp.yp_bytes = ((size_t)nkb * nct * 3 * 64 * sizeof(uint4) + 255) & ~size_t(255);
  sp.p = plan_split(K, N, use_tn16(nn, md) ? TN16_W : 16 * jt, 32, cu_count, 4);
  if (const int tn = tuned_ns(md, nn, K, N, ell); tn > 0) {
    // an autotuned split, within the partial buffers stream_ws_bytes provides (nkb / 4)
    const int64_t ns = std::max<int64_t>(1, std::min<int64_t>(tn, std::max<int64_t>(1, nkb / 4)));
    sp.p.kb_per_split = (int)((nkb + ns - 1) / ns);
    sp.p.nsplit = (int)((nkb + sp.p.kb_per_split - 1) / sp.p.kb_per_split);
  }
  sp.part_bytes = sp.p.nsplit > 1 ? (size_t)sp.p.nsplit * N * ell * sizeof(float) : 0;
  return sp;
}

int stream_any(hipStream_t st, bool nn, const void *X, int dtype, int64_t K, int64_t N, int64_t ldx,
               const void *Y, int ell, void *out, int64_t ldo, int mode, void *ws, int cu_count,
               hipEvent_t ev0, hipEvent_t ev1) {
  if (ell < 1 || ell > 128) return -1;
  char *w = reinterpret_cast<char *>(ws);
  const StreamPlan sp = stream_plan(nn, dtype, K, N, ell, mode, cu_count);
  if (dtype == DSK_F64) {
    const int ellp = ell <= 16 ? 16 : ell <= 32 ? 32 : ell <= 64 ? 64 : 128;
    const Plan p = sp.p;
    double *dst = reinterpret_cast<double *>(out);
    int64_t ldd = ldo;
    if (p.nsplit > 1) { dst = reinterpret_cast<double *>(w); ldd = ell; }
    dim3 grid(p.gx, (unsigned)p.nsplit);
    if (ev0) DSK_TRY(hipEventRecord(ev0, st));
    int r = nn ? launch_f64_t<true>(st, grid, ellp, (const double *)X, K, N, ldx, (const double *)Y, ell, dst, ldd,
                                    p.kb_per_split)
               : launch_f64_t<false>(st, grid, ellp, (const double *)X, K, N, ldx, (const double *)Y, ell, dst, ldd,
                                     p.kb_per_split);
    if (ev1) DSK_TRY(hipEventRecord(ev1, st));
    if (r) return r;
    if (p.nsplit > 1) {
      const unsigned blocks = (unsigned)std::min<int64_t>((N * ell + 255) / 256, 4096);
      hipLaunchKernelGGL(k_split_reduce<double>, dim3(blocks), dim3(256), 0, st, (const double *)dst, p.nsplit, N,
                         ell, (int64_t)ell, (double *)out, ldo);
      DSK_TRY(hipGetLastError());
    }
    return 0;
  }
  const int md = mode_of(dtype, mode);
  const int nct = (ell + 15) / 16;
  const int64_t nkb = (K + 31) / 32;
  // packed Y
  uint4 *Yp = reinterpret_cast<uint4 *>(w);
  const size_t yp_bytes = sp.yp_bytes;
  dim3 pgrid((unsigned)nkb, (unsigned)nct);
  switch (md) {
    case MODE_SPLIT6:
      hipLaunchKernelGGL((k_pack_y<MODE_SPLIT6, float>), pgrid, dim3(64), 0, st, (const float *)Y, K, ell,
                         (int64_t)ell, nct, Yp);
      break;
    case MODE_SPLIT3:
    case MODE_BF16X:
      hipLaunchKernelGGL((k_pack_y<MODE_SPLIT3, float>), pgrid, dim3(64), 0, st, (const float *)Y, K, ell,
                         (int64_t)ell, nct, Yp);
      break;
    case MODE_F16X:
      hipLaunchKernelGGL((k_pack_y<MODE_F16X, float>), pgrid, dim3(64), 0, st, (const float *)Y, K, ell,
                         (int64_t)ell, nct, Yp);
      break;
    default:
      hipLaunchKernelGGL((k_pack_y<MODE_F32, float>), pgrid, dim3(64), 0, st, (const float *)Y, K, ell,
                         (int64_t)ell, nct, Yp);
  }
  DSK_TRY(hipGetLastError());
  const Plan p = sp.p;
  float *dst = reinterpret_cast<float *>(out);
  int64_t ldd = ldo;
  if (p.nsplit > 1) { dst = reinterpret_cast<float *>(w + yp_bytes); ldd = ell; }
  dim3 grid(p.gx, (unsigned)p.nsplit);
  if (ev0) DSK_TRY(hipEventRecord(ev0, st));
  int r;
  if (use_tn16(nn, md)) {
    r = md == MODE_BF16X ? launch_tn16<MODE_BF16X>(st, nct, grid, X, K, N, ldx, Yp, ell, dst, ldd, p.kb_per_split)
                         : launch_tn16<MODE_F16X>(st, nct, grid, X, K, N, ldx, Yp, ell, dst, ldd, p.kb_per_split);
  } else {
  switch (md) {
    case MODE_SPLIT6:
      r = nn ? launch_mfma_nct<MODE_SPLIT6, true>(st, nct, grid, X, K, N, ldx, Yp, ell, dst, ldd, p.kb_per_split)
             : launch_mfma_nct<MODE_SPLIT6, false>(st, nct, grid, X, K, N, ldx, Yp, ell, dst, ldd, p.kb_per_split);
      break;
    case MODE_SPLIT3:
      r = nn ? launch_mfma_nct<MODE_SPLIT3, true>(st, nct, grid, X, K, N, ldx, Yp, ell, dst, ldd, p.kb_per_split)
             : launch_mfma_nct<MODE_SPLIT3, false>(st, nct, grid, X, K, N, ldx, Yp, ell, dst, ldd, p.kb_per_split);
      break;
    case MODE_F32:
      r = nn ? launch_mfma_nct<MODE_F32, true>(st, nct, grid, X, K, N, ldx, Yp, ell, dst, ldd, p.kb_per_split)
             : launch_mfma_nct<MODE_F32, false>(st, nct, grid, X, K, N, ldx, Yp, ell, dst, ldd, p.kb_per_split);
      break;
    case MODE_BF16X:   // NN form (the TN form took k_stream_tn16 above)
      r = launch_mfma_nct<MODE_BF16X, true>(st, nct, grid, X, K, N, ldx, Yp, ell, dst, ldd, p.kb_per_split);
      break;
    default:
      r = launch_mfma_nct<MODE_F16X, true>(st, nct, grid, X, K, N, ldx, Yp, ell, dst, ldd, p.kb_per_split);
  }
  }
  if (ev1) DSK_TRY(hipEventRecord(ev1, st));
  if (r) return r;
  if (p.nsplit > 1) {
    const unsigned blocks = (unsigned)std::min<int64_t>((N * ell + 255) / 256, 4096);
    hipLaunchKernelGGL(k_split_reduce<float>, dim3(blocks), dim3(256), 0, st, (const float *)dst, p.nsplit, N, ell,
                       (int64_t)ell, (float *)out, ldo);
    DSK_TRY(hipGetLastError());
  }
  return 0;
}

}  // namespace

size_t stream_ws_bytes(int dtype, int64_t K, int64_t N, int ell, int mode) {
  (void)mode;
  if (dtype == DSK_F64) {
    // worst case split partials
    const int64_t nkb = (K + 15) / 16;
    const int64_t ns = std::min<int64_t>(nkb, 1024);
    return (size_t)ns * N * ell * sizeof(double) + 256;
  }
  const int nct = (ell + 15) / 16;
  const int64_t nkb = (K + 31) / 32;
  size_t yp = ((size_t)nkb * nct * 3 * 64 * sizeof(uint4) + 255) & ~size_t(255);   // same as stream_any
  const int64_t ns = std::min<int64_t>(std::max<int64_t>(1, nkb / 4), 1024);
  return yp + (size_t)ns * N * ell * sizeof(float) + 256;
}

size_t stream_scratch_bytes(int dtype, int64_t K, int64_t N, int ell, int mode, int cu_count) {
  const StreamPlan sp = stream_plan(false, dtype, K, N, ell, mode, cu_count);
  return sp.yp_bytes + sp.part_bytes;
}

int launch_stream(hipStream_t st, const void *X, int dtype, int64_t K, int64_t N, int64_t ldx, const void *Y,
                  int f64y, int ell, void *out, int64_t ldo, int mode, void *ws, int cu_count, hipEvent_t ev0,
                  hipEvent_t ev1) {
  (void)f64y;
  return stream_any(st, false, X, dtype, K, N, ldx, Y, ell, out, ldo, mode, ws, cu_count, ev0, ev1);
}

int launch_stream_nn(hipStream_t st, const void *X, int dtype, int64_t M, int64_t K, int64_t ldx, const void *Y,
                     int ell, void *out, int64_t ldo, int mode, void *ws, int cu_count) {
  return stream_any(st, true, X, dtype, K, M, ldx, Y, ell, out, ldo, mode, ws, cu_count, nullptr, nullptr);
}

int stream_autotune(hipStream_t st, const void *X, int dtype, int64_t K, int64_t N, int64_t ldx, int ell, int mode,
                    void *ws, void *Y, void *out, int cu_count, int *best_ns, float *best_ms) {
  if (dtype == DSK_F64 || ell < 1 || ell > 128) return -1;
  const int md = mode_of(dtype, mode);
  const int64_t nkb = (K + 31) / 32;
  const int64_t cap = std::max<int64_t>(1, nkb / 4);
  hipEvent_t e0, e1;
  DSK_TRY(hipEventCreate(&e0));
  DSK_TRY(hipEventCreate(&e1));
  int best = 1;
  float bms = 1e30f;
  int rc = 0;
  for (int ns : {1, 2, 3, 4, 6, 8, 12, 16}) {
    if (ns > cap) break;
    set_tuned_ns(md, false, K, N, ell, ns);
    rc = stream_any(st, false, X, dtype, K, N, ldx, Y, ell, out, ell, mode, ws, cu_count, nullptr, nullptr);
    if (rc) break;
    if ((rc = (int)hipEventRecord(e0, st)) != 0) { rc += DSK_ERR_BASE; break; }
    for (int r = 0; r < 3 && !rc; ++r)
      rc = stream_any(st, false, X, dtype, K, N, ldx, Y, ell, out, ell, mode, ws, cu_count, nullptr, nullptr);
    if (rc) break;
    if ((rc = (int)hipEventRecord(e1, st)) != 0) { rc += DSK_ERR_BASE; break; }
    if ((rc = (int)hipEventSynchronize(e1)) != 0) { rc += DSK_ERR_BASE; break; }
    float ms = 0.f;
    if ((rc = (int)hipEventElapsedTime(&ms, e0, e1)) != 0) { rc += DSK_ERR_BASE; break; }
    ms /= 3.f;
    if (ms < bms) { bms = ms; best = ns; }
  }
  set_tuned_ns(md, false, K, N, ell, best);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_ns) *best_ns = best;
  if (best_ms) *best_ms = bms;
  return rc;
}

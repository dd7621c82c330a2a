// One-wave building blocks shared by the small factorizations: lane-uniform
// reads, wave-local LDS ordering, refined hardware reciprocal / reciprocal
// square root, 16-lane DPP sums, the FP64 16 x 16 x 4 MFMA, and a blocked
// Cholesky of an ell x ell (ell <= 64) symmetric positive definite matrix.
#pragma once

#include "dsk_internal.h"

namespace wc {

constexpr int LDL = 65;   // row stride of the 64 x 64 LDS factor buffers (odd: conflict-free row walks)

// Value of v held by lane `src` (uniform result).
__device__ __forceinline__ double readlane_f64(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Orders this wave's LDS accesses (no other wave takes part).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1/sqrt(d) for finite d > 0: hardware estimate plus two Newton steps
// (y <- y (3 - d y^2) / 2), which reach full double precision.
__device__ __forceinline__ double rsq_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// 1/x for finite nonzero x: hardware estimate plus two Newton steps.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over each aligned group of 16 lanes (a DPP row); every lane of the row
// gets the same value: quad xor 1, quad xor 2, half-row mirror, row mirror.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  return v;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// D = A B + C for 16 x 16 FP64 tiles, k = 4: A(i, k) in lane i + 16 k, B(k, j) in
// lane j + 16 k, D(i, j) in lane j + 16 (i mod 4), register i / 4.
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Cholesky of the lower triangle of A (LDS, 64 x LDL, the shift already added;
// rows and columns past ell zero), ell <= 64, by the calling wave, no
// barriers: four 16-column panels, each factored in registers, then the
// trailing tiles A_IJ -= L_IK L_JK^T (K < J <= I) on MFMA.  In a panel step
// lane i keeps row i; the pivot column goes to every lane through one LDS
// write and uniform-address reads (colb: 64 doubles of LDS), the pivot itself
// by v_readlane, and the update A(i, c) -= A(i, p) A(c, p) / d needs no square
// root, so only 1 / d is on the chain from one pivot to the next.  Branch-free
// steps (a padded column p >= ell is an identity column).  A is overwritten.
// L goes to Lf (LDS, 64 x LDL, zero above the diagonal, identity past ell),
// dinv[j] = 1 / L(j, j).  Returns false at a pivot <= thr or non-finite.
__device__ __forceinline__ bool chol64_blocked(double *A, int ell, double thr, double *Lf, double *dinv,
                                               double *colb) {
  const int i = threadIdx.x & 63;
  bool ok = true;
  double mydinv = 1.0;
  for (int K = 0; K < 4; ++K) {
    const int c0 = 16 * K;
    double g[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) g[j] = A[i * LDL + c0 + j];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int p = c0 + j;
      const bool live = p < ell;
      const double dp = readlane_f64(g[j], p);
      colb[i] = g[j];
      wave_lds_sync();
      // uniform-address reads; colb is only 8-byte aligned (the dynamic LDS base
      // follows the static segment), so no wider access is assumed
      double lc[16];
#pragma unroll
      for (int c = j + 1; c < 16; ++c) lc[c] = colb[c0 + c];
      const double d = live ? dp : 1.0;
      ok = ok && (!live || (d > thr && isfinite(d)));
      const double inv = rcp_nr(d), rs = rsq_nr(d);
      const double ti = g[j] * inv;
#pragma unroll
      for (int c = j + 1; c < 16; ++c) g[c] = fma(-ti, lc[c], g[c]);
      g[j] = live ? (i > p ? g[j] * rs : (i == p ? d * rs : 0.0)) : (i == p ? 1.0 : 0.0);
      mydinv = (i == p) ? (live ? rs : 1.0) : mydinv;
      wave_lds_sync();   // colb is rewritten by the next step
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) Lf[i * LDL + c0 + j] = (i >= c0 + j) ? g[j] : 0.0;
    wave_lds_sync();
    // A(i, k) = L(16 I + i, c0 + k) in lane i + 16 k, B(k, j) = L(16 J + j, c0 + k) in lane j + 16 k
    for (int I = K + 1; I < 4; ++I)
      for (int J = K + 1; J <= I; ++J) {
        d4 c;
#pragma unroll
        for (int v = 0; v < 4; ++v) c[v] = A[(16 * I + (i >> 4) + 4 * v) * LDL + 16 * J + (i & 15)];
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4)
          c = mfma(-Lf[(16 * I + (i & 15)) * LDL + c0 + 4 * k4 + (i >> 4)],
                   Lf[(16 * J + (i & 15)) * LDL + c0 + 4 * k4 + (i >> 4)], c);
#pragma unroll
        for (int v = 0; v < 4; ++v) A[(16 * I + (i >> 4) + 4 * v) * LDL + 16 * J + (i & 15)] = c[v];
      }
    wave_lds_sync();
  }
  dinv[i] = mydinv;
  wave_lds_sync();
  return ok;
}

}  // namespace wc

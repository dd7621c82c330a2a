// One-wave building blocks shared by the small factorizations: lane-uniform
// reads, wave-local LDS ordering, refined hardware reciprocal / reciprocal
// square root, 16-lane DPP sums, and a register-resident Cholesky of an
// ell x ell (ell <= 64) symmetric positive definite matrix.
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

// Step J of the right-looking register Cholesky: lane i keeps row i of the
// working matrix in g (compile-time J keeps every register index static); the
// pivot column L(:, J) is broadcast lane by lane with v_readlane (no memory
// round trip on the dependent chain).  On success g[c] holds L(i, c) for
// c <= i; dinv[J] = 1 / L(J, J).  Rows and columns past ell hold the identity.
template <int J>
__device__ __forceinline__ void chol_step(double (&g)[64], int ell, int lane, double thr, bool &ok, double *dinv) {
  if constexpr (J < 64) {
    if (J < ell && ok) {
      const double d = readlane_f64(g[J], J);
      if (!(d > thr) || !isfinite(d)) {
        ok = false;
        return;
      }
      const double inv = rsq_nr(d), piv = d * inv;
      // lanes below the pivot get L(i, J); the pivot lane's own update only
      // touches its (unused) upper triangle
      const double l = lane > J ? g[J] * inv : (lane == J ? piv : 0.0);
      g[J] = l;
      if (lane == 0) dinv[J] = inv;
      double lc[64 - J];
#pragma unroll
      for (int c = J + 1; c < 64; ++c) lc[c - J] = readlane_f64(l, c);
#pragma unroll
      for (int c = J + 1; c < 64; ++c) g[c] = fma(-l, lc[c - J], g[c]);
      chol_step<J + 1>(g, ell, lane, thr, ok, dinv);
    }
  }
}

// Cholesky of S = A + shift I by the calling wave (lanes 0..63), ell <= 64.
// A: LDS or global, row-major with leading dimension lda.  On success L is
// written to Lout (LDS, 64 x LDL, row i = L(i, :), zero above the diagonal and
// identity past ell) and dinv[j] = 1 / L(j, j); returns false at a pivot
// <= thr (or non-finite).  col: unused (kept for the LDS layout of callers).
__device__ __forceinline__ bool chol64(const double *A, int lda, int ell, double shift, double thr, double *Lout,
                                       double *dinv, double *col) {
  const int lane = threadIdx.x & 63;
  double g[64];
#pragma unroll
  for (int c = 0; c < 64; ++c)
    g[c] = (lane < ell && c < ell) ? A[lane * lda + c] + (c == lane ? shift : 0.0) : (c == lane ? 1.0 : 0.0);
  bool ok = true;
  (void)col;
  chol_step<0>(g, ell, lane, thr, ok, dinv);
  if (!ok) return false;
#pragma unroll
  for (int c = 0; c < 64; ++c) Lout[lane * LDL + c] = c <= lane ? g[c] : 0.0;
  if (lane >= ell) dinv[lane] = 1.0;
  wave_lds_sync();
  return true;
}

}  // namespace wc

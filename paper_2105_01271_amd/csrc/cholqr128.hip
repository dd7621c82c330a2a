// CholeskyQR for blocks 65 .. 128 wide: the QR steps of Alg. 2 and Alg. 7
// (range finder, power-iteration bases) when ell = k + p exceeds 64.  Same
// contract and numerics as the 64-wide path: Q = Y L^{-T} with L L^T = Y^T Y,
// FP64 Gram, FP64 factorization, FP64 products; on a non-positive or
// negligible pivot the factorization is retried with the shift
// 11 (rows ell + ell (ell + 1)) u tr(Y^T Y), DSK_FLAG_FALLBACK is raised and a
// third pass restores orthonormality (shifted CholeskyQR3).
//
// A pass is three launches:
//  * Gram partials of the block (gram64.hip, tile-major lower 16 x 16 tiles,
//    one partial per 64 rows);
//  * fold + factor: every workgroup sums 64 entries of the partials in a
//    fixed order (four threads per entry, partials strided by four, then the
//    four in order) and publishes them; the last workgroup to arrive factors
//    G = L L^T in LDS, blocked by 16 columns: one wave factors the diagonal
//    block A_KK in registers (pivot columns by DPP row broadcasts, only 1 / d
//    on the chain from pivot to pivot) and inverts it, W_K = L_KK^{-1}; the
//    four waves then form the panel below it, L_IK = A_IK W_K^T, on MFMA; the
//    trailing tiles A_IJ -= L_IK L_JK^T go to three waves while the fourth
//    updates and factors the next diagonal block: two barriers per block;
//  * apply: each wave owns 16 rows of a 64-row chunk and forms
//    Q_J = (Y_J - sum_{K<J} Q_K L_JK^T) W_J^T block column by block column
//    on MFMA, with no barrier; when the next pass needs the Gram of the
//    rounded Q, the workgroup accumulates its tiles (two barriers per chunk).
// All sums run in fixed orders, so repeated runs give identical bytes.
#include <algorithm>

#include "devsync.h"
#include "dsk_internal.h"
#include "gramtile.h"

namespace {

using wc::d4;
using wc::mfma;

constexpr int NBM = 8;                    // 16-column blocks at most
constexpr int EMAX = 16 * NBM;            // widest block
constexpr int NTM = NBM * (NBM + 1) / 2;  // lower tiles at most
constexpr int TILE = 256;
constexpr int PART = NTM * TILE;          // doubles of a (largest) partial
constexpr int PMAX = 256;                 // partials at most
constexpr int GRPB = 64;                  // rows per Gram partial (at least)
constexpr int LDA = EMAX + 2;             // LDS row stride of the factor (conflict-free MFMA operand reads)
constexpr int RCH = 64;                   // rows per apply chunk (16 per wave)
constexpr int LDQ = EMAX + 2;             // LDS row stride of the apply chunk
constexpr int MST = 16 * 17;              // LDS footprint of a factor tile (row stride 17)
constexpr int FE = 64;                    // entries per fold workgroup
constexpr double U64 = 1.1102230246251565e-16;

constexpr int FACT_LDS = EMAX * LDA + NBM * 16 * 17 + 8;   // A, W_K tiles, words
constexpr int APPLY_LDS = NTM * MST + RCH * LDQ + 4 * MST;  // factor tiles, chunk, per-wave S

__device__ __forceinline__ int ltile(int J, int K) { return J * (J + 1) / 2 + K; }

__device__ __forceinline__ void tile_ij(int id, int &I, int &J) {
  I = 0;
  while ((I + 1) * (I + 2) / 2 <= id) ++I;
  J = id - I * (I + 1) / 2;
}

// A (LDS, lower triangle) from the folded Gram (tile-major, published by other
// workgroups of this launch); identity past ell; shift added to the diagonal.
// Thread t reads entry t of every tile (so the tile of each load is a
// compile-time constant); its loads go out in two batches, each issued
// before its first use.
__device__ __forceinline__ void load_gram(const double *G, int ell, int nb, double shift, double *A) {
  constexpr int LG = NTM / 2;
  const int nt = nb * (nb + 1) / 2, t = threadIdx.x, r16 = t >> 4, c16 = t & 15;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double v[LG];
#pragma unroll
    for (int u = 0; u < LG; ++u) {
      const int id = u + LG * h;
      v[u] = id < nt ? ds::ld_dev(&G[id * TILE + t]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < LG; ++u) {
      const int id = u + LG * h;
      if (id >= nt) continue;
      int I, J;
      tile_ij(id, I, J);
      const int r = 16 * I + r16, c = 16 * J + c16;
      double x = v[u];
      if (r >= ell || c >= ell) x = (r == c) ? 1.0 : 0.0;
      else if (r == c) x += shift;
      A[r * LDA + c] = x;
    }
  }
}

// Lane c of each row of 16 lanes, in every lane of that row (DPP
// row_newbcast: a vector-register move, no scalar register on the way).
__device__ __forceinline__ double row_bcast(double v, int c) {
  switch (c) {
    case 0: return wc::dpp_f64<0x150>(v);
    case 1: return wc::dpp_f64<0x151>(v);
    case 2: return wc::dpp_f64<0x152>(v);
    case 3: return wc::dpp_f64<0x153>(v);
    case 4: return wc::dpp_f64<0x154>(v);
    case 5: return wc::dpp_f64<0x155>(v);
    case 6: return wc::dpp_f64<0x156>(v);
    case 7: return wc::dpp_f64<0x157>(v);
    case 8: return wc::dpp_f64<0x158>(v);
    case 9: return wc::dpp_f64<0x159>(v);
    case 10: return wc::dpp_f64<0x15A>(v);
    case 11: return wc::dpp_f64<0x15B>(v);
    case 12: return wc::dpp_f64<0x15C>(v);
    case 13: return wc::dpp_f64<0x15D>(v);
    case 14: return wc::dpp_f64<0x15E>(v);
    default: return wc::dpp_f64<0x15F>(v);
  }
}

// Diagonal block K by the calling wave: lane i (mod 16) holds row i of the
// trailing-updated A_KK (each row of 16 lanes a copy).  Pivot by pivot, the
// pivot column reaches every lane by DPP row broadcasts, so no LDS round trip
// sits on the chain from one pivot to the next; A(i, c) -= A(i, p) A(c, p) / d
// needs no square root on it.  Then W_K = L_KK^{-1} by forward substitution,
// column c in lane c, the entries of L read back from LDS at uniform
// addresses.  Lanes 0 .. 15 write L_KK (zero above the diagonal) to A, W_K to
// Wl and to its factor tile.  Padded pivots (p >= ell) are identity columns.
__device__ __forceinline__ bool diag_block(double *A, double *Wl, double *Mf, int K, int ell, double thr) {
  const int l = threadIdx.x & 63, i = l & 15, c0 = 16 * K;
  double a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) a[c] = A[(c0 + i) * LDA + c0 + c];
  bool ok = true;
  double rsv[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const bool live = c0 + j < ell;
    const double dp = row_bcast(a[j], j);
    const double d = live ? dp : 1.0;
    ok = ok & (!live | ((d > thr) & isfinite(d)));
    const double inv = wc::rcp_nr(d), rs = wc::rsq_nr(d);
    const double t = a[j] * inv;
#pragma unroll
    for (int c = j + 1; c < 16; ++c) a[c] = fma(-t, row_bcast(a[j], c), a[c]);
    a[j] = live ? (i > j ? a[j] * rs : (i == j ? d * rs : 0.0)) : (i == j ? 1.0 : 0.0);
    rsv[j] = live ? rs : 1.0;
  }
  if (l < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c) A[(c0 + i) * LDA + c0 + c] = (c <= i) ? a[c] : 0.0;
  }
  wc::wave_lds_sync();
  // x_r = (delta_rc - sum_{m < r} L(r, m) x_m) / L(r, r), L(r, m) by
  // uniform-address LDS reads; zero above the diagonal by construction
  const double *Lk = A + c0 * LDA + c0;
  double x[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    double s = (r == i) ? 1.0 : 0.0;
#pragma unroll
    for (int m = 0; m < r; ++m) s = fma(-Lk[r * LDA + m], x[m], s);
    x[r] = s * rsv[r];
  }
  if (l < 16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      Wl[K * MST + r * 17 + i] = x[r];
      Mf[ltile(K, K) * TILE + r * 16 + i] = x[r];
    }
  }
  return ok;
}

// L_IK = A_IK W_K^T for K < I < nb, tiles dealt to the four waves (in place:
// a wave reads its whole tile before it writes it), also stored as factor tiles.
__device__ __forceinline__ void below(double *A, const double *Wl, double *Mf, int K, int nb) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, c0 = 16 * K;
  for (int I = K + 1 + w; I < nb; I += 4) {
    d4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4)
      c = mfma(A[(16 * I + (l & 15)) * LDA + c0 + 4 * k4 + (l >> 4)], Wl[K * MST + (l & 15) * 17 + 4 * k4 + (l >> 4)],
               c);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      A[(16 * I + (l >> 4) + 4 * v) * LDA + c0 + (l & 15)] = c[v];
      Mf[ltile(I, K) * TILE + ((l >> 4) + 4 * v) * 16 + (l & 15)] = c[v];
    }
  }
}

// A_IJ -= L_IK L_JK^T for one tile (K < J <= I), by the calling wave.
// MFMA operands: A(i, k) = L(16 I + i, 16 K + k) in lane i + 16 k,
// B(k, j) = L(16 J + j, 16 K + k) in lane j + 16 k.
__device__ __forceinline__ void trail_tile(double *A, int K, int I, int J) {
  const int l = threadIdx.x & 63, c0 = 16 * K;
  d4 c;
#pragma unroll
  for (int v = 0; v < 4; ++v) c[v] = A[(16 * I + (l >> 4) + 4 * v) * LDA + 16 * J + (l & 15)];
#pragma unroll
  for (int k4 = 0; k4 < 4; ++k4)
    c = mfma(-A[(16 * I + (l & 15)) * LDA + c0 + 4 * k4 + (l >> 4)],
             A[(16 * J + (l & 15)) * LDA + c0 + 4 * k4 + (l >> 4)], c);
#pragma unroll
  for (int v = 0; v < 4; ++v) A[(16 * I + (l >> 4) + 4 * v) * LDA + 16 * J + (l & 15)] = c[v];
}

// The trailing tiles of block K but the next diagonal one (tile 0 of the
// enumeration), dealt to the calling waves: tile id0, id0 + stride, ...
__device__ __forceinline__ void trailing(double *A, int K, int nb, int id0, int stride) {
  const int mrest = nb - 1 - K, cnt = mrest * (mrest + 1) / 2;
  for (int id = id0; id < cnt; id += stride) {
    int I, J;
    tile_ij(id, I, J);
    trail_tile(A, K, I + K + 1, J + K + 1);
  }
}

// The last workgroup of the fold: factor (with the shifted retry), invert the
// diagonal blocks, write the factor tiles Mf: tile (J, K), K < J, is L_JK and
// tile (J, J) is W_J = L_JJ^{-1}, each 16 x 16 row-major.
__device__ __forceinline__ void factor(const double *G, int ell, int64_t rows, double *Mf, int *dflags, double *pool) {
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int nb = (ell + 15) / 16, ntile = nb * (nb + 1) / 2;
  double *A = pool, *Wl = A + EMAX * LDA, *word = Wl + NBM * MST;
  load_gram(G, ell, nb, 0.0, A);
  __syncthreads();
  if (w == 0) {
    double v = 0.0;
    for (int i = l; i < ell; i += 64) v += A[i * LDA + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (l == 0) word[0] = v;
  }
  __syncthreads();
  const double tr = word[0];
  const bool trok = tr > 0.0 && isfinite(tr);
  bool ok = false;
#pragma nounroll
  for (int attempt = 0; attempt < 2 && trok && !ok; ++attempt) {
    if (attempt) {
      load_gram(G, ell, nb, 11.0 * ((double)rows * ell + (double)ell * (ell + 1)) * U64 * tr, A);
      __syncthreads();
    }
    // block K + 1's diagonal tile is updated and factored by wave 0 while the
    // other three waves update the rest of block K's trailing tiles
    const double thr = 1e-15 * tr;
    bool okw = true;
    if (w == 0) okw = diag_block(A, Wl, Mf, 0, ell, thr);
    __syncthreads();
    below(A, Wl, Mf, 0, nb);
    __syncthreads();
    for (int K = 0; K + 1 < nb; ++K) {
      if (w == 0) {
        trail_tile(A, K, K + 1, K + 1);
        wc::wave_lds_sync();
        okw = diag_block(A, Wl, Mf, K + 1, ell, thr) && okw;
      } else {
        trailing(A, K, nb, w, 3);
      }
      __syncthreads();
      below(A, Wl, Mf, K + 1, nb);
      __syncthreads();
    }
    if (t == 0) word[1] = okw ? 1.0 : 0.0;
    __syncthreads();
    ok = word[1] != 0.0;
    if (!ok && attempt == 0 && t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_FALLBACK);
    __syncthreads();
  }
  if (!ok) {
    // non-finite or zero input: identity factor keeps the pipeline finite
    if (t == 0) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_FALLBACK | DSK_FLAG_RANK_DEFICIENT | DSK_FLAG_NONFINITE);
    for (int e = t; e < ntile * TILE; e += 256) {
      int I, J;
      tile_ij(e >> 8, I, J);
      Mf[e] = (I == J && ((e >> 4) & 15) == (e & 15)) ? 1.0 : 0.0;
    }
    return;
  }
}

// ---------------------------------------------------------------- launches
// G = sum of the P partials (fixed order); the last workgroup factors G.
// cond = 1: only after a shifted first pass.
__global__ void __launch_bounds__(256) k_q8_fold_factor(const double *__restrict__ part, int P, int ell,
                                                        int64_t rows, double *G, double *__restrict__ Mf,
                                                        unsigned *ticket, int *dflags, int cond) {
  if (cond && !(dflags[FLAGW_BITS] & DSK_FLAG_FALLBACK)) return;
  extern __shared__ double pool[];
  __shared__ double red[4][FE];
  const int nb = (ell + 15) / 16, ne = nb * (nb + 1) / 2 * TILE;
  const int t = threadIdx.x, q = t >> 6, el = t & 63;
  const int e = blockIdx.x * FE + el;
  double s = 0.0;
  if (e < ne) {
    for (int p0 = q; p0 < P; p0 += 64) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int p = p0 + 4 * u;
        v[u] = p < P ? part[(int64_t)p * ne + e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) s += v[u];
    }
  }
  red[q][el] = s;
  __syncthreads();
  if (q == 0 && e < ne) ds::st_dev(&G[e], (red[0][el] + red[1][el]) + (red[2][el] + red[3][el]));
  if (ds::last_arrival(ticket)) factor(G, ell, rows, Mf, dflags, pool);
}

// Q = Y L^{-T} for the rows of this workgroup (Q may alias Y: each wave reads
// its rows before it writes them).  With part, also the Gram partial of the
// rounded Q.  cond = 1: only after a shifted pass; gram_cond = 1: the Gram
// only after a shifted pass.
template <typename T>
__global__ void __launch_bounds__(256) k_q8_apply(const T *Y, int64_t rows, int ell, const double *__restrict__ Mf,
                                                  T *Q, int64_t rpw, double *__restrict__ part, int *dflags,
                                                  int cond, int gram_cond) {
  const bool fallback = (dflags[FLAGW_BITS] & DSK_FLAG_FALLBACK) != 0;
  if (cond && !fallback) return;
  if (gram_cond && !fallback) part = nullptr;
  extern __shared__ double pool[];
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int nb = (ell + 15) / 16, ellp = 16 * nb, ntile = nb * (nb + 1) / 2;
  double *Ms = pool, *YQ = Ms + NTM * MST, *Sw = YQ + RCH * LDQ + w * MST;
  {
    // all of a thread's factor loads in flight at once
    constexpr int LM = NTM * TILE / 256;
    double mv[LM];
#pragma unroll
    for (int u = 0; u < LM; ++u) {
      const int e = t + 256 * u;
      mv[u] = e < ntile * TILE ? Mf[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < LM; ++u) {
      const int e = t + 256 * u;
      if (e < ntile * TILE) Ms[(e >> 8) * MST + ((e >> 4) & 15) * 17 + (e & 15)] = mv[u];
    }
  }
  __syncthreads();
  const gt::Tiles tl = gt::tiles_of(w, nb);
  d4 acc[gt::MAXT];
  gt::zero(acc);
  const int i16 = l & 15, kk = l >> 4, rb = 16 * w;
  const int64_t r0 = (int64_t)blockIdx.x * rpw, r1 = std::min<int64_t>(rows, r0 + rpw);
  for (int64_t c0 = r0; c0 < r1; c0 += RCH) {
    // this wave's 16 rows, FP64, zero padded (all loads in flight at once)
    // (lane l takes columns l and l + 64 of every row: no index division)
    {
      T yv[16][2];
#pragma unroll
      for (int rr = 0; rr < 16; ++rr)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int c = l + 64 * h;
          const int64_t r = c0 + rb + rr;
          yv[rr][h] = (r < r1 && c < ell) ? Y[r * ell + c] : T(0);
        }
#pragma unroll
      for (int rr = 0; rr < 16; ++rr)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int c = l + 64 * h;
          if (c < ellp) YQ[(rb + rr) * LDQ + c] = (double)yv[rr][h];
        }
    }
    wc::wave_lds_sync();
    for (int J = 0; J < nb; ++J) {
      // S = Y_J - sum_{K<J} Q_K L_JK^T: one accumulator per K (independent MFMA chains), summed in K order
      d4 c, ck[NBM - 1];
#pragma unroll
      for (int v = 0; v < 4; ++v) c[v] = YQ[(rb + kk + 4 * v) * LDQ + 16 * J + i16];
#pragma unroll
      for (int K = 0; K < NBM - 1; ++K) ck[K] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
        for (int K = 0; K < NBM - 1; ++K)
          if (K < J)
            ck[K] = mfma(-YQ[(rb + i16) * LDQ + 16 * K + 4 * k4 + kk], Ms[ltile(J, K) * MST + i16 * 17 + 4 * k4 + kk],
                         ck[K]);
#pragma unroll
      for (int K = 0; K < NBM - 1; ++K)
        if (K < J) c += ck[K];
#pragma unroll
      for (int v = 0; v < 4; ++v) Sw[(kk + 4 * v) * 17 + i16] = c[v];
      wc::wave_lds_sync();
      const double *Wt = Ms + ltile(J, J) * MST;
      d4 qv = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) qv = mfma(Sw[i16 * 17 + 4 * k4 + kk], Wt[i16 * 17 + 4 * k4 + kk], qv);
#pragma unroll
      for (int v = 0; v < 4; ++v) YQ[(rb + kk + 4 * v) * LDQ + 16 * J + i16] = qv[v];
      wc::wave_lds_sync();
    }
    // round this wave's rows to the output type (the Gram describes the stored Q)
#pragma unroll
    for (int rr = 0; rr < 16; ++rr)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = l + 64 * h;
        if (c >= ellp) continue;
        const int64_t r = c0 + rb + rr;
        double *p = &YQ[(rb + rr) * LDQ + c];
        const T v = (T)(*p);
        *p = (double)v;
        if (r < r1 && c < ell) Q[r * ell + c] = v;
      }
    if (part) {
      __syncthreads();
      gt::accum<RCH / 4>(YQ, LDQ, tl, acc);
      __syncthreads();
    } else {
      wc::wave_lds_sync();
    }
  }
  if (part) gt::store_tiles(acc, tl, w, part + (int64_t)blockIdx.x * ntile * TILE);
}

int pick_parts(int64_t rows, int64_t unit, int64_t &rpw) {
  rpw = unit;
  if ((rows + rpw - 1) / rpw > PMAX) rpw = ((rows + PMAX - 1) / PMAX + unit - 1) / unit * unit;
  return (int)((rows + rpw - 1) / rpw);
}

template <typename T>
int cholqr128_typed(hipStream_t st, const T *Y, int64_t rows, int ell, T *Q, void *ws, int *dflags, int passes) {
  double *part = reinterpret_cast<double *>(ws);
  double *G = part + (size_t)PMAX * PART;
  double *Mf = G + PART;
  T *Q1 = reinterpret_cast<T *>(Mf + PART);
  unsigned *ticket = reinterpret_cast<unsigned *>(dflags + FLAGW_TICKET);
  const int nb = (ell + 15) / 16;
  const int nfold = (nb * (nb + 1) / 2 * TILE + FE - 1) / FE;
  const size_t flds = (size_t)FACT_LDS * sizeof(double), alds = (size_t)APPLY_LDS * sizeof(double);
  allow_lds(k_q8_fold_factor, flds);
  allow_lds(k_q8_apply<T>, alds);
  int64_t grpb, arpw;
  const int gparts = pick_parts(rows, GRPB, grpb);
  const int aparts = pick_parts(rows, RCH, arpw);
  DSK_RET(launch_gram_tiles(st, Y, sizeof(T) == 8, rows, ell, grpb, part));
  auto fold = [&](int P, int cond) {
    hipLaunchKernelGGL(k_q8_fold_factor, dim3(nfold), dim3(256), flds, st, (const double *)part, P, ell, rows, G, Mf,
                       ticket, dflags, cond);
  };
  auto apply = [&](const T *src, T *dst, double *prt, int cond, int gcond) {
    hipLaunchKernelGGL(k_q8_apply<T>, dim3(aparts), dim3(256), alds, st, src, rows, ell, (const double *)Mf, dst,
                       arpw, prt, dflags, cond, gcond);
  };
  fold(gparts, 0);
  if (passes == 1) {
    apply(Y, Q, nullptr, 0, 0);   // span only
  } else {
    apply(Y, Q1, part, 0, 0);     // second factorization
    fold(aparts, 0);
    apply(Q1, Q, part, 0, 1);     // third factorization only after a shifted first pass
    fold(aparts, 1);
    apply(Q, Q, nullptr, 1, 0);   // third application only after a shifted first pass
  }
  DSK_TRY(hipGetLastError());
  return 0;
}

}  // namespace

size_t cholqr128_ws_bytes(int64_t rows, int ell) {
  (void)ell;
  return ((size_t)PMAX * PART + 2 * (size_t)PART) * sizeof(double) + (size_t)rows * EMAX * sizeof(double) + 256;
}

int launch_cholqr128_apply(hipStream_t st, const void *X, int f64, int64_t rows, int ell, const void *ws, void *out,
                           int *dflags) {
  if (ell < 1 || ell > EMAX || rows < 1) return -1;
  // the factor tiles the last factorization on ws left (after the Gram partials and G)
  const double *Mf = reinterpret_cast<const double *>(ws) + (size_t)PMAX * PART + PART;
  // about two workgroups per compute unit's worth of row ranges, each a multiple of RCH rows
  const int64_t rpw = std::max<int64_t>(RCH, ((rows + 511) / 512 + RCH - 1) / RCH * RCH);
  const unsigned grid = (unsigned)((rows + rpw - 1) / rpw);
  const size_t alds = (size_t)APPLY_LDS * sizeof(double);
  if (f64) {
    allow_lds(k_q8_apply<double>, alds);
    hipLaunchKernelGGL(k_q8_apply<double>, dim3(grid), dim3(256), alds, st, (const double *)X, rows, ell, Mf,
                       (double *)out, rpw, (double *)nullptr, dflags, 0, 0);
  } else {
    allow_lds(k_q8_apply<float>, alds);
    hipLaunchKernelGGL(k_q8_apply<float>, dim3(grid), dim3(256), alds, st, (const float *)X, rows, ell, Mf,
                       (float *)out, rpw, (double *)nullptr, dflags, 0, 0);
  }
  DSK_TRY(hipGetLastError());
  return 0;
}

int launch_cholqr128(hipStream_t st, const void *Y, int f64, int64_t rows, int ell, void *Q, void *ws, int *dflags,
                     int passes) {
  if (ell < 1 || ell > EMAX || rows < 1 || passes < 1 || passes > 2) return -1;
  if (f64) return cholqr128_typed<double>(st, (const double *)Y, rows, ell, (double *)Q, ws, dflags, passes);
  return cholqr128_typed<float>(st, (const float *)Y, rows, ell, (float *)Q, ws, dflags, passes);
}

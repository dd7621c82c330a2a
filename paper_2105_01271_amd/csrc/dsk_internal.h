// Internal declarations shared by the HIP translation units of libdsketch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <functional>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/dsketch.h"

#define DSK_ERR_BASE 100
#define DSK_TRY(expr)                                          \
  do {                                                         \
    hipError_t e__ = (expr);                                   \
    if (e__ != hipSuccess) return DSK_ERR_BASE + (int)e__;     \
  } while (0)
#define DSK_RET(expr)                                          \
  do {                                                         \
    int r__ = (expr);                                          \
    if (r__ != 0) return r__;                                  \
  } while (0)

// Device-side status words: [0] DSK_FLAG_* bits, [1] workgroup ticket counter of
// the fused reduce-and-factor kernels (returns to 0 after every launch), [2]
// Jacobi sweeps of the last core factorization.
enum { FLAGW_BITS = 0, FLAGW_TICKET = 1, FLAGW_SWEEPS = 2, FLAGW_COUNT = 4 };

// A handle's persistent device allocation: the status words, then (from byte
// STATUS_BYTES) the composed filters the learned restriction's forward pass
// builds per call (used only on the handle's own stream, like the status words).
constexpr size_t STATUS_BYTES = 256;
constexpr size_t CONV_FILTER_BYTES = 16 * 1024;
constexpr size_t HANDLE_DEV_BYTES = STATUS_BYTES + CONV_FILTER_BYTES;
inline float *conv_filter_ws(int *dflags) {
  return reinterpret_cast<float *>(reinterpret_cast<char *>(dflags) + STATUS_BYTES);
}

struct dsk_handle {
  int device;
  hipStream_t stream;
  char *arena;
  size_t arena_bytes;
  int *dflags;        // device flag words (FLAGW_COUNT ints), persistent
  int cu_count;
  size_t max_lds;
  // optional event timing of the projection kernel (B^T = A^T Q)
  int timing;
  int tcount;
  hipEvent_t *tev;    // 2 * TIMING_CAP events
  // batched execution: worker sub-handles (own stream, arena and status words),
  // fork/join events, and the cache of instantiated graphs keyed by batch contents
  std::vector<dsk_handle *> workers;
  std::vector<hipEvent_t> wev;        // [0] fork, [1 + w] join of worker w
  hipStream_t capst = nullptr;        // capture origin (the caller's stream may be the legacy NULL stream)
  std::unordered_map<uint64_t, hipGraphExec_t> graphs;
  std::vector<uint64_t> graph_order;
};

constexpr int TIMING_CAP = 4096;
constexpr int ELL_CAP = 112;       // widest range finder / projection tile set
constexpr int ELL_CAP_F64 = 100;   // widest range finder of FP64 input (the FP64 core SVD's LDS)

// next (start, stop) event pair for a timed projection launch, or nulls
inline void timing_slot(dsk_handle *h, hipEvent_t *e0, hipEvent_t *e1) {
  *e0 = *e1 = nullptr;
  if (h->timing && h->tev && h->tcount < TIMING_CAP) {
    *e0 = h->tev[2 * h->tcount];
    *e1 = h->tev[2 * h->tcount + 1];
    ++h->tcount;
  }
}

// Bump allocator over the handle arena; sizes are 256-byte aligned.
struct Carve {
  char *base;
  size_t off;
  size_t cap;
  bool dry;           // true: only count bytes
  template <class T>
  T *take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T *p = dry ? nullptr : reinterpret_cast<T *>(base + off);
    off += bytes;
    return p;
  }
};

int arena_reserve(dsk_handle *h, size_t bytes);
void destroy_workers(dsk_handle *h);   // batch.hip

// Kernels whose dynamic LDS exceeds 64 KB must opt in (gfx950 offers 160 KB per
// workgroup).  The largest size granted so far is remembered per kernel, so the
// attribute call is made once per growth (never again while a stream is being
// captured into a graph for sizes already granted).
void allow_lds_raw(const void *kernel, size_t bytes);
template <typename K>
inline void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) allow_lds_raw(reinterpret_cast<const void *>(kernel), bytes);
}

// api.hip: the sketch-SVD sequence, shared with the batched entry point
int svd_check(const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k, const dsk_restriction *R,
              int32_t q, const dsk_opts *o, void *U, double *S, void *V, dsk_opts *odp, int64_t *s_out, int *L_out);
// after_projection (may be null) is called once B^T = A^T Q has been enqueued
// (work forked from the handle's stream at that point starts after it).
// single_pass: SPC-SVD (Alg. 3, q must be 0): the pass over A forms H = A^T Y
// while a worker stream orthonormalises Y, then B^T = H R^{-1}.
// orth_z = false: each power step forms Y = A_g (A_g^T Q) without
// orthonormalising the middle block (the same span; used where the steps are
// plain subspace iteration, not the paper's C-PWR).
int svd_run(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k,
            const dsk_restriction *R, int32_t q, const dsk_opts &od, int64_t s, int L, void *U, double *S, void *V,
            dsk_info *info, size_t *need, const std::function<int()> *after_projection = nullptr,
            bool single_pass = false, bool orth_z = true);
int ensure_workers(dsk_handle *h, int nw);   // batch.hip
int id_check(const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k, const dsk_restriction *R,
             int32_t q, const dsk_opts *o, int64_t *skel, double *P, dsk_opts *odp, int64_t *s_out, int64_t *cols_out,
             int64_t *ell_out);
// phase 0: the whole row ID.  phase 1 then phase 2 on the same stream: the
// same work split where the one-launch pivoted QR reads the restricted columns
// in their storage dtype (phase 1: the status reset and that gather, which need
// only A; phase 2: the rest); on the other paths phase 1 does nothing and
// phase 2 everything.
int id_run(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k,
           const dsk_restriction *R, int32_t q, const dsk_opts &od, int64_t s, int64_t cols, int64_t ell,
           int64_t *skel, double *P, void *skel_rows, dsk_info *info, size_t *need, int phase = 0);
int read_info_words(dsk_handle *h, dsk_info *info, int ell);

// ---------------------------------------------------------------- launchers
// restrict.hip
int launch_restrict(hipStream_t st, const void *A, int dtype, int64_t m, int64_t n, int64_t lda,
                    const dsk_restriction *R, int64_t s, int work_f64, void *Ac, void *AcT, int *dflags);
// A_g = A(:, I), C-PWR's Gram sub-sample (Alg. 7): the index set of an index
// restriction, else the direct-injection points of the restriction's grid
// (factor 4 x 4 for the learned conv); m x s compact in the work dtype.
int launch_gram_sample(hipStream_t st, const void *A, int dtype, int64_t m, int64_t n, int64_t lda,
                       const dsk_restriction *R, int64_t s, int work_f64, void *Ag, int *dflags);
int launch_select_cols(hipStream_t st, const void *Ac, int work_f64, int64_t m, int64_t s,
                       int64_t ldc, int ell, void *Y);
int launch_gather_rows(hipStream_t st, const void *A, int dtype, int64_t m, int64_t n, int64_t lda,
                       const int64_t *rows, int k, void *out);
// out (m x s, 16-bit) = A(:, index) of a DSK_R_INDEX restriction, A 16-bit, bits unchanged
int launch_gather_cols16(hipStream_t st, const void *A, int64_t m, int64_t n, int64_t lda, const dsk_restriction *R,
                         int64_t s, void *out);
int launch_convert(hipStream_t st, const void *src, int src_f64, void *dst, int dst_f64, int64_t count);
int launch_transpose(hipStream_t st, const void *src, int f64, int64_t rows, int64_t cols, void *dst);

// conv.hip (learned linear restriction)
int conv_shape_ok(int64_t n, int ny, int nx, int C);
int launch_conv_fwd(hipStream_t st, const void *A, int dtype, int64_t m, int64_t lda, int ny, int nx, int C,
                    const float *w1, const float *w2, int out_f64, void *Ac, int64_t ldc, float *filt_ws);
size_t conv_bwd_ws_bytes(int64_t m, int ny, int nx, int C);
int launch_conv_bwd(hipStream_t st, const void *A, int dtype, int64_t m, int64_t lda, int ny, int nx, int C,
                    const float *w1, const float *w2, const void *gAc, int g_f64, int64_t ldg, float *gw1,
                    float *gw2, void *ws);

// spc.hip: M = R^{-1} (FP64, upper triangular) from an upper-triangular R
// (ell x ell row-major); ell <= 112; u_data = unit roundoff of Y's data (rank test)
int launch_spc_rinv(hipStream_t st, const double *G, int ell, double u_data, double *M, int *dflags);

// smallmat.hip (tall-skinny orthonormalisation, small factorizations)
size_t cholqr2_ws_bytes(int64_t rows, int ell);
// ell <= 64 (cholqr64.hip): MFMA Gram partials, one-workgroup factorization,
// blocked forward substitution; same contract as launch_cholqr2.
size_t cholqr64_ws_bytes(int64_t rows, int ell);
int launch_cholqr64(hipStream_t st, const void *Y, int f64, int64_t rows, int ell, void *Q, void *ws, int *dflags,
                    int passes);
// out = X L^{-T} (rows x ell, one 64-row chunk per workgroup) with the factor L that
// the last launch_cholqr64 on ws computed (with passes = 1: Y^T Y = L L^T)
int launch_cholqr64_apply(hipStream_t st, const void *X, int f64, int64_t rows, int ell, const void *ws, void *out,
                          int *dflags);
// 64 < ell <= 128 (cholqr128.hip): the same contract, Gram partials + fold/factor
// + blocked-substitution apply per pass.
size_t cholqr128_ws_bytes(int64_t rows, int ell);
// out = X L^{-T} with the factor L the last launch_cholqr128 on ws computed
// (with passes = 1: Y^T Y = L L^T), by the same blocked substitution
int launch_cholqr128_apply(hipStream_t st, const void *X, int f64, int64_t rows, int ell, const void *ws, void *out,
                           int *dflags);
int launch_cholqr128(hipStream_t st, const void *Y, int f64, int64_t rows, int ell, void *Q, void *ws, int *dflags,
                     int passes);
// passes = 2: CholeskyQR2 (orthonormal to working precision); passes = 1: one
// CholeskyQR pass, an orthonormal-up-to-kappa^2 u basis of span(Y) (enough
// where only the span is used, as in the intermediate power steps).
int launch_cholqr2(hipStream_t st, const void *Y, int f64, int64_t rows, int ell, void *Q,
                   void *ws, int *dflags, double *Rout, int passes = 2);
int launch_hhqr(hipStream_t st, double *X, int64_t rows, int ell, double *Q, double *R, int *dflags);
int launch_gram(hipStream_t st, const void *X, int f64, int64_t rows, int ell, double *G,
                double *part, int nparts);
// gram64.hip: the same on the FP64 matrix cores (ell <= 128), at most
// gram_mfma_blocks(rows) <= nparts partials
int gram_mfma_blocks(int64_t rows);
int launch_gram_mfma(hipStream_t st, const void *X, int f64, int64_t rows, int ell, double *G, double *part,
                     int nparts);
// tile-major lower-tile partials (16 x 16 tiles numbered I (I + 1) / 2 + J), one per
// rows_per_blk rows (a multiple of 32): ceil(rows / rows_per_blk) partials of
// nb (nb + 1) / 2 * 256 doubles each, nb = ceil(ell / 16)
int launch_gram_tiles(hipStream_t st, const void *X, int f64, int64_t rows, int ell, int64_t rows_per_blk,
                      double *part);
// refine.hip: FP64 re-orthonormalisation of the assembled FP32 factors (U0 m x k,
// V0 n x k, S k) into U, V, S with U S V^T unchanged (k <= 100); ws: refine_ws_bytes(k);
// sws: the stream workspace of an n-row product with K = k (the mode's FP32 products)
size_t refine_ws_bytes(int k);
int launch_refine(hipStream_t st, const float *U0, int64_t m, const float *V0, int64_t n, int k, double *S,
                  float *U, float *V, double *part, int nparts, double *ws, int *dflags, int mode, void *sws,
                  int cu_count);
// jacobi.hip
int launch_core_eig(hipStream_t st, const double *G, int ell, double *lam, double *U, int *dflags);
// the same, run only where *gate != 0 (gate may be null: always); count matrices, one workgroup each
int launch_core_eig_gated(hipStream_t st, const double *G, int ell, double *lam, double *U, int *dflags,
                          const int *gate, int count);
// eigtri.hip: the same eigenpairs by Householder tridiagonalisation, multisection and
// twisted-factorisation eigenvectors (3 <= ell <= 112), with the Jacobi core as a gated
// fallback; ws: core_eig_tri_ws_bytes(ell)
size_t core_eig_tri_ws_bytes(int ell);
int launch_core_eig_tri(hipStream_t st, const double *G, int ell, double *lam, double *U, double *ws, int *dflags);
// count independent ell x ell matrices (consecutive), one workgroup each
int launch_core_eig_batched(hipStream_t st, const double *G, int ell, double *lam, double *U, int *dflags,
                            int count);
// spcerr.hip: row Gram G = X X^T (r <= 112 rows of length ncols, row stride ldx) in FP64;
// part: spc_err_parts(ncols) * r^2 doubles
int spc_err_parts(int64_t ncols);
int launch_row_gram(hipStream_t st, const void *X, int dtype, int r, int64_t ncols, int64_t ldx, double *part,
                    double *G);
// eps[i] = c lambda_max(Gf - taus[i] Gc) for i < ntau (Mb: ntau r^2, sig: ntau, lam: ntau r, Ub: ntau r^2)
int launch_eps_curve(hipStream_t st, const double *Gf, const double *Gc, int r, const double *taus, int ntau,
                     double c, double *Mb, double *sig, double *lam, double *Ub, double *eps, double *rho,
                     int *dflags);
int launch_jacobi_svd(hipStream_t st, const double *Rm, int ell, double *sig, double *Vr,
                      double *Ur, int *dflags);
int launch_tsmm(hipStream_t st, const void *X, int f64, int64_t rows, int ell, int64_t ldx,
                const double *M, int ldm, int kout, const double *colscale, void *out, int64_t ldo);
int launch_sign_fix(hipStream_t st, void *U, int f64, int64_t m, int k, double *sign);
int launch_fro2(hipStream_t st, const void *A, int dtype, int64_t m, int64_t n, int64_t lda,
                double *part, int nparts, double *out);

// stream.hip (B^T = X^T Y and X Y for tall-skinny Y)
// argument checks of dsk_project (0 or -i for argument i)
int project_args(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, const void *Q,
                 int32_t ell, void *Bt, int32_t mode);
// noalloc.hip: takes the device address of dsk_project_noalloc's fixed scratch
// on `device` (current); called by dsk_create
int noalloc_setup(int device);
size_t stream_ws_bytes(int dtype, int64_t K, int64_t N, int ell, int mode);
// the workspace launch_stream (X^T Y) uses at these sizes on a device with cu_count CUs
// (at most stream_ws_bytes)
size_t stream_scratch_bytes(int dtype, int64_t K, int64_t N, int ell, int mode, int cu_count);
int launch_stream(hipStream_t st, const void *X, int dtype, int64_t K, int64_t N, int64_t ldx,
                  const void *Y, int f64y, int ell, void *out, int64_t ldo, int mode, void *ws,
                  int cu_count, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
int launch_stream_nn(hipStream_t st, const void *X, int dtype, int64_t M, int64_t K, int64_t ldx,
                     const void *Y, int ell, void *out, int64_t ldo, int mode, void *ws, int cu_count);
// autotuner of the TN projection's K-split for one (dtype/mode, K, N, ell) shape:
// times the candidates on X with scratch Y (K x ell f32) and out (N x ell f32),
// records the fastest in the process-wide table the launchers consult.
int stream_autotune(hipStream_t st, const void *X, int dtype, int64_t K, int64_t N, int64_t ldx, int ell, int mode,
                    void *ws, void *Y, void *out, int cu_count, int *best_ns, float *best_ms);

// cpqr.hip (row ID)
int launch_cpqr(hipStream_t st, double *W, int64_t m, int64_t s, int k, double *nu0, double *nu1,
                double *Rk, int64_t *piv, int *dflags);
// rowid_reg.hip: all k pivot steps in one launch with W's rows in registers
// (left-looking form, downdated norms); 0 bytes = shape not supported.  W's
// dtype wdt: DSK_F64, or DSK_F32 / DSK_BF16 / DSK_F16 holding the stored values
// exactly (products and sums in FP64 either way).  Outputs as launch_cpqr's,
// final norms in nu_final.
size_t rowid_reg_ws_bytes(int64_t m, int64_t s, int k, int wdt, int cu_count);
int launch_rowid_reg(hipStream_t st, const void *W, int wdt, int64_t m, int64_t s, int k, double *nu_final,
                     double *Rk, int64_t *piv, void *ws, int cu_count, int *dflags);
int launch_id_solve(hipStream_t st, const double *Rk, const int64_t *piv, const double *nu_final,
                    int64_t m, int k, double *P, int *dflags);

// gemm64.hip (small FP64 GEMM for the full-sketch ID power block)
int launch_gemm64(hipStream_t st, int transA, int transB, int64_t M, int64_t N, int64_t K,
                  double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                  double *C, int64_t ldc, double beta = 0.0);

// device helpers
__device__ __forceinline__ float bf16_bits_to_f32(unsigned short b) {
  return __uint_as_float(((unsigned)b) << 16);
}
__device__ __forceinline__ float f16_bits_to_f32(unsigned short b) {
  return (float)__builtin_bit_cast(_Float16, b);
}

/*
 * dsketch.h -- C ABI of the deterministic-sketch low-rank SVD / row-ID path
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Dunton & Doostan, "Deterministic matrix sketches for low-rank
 * compression of high-dimensional simulation data" (arXiv 2105.01271).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * A is an m x n snapshot matrix, ROW-MAJOR with leading dimension lda >= n:
 *    one row per snapshot (time step / parameter), one column per fine-grid
 *    dof (Sec. 2).  A 2-D field on an ny x nx grid is flattened y-major
 *    (column = iy*nx + ix).
 *  * Every array argument is a DEVICE pointer owned by the caller unless it is
 *    marked "host".  The library never frees caller memory and keeps no
 *    pointer past the call.
 *  * Storage dtypes of A: DSK_F64, DSK_F32, DSK_BF16, DSK_F16.  The work dtype
 *    (dtype of every floating output except S and P) is F64 for F64 input and
 *    F32 otherwise.  Singular values S and the interpolation matrix P are F64.
 *  * Work is enqueued on the handle's stream and is asynchronous: outputs are
 *    valid after the stream is synchronised.  Passing a non-NULL dsk_info
 *    makes the call synchronise the stream before it returns.
 *  * Return value: 0 on success; -i when argument i (1-based) is invalid,
 *    detected on the host before anything is enqueued (no side effects);
 *    DSK_ERR_* (> 100) for HIP runtime errors (100 + hipError_t);
 *    DSK_ERR_SCRATCH (90) from dsk_project_noalloc (size beyond its fixed scratch).
 *    Numerical events (fallback taken, rank deficiency, non-finite input)
 *    are reported through dsk_info.flags, not through the return value.
 *  * Scratch memory comes from a per-handle arena that grows on demand
 *    (hipMalloc) and is reused across calls; the first call at a new largest
 *    size allocates.
 *  * A handle is bound to one device and one stream and must not be used by
 *    two host threads at once.
 */
#ifndef DSKETCH_H
#define DSKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dsk_handle dsk_handle;

enum { DSK_F64 = 0, DSK_F32 = 1, DSK_BF16 = 2, DSK_F16 = 3 };

/* Restriction kinds: the sketch D of A_c = A D (Sec. 2), never formed. */
enum {
  DSK_R_INDEX = 0,   /* direct injection / Gram sub-sample: A_c = A(:, index) (Sec. 2; Alg. 7) */
  DSK_R_NN = 1,      /* nearest neighbour, weights (1/4,1/2,1/4) per axis around DI points (Sec. 2) */
  DSK_R_GLOBAL = 2,  /* global sketch: mean over the sy x sx block at each DI point (Sec. 2) */
  DSK_R_LEARNED = 3  /* learned linear 2-layer strided conv (not in the paper) */
};

/* Product modes for F32 input (B = Q^T A and the coarse power products). */
enum {
  DSK_MODE_DEFAULT = 0,  /* = DSK_MODE_SPLIT6 */
  DSK_MODE_SPLIT3 = 1,   /* A and Q split into bf16 hi+lo halves, 3 bf16 MFMA products (~2^-16 relative) */
  DSK_MODE_F32 = 2,      /* plain f32 MFMA products */
  DSK_MODE_SPLIT6 = 3    /* A and Q split exactly into three bf16 pieces, the 6 products of order >= 2^-16
                            kept (~2^-24 relative, f32 rounding level), f32 accumulation */
};

/* flag bits reported in dsk_info.flags */
enum {
  DSK_FLAG_FALLBACK = 1,        /* a shifted Cholesky-QR fallback was taken */
  DSK_FLAG_RANK_DEFICIENT = 2,  /* a triangular factor had a negligible pivot */
  DSK_FLAG_NONFINITE = 4,       /* NaN/Inf met in a Gram or residual norm */
  DSK_FLAG_BAD_INDEX = 8,       /* an index of the restriction was outside [0, n); column 0 was used */
  DSK_FLAG_SYNC_TIMEOUT = 16    /* a workgroup of the one-launch pivoted QR waited past its spin limit (its
                                   workgroups were not all resident); a one-workgroup kernel then redid the
                                   factorization, so the ID outputs are valid (but slow to come) */
};

typedef struct {
  int32_t kind;            /* DSK_R_* */
  int64_t s;               /* DSK_R_INDEX: number of coarse columns |I| */
  const int64_t *index;    /* DSK_R_INDEX: device, s distinct column indices in [0, n) */
  int32_t ny, nx;          /* NN / GLOBAL / LEARNED: fine grid, n = ny*nx */
  int32_t sy, sx;          /* NN / GLOBAL: coarse factor per axis (coarse grid ceil(ny/sy) x ceil(nx/sx)) */
  int32_t channels;        /* LEARNED: hidden channels C */
  const float *w1;         /* LEARNED: device, layer-1 taps [C][5][5], stride 2, pad 2 */
  const float *w2;         /* LEARNED: device, layer-2 taps [C][5][5], stride 2, pad 2 */
} dsk_restriction;

typedef struct {
  int32_t p;          /* oversampling; range-finder width ell = min(k+p, s, m); default 10 */
  const void *S;      /* optional device s x ell second-level sketch, row-major, work dtype;
                         NULL = nested direct injection (every floor(s/ell)-th coarse column) */
  int32_t ell;        /* width of S when S != NULL: 1 <= ell <= min(s, 112) (and <= m, and <= 100 for FP64 input, for the SVD) */
  double tau;         /* coarse Gram scale (Sec. 5); <= 0 means n/s */
  int32_t id_projected; /* sketch_id: 0 = ID of W_q = (tau A_c A_c^T)^q A_c (full coarse sketch),
                           1 = ID of the ell-wide block (tau A_c A_c^T)^q A_c S */
  int32_t mode;       /* DSK_MODE_* (F32 input only) */
  int32_t refine;     /* sketch_svd with FP32 / 16-bit input: 1 = one FP64 refinement sweep of the
                         assembled factors: with FP64 Grams U^T U = R_U^T R_U and V^T V = R_V^T R_V,
                         the k x k matrix R_U diag(S) R_V^T = U_m S' V_m^T is decomposed and
                         U <- U R_U^-1 U_m, V <- V R_V^-1 V_m, S <- S', so that U S V^T is unchanged
                         and U, V are orthonormal to the rounding of their storage (requires k <= 100;
                         ignored for FP64 input) */
  int32_t id_per_step; /* sketch_id pivoted QR: 0 = all k pivot steps in one launch when the ID matrix's
                          rows fit the registers of one workgroup per compute unit (m <= 4 or 8 x compute
                          units, m <= 2048, at most 8192 wide), else one launch per step; 1 = always one
                          launch per pivot step.  The one launch takes the left-looking form of the pivoted
                          QR with downdated residual norms, the per-step launches the right-looking form
                          with recomputed norms: the same pivots wherever they are separated, P to rounding. */
} dsk_opts;

typedef struct {       /* host struct, filled when passed */
  int32_t ell;         /* range-finder width used */
  int32_t flags;       /* DSK_FLAG_* bits */
  double normA_fro2;   /* ||A||_F^2 (sketch_svd only) */
  double normB_fro2;   /* ||Q^T A||_F^2 (sketch_svd only): projection error^2 = normA - normB */
  double sigma_tail;   /* sigma_{k+1} of B = Q^T A when ell > k, else 0 */
  int32_t core_sweeps; /* Jacobi sweeps of the ell x ell core factorization (sketch_svd) */
  int32_t reserved;    /* 0 */
} dsk_info;

/* Fill *o with the defaults listed above. */
void dsk_opts_default(dsk_opts *o);

/* Create a handle bound to `device` and `stream` (a hipStream_t; NULL = default stream).
   *h receives the handle.  A handle owns a device arena (grown on demand), status
   words and, once a call needs them, worker streams with arenas of their own; calls
   on one handle must not overlap (one host thread at a time).
   Errors: -1 (h NULL), DSK_ERR_* (HIP). */
int dsk_create(dsk_handle **h, int device, void *stream);
/* Wait for the handle's stream and worker streams, then free everything the handle
   owns (arenas, status words, worker streams, events).  Errors: -1 (h NULL). */
int dsk_destroy(dsk_handle *h);
/* Rebind the handle's stream: later calls enqueue on `stream` (a hipStream_t, NULL =
   default stream).  Work already enqueued stays where it is; ordering the old stream
   before the new one is the caller's.  Errors: -1 (h NULL). */
int dsk_set_stream(dsk_handle *h, void *stream);

/*
 * dsk_restrict -- A_c = A D for the given restriction (Sec. 2 sketch equation;
 * direct injection, nearest-neighbour and global sketch equations; learned conv).
 *   A    (1) device m x n, row-major, lda
 *   Ac   (8) device m x s output, row-major compact, work dtype
 * Argument numbers: h=1, A=2, dtype=3, m=4, n=5, lda=6, R=7, Ac=8.
 */
int dsk_restrict(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                 const dsk_restriction *R, void *Ac);

/*
 * dsk_project -- B^T = A^T Q, the projection B = Q^T A of TPC-SVD (Alg. 2;
 * Sec. 3.1) written transposed: the one full pass over A.
 * Arguments: h=1, A=2, dtype=3, m=4, n=5, lda=6, Q=7 (m x ell row-major, work dtype),
 *   ell=8 (1..112), Bt=9 (n x ell row-major, work dtype), mode=10 (DSK_MODE_*).
 */
int dsk_project(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                const void *Q, int32_t ell, void *Bt, int32_t mode);

/*
 * dsk_project_noalloc -- dsk_project without any device allocation, for callers
 * that cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernels and launch plan as
 * dsk_project, so the same bytes in Bt.  The workspace (the packed Q and, when
 * the pass is split over the rows of A, the per-split partial outputs) is a
 * fixed device array of DSK_NOALLOC_SCRATCH_BYTES (32 MiB) that the library
 * holds on every device it runs on, from the first dsk_create on that device
 * until the process ends.  The caller passes A, Q and Bt and creates the handle
 * beforehand; the call itself allocates nothing (no hipMalloc, no arena growth).
 * Calls on one device share the array: calls that overlap on a device (other
 * streams, handles or threads) race.  Errors: as dsk_project; DSK_ERR_SCRATCH
 * when this size's plan needs more than DSK_NOALLOC_SCRATCH_BYTES (nothing is
 * enqueued).  The plan needs 3 ceil(m / 32) ceil(ell / 16) KiB (rounded up to
 * 256 bytes) for F32 / 16-bit input, plus split partials (4 or 8 bytes per
 * n * ell per split) when n alone is too small to fill the device.
 */
#define DSK_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
#define DSK_ERR_SCRATCH 90
int dsk_project_noalloc(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                        const void *Q, int32_t ell, void *Bt, int32_t mode);

/*
 * dsk_sketch_svd -- rank-k SVD A ~ U diag(S) V^T by TPC-SVD (Alg. 2) with q
 * steps of the single-pass coarse power iteration C-PWR (Alg. 7):
 *   A_c = A D; Y = A_c S_ell; Q = orth(Y); q times { Z = orth(tau A_g^T Q); Q = orth(A_g Z) };
 *   B = Q^T A (the one full pass over A); SVD(B) = U_B Sigma V_B^T;
 *   U = Q U_B(:, :k), S = Sigma(:k), V = V_B(:, :k).
 * A_g = A(:, I) is C-PWR's Gram sub-sample, which Alg. 7 keeps apart from the
 * sketch D: for DSK_R_INDEX the restriction's own index set (A_g = A_c), for
 * NN / GLOBAL the direct-injection points of the same grid and factor, for
 * LEARNED those of its stride-4 output grid (s columns in every case).
 * Each (u_j, v_j) is sign-normalised so the largest-magnitude entry of u_j
 * (lowest index on ties) is positive.
 * Range finder width ell = min(k + p, s, m, 112), or the given S's width; at most
 * 100 for FP64 input (its core SVD holds two ell x ell FP64 blocks in LDS).
 * Arguments: h=1, A=2, dtype=3, m=4, n=5, lda=6, k=7 (1 <= k <= ell), R=8, q=9 (>= 0),
 *   o=10 (host, may be NULL = defaults), U=11 (m x k row-major, work dtype),
 *   S=12 (k, F64), V=13 (n x k row-major, work dtype), info=14 (host, may be NULL).
 */
int dsk_sketch_svd(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                   int32_t k, const dsk_restriction *R, int32_t q, const dsk_opts *o,
                   void *U, double *S, void *V, dsk_info *info);

/*
 * dsk_sketch_svd_sp -- rank-k SVD by the single-pass SPC-SVD (Alg. 3): the one
 * pass over A forms H = A^T Y for the start block Y = A_c S_ell (same Y as
 * dsk_sketch_svd), Y = Q R, and B^T = H R^{-1} = A^T Q (the identity derived
 * under Alg. 3) replaces the second pass; then SVD(B) and U, S, V as in
 * dsk_sketch_svd.  No power iteration (Alg. 3 has none).  In exact arithmetic
 * the result equals dsk_sketch_svd with q = 0; in floating point the rounding
 * of H is amplified by kappa(Y) = ||Y|| ||R^{-1}||, as the formula implies, so
 * the two agree to about u kappa(Y) sigma_1 (u = 2^-24 for FP32 input).
 * R: FP64, the Cholesky factor of the FP64 Gram Y^T Y with Q = Y R^{-1} (FP32 /
 * 16-bit input; one CholeskyQR pass, and B^T = H R^{-1} by the same blocked
 * substitution) or the Householder R of Y (FP64 input).  A numerically
 * rank-deficient Y (where the formula breaks down) raises DSK_FLAG_FALLBACK
 * (shifted factor) or DSK_FLAG_RANK_DEFICIENT.  The orthonormalisation of Y runs
 * on a worker stream of the handle, concurrently with the pass.
 * Arguments: h=1, A=2, dtype=3, m=4, n=5, lda=6, k=7 (1 <= k <= ell), R=8,
 *   o=9 (host, may be NULL; refine must be 0), U=10 (m x k row-major, work dtype),
 *   S=11 (k, F64), V=12 (n x k row-major, work dtype), info=13 (host, may be NULL).
 */
int dsk_sketch_svd_sp(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                      int32_t k, const dsk_restriction *R, const dsk_opts *o,
                      void *U, double *S, void *V, dsk_info *info);

/*
 * dsk_spc_id_err -- the single-pass error estimate of SPC-ID (SPC-ID-ERR,
 * Alg. 6) at given scales tau:
 *   eps[i] = c lambda_max(B_f B_f^T - taus[i] B_c B_c^T),  c = floor(m / mc),
 * where B_f holds the rows i of A with (i + 1) mod c == 0 (floor(m / c) rows,
 * the rows Alg. 6 keeps while streaming A) and B_c = B_f D their coarse rows;
 * with every row kept (mc = m) this is eps(tau) of the SPC-ID bound (Sec. 4).
 * Alg. 6 writes a minimum over tau; lambda_max(B_f B_f^T - tau B_c B_c^T) is
 * non-increasing in tau (B_c B_c^T is positive semidefinite), so the scales
 * are chosen by the caller and the minimum over them is eps's minimum.
 * Grams in FP64 from the stored values; eigenvalues by the core eigensolver on
 * the positive semidefinite shift M + ||M||_F I (absolute error about
 * 1e-12 c (|tr M| + r ||M||_F)).
 * With rho, the same kept rows also give the estimate of the Gram mismatch
 * rho(tau) = ||A_f A_f^T - tau A_c A_c^T||_2 of the C-PWR analysis (Sec. 5):
 *   rho[i] = c ||B_f B_f^T - taus[i] B_c B_c^T||_2 = c max(lambda_max, -lambda_min),
 * from the same eigenvalues (rho(tau) itself when mc = m).
 * Arguments: h=1, A=2, dtype=3, m=4, n=5, lda=6, R=7, mc=8 (1 <= mc <= m, with
 *   floor(m / floor(m / mc)) <= 112 kept rows), taus=9 (device F64, ntau values),
 *   ntau=10 (1..1024), eps=11 (device F64, ntau), rho=12 (device F64, ntau; NULL
 *   when not wanted).
 * Errors: -1..-7 as for dsk_restrict's arguments 1..7 (-7: restriction invalid),
 *   -8 mc, -9 taus NULL, -10 ntau, -11 eps NULL.
 */
int dsk_spc_id_err(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                   const dsk_restriction *R, int32_t mc, const double *taus, int32_t ntau, double *eps,
                   double *rho);

/*
 * dsk_sketch_id -- rank-k row interpolative decomposition A ~ P A(I, :) by
 * TPC-ID (Alg. 4): column-pivoted QR of W^T (Sec. 4, row ID) with W = A_c, or
 * W = (tau A_g A_g^T)^q A_c for q >= 1 (C-PWR without re-orthonormalisation,
 * A_g the Gram sub-sample described under dsk_sketch_svd), pivots = largest
 * residual norm (squared norms ranked at 34 mantissa bits, lowest index on
 * ties; downdated while the pivot's squared norm stays above 1e-5 of the
 * first pivot's, recomputed from the residuals after that);
 * C = R_1^{-1} R_2; P(I, :) = I_k, P(rest, :) = C^T.  When R_1 has negligible
 * pivots (|r_jj| <= 1e-14 |r_11|, a suffix of its diagonal) the least-squares
 * problem R_1 C = R_2 has many solutions and the basic one is returned: zero
 * coefficients for those pivots, the leading triangle solved for the rest;
 * DSK_FLAG_RANK_DEFICIENT is raised.
 * Arguments: h=1, A=2, dtype=3, m=4, n=5, lda=6, k=7 (1 <= k <= min(m, s) or ell),
 *   R=8, q=9, o=10 (host, may be NULL), skel=11 (k int64, 0-based row indices in pivot order),
 *   P=12 (m x k row-major F64), skel_rows=13 (k x n row-major in A's dtype, or NULL),
 *   info=14 (host, may be NULL).
 */
int dsk_sketch_id(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                  int32_t k, const dsk_restriction *R, int32_t q, const dsk_opts *o,
                  int64_t *skel, double *P, void *skel_rows, dsk_info *info);

/*
 * dsk_spc_id -- rank-k row ID by the single-pass SPC-ID (Alg. 5, Sec. 4):
 *   A ~ P X,  X = A_c(I, :) T_r,  T_r = A_c^+ U_r U_r^T A = V_r S_r^{-2} V_r^T H^T,
 * where the one pass over A forms A_c = A D and H = A^T A_c (n x s), U_r S_r V_r^T
 * are the leading r singular triplets of A_c (the lifting operator's rank r acts
 * as a regulariser, k <= r <= rank(A_c)), and (I, P) is the row ID of A_c, i.e.
 * exactly dsk_sketch_id's at q = 0.  The singular triplets of A_c come from the
 * sketch SVD of A_c with every coarse column kept and qc subspace-iteration
 * steps (range finder width ell = min(m, s, 112), 100 for FP64 input): the r-th singular
 * direction's error falls like (sigma_{ell+1} / sigma_r)^(2 qc + 1), so qc sets
 * how close this is to the exact SVD of Alg. 5.  Singular values at or below
 * max(m, s) eps sigma_1 (eps the machine epsilon of the work precision) are
 * dropped from S_r^{-2} (the pseudo-inverse) and raise DSK_FLAG_RANK_DEFICIENT.  T_r is never formed:
 * X = (A_c(I, :) V_r) W_r with W_r = S_r^{-2} V_r^T H^T, and T_r = V_r W_r.
 * Work precision: FP64 for FP64 input, else FP32 (H on the projection kernel:
 * FP32 to about 2^-24 relative, exact products for 16-bit storage); the
 * rounding of H is amplified by about sigma_1 / sigma_r in X.
 * The row ID and the SVD of A_c run on two worker streams of the handle beside
 * the pass over A; the call is ordered on the handle's stream like any other.
 * Arguments: h=1, A=2, dtype=3, m=4, n=5, lda=6, k=7 (1 <= k <= min(m, s)),
 *   r=8 (k <= r <= ell), R=9, qc=10 (0..64), o=11 (host, may be NULL;
 *   mode is used, S and id_projected must be unset), skel=12 (device, k
 *   int64), P=13 (device, m x k row-major F64), X=14 (device, k x n row-major,
 *   work dtype), Vr=15 (device, s x r row-major, work dtype, or NULL),
 *   Wr=16 (device, r x n row-major, work dtype, or NULL), info=17 (host, may be
 *   NULL: flags of all three streams, core_sweeps and ell of the SVD of A_c).
 * Workspace: n s (H) + about (m + n + 3 s) r + (n + 2 s) k elements of the work
 * dtype in the handle's arena, plus the two workers' arenas.
 * Errors: -1..-7 and -9 as dsk_sketch_id's arguments 1..8, -8 r, -10 qc,
 *   -11 o (a second-level sketch or projected ID asked for), -12 skel NULL,
 *   -13 P NULL, -14 X NULL.
 */
int dsk_spc_id(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k,
               int32_t r, const dsk_restriction *R, int32_t qc, const dsk_opts *o, int64_t *skel, double *P,
               void *X, void *Vr, void *Wr, dsk_info *info);

/*
 * dsk_power_iter -- the C-PWR loop alone (Alg. 7):
 *   q times { G = tau A_c^T G; [G = orth(G)]; G = A_c G; [G = orth(G)] }
 * starting from G = Q0, where Ac is the caller's Gram sub-sample A(:, I).  reorth = 1 orthonormalises after every product
 * (result = orthonormal m x ell basis), reorth = 0 returns the raw block.
 * Arguments: h=1, Ac=2 (m x s row-major, ldc), dtype=3 (DSK_F64 or DSK_F32), m=4, s=5,
 *   ldc=6, Q0=7 (m x ell row-major), ell=8, q=9, tau=10, reorth=11, Qout=12 (m x ell).
 */
int dsk_power_iter(dsk_handle *h, const void *Ac, int32_t dtype, int64_t m, int64_t s, int64_t ldc,
                   const void *Q0, int32_t ell, int32_t q, double tau, int32_t reorth, void *Qout);

/*
 * Batched execution (extension; not in the paper): independent sketch-SVD
 * problems of different shapes, dtypes and restrictions in one call.
 */
typedef struct {
  const void *A;       /* device m x n, row-major, lda */
  int32_t dtype;       /* DSK_F64 / F32 / BF16 / F16 */
  int64_t m, n, lda;
  int32_t k, q;        /* rank and power steps, as in dsk_sketch_svd */
  dsk_restriction R;   /* by value; its device arrays must stay valid for the call (and for graph replays) */
  void *U;             /* device m x k, work dtype */
  double *S;           /* device k */
  void *V;             /* device n x k, work dtype */
} dsk_problem;

enum { DSK_BATCH_GRAPH = 1 };   /* capture the batch into a HIP graph on first use, replay afterwards
                                   (currently disabled: the call returns -5, see below) */

/*
 * dsk_sketch_svd_batched -- dsk_sketch_svd (Alg. 2 + Alg. 7) for nprob problems.
 * The problems run concurrently on up to 8 worker streams owned by the handle
 * (longest-processing-time assignment on m*n), forked from and joined back
 * into the handle's stream.  With DSK_BATCH_GRAPH the launch sequence of a
 * given batch description (every field of every problem, the options, the
 * stream) is captured into a HIP graph on its first call (which also runs it)
 * and replayed with one graph launch on later calls; up to 16 graphs are kept.
 * Results are identical to nprob separate dsk_sketch_svd calls.
 * Arguments: h=1, nprob=2 (>= 1), probs=3 (host array), o=4 (host, may be NULL; shared),
 *   flags=5 (0 or DSK_BATCH_GRAPH), nworkers=6 (host int, may be NULL: workers used).
 * Errors: -1..-5 as numbered; -(1000 + i) when problem i fails the checks of
 *   dsk_sketch_svd; DSK_ERR_* (HIP).  No per-problem dsk_info is produced.
 *   DSK_BATCH_GRAPH is currently disabled and returns -5: a memory fault was
 *   observed on the capture-and-replay path and its cause has not been
 *   identified.  The eager path (flags = 0) is unaffected.
 */
int dsk_sketch_svd_batched(dsk_handle *h, int32_t nprob, const dsk_problem *probs, const dsk_opts *o, int32_t flags,
                           int32_t *nworkers);

/*
 * dsk_sketch_svd_id -- dsk_sketch_svd (TPC-SVD + C-PWR, Alg. 2 and Alg. 7) and
 * dsk_sketch_id (TPC-ID, Alg. 4) of the same matrix in one call: the row ID runs
 * on a worker stream of the handle, concurrently with the SVD on the handle's
 * stream, and joins back before the call's work ends on the handle's stream.
 * Outputs are identical to the two separate calls.
 * Arguments: h=1, A=2, dtype=3, m=4, n=5, lda=6, k=7, R=8, q_svd=9, q_id=10, o=11 (host, may be NULL),
 *   U=12, S=13, V=14 (as in dsk_sketch_svd), skel=15, P=16, skel_rows=17 (as in dsk_sketch_id),
 *   info_svd=18, info_id=19 (host, may be NULL).
 */
int dsk_sketch_svd_id(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k,
                      const dsk_restriction *R, int32_t q_svd, int32_t q_id, const dsk_opts *o, void *U, double *S,
                      void *V, int64_t *skel, double *P, void *skel_rows, dsk_info *info_svd, dsk_info *info_id);

/*
 * dsk_autotune -- time the K-split candidates of the projection B^T = A^T Q
 * (the one full pass over A) for this (dtype, mode, m, n, ell) on A itself,
 * and keep the fastest in a process-wide table that every later launch of that
 * shape uses.  Synchronises the handle's stream.
 * Arguments: h=1, A=2, dtype=3 (F32 / BF16 / F16), m=4, n=5, lda=6, ell=7 (1..112),
 *   mode=8 (DSK_MODE_*), nsplit=9 (host int, may be NULL), ms=10 (host float, may be NULL:
 *   time of one projection with the chosen split).
 */
int dsk_autotune(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t ell,
                 int32_t mode, int32_t *nsplit, float *ms);

/*
 * Learned linear restriction (extension; not in the paper).  R->kind ==
 * DSK_R_LEARNED: two 5x5 stride-2 zero-padded linear convolutions of every
 * row viewed as an ny x nx image, 1 -> C channels -> 1, no bias, no
 * activation (ny, nx multiples of 4, 1 <= C <= 32), so A_c = A D with s =
 * (ny/4)(nx/4) and the D of Sec. 2 replaced by the conv.  Weights: device
 * FP32, w1 [C][5][5] and w2 [C][5][5]; FP32 arithmetic.  dsk_restrict,
 * dsk_sketch_svd and dsk_sketch_id accept it like any other restriction.
 *
 * dsk_conv_restrict_bwd -- weight gradients of <gAc, A_c(w)>:
 *   gw1, gw2 (device FP32, C x 25 each) = d/dw1, d/dw2 of sum(gAc .* conv(A)).
 * Arguments: h=1, A=2, dtype=3, m=4, n=5, lda=6, R=7 (learned), gAc=8 (device
 *   m x s FP32 row-major), gw1=9, gw2=10.
 */
int dsk_conv_restrict_bwd(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                          const dsk_restriction *R, const float *gAc, float *gw1, float *gw2);

/*
 * dsk_learned_loss_grad -- training objective of the learned restriction: the
 * sketch error of Thm 3.2 in the Frobenius norm, normalised,
 *   L = ||A - Q Q^T A||_F^2 / ||A||_F^2,
 * with Q the ell-wide orthonormal block of the SVD path built from A_c = conv(A)
 * (nested direct-injection start block, q power steps with re-orthonormalisation,
 * Alg. 7), and its weight gradients (every QR factor R held constant: L depends
 * on Q only through its span).  Coarse algebra in FP64.
 * Arguments: h=1, A=2, dtype=3, m=4, n=5, lda=6, R=7 (learned), ell=8 (1..min(s, m, 112)),
 *   q=9 (0..8), loss=10 (host double), gw1=11, gw2=12 (device FP32, C x 25).
 * Synchronises the handle's stream (the loss is returned on the host).
 */
int dsk_learned_loss_grad(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                          const dsk_restriction *R, int32_t ell, int32_t q, double *loss, float *gw1, float *gw2);

/*
 * dsk_adam_step -- one Adam update (Kingma and Ba) of count FP32 parameters on
 * the device: m1 = b1 m1 + (1 - b1) g, m2 = b2 m2 + (1 - b2) g^2,
 * p -= lr (m1 / (1 - b1^t)) / (sqrt(m2 / (1 - b2^t)) + eps).
 * Arguments: h=1, param=2, grad=3, m1=4, m2=5 (device FP32), count=6, lr=7, beta1=8,
 *   beta2=9, eps=10, step=11 (t >= 1).
 */
int dsk_adam_step(dsk_handle *h, float *param, const float *grad, float *m1, float *m2, int64_t count, float lr,
                  float beta1, float beta2, float eps, int32_t step);

/*
 * Event timing of the projection kernel B^T = A^T Q (the dominant pass), for
 * benchmarks.  While enabled, dsk_sketch_svd and dsk_project bracket that one
 * kernel with two hipEvents recorded on the handle's stream (up to 4096 launches).
 * dsk_timing_read synchronises the stream, returns the number of timed launches
 * and their summed duration in milliseconds, and restarts the count.
 * Arguments: h=1, enable=2 / h=1, count=2 (host), total_ms=3 (host).
 */
int dsk_timing_enable(dsk_handle *h, int enable);
int dsk_timing_read(dsk_handle *h, int *count, double *total_ms);

/* Human-readable text of a return code. */
const char *dsk_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* DSKETCH_H */

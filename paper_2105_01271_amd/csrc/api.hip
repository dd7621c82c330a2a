// extern "C" entry points of libdsketch: argument validation, workspace
// carving and the launch sequence of each operation.  Every numerical step is
// one of the HIP kernels of this library; the host only validates, carves the
// arena and enqueues work on the handle's stream.
#include <string.h>

#include <algorithm>

#include "dsk_internal.h"

namespace {

__global__ void k_zero_flags(int *f) {
  if (threadIdx.x < FLAGW_COUNT) f[threadIdx.x] = 0;
}

__global__ void k_scale(void *x, int f64, int64_t count, double a) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    if (f64) reinterpret_cast<double *>(x)[t] *= a;
    else reinterpret_cast<float *>(x)[t] = (float)(reinterpret_cast<float *>(x)[t] * a);
  }
}

// sigma_c from eigenvalues (is_lam) or singular values
__device__ __forceinline__ double finish_sigma(const double *vals, int is_lam, int c) {
  const double v = vals[c];
  return is_lam ? sqrt(v > 0.0 ? v : 0.0) : v;
}

// the column scale of singular value c: its sign, divided by sigma_c when
// asked (zero for a negligible sigma_c)
__device__ __forceinline__ double finish_scale(const double *vals, int is_lam, const double *sign, int divide,
                                               int c) {
  const double sg = finish_sigma(vals, is_lam, c), s1 = finish_sigma(vals, is_lam, 0);
  double cs = sign ? sign[c] : 1.0;
  if (divide) cs = (sg > 1e-300 && sg > 1e-13 * s1) ? cs / sg : 0.0;
  return cs;
}

// Block 0: S, the V column scales and the info scalars ([0] = sum of all
// sigma^2 = ||B||_F^2, [1] = sigma_{k+1}), one thread per singular value
// (ell <= 128).  With Mv (FP32 path), every block also writes 256 entries of
// Mv = U_B(:, :k) diag(scale) in FP32 (ell x k, the right factor of
// V = B^T Mv; grid ceil(ell k / 256) blocks, each entry's scale recomputed by
// the same operations as block 0's).
__global__ void __launch_bounds__(256) k_finish(const double *__restrict__ vals, int is_lam, int ell, int k,
                                                const double *__restrict__ sign, int divide, double *__restrict__ S,
                                                double *__restrict__ colscale, double *__restrict__ info,
                                                const double *__restrict__ UB, float *__restrict__ Mv) {
  const int t = threadIdx.x;
  if (Mv) {
    const int e = blockIdx.x * 256 + t;
    if (e < ell * k) {
      const int i = e / k, c = e - (e / k) * k;
      Mv[e] = (float)(UB[i * ell + c] * finish_scale(vals, is_lam, sign, divide, c));
    }
  }
  if (blockIdx.x != 0) return;
  __shared__ double sq_sh[128];
  double sg = 0.0;
  if (t < ell) {
    sg = finish_sigma(vals, is_lam, t);
    sq_sh[t] = sg * sg;
  }
  if (t < k) {
    S[t] = sg;
    colscale[t] = finish_scale(vals, is_lam, sign, divide, t);
  }
  __syncthreads();
  if (t == 0) {
    double tot = 0.0;   // fixed order
    for (int j = 0; j < ell; ++j) tot += sq_sh[j];
    info[0] = tot;
    info[1] = (ell > k) ? finish_sigma(vals, is_lam, k) : 0.0;
  }
}

void launch_scale(hipStream_t st, void *x, int f64, int64_t count, double a) {
  const unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 2048);
  hipLaunchKernelGGL(k_scale, dim3(blocks), dim3(256), 0, st, x, f64, count, a);
}

int valid_dtype(int dt) { return dt >= DSK_F64 && dt <= DSK_F16; }

// coarse size of a restriction, or a negative value when invalid
int64_t coarse_size(const dsk_restriction *R, int64_t n) {
  if (!R) return -1;
  switch (R->kind) {
    case DSK_R_INDEX:
      if (R->s < 1 || R->s > n || !R->index) return -1;
      return R->s;
    case DSK_R_NN:
    case DSK_R_GLOBAL:
      if (R->ny < 1 || R->nx < 1 || (int64_t)R->ny * R->nx != n || R->sy < 1 || R->sx < 1) return -1;
      return (int64_t)((R->ny + R->sy - 1) / R->sy) * ((R->nx + R->sx - 1) / R->sx);
    case DSK_R_LEARNED:
      if (!conv_shape_ok(n, R->ny, R->nx, R->channels) || !R->w1 || !R->w2) return -1;
      return (int64_t)(R->ny / 4) * (R->nx / 4);
    default:
      return -1;
  }
}

struct Finish {
  dsk_handle *h;
  int flags_on_host;
};

int read_info(dsk_handle *h, const double *dinfo, dsk_info *info, int ell) {
  if (!info) return 0;
  int words[FLAGW_COUNT] = {0, 0, 0, 0};
  double vals[3] = {0, 0, 0};
  DSK_TRY(hipMemcpyAsync(words, h->dflags, sizeof(words), hipMemcpyDeviceToHost, h->stream));
  if (dinfo) DSK_TRY(hipMemcpyAsync(vals, dinfo, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  DSK_TRY(hipStreamSynchronize(h->stream));
  info->ell = ell;
  info->flags = words[FLAGW_BITS];
  info->core_sweeps = words[FLAGW_SWEEPS];
  info->reserved = 0;
  info->normA_fro2 = vals[2];
  info->normB_fro2 = vals[0];
  info->sigma_tail = vals[1];
  return 0;
}

// Orthonormalise a rows x ell block in place-ish: Q = orth(Y).  f64 uses
// Householder (tmp: rows*ell f64 scratch, R: ell^2), f32 uses CholeskyQR2, or
// a single CholeskyQR pass when span_only (a basis of span(Y) whose
// orthogonality only needs to keep the next product well conditioned).
int orth(dsk_handle *h, const void *Y, int f64, int64_t rows, int ell, void *Q, void *tmp, void *cws, double *R,
         bool span_only = false) {
  if (f64) {
    DSK_RET(launch_convert(h->stream, Y, 1, tmp, 1, rows * ell));
    return launch_hhqr(h->stream, (double *)tmp, rows, ell, (double *)Q, R, h->dflags);
  }
  return launch_cholqr2(h->stream, Y, 0, rows, ell, Q, cws, h->dflags, R, span_only ? 1 : 2);
}

}  // namespace

void allow_lds_raw(const void *kernel, size_t bytes) {
  static std::mutex mu;
  static std::unordered_map<const void *, size_t> granted;
  std::lock_guard<std::mutex> lock(mu);
  size_t &g = granted[kernel];
  if (bytes <= g) return;
  if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess) g = bytes;
}

int read_info_words(dsk_handle *h, dsk_info *info, int ell) { return read_info(h, nullptr, info, ell); }

int arena_reserve(dsk_handle *h, size_t bytes) {
  if (bytes <= h->arena_bytes) return 0;
  if (h->arena) {
    DSK_TRY(hipStreamSynchronize(h->stream));
    DSK_TRY(hipFree(h->arena));
    h->arena = nullptr;
    h->arena_bytes = 0;
  }
  const size_t want = (bytes + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
  DSK_TRY(hipMalloc(&h->arena, want));
  h->arena_bytes = want;
  return 0;
}

int project_args(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, const void *Q,
                 int32_t ell, void *Bt, int32_t mode) {
  if (!h) return -1;
  if (!A) return -2;
  if (!valid_dtype(dtype)) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < n) return -6;
  if (!Q) return -7;
  if (ell < 1 || ell > ELL_CAP) return -8;
  if (!Bt) return -9;
  if (mode < 0 || mode > DSK_MODE_SPLIT6) return -10;
  return 0;
}

extern "C" {

void dsk_opts_default(dsk_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->p = 10;
  o->tau = 0.0;
  o->mode = DSK_MODE_DEFAULT;
}

int dsk_create(dsk_handle **h, int device, void *stream) {
  if (!h) return -1;
  *h = nullptr;
  DSK_TRY(hipSetDevice(device));
  DSK_RET(noalloc_setup(device));   // the fixed scratch of dsk_project_noalloc on this device
  dsk_handle *x = new dsk_handle();
  x->device = device;
  x->stream = reinterpret_cast<hipStream_t>(stream);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 256;
  x->cu_count = cus;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 65536;
  x->max_lds = (size_t)lds;
  if (hipMalloc(&x->dflags, HANDLE_DEV_BYTES) != hipSuccess) {
    delete x;
    return DSK_ERR_BASE + (int)hipErrorOutOfMemory;
  }
  hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, x->stream, x->dflags);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(x->stream) != hipSuccess) {
    hipFree(x->dflags);
    delete x;
    return DSK_ERR_BASE + (int)hipErrorLaunchFailure;
  }
  *h = x;
  return 0;
}

int dsk_destroy(dsk_handle *h) {
  if (!h) return -1;
  hipSetDevice(h->device);
  hipStreamSynchronize(h->stream);
  destroy_workers(h);
  if (h->arena) (void)hipFree(h->arena);
  if (h->dflags) (void)hipFree(h->dflags);
  if (h->tev) {
    for (int i = 0; i < 2 * TIMING_CAP; ++i) (void)hipEventDestroy(h->tev[i]);
    delete[] h->tev;
  }
  delete h;
  return 0;
}

int dsk_set_stream(dsk_handle *h, void *stream) {
  if (!h) return -1;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  return 0;
}

const char *dsk_status_string(int status) {
  if (status == 0) return "success";
  if (status < 0) {
    static const char *names[] = {"", "argument 1 invalid", "argument 2 invalid", "argument 3 invalid",
                                  "argument 4 invalid", "argument 5 invalid", "argument 6 invalid",
                                  "argument 7 invalid", "argument 8 invalid", "argument 9 invalid",
                                  "argument 10 invalid", "argument 11 invalid", "argument 12 invalid",
                                  "argument 13 invalid", "argument 14 invalid"};
    const int i = -status;
    return i < 15 ? names[i] : "invalid argument";
  }
  if (status == DSK_ERR_SCRATCH) return "size exceeds the fixed scratch of the allocation-free entry point";
  if (status >= DSK_ERR_BASE) return hipGetErrorString((hipError_t)(status - DSK_ERR_BASE));
  return "unknown status";
}

int dsk_restrict(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                 const dsk_restriction *R, void *Ac) {
  if (!h) return -1;
  if (!A) return -2;
  if (!valid_dtype(dtype)) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < n) return -6;
  const int64_t s = coarse_size(R, n);
  if (s < 1) return -7;
  if (!Ac) return -8;
  DSK_TRY(hipSetDevice(h->device));
  hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, h->stream, h->dflags);
  return launch_restrict(h->stream, A, dtype, m, n, lda, R, s, dtype == DSK_F64, Ac, nullptr, h->dflags);
}

int dsk_project(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, const void *Q,
                int32_t ell, void *Bt, int32_t mode) {
  if (const int bad = project_args(h, A, dtype, m, n, lda, Q, ell, Bt, mode)) return bad;
  DSK_TRY(hipSetDevice(h->device));
  DSK_RET(arena_reserve(h, stream_ws_bytes(dtype, m, n, ell, mode)));
  hipEvent_t e0, e1;
  timing_slot(h, &e0, &e1);
  return launch_stream(h->stream, A, dtype, m, n, lda, Q, dtype == DSK_F64, ell, Bt, ell, mode, h->arena,
                       h->cu_count, e0, e1);
}

int dsk_timing_enable(dsk_handle *h, int enable) {
  if (!h) return -1;
  DSK_TRY(hipSetDevice(h->device));
  if (enable && !h->tev) {
    h->tev = new hipEvent_t[2 * TIMING_CAP];
    for (int i = 0; i < 2 * TIMING_CAP; ++i) DSK_TRY(hipEventCreate(&h->tev[i]));
  }
  h->timing = enable ? 1 : 0;
  h->tcount = 0;
  return 0;
}

int dsk_timing_read(dsk_handle *h, int *count, double *total_ms) {
  if (!h) return -1;
  if (!count) return -2;
  if (!total_ms) return -3;
  *count = 0;
  *total_ms = 0.0;
  if (!h->tev || h->tcount == 0) return 0;
  DSK_TRY(hipStreamSynchronize(h->stream));
  double tot = 0.0;
  for (int i = 0; i < h->tcount; ++i) {
    float ms = 0.f;
    DSK_TRY(hipEventElapsedTime(&ms, h->tev[2 * i], h->tev[2 * i + 1]));
    tot += ms;
  }
  *count = h->tcount;
  *total_ms = tot;
  h->tcount = 0;
  return 0;
}

}  // extern "C"

// Argument checks of dsk_sketch_svd (codes are its argument numbers); fills the
// effective options, the coarse size s and the range-finder width L.
int svd_check(const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k, const dsk_restriction *R,
              int32_t q, const dsk_opts *o, void *U, double *S, void *V, dsk_opts *odp, int64_t *s_out, int *L_out) {
  if (!A) return -2;
  if (!valid_dtype(dtype)) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < n) return -6;
  const int64_t s = coarse_size(R, n);
  dsk_opts od;
  dsk_opts_default(&od);
  if (o) od = *o;
  if (od.p < 0) return -10;
  int64_t ell = od.S ? od.ell : std::min<int64_t>(std::min<int64_t>((int64_t)k + od.p, s), m);
  if (s < 1) return -8;
  // the FP64 core SVD (one-sided Jacobi on R of B^T) holds two ell x ell blocks in LDS
  const int cap = dtype == DSK_F64 ? ELL_CAP_F64 : ELL_CAP;
  if (od.S && (od.ell < 1 || od.ell > std::min<int64_t>(s, m) || od.ell > cap)) return -10;
  ell = std::min<int64_t>(ell, cap);
  if (k < 1 || k > ell) return -7;
  if (q < 0 || q > 64) return -9;
  if (od.mode < 0 || od.mode > DSK_MODE_SPLIT6) return -10;
  if (od.refine && dtype != DSK_F64 && k > 100) return -10;
  if (!U) return -11;
  if (!S) return -12;
  if (!V) return -13;
  *odp = od;
  *s_out = s;
  *L_out = (int)ell;
  return 0;
}

// The sketch-SVD launch sequence on h's stream and arena.  With need != NULL
// only the arena size is computed (nothing is allocated or enqueued).
int svd_run(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k,
            const dsk_restriction *R, int32_t q, const dsk_opts &od, int64_t s, int L, void *U, double *S, void *V,
            dsk_info *info, size_t *need, const std::function<int()> *after_projection, bool single_pass,
            bool orth_z) {
  hipStream_t st = h->stream;
  const int f64 = dtype == DSK_F64;
  const size_t we = f64 ? 8 : 4;
  const int64_t rmax = std::max<int64_t>(std::max<int64_t>(m, s), n);
  // ---- workspace
  Carve c{nullptr, 0, 0, true};
  for (int pass = 0; pass < 2; ++pass) {
    c.off = 0;
    char *Ac = c.take<char>((size_t)m * s * we);
    char *Y = c.take<char>((size_t)m * L * we);
    char *Q = c.take<char>((size_t)m * L * we);
    char *Z = c.take<char>((size_t)s * L * we);
    char *Bt = c.take<char>((size_t)n * L * we);
    double *tmp = f64 ? c.take<double>((size_t)rmax * L) : nullptr;
    double *QB = f64 ? c.take<double>((size_t)n * L) : nullptr;
    char *cws = c.take<char>(cholqr2_ws_bytes(std::max(m, s), L));
    size_t sws_b = std::max(stream_ws_bytes(dtype, m, n, L, od.mode), stream_ws_bytes(f64 ? DSK_F64 : DSK_F32, m, s, L, od.mode));
    sws_b = std::max(sws_b, stream_ws_bytes(f64 ? DSK_F64 : DSK_F32, s, m, L, od.mode));
    sws_b = std::max(sws_b, stream_ws_bytes(f64 ? DSK_F64 : DSK_F32, L, n, k, od.mode));
    char *sws = c.take<char>(sws_b);
    float *Mv = c.take<float>((size_t)L * k);
    const int nparts = gram_mfma_blocks(n);
    double *part = c.take<double>((size_t)nparts * L * L);
    double *GB = c.take<double>((size_t)L * L);
    double *lam = c.take<double>(L);
    double *UB = c.take<double>((size_t)L * L);
    double *Ur = c.take<double>((size_t)L * L);
    double *RB = c.take<double>((size_t)L * L);
    double *Rsm = c.take<double>((size_t)L * L);
    double *sign = c.take<double>(L);
    double *colscale = c.take<double>(L);
    double *dinfo = c.take<double>(4);
    double *fpart = c.take<double>(1024);
    // single pass: H = A^T Y, M = R^{-1} (FP64 input)
    char *Hb = single_pass ? c.take<char>((size_t)n * L * we) : nullptr;
    double *Mr = single_pass ? c.take<double>((size_t)L * L) : nullptr;
    // C-PWR's Gram sub-sample A(:, I) (Alg. 7) when the restriction is not an index set
    const bool own_gram = q > 0 && R->kind != DSK_R_INDEX;
    char *Ag = own_gram ? c.take<char>((size_t)m * s * we) : nullptr;
    // refinement sweep (FP32 / 16-bit input): unrefined factors, then FP64 re-orthonormalisation
    const bool refine = od.refine && !f64;
    float *U0 = refine ? c.take<float>((size_t)m * k) : nullptr;
    float *V0 = refine ? c.take<float>((size_t)n * k) : nullptr;
    double *rws = refine ? c.take<double>(refine_ws_bytes(k) / sizeof(double)) : nullptr;
    double *ews = f64 ? nullptr : c.take<double>(core_eig_tri_ws_bytes(L) / sizeof(double));
    if (pass == 0) {
      if (need) {
        *need = c.off;
        return 0;
      }
      DSK_RET(arena_reserve(h, c.off));
      c.base = h->arena;
      c.cap = h->arena_bytes;
      c.dry = false;
      continue;
    }
    // ---- launch sequence
    hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, st, h->dflags);
    const int wdt = f64 ? DSK_F64 : DSK_F32;
    DSK_RET(launch_restrict(st, A, dtype, m, n, lda, R, s, f64, Ac, nullptr, h->dflags));
    if (od.S) DSK_RET(launch_stream_nn(st, Ac, wdt, m, s, s, od.S, L, Y, L, od.mode, sws, h->cu_count));
    else DSK_RET(launch_select_cols(st, Ac, f64, m, s, s, L, Y));
    if (single_pass) {
      // SPC-SVD (Alg. 3): the pass over A needs Y only, so it starts at once; a
      // worker stream meanwhile orthonormalises Y (Q for U = Q U_B) and forms
      // M = R^{-1}; then B^T = A^T Q = H M.
      dsk_handle *wk = h->workers[0];
      hipStream_t wst = wk->stream;
      DSK_TRY(hipEventRecord(h->wev[0], st));
      DSK_TRY(hipStreamWaitEvent(wst, h->wev[0], 0));
      // FP32 / 16-bit: one CholeskyQR pass, Y^T Y = L L^T (FP64), Q = Y L^{-T};
      // then B^T = H L^{-T} by the same blocked substitution (the 64- or the
      // 128-wide factorization's tiles)
      const bool chol_tiles = !f64;
      if (f64) {
        DSK_RET(launch_convert(wst, Y, 1, tmp, 1, m * L));
        DSK_RET(launch_hhqr(wst, tmp, m, L, (double *)Q, Rsm, h->dflags));
        DSK_RET(launch_spc_rinv(wst, Rsm, L, 0x1p-53, Mr, h->dflags));
      } else if (L <= 64) {
        DSK_RET(launch_cholqr64(wst, Y, 0, m, L, Q, cws, h->dflags, 1));
      } else {
        DSK_RET(launch_cholqr128(wst, Y, 0, m, L, Q, cws, h->dflags, 1));
      }
      DSK_TRY(hipEventRecord(h->wev[1], wst));
      hipEvent_t e0, e1;
      timing_slot(h, &e0, &e1);
      DSK_RET(launch_stream(st, A, dtype, m, n, lda, Y, f64, L, Hb, L, od.mode, sws, h->cu_count, e0, e1));
      DSK_TRY(hipStreamWaitEvent(st, h->wev[1], 0));
      if (chol_tiles && L <= 64) DSK_RET(launch_cholqr64_apply(st, Hb, 0, n, L, cws, Bt, h->dflags));
      else if (chol_tiles) DSK_RET(launch_cholqr128_apply(st, Hb, 0, n, L, cws, Bt, h->dflags));
      else DSK_RET(launch_tsmm(st, Hb, f64, n, L, L, Mr, L, L, nullptr, Bt, L));
    } else {
    // intermediate bases of the power iteration only carry a span (one
    // CholeskyQR pass); the block that B is projected on is orthonormalised fully
    DSK_RET(orth(h, Y, f64, m, L, Q, tmp, cws, Rsm, q > 0));
    const char *Gs = Ac;
    if (own_gram) {
      DSK_RET(launch_gram_sample(st, A, dtype, m, n, lda, R, s, f64, Ag, h->dflags));
      Gs = Ag;
    }
    for (int it = 0; it < q; ++it) {
      // Z = A_g^T Q (s x ell), orthonormalised; Q = orth(A_g Z), A_g = A(:, I) the Gram
      // sub-sample of Alg. 7.  tau cancels under re-orthonormalisation.
      DSK_RET(launch_stream(st, Gs, wdt, m, s, s, Q, f64, L, Z, L, od.mode, sws, h->cu_count));
      if (orth_z) DSK_RET(orth(h, Z, f64, s, L, Z, tmp, cws, Rsm, true));
      DSK_RET(launch_stream_nn(st, Gs, wdt, m, s, s, Z, L, Y, L, od.mode, sws, h->cu_count));
      DSK_RET(orth(h, Y, f64, m, L, Q, tmp, cws, Rsm, it + 1 < q));
    }
    // B^T = A^T Q: the single full pass over A
    hipEvent_t e0, e1;
    timing_slot(h, &e0, &e1);
    DSK_RET(launch_stream(st, A, dtype, m, n, lda, Q, f64, L, Bt, L, od.mode, sws, h->cu_count, e0, e1));
    if (after_projection) DSK_RET((*after_projection)());
    }
    if (!f64) {
      void *Ua = refine ? (void *)U0 : U;
      void *Va = refine ? (void *)V0 : V;
      DSK_RET(launch_gram(st, Bt, 0, n, L, GB, part, nparts));
      DSK_RET(launch_core_eig_tri(st, GB, L, lam, UB, ews, h->dflags));
      DSK_RET(launch_tsmm(st, Q, 0, m, L, L, UB, L, k, nullptr, Ua, k));
      DSK_RET(launch_sign_fix(st, Ua, 0, m, k, sign));
      hipLaunchKernelGGL(k_finish, dim3((unsigned)((L * k + 255) / 256)), dim3(256), 0, st, lam, 1, L, k, sign, 1, S,
                         colscale, dinfo, (const double *)UB, Mv);
      // V = B^T U_B(:, :k) diag(sign / sigma) on the MFMA stream kernel (n rows, K = ell)
      DSK_RET(launch_stream_nn(st, Bt, DSK_F32, n, L, L, Mv, k, Va, k, od.mode, sws, h->cu_count));
      if (refine)
        DSK_RET(launch_refine(st, U0, m, V0, n, k, S, (float *)U, (float *)V, part, nparts, rws, h->dflags,
                              od.mode, sws, h->cu_count));
    } else {
      DSK_RET(launch_convert(st, Bt, 1, tmp, 1, n * L));
      DSK_RET(launch_hhqr(st, tmp, n, L, QB, RB, h->dflags));
      DSK_RET(launch_jacobi_svd(st, RB, L, lam, UB, Ur, h->dflags));
      DSK_RET(launch_tsmm(st, Q, 1, m, L, L, UB, L, k, nullptr, U, k));
      DSK_RET(launch_sign_fix(st, U, 1, m, k, sign));
      hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, st, lam, 0, L, k, sign, 0, S, colscale, dinfo,
                         (const double *)nullptr, (float *)nullptr);
      DSK_RET(launch_tsmm(st, QB, 1, n, L, L, Ur, L, k, colscale, V, k));
    }
    DSK_TRY(hipGetLastError());
    if (info) {
      DSK_RET(launch_fro2(st, A, dtype, m, n, lda, fpart, 1024, dinfo + 2));
    }
    return read_info(h, dinfo, info, L);
  }
  return 0;
}

extern "C" {

int dsk_sketch_svd(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k,
                   const dsk_restriction *R, int32_t q, const dsk_opts *o, void *U, double *S, void *V,
                   dsk_info *info) {
  if (!h) return -1;
  dsk_opts od;
  int64_t s = 0;
  int L = 0;
  DSK_RET(svd_check(A, dtype, m, n, lda, k, R, q, o, U, S, V, &od, &s, &L));
  DSK_TRY(hipSetDevice(h->device));
  return svd_run(h, A, dtype, m, n, lda, k, R, q, od, s, L, U, S, V, info, nullptr);
}

int dsk_spc_id_err(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                   const dsk_restriction *R, int32_t mc, const double *taus, int32_t ntau, double *eps,
                   double *rho) {
  if (!h) return -1;
  if (!A) return -2;
  if (!valid_dtype(dtype)) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < n) return -6;
  const int64_t s = coarse_size(R, n);
  if (s < 1) return -7;
  if (mc < 1 || mc > m) return -8;
  const int64_t c = m / mc;         // keep rows i with (i + 1) mod c == 0
  const int64_t r = m / c;
  if (r > 112) return -8;
  if (!taus) return -9;
  if (ntau < 1 || ntau > 1024) return -10;
  if (!eps) return -11;
  DSK_TRY(hipSetDevice(h->device));
  hipStream_t st = h->stream;
  const size_t esz = dtype == DSK_F64 ? 8 : (dtype == DSK_F32 ? 4 : 2);
  const int nparts = std::max(spc_err_parts(n), spc_err_parts(s));
  Carve cv{nullptr, 0, 0, true};
  for (int pass = 0; pass < 2; ++pass) {
    cv.off = 0;
    double *Bc = cv.take<double>((size_t)r * s);
    double *part = cv.take<double>((size_t)nparts * r * r);
    double *Gf = cv.take<double>((size_t)r * r);
    double *Gc = cv.take<double>((size_t)r * r);
    double *Mb = cv.take<double>((size_t)ntau * r * r);
    double *sig = cv.take<double>(ntau);
    double *lam = cv.take<double>((size_t)ntau * r);
    double *Ub = cv.take<double>((size_t)ntau * r * r);
    if (pass == 0) {
      DSK_RET(arena_reserve(h, cv.off));
      cv.base = h->arena;
      cv.cap = h->arena_bytes;
      cv.dry = false;
      continue;
    }
    hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, st, h->dflags);
    // the kept rows: a strided view of A (first row c - 1, row stride c lda)
    const void *Ak = reinterpret_cast<const char *>(A) + (size_t)(c - 1) * lda * esz;
    const int64_t ldk = c * lda;
    DSK_RET(launch_restrict(st, Ak, dtype, r, n, ldk, R, s, 1, Bc, nullptr, h->dflags));
    DSK_RET(launch_row_gram(st, Ak, dtype, (int)r, n, ldk, part, Gf));
    DSK_RET(launch_row_gram(st, Bc, DSK_F64, (int)r, s, s, part, Gc));
    DSK_RET(launch_eps_curve(st, Gf, Gc, (int)r, taus, ntau, (double)c, Mb, sig, lam, Ub, eps, rho, h->dflags));
  }
  return 0;
}

int dsk_sketch_svd_sp(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k,
                      const dsk_restriction *R, const dsk_opts *o, void *U, double *S, void *V, dsk_info *info) {
  if (!h) return -1;
  dsk_opts od;
  int64_t s = 0;
  int L = 0;
  const int r = svd_check(A, dtype, m, n, lda, k, R, 0, o, U, S, V, &od, &s, &L);
  if (r) return r <= -10 ? r + 1 : r;   // dsk_sketch_svd numbering -> this one (no q argument)
  if (od.refine) return -9;
  DSK_TRY(hipSetDevice(h->device));
  DSK_RET(ensure_workers(h, 1));
  return svd_run(h, A, dtype, m, n, lda, k, R, 0, od, s, L, U, S, V, info, nullptr, nullptr, true);
}

}  // extern "C"

// Argument checks of dsk_sketch_id (codes are its argument numbers).
int id_check(const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k, const dsk_restriction *R,
             int32_t q, const dsk_opts *o, int64_t *skel, double *P, dsk_opts *odp, int64_t *s_out, int64_t *cols_out,
             int64_t *ell_out) {
  if (!A) return -2;
  if (!valid_dtype(dtype)) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < n) return -6;
  const int64_t s = coarse_size(R, n);
  if (s < 1) return -8;
  dsk_opts od;
  dsk_opts_default(&od);
  if (o) od = *o;
  if (od.p < 0) return -10;
  int64_t cols = s;
  int64_t ell = 0;
  if (od.id_projected) {
    ell = od.S ? od.ell : std::min<int64_t>(std::min<int64_t>((int64_t)k + od.p, s), m);
    if (od.S && (od.ell < 1 || od.ell > s || od.ell > ELL_CAP)) return -10;
    ell = std::min<int64_t>(ell, ELL_CAP);
    cols = ell;
  }
  if (k < 1 || k > std::min<int64_t>(m, cols) || k > 112) return -7;
  if (q < 0 || q > 64) return -9;
  if (!skel) return -11;
  if (!P) return -12;
  *odp = od;
  *s_out = s;
  *cols_out = cols;
  *ell_out = ell;
  return 0;
}

// The row-ID launch sequence on h's stream and arena (need != NULL: size only).
int id_run(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k,
           const dsk_restriction *R, int32_t q, const dsk_opts &od, int64_t s, int64_t cols, int64_t ell,
           int64_t *skel, double *P, void *skel_rows, dsk_info *info, size_t *need, int phase) {
  hipStream_t st = h->stream;
  const double tau = od.tau > 0.0 ? od.tau : (double)n / (double)s;
  Carve c{nullptr, 0, 0, true};
  for (int pass = 0; pass < 2; ++pass) {
    c.off = 0;
    double *Ac = c.take<double>((size_t)m * s);
    // C-PWR's Gram sub-sample A(:, I) (Alg. 7) when the restriction is not an index set
    double *Ag = (q > 0 && R->kind != DSK_R_INDEX) ? c.take<double>((size_t)m * s) : nullptr;
    double *W = c.take<double>((size_t)m * cols);
    double *W2 = c.take<double>((size_t)m * cols);
    double *M = (q > 0 && !od.id_projected) ? c.take<double>((size_t)m * m) : nullptr;
    double *Zs = od.id_projected ? c.take<double>((size_t)s * cols) : nullptr;
    char *sws = c.take<char>(std::max(stream_ws_bytes(DSK_F64, m, s, (int)std::max<int64_t>(ell, 1), 0),
                                      stream_ws_bytes(DSK_F64, s, m, (int)std::max<int64_t>(ell, 1), 0)));
    double *nu0 = c.take<double>(m);
    double *nu1 = c.take<double>(m);
    double *Rk = c.take<double>((size_t)k * m);
    // one launch for all pivot steps when the rows fit the registers of one
    // workgroup per compute unit; W = A_c held in the storage dtype where it is
    // a plain gather of stored values (an index restriction of FP32 / 16-bit
    // data, no power step): FP32, or the 16-bit values themselves
    const bool wstore = dtype != DSK_F64 && q == 0 && !od.id_projected && R->kind == DSK_R_INDEX;
    const int wdt = wstore ? dtype : DSK_F64;
    const size_t rwsb = od.id_per_step ? 0 : rowid_reg_ws_bytes(m, cols, k, wdt, h->cu_count);
    char *rws = rwsb ? c.take<char>(rwsb) : nullptr;
    // (carved in the dry pass too)
    char *Acs = (rwsb && wstore) ? c.take<char>((size_t)m * s * (dtype == DSK_F32 ? 4 : 2)) : nullptr;
    // a given S arrives in the work dtype; the ID works in FP64
    const bool s_conv = od.id_projected && od.S && dtype != DSK_F64;
    double *S64 = s_conv ? c.take<double>((size_t)s * ell) : nullptr;
    if (pass == 0) {
      if (need) {
        *need = c.off;
        return 0;
      }
      DSK_RET(arena_reserve(h, c.off));
      c.base = h->arena;
      c.cap = h->arena_bytes;
      c.dry = false;
      continue;
    }
    const bool split = rwsb && wstore;   // the phases of the one-launch path (see dsk_internal.h)
    if (phase == 1 && !split) return 0;
    if (phase != 2 || !split) hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, st, h->dflags);
    if (split) {
      if (phase != 2) {
        if (dtype == DSK_F32) DSK_RET(launch_restrict(st, A, dtype, m, n, lda, R, s, 0, Acs, nullptr, h->dflags));
        else DSK_RET(launch_gather_cols16(st, A, m, n, lda, R, s, Acs));
        if (phase == 1) {
          DSK_TRY(hipGetLastError());
          return 0;
        }
      }
      DSK_RET(launch_rowid_reg(st, Acs, wdt, m, s, k, nu0, Rk, skel, rws, h->cu_count, h->dflags));
      DSK_RET(launch_id_solve(st, Rk, skel, nu0, m, k, P, h->dflags));
      if (skel_rows) DSK_RET(launch_gather_rows(st, A, dtype, m, n, lda, skel, k, skel_rows));
      DSK_TRY(hipGetLastError());
      return read_info(h, nullptr, info, 0);
    }
    // A_c in FP64 (exact for every storage dtype)
    DSK_RET(launch_restrict(st, A, dtype, m, n, lda, R, s, 1, Ac, nullptr, h->dflags));
    const double *Gs = Ac;
    if (Ag) {
      DSK_RET(launch_gram_sample(st, A, dtype, m, n, lda, R, s, 1, Ag, h->dflags));
      Gs = Ag;
    }
    double *Wcur = nullptr;
    if (od.id_projected) {
      if (od.S) {
        const void *S = od.S;
        if (s_conv) {
          DSK_RET(launch_convert(st, od.S, 0, S64, 1, s * ell));
          S = S64;
        }
        DSK_RET(launch_stream_nn(st, Ac, DSK_F64, m, s, s, S, (int)ell, W, ell, 0, sws, h->cu_count));
      } else {
        DSK_RET(launch_select_cols(st, Ac, 1, m, s, s, (int)ell, W));
      }
      for (int it = 0; it < q; ++it) {
        DSK_RET(launch_stream(st, Gs, DSK_F64, m, s, s, W, 1, (int)ell, Zs, ell, 0, sws, h->cu_count));
        launch_scale(st, Zs, 1, s * ell, tau);
        DSK_RET(launch_stream_nn(st, Gs, DSK_F64, m, s, s, Zs, (int)ell, W, ell, 0, sws, h->cu_count));
      }
      Wcur = W;
    } else if (q > 0) {
      // (tau A_g A_g^T)^q A_c evaluated as M = tau A_g A_g^T, W <- M W (same product, reassociated)
      DSK_RET(launch_gemm64(st, 0, 1, m, m, s, tau, Gs, s, Gs, s, M, m));
      const double *src = Ac;
      double *bufs[2] = {W, W2};
      for (int it = 0; it < q; ++it) {
        DSK_RET(launch_gemm64(st, 0, 0, m, s, m, 1.0, M, m, src, s, bufs[it & 1], s));
        src = bufs[it & 1];
      }
      Wcur = const_cast<double *>(src);
    } else {
      Wcur = Ac;
    }
    const double *nu_final;
    if (rwsb) {
      DSK_RET(launch_rowid_reg(st, Wcur, DSK_F64, m, cols, k, nu0, Rk, skel, rws, h->cu_count, h->dflags));
      nu_final = nu0;
    } else {
      DSK_RET(launch_cpqr(st, Wcur, m, cols, k, nu0, nu1, Rk, skel, h->dflags));
      nu_final = ((k - 1) & 1) ? nu0 : nu1;
    }
    DSK_RET(launch_id_solve(st, Rk, skel, nu_final, m, k, P, h->dflags));
    if (skel_rows) DSK_RET(launch_gather_rows(st, A, dtype, m, n, lda, skel, k, skel_rows));
    DSK_TRY(hipGetLastError());
    return read_info(h, nullptr, info, (int)(od.id_projected ? ell : 0));
  }
  return 0;
}

extern "C" {

int dsk_sketch_id(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k,
                  const dsk_restriction *R, int32_t q, const dsk_opts *o, int64_t *skel, double *P, void *skel_rows,
                  dsk_info *info) {
  if (!h) return -1;
  dsk_opts od;
  int64_t s = 0, cols = 0, ell = 0;
  DSK_RET(id_check(A, dtype, m, n, lda, k, R, q, o, skel, P, &od, &s, &cols, &ell));
  DSK_TRY(hipSetDevice(h->device));
  return id_run(h, A, dtype, m, n, lda, k, R, q, od, s, cols, ell, skel, P, skel_rows, info, nullptr);
}

int dsk_power_iter(dsk_handle *h, const void *Ac, int32_t dtype, int64_t m, int64_t s, int64_t ldc, const void *Q0,
                   int32_t ell, int32_t q, double tau, int32_t reorth, void *Qout) {
  if (!h) return -1;
  if (!Ac) return -2;
  if (dtype != DSK_F64 && dtype != DSK_F32) return -3;
  if (m < 1) return -4;
  if (s < 1) return -5;
  if (ldc < s) return -6;
  if (!Q0) return -7;
  if (ell < 1 || ell > std::min<int64_t>(std::min<int64_t>(m, s), ELL_CAP)) return -8;
  if (q < 0 || q > 64) return -9;
  if (!(tau > 0.0)) return -10;
  if (!Qout) return -12;
  DSK_TRY(hipSetDevice(h->device));
  hipStream_t st = h->stream;
  const int f64 = dtype == DSK_F64;
  const size_t we = f64 ? 8 : 4;
  Carve c{nullptr, 0, 0, true};
  for (int pass = 0; pass < 2; ++pass) {
    c.off = 0;
    char *Z = c.take<char>((size_t)s * ell * we);
    char *G = c.take<char>((size_t)m * ell * we);
    double *tmp = c.take<double>((size_t)std::max(m, s) * ell);
    char *cws = c.take<char>(cholqr2_ws_bytes(std::max(m, s), ell));
    char *sws = c.take<char>(std::max(stream_ws_bytes(dtype, m, s, ell, 0), stream_ws_bytes(dtype, s, m, ell, 0)));
    double *Rsm = c.take<double>((size_t)ell * ell);
    if (pass == 0) {
      DSK_RET(arena_reserve(h, c.off));
      c.base = h->arena;
      c.cap = h->arena_bytes;
      c.dry = false;
      continue;
    }
    hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, st, h->dflags);
    DSK_RET(launch_convert(st, Q0, f64, Qout, f64, m * ell));
    for (int it = 0; it < q; ++it) {
      DSK_RET(launch_stream(st, Ac, dtype, m, s, ldc, Qout, f64, ell, Z, ell, 0, sws, h->cu_count));
      if (reorth) DSK_RET(orth(h, Z, f64, s, ell, Z, tmp, cws, Rsm));
      else launch_scale(st, Z, f64, s * ell, tau);
      DSK_RET(launch_stream_nn(st, Ac, dtype, m, s, ldc, Z, ell, G, ell, 0, sws, h->cu_count));
      if (reorth) DSK_RET(orth(h, G, f64, m, ell, Qout, tmp, cws, Rsm));
      else DSK_RET(launch_convert(st, G, f64, Qout, f64, m * ell));
    }
    DSK_TRY(hipGetLastError());
    return 0;
  }
  return 0;
}

}  // extern "C"

// Single-pass coarse-grid row ID, SPC-ID (Alg. 5, Sec. 4): A ~ P_c A_c(I_c, :) T_r
// with the lifting operator T_r = V_c S_c^+ U_c^T U_r U_r^T U_c S_c^+ V_c^T H^T.
//
// U_c^T U_r U_r^T U_c is the identity on the first r singular directions and
// zero elsewhere, so T_r = V_r S_r^{-2} V_r^T H^T (s x n), kept factored:
// T_r = V_r W_r with W_r = S_r^{-2} V_r^T H^T (r x n), and the lifted skeleton
// rows X = A_c(I_c, :) T_r = (A_c(I_c, :) V_r) W_r (k x n) are formed without
// the s x n operator.  Launch sequence, on three streams of the handle:
//
//   main      A_c = A D; H = A^T A_c (n x s), the pass over A, as blocks of up
//             to 112 columns of A_c on the projection kernel (each block a
//             strided column slice of H)
//   worker 0  top r singular triplets of A_c: the sketch SVD of A_c itself with
//             every coarse column kept (start block of ell = min(m, s, 112)
//             nested columns, 100 for FP64 input, qc subspace-iteration steps
//             Q <- orth(A_c A_c^T Q), core eigensolver);
//             exact as qc grows, the error of the r-th direction falling like
//             (sigma_{ell+1} / sigma_r)^(2 qc + 1)
//   worker 1  the row ID of A_c (TPC-ID at q = 0: the same skeleton and P)
//   main      W_r^T = H (V_r S_r^{-2}) (n x r, one read of H); M^T = V_r^T
//             A_c(I_c, :)^T (r x k); X^T = W_r^T M^T; X = (X^T)^T
//
// Singular values at or below max(m, s) eps sigma_1 (eps the machine epsilon of
// the work precision) are treated as zero in S_r^{-2} (the pseudo-inverse
// S_c^+) and raise DSK_FLAG_RANK_DEFICIENT.
#include <algorithm>
#include <cstdlib>
#include <thread>

#include "dsk_internal.h"

namespace {

constexpr int NT = 256;
constexpr int HBLK = 112;   // columns of A_c per projection launch (the kernel's widest tile set)

__global__ void k_zero_flags_spc(int *f) {
  if (threadIdx.x < FLAGW_COUNT) f[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(NT) k_iota(int64_t *__restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) x[i] = i;
}

// dst (rows x b, contiguous) = src(:, c0 : c0 + b), src row-major with leading dimension ld
template <typename T>
__global__ void __launch_bounds__(NT) k_col_block(const T *__restrict__ src, int64_t ld, int64_t rows, int64_t c0,
                                                  int b, T *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= rows * b) return;
  const int64_t i = e / b;
  const int j = (int)(e - i * b);
  dst[e] = src[i * ld + c0 + j];
}

// Z(:, j) = V(:, j) / sigma_j^2 for sigma_j above the pseudo-inverse threshold
// u_thr max(rows, cols) sigma_1, else 0 (and the rank-deficient flag).
template <typename T>
__global__ void __launch_bounds__(NT) k_scale_inv2(const T *__restrict__ V, int64_t s, int r,
                                                   const double *__restrict__ S, double thr_rel,
                                                   T *__restrict__ Z, int *__restrict__ dflags) {
  const double thr = thr_rel * S[0];
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x < r) {
    const double sg = S[threadIdx.x];
    if (!(sg > thr)) atomicOr(&dflags[FLAGW_BITS], DSK_FLAG_RANK_DEFICIENT);
  }
  if (e >= s * r) return;
  const int j = (int)(e % r);
  const double sg = S[j];
  const double f = sg > thr ? 1.0 / (sg * sg) : 0.0;
  Z[e] = (T)((double)V[e] * f);
}

// DSK_SERIAL_ENQUEUE=1: enqueue everything from the calling thread (for
// runtimes that are not thread-safe, such as a host emulation of the kernels)
bool serial_enqueue() {
  static const bool serial = [] {
    const char *e = std::getenv("DSK_SERIAL_ENQUEUE");
    return e && e[0] == '1';
  }();
  return serial;
}

template <typename T>
int col_block(hipStream_t st, const void *src, int64_t ld, int64_t rows, int64_t c0, int b, void *dst) {
  const int64_t cnt = rows * b;
  hipLaunchKernelGGL(k_col_block<T>, dim3((unsigned)((cnt + NT - 1) / NT)), dim3(NT), 0, st, (const T *)src, ld,
                     rows, c0, b, (T *)dst);
  DSK_TRY(hipGetLastError());
  return 0;
}

}  // namespace

extern "C" {

int dsk_spc_id(dsk_handle *h, const void *A, int32_t dtype, int64_t m, int64_t n, int64_t lda, int32_t k, int32_t r,
               const dsk_restriction *R, int32_t qc, const dsk_opts *o, int64_t *skel, double *P, void *X, void *Vr,
               void *Wr, dsk_info *info) {
  if (!h) return -1;
  dsk_opts oid;
  int64_t s = 0, cols = 0, ell_id = 0;
  {
    // dsk_sketch_id's checks at q = 0, renumbered to this entry point
    const int rc = id_check(A, dtype, m, n, lda, k, R, 0, o, skel, P, &oid, &s, &cols, &ell_id);
    if (rc) {
      static const int map[13] = {0, -1, -2, -3, -4, -5, -6, -7, -9, -10, -11, -12, -13};
      return (rc <= -1 && rc >= -12) ? map[-rc] : rc;
    }
  }
  const int cap = dtype == DSK_F64 ? ELL_CAP_F64 : ELL_CAP;
  if (r < k || (int64_t)r > std::min<int64_t>(std::min<int64_t>(m, s), cap)) return -8;
  if (qc < 0 || qc > 64) return -10;
  if (oid.S || oid.id_projected) return -11;   // no second-level sketch here
  if (!X) return -14;
  DSK_TRY(hipSetDevice(h->device));
  DSK_RET(ensure_workers(h, 2));
  dsk_handle *wsv = h->workers[0];
  dsk_handle *wid = h->workers[1];
  hipStream_t st = h->stream;
  const int f64 = dtype == DSK_F64;
  const int wdt = f64 ? DSK_F64 : DSK_F32;
  const size_t we = f64 ? 8 : 4;
  // the sketch SVD of A_c (m x s) with every column kept
  dsk_opts osv;
  dsk_opts_default(&osv);
  osv.mode = oid.mode;
  // the widest range finder: the r-th direction converges like (sigma_{Lc+1} / sigma_r)^(2 qc + 1)
  const int Lc = (int)std::min<int64_t>(std::min<int64_t>(s, m), cap);
  dsk_restriction Rall{};
  Rall.kind = DSK_R_INDEX;
  Rall.s = s;
  Rall.index = nullptr;   // set once the arena is carved
  // ---- workspace (main arena); the workers size their own
  size_t need_sv = 0, need_id = 0;
  {
    int64_t dummy = 0;
    Rall.index = &dummy;   // only the sizing pass reads it (never dereferenced there)
    DSK_RET(svd_run(wsv, nullptr, wdt, m, s, s, r, &Rall, qc, osv, s, Lc, nullptr, nullptr, nullptr, nullptr, &need_sv,
                    nullptr, false, false));
    Rall.index = nullptr;
  }
  DSK_RET(id_run(wid, A, dtype, m, n, lda, k, R, 0, oid, s, cols, ell_id, skel, P, nullptr, nullptr, &need_id));
  DSK_RET(arena_reserve(wsv, need_sv));
  DSK_RET(arena_reserve(wid, need_id));
  Carve c{nullptr, 0, 0, true};
  for (int pass = 0; pass < 2; ++pass) {
    c.off = 0;
    char *Ac = c.take<char>((size_t)m * s * we);
    int64_t *iota = c.take<int64_t>((size_t)s);
    char *Qb = c.take<char>((size_t)m * HBLK * we);
    char *H = c.take<char>((size_t)n * s * we);
    char *Ur = c.take<char>((size_t)m * r * we);
    double *Sr = c.take<double>((size_t)r);
    char *Vv = Vr ? (char *)Vr : c.take<char>((size_t)s * r * we);
    char *Zs = c.take<char>((size_t)s * r * we);
    char *WT = c.take<char>((size_t)n * r * we);
    char *AcI = c.take<char>((size_t)k * s * we);
    char *AcIT = c.take<char>((size_t)s * k * we);
    char *Mt = c.take<char>((size_t)r * k * we);
    double *Mt64 = f64 ? (double *)Mt : c.take<double>((size_t)r * k);
    char *XT = c.take<char>((size_t)n * k * we);
    size_t sws_b = stream_ws_bytes(dtype, m, n, HBLK, oid.mode);
    sws_b = std::max(sws_b, stream_ws_bytes(wdt, s, n, r, oid.mode));
    sws_b = std::max(sws_b, stream_ws_bytes(wdt, s, r, k, oid.mode));
    char *sws = c.take<char>(sws_b);
    if (pass == 0) {
      DSK_RET(arena_reserve(h, c.off));
      c.base = h->arena;
      c.cap = h->arena_bytes;
      c.dry = false;
      continue;
    }
    hipLaunchKernelGGL(k_zero_flags_spc, dim3(1), dim3(64), 0, st, h->dflags);
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((s + NT - 1) / NT)), dim3(NT), 0, st, iota, s);
    DSK_TRY(hipGetLastError());
    Rall.index = iota;
    // A_c, then fork: the SVD of A_c and the row ID run beside the pass over A
    DSK_RET(launch_restrict(st, A, dtype, m, n, lda, R, s, f64, Ac, nullptr, h->dflags));
    DSK_TRY(hipEventRecord(h->wev[0], st));
    DSK_TRY(hipStreamWaitEvent(wsv->stream, h->wev[0], 0));
    DSK_TRY(hipStreamWaitEvent(wid->stream, h->wev[0], 0));
    DSK_RET(id_run(wid, A, dtype, m, n, lda, k, R, 0, oid, s, cols, ell_id, skel, P, nullptr, nullptr, nullptr));
    DSK_TRY(hipEventRecord(h->wev[2], wid->stream));
    // The SVD of A_c is several hundred small launches and the pass over A a
    // hundred; the runtime holds the enqueuing thread back while a stream has
    // many launches pending, so one host thread would feed the two streams one
    // after the other.  The SVD sequence is enqueued from a second thread while
    // this one enqueues the pass.
    auto enqueue_svd = [&]() -> int {
      DSK_TRY(hipSetDevice(h->device));
      DSK_RET(svd_run(wsv, Ac, wdt, m, s, s, r, &Rall, qc, osv, s, Lc, Ur, Sr, Vv, nullptr, nullptr, nullptr, false,
                      false));
      DSK_TRY(hipEventRecord(h->wev[1], wsv->stream));
      return 0;
    };
    // H = A^T A_c (n x s), block by block: H(:, c0 : c0 + b) = A^T A_c(:, c0 : c0 + b)
    auto enqueue_pass = [&]() -> int {
      for (int64_t c0 = 0; c0 < s; c0 += HBLK) {
        const int b = (int)std::min<int64_t>(HBLK, s - c0);
        DSK_RET(f64 ? col_block<double>(st, Ac, s, m, c0, b, Qb) : col_block<float>(st, Ac, s, m, c0, b, Qb));
        hipEvent_t e0, e1;
        timing_slot(h, &e0, &e1);
        DSK_RET(launch_stream(st, A, dtype, m, n, lda, Qb, f64, b, H + c0 * we, s, oid.mode, sws, h->cu_count, e0,
                              e1));
      }
      return 0;
    };
    if (serial_enqueue()) {
      DSK_RET(enqueue_pass());
      DSK_RET(enqueue_svd());
    } else {
      int svd_rc = 0;
      std::thread worker([&] { svd_rc = enqueue_svd(); });
      const int pass_rc = enqueue_pass();
      worker.join();
      DSK_RET(pass_rc);
      DSK_RET(svd_rc);
    }
    // lifting: W_r^T = H V_r S_r^{-2}
    DSK_TRY(hipStreamWaitEvent(st, h->wev[1], 0));
    {
      const double u = f64 ? 0x1p-52 : 0x1p-23;   // machine epsilon of the work precision
      const double thr_rel = (double)std::max<int64_t>(m, s) * u;
      const int64_t cnt = s * r;
      const unsigned blocks = (unsigned)((cnt + NT - 1) / NT);
      if (f64)
        hipLaunchKernelGGL(k_scale_inv2<double>, dim3(blocks), dim3(NT), 0, st, (const double *)Vv, s, r, Sr, thr_rel,
                           (double *)Zs, h->dflags);
      else
        hipLaunchKernelGGL(k_scale_inv2<float>, dim3(blocks), dim3(NT), 0, st, (const float *)Vv, s, r, Sr, thr_rel,
                           (float *)Zs, h->dflags);
      DSK_TRY(hipGetLastError());
    }
    DSK_RET(launch_stream_nn(st, H, wdt, n, s, s, Zs, r, WT, r, oid.mode, sws, h->cu_count));
    if (Wr) DSK_RET(launch_transpose(st, WT, f64, n, r, Wr));
    // X = (A_c(I, :) V_r) W_r, once the skeleton is known
    DSK_TRY(hipStreamWaitEvent(st, h->wev[2], 0));
    DSK_RET(launch_gather_rows(st, Ac, wdt, m, s, s, skel, k, AcI));
    DSK_RET(launch_transpose(st, AcI, f64, k, s, AcIT));
    DSK_RET(launch_stream(st, Vv, wdt, s, r, r, AcIT, f64, k, Mt, k, oid.mode, sws, h->cu_count));
    if (!f64) DSK_RET(launch_convert(st, Mt, 0, Mt64, 1, (int64_t)r * k));
    DSK_RET(launch_tsmm(st, WT, f64, n, r, r, Mt64, k, k, nullptr, XT, k));
    DSK_RET(launch_transpose(st, XT, f64, n, k, X));
    DSK_TRY(hipGetLastError());
    if (info) {
      dsk_info a{}, b{}, d{};
      DSK_RET(read_info_words(h, &d, 0));
      DSK_RET(read_info_words(wsv, &a, Lc));
      DSK_RET(read_info_words(wid, &b, 0));
      *info = a;
      info->flags = a.flags | b.flags | d.flags;
      info->normA_fro2 = info->normB_fro2 = info->sigma_tail = 0.0;
    }
    return 0;
  }
  return 0;
}

}  // extern "C"

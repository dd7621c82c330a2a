// Calls the C ABI of the host-emulated library on host buffers.  Built with
// AddressSanitizer, any out-of-bounds access of a kernel (device buffers and
// LDS) aborts the run with a report; a missing barrier shows up as a deadlock.
// Modes: "quick" (one configuration per path), "svd", "batch", "more", "persist"
// ("persist-quick": its two smaller cases), "files <dir>" (inputs from and outputs
// to raw files, for comparison with the oracle), "streams" ("streams-quick": one small
// case each, nine small batch problems), "all".  SIMT_STREAMS=defer:<order> runs
// the streams' work in another interleaving (see simt_rt.cpp).  "persist" runs the one-launch pivoted QR (its workgroups waiting on
// each other's published words) with all blocks of the launch resident together,
// and compares it bitwise with the per-step factorization.
#include <cmath>
#include <initializer_list>
#include <utility>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>
#include "dsketch.h"
#include <cstdint>

namespace simt {
extern long long g_resident_launches;
void sync_all();   // run every queued stream item (deferred streams)
}

// FNV-1a over a set of output buffers
static unsigned long long fnv(std::initializer_list<std::pair<const void *, size_t>> bufs) {
  unsigned long long hsh = 1469598103934665603ull;
  for (const auto &b : bufs) {
    const unsigned char *p = (const unsigned char *)b.first;
    for (size_t i = 0; i < b.second; ++i) hsh = (hsh ^ p[i]) * 1099511628211ull;
  }
  return hsh;
}

static std::vector<double> make_A(int64_t m, int N, int r, unsigned seed, double noise) {
  // sum of r smooth separable modes with decaying weights plus noise
  std::mt19937_64 g(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  const int64_t n = (int64_t)N * N;
  std::vector<double> A(m * n, 0.0);
  for (int q = 0; q < r; ++q) {
    const double w = 1.0 / std::sqrt(1.0 + q);
    const int kx = 1 + q % 7, ky = 1 + q / 7;
    const double ph = nd(g);
    std::vector<double> tt(m);
    for (int64_t i = 0; i < m; ++i) tt[i] = nd(g);
    for (int64_t i = 0; i < m; ++i)
      for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x)
          A[i * n + y * N + x] += w * tt[i] * std::cos(6.283185307 * (kx * x + ky * y) / N + ph);
  }
  for (auto &v : A) v += noise * nd(g);
  return A;
}

static std::vector<int64_t> di_index(int N, int f) {
  std::vector<int64_t> idx;
  for (int y = 0; y < N; y += f)
    for (int x = 0; x < N; x += f) idx.push_back((int64_t)y * N + x);
  return idx;
}


// raw little-endian arrays for the file mode
template <class T>
static bool read_bin(const std::string &path, std::vector<T> &v) {
  FILE *f = fopen(path.c_str(), "rb");
  if (!f) return false;
  const size_t got = fread(v.data(), sizeof(T), v.size(), f);
  fclose(f);
  return got == v.size();
}
static void write_bin(const std::string &path, const void *p, size_t bytes) {
  FILE *f = fopen(path.c_str(), "wb");
  if (!f) return;
  fwrite(p, 1, bytes, f);
  fclose(f);
}

static int check(const char *what, int rc) {
  simt::sync_all();
  printf("%-44s rc=%d\n", what, rc);
  fflush(stdout);
  return rc;
}

int main(int argc, char **argv) {
  const std::string which = argc > 1 ? argv[1] : "quick";
  const bool quick = which == "quick";
  // enough emulated compute units for the one-launch factorization (m <= 4 x units)
  const bool persist = which == "persist" || which == "persist-quick";
  if (persist) setenv("SIMT_CU", "48", 1);
  setenv("DSK_SERIAL_ENQUEUE", "1", 1);   // the emulated runtime is single-threaded
  dsk_handle *h = nullptr;
  if (dsk_create(&h, 0, nullptr)) return 1;
  dsk_opts o;
  dsk_opts_default(&o);
  auto want = [&](const char *w) { return which == "all" || quick || which == w; };

  // ---- sketch SVD, FP32 and FP64, q = 0..2, ell = 30 and 60
  for (int f64 = 0; f64 < 2; ++f64)
    for (int cfg = 0; cfg < (quick ? 1 : 2) && want("svd"); ++cfg) {
      const int64_t m = cfg ? 300 : 200;
      const int N = 32, fct = cfg ? 2 : 4, k = cfg ? 50 : 20;
      const int64_t n = (int64_t)N * N;
      auto A64 = make_A(m, N, 40, 7 + cfg, 1e-3);
      std::vector<float> A32(A64.begin(), A64.end());
      auto idx = di_index(N, fct);
      int64_t *didx = nullptr;
      double *dA = nullptr;
      void *dAv = nullptr;
      dsk_restriction R{};
      R.kind = DSK_R_INDEX;
      R.s = (int64_t)idx.size();
      R.index = idx.data();
      R.ny = R.nx = N;
      R.sy = R.sx = fct;
      (void)didx;
      (void)dA;
      dAv = f64 ? (void *)A64.data() : (void *)A32.data();
      const size_t we = f64 ? 8 : 4;
      std::vector<char> U(m * k * we), V(n * k * we);
      std::vector<double> S(k);
      for (int q = 0; q < (quick ? (f64 ? 1 : 2) : 3); ++q) {
        dsk_info info{};
        char nm[128];
        snprintf(nm, sizeof nm, "svd f64=%d cfg=%d q=%d", f64, cfg, q);
        check(nm, dsk_sketch_svd(h, dAv, f64 ? DSK_F64 : DSK_F32, m, n, n, k, &R, q, &o, U.data(), S.data(),
                                 V.data(), &info));
        printf("   S0 %.10g S%d %.10g flags %d sweeps %d\n", S[0], k - 1, S[k - 1], info.flags, info.core_sweeps);
      }
      // row ID and the combined call
      if (want("svd") && !(quick && f64)) {
        std::vector<int64_t> I(k);
        std::vector<double> P(m * k);
        std::vector<char> rows(k * n * we);
        dsk_info ii{};
        check("id q=0", dsk_sketch_id(h, dAv, f64 ? DSK_F64 : DSK_F32, m, n, n, k, &R, 0, &o, I.data(), P.data(),
                                      rows.data(), &ii));
        printf("   I0 %lld I1 %lld flags %d\n", (long long)I[0], (long long)I[1], ii.flags);
        dsk_info a{}, b{};
        check("svd_id q=1", dsk_sketch_svd_id(h, dAv, f64 ? DSK_F64 : DSK_F32, m, n, n, k, &R, 1, 0, &o, U.data(),
                                               S.data(), V.data(), I.data(), P.data(), rows.data(), &a, &b));
        check("svd single pass", dsk_sketch_svd_sp(h, dAv, f64 ? DSK_F64 : DSK_F32, m, n, n, k, &R, &o, U.data(),
                                                   S.data(), V.data(), &a));
        printf("   S0 %.10g flags %d\n", S[0], a.flags);
        std::vector<double> taus = {0.0, 1.0, 4.0, 16.0}, eps(4);
        check("spc_id_err", dsk_spc_id_err(h, dAv, f64 ? DSK_F64 : DSK_F32, m, n, n, &R, (int)(m / 10), taus.data(), 4,
                                           eps.data(), nullptr));
        printf("   eps %.6g %.6g %.6g %.6g\n", eps[0], eps[1], eps[2], eps[3]);
      }
    }

  // ---- batched ragged instances (eager), shapes of the batched tests
  if (want("batch")) {
    struct Inst { int64_t m; int N, k, f, f64, q; };
    std::vector<Inst> ins = {{331, 32, 18, 2, 1, 2}, {199, 64, 22, 4, 0, 1}, {238, 32, 11, 4, 0, 2},
                             {386, 32, 12, 4, 0, 1}, {198, 64, 19, 4, 0, 0}, {273, 32, 37, 4, 1, 0},
                             {144, 32, 16, 2, 0, 2}, {388, 32, 14, 4, 0, 0}, {338, 64, 11, 4, 0, 1}};
    std::vector<std::vector<double>> A64s;
    std::vector<std::vector<float>> A32s;
    std::vector<std::vector<int64_t>> idxs;
    std::vector<std::vector<char>> Us, Vs;
    std::vector<std::vector<double>> Ss;
    std::vector<dsk_problem> pr;
    if (quick) ins.resize(3);
    for (size_t i = 0; i < ins.size(); ++i) {
      const Inst &t = ins[i];
      A64s.push_back(make_A(t.m, t.N, 30, 100 + (unsigned)i, 1e-3));
      A32s.emplace_back(A64s.back().begin(), A64s.back().end());
      idxs.push_back(di_index(t.N, t.f));
    }
    for (size_t i = 0; i < ins.size(); ++i) {
      const Inst &t = ins[i];
      const int64_t n = (int64_t)t.N * t.N;
      const size_t we = t.f64 ? 8 : 4;
      Us.emplace_back(t.m * t.k * we);
      Vs.emplace_back(n * t.k * we);
      Ss.emplace_back(t.k);
      dsk_problem p{};
      p.A = t.f64 ? (const void *)A64s[i].data() : (const void *)A32s[i].data();
      p.dtype = t.f64 ? DSK_F64 : DSK_F32;
      p.m = t.m;
      p.n = n;
      p.lda = n;
      p.k = t.k;
      p.q = t.q;
      p.R.kind = DSK_R_INDEX;
      p.R.s = (int64_t)idxs[i].size();
      p.R.index = idxs[i].data();
      p.U = Us.back().data();
      p.S = Ss.back().data();
      p.V = Vs.back().data();
      pr.push_back(p);
    }
    int nw = 0;
    check("batched eager", dsk_sketch_svd_batched(h, (int)pr.size(), pr.data(), &o, 0, &nw));
    printf("   workers %d S0 %.8g\n", nw, Ss[0][0]);
    // graph path: fresh outputs, first call = eager run + capture, then replays after clearing the outputs
    std::vector<std::vector<char>> U2, V2;
    std::vector<std::vector<double>> S2;
    std::vector<dsk_problem> pr2 = pr;
    for (size_t i = 0; i < pr.size(); ++i) {
      U2.emplace_back(Us[i].size());
      V2.emplace_back(Vs[i].size());
      S2.emplace_back(Ss[i].size());
      pr2[i].U = U2.back().data();
      pr2[i].S = S2.back().data();
      pr2[i].V = V2.back().data();
    }
    const int rg = check("batched graph (first call; -5 while graph replay is disabled)", dsk_sketch_svd_batched(h, (int)pr2.size(), pr2.data(), &o,
                                                                             DSK_BATCH_GRAPH, &nw));
    if (rg == 0) {
      for (int rep = 0; rep < 3; ++rep) {
        for (size_t i = 0; i < pr.size(); ++i) {
          memset(U2[i].data(), 0, U2[i].size());
          memset(V2[i].data(), 0, V2[i].size());
          memset(S2[i].data(), 0, S2[i].size() * 8);
        }
        check("batched graph replay", dsk_sketch_svd_batched(h, (int)pr2.size(), pr2.data(), &o, DSK_BATCH_GRAPH, &nw));
        int bad = 0;
        for (size_t i = 0; i < pr.size(); ++i)
          bad += memcmp(U2[i].data(), Us[i].data(), Us[i].size()) != 0 || memcmp(V2[i].data(), Vs[i].data(), Vs[i].size()) != 0 ||
                 memcmp(S2[i].data(), Ss[i].data(), Ss[i].size() * 8) != 0;
        printf("   replay %d: %d instances differ from the eager results\n", rep, bad);
      }
    }
  }
  // ---- wide range finder (ell = 110), 16-bit storage with refinement, stencil restrictions, projected ID
  if (which == "all" || which == "more") {
    const int64_t m = 300;
    const int N = 32;
    const int64_t n = (int64_t)N * N;
    auto A64 = make_A(m, N, 60, 21, 1e-3);
    std::vector<float> A32(A64.begin(), A64.end());
    std::vector<uint16_t> Abf(m * n), Ah(m * n);
    for (int64_t i = 0; i < m * n; ++i) {
      const __bf16 b = (__bf16)A32[i];
      const _Float16 hv = (_Float16)A32[i];
      memcpy(&Abf[i], &b, 2);
      memcpy(&Ah[i], &hv, 2);
    }
    auto idx2 = di_index(N, 2);
    dsk_restriction R{};
    R.kind = DSK_R_INDEX;
    R.s = (int64_t)idx2.size();
    R.index = idx2.data();
    const int k = 100;
    std::vector<float> U(m * k), V(n * k);
    std::vector<double> S(k);
    dsk_info info{};
    check("svd wide ell=110 q=1", dsk_sketch_svd(h, A32.data(), DSK_F32, m, n, n, k, &R, 1, &o, U.data(), S.data(),
                                                 V.data(), &info));
    printf("   ell %d S0 %.10g S99 %.6g flags %d\n", info.ell, S[0], S[99], info.flags);
    const int k2 = 20;
    dsk_opts orf = o;
    orf.refine = 1;
    check("svd bf16 q=1 refine", dsk_sketch_svd(h, Abf.data(), DSK_BF16, m, n, n, k2, &R, 1, &orf, U.data(),
                                                S.data(), V.data(), &info));
    printf("   S0 %.10g flags %d\n", S[0], info.flags);
    check("svd f16 q=0", dsk_sketch_svd(h, Ah.data(), DSK_F16, m, n, n, k2, &R, 0, &o, U.data(), S.data(), V.data(),
                                        &info));
    printf("   S0 %.10g flags %d\n", S[0], info.flags);
    for (int kind : {DSK_R_NN, DSK_R_GLOBAL}) {
      dsk_restriction Rs{};
      Rs.kind = kind;
      Rs.ny = Rs.nx = N;
      Rs.sy = Rs.sx = 4;
      check(kind == DSK_R_NN ? "svd nn q=1" : "svd global q=1",
            dsk_sketch_svd(h, A64.data(), DSK_F64, m, n, n, k2, &Rs, 1, &o, U.data(), S.data(), V.data(), &info));
      std::vector<int64_t> I(k2);
      std::vector<double> P(m * k2);
      check(kind == DSK_R_NN ? "id nn q=1" : "id global q=1",
            dsk_sketch_id(h, A64.data(), DSK_F64, m, n, n, k2, &Rs, 1, &o, I.data(), P.data(), nullptr, &info));
    }
    // projected ID with a given FP32 second level (widened to FP64 inside)
    std::vector<float> Om(idx2.size() * 30);
    std::mt19937_64 g(5);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (auto &v : Om) v = (float)nd(g);
    dsk_opts op = o;
    op.S = Om.data();
    op.ell = 30;
    op.id_projected = 1;
    std::vector<int64_t> I(k2);
    std::vector<double> P(m * k2);
    check("id projected given S q=1", dsk_sketch_id(h, A32.data(), DSK_F32, m, n, n, k2, &R, 1, &op, I.data(), P.data(),
                                                    nullptr, &info));
    check("svd given S q=1", dsk_sketch_svd(h, A32.data(), DSK_F32, m, n, n, k2, &R, 1, &op, U.data(), S.data(),
                                            V.data(), &info));
    // restriction, projection and power iteration alone
    std::vector<float> Ac(m * idx2.size()), Q(m * 30), Bt(n * 30), Qo(m * 30);
    for (auto &v : Q) v = (float)nd(g);
    check("restrict", dsk_restrict(h, A32.data(), DSK_F32, m, n, n, &R, Ac.data()));
    check("project", dsk_project(h, A32.data(), DSK_F32, m, n, n, Q.data(), 30, Bt.data(), DSK_MODE_DEFAULT));
    check("power_iter q=2", dsk_power_iter(h, Ac.data(), DSK_F32, m, (int64_t)idx2.size(), (int64_t)idx2.size(),
                                           Q.data(), 30, 2, 1.0, 1, Qo.data()));
    // learned restriction: forward, backward, loss gradient, Adam
    const int C = 4;
    std::vector<float> w1(C * 25), w2(C * 25), gw1(C * 25), gw2(C * 25), m1(C * 25, 0.f), m2(C * 25, 0.f);
    for (auto &v : w1) v = (float)(0.2 * nd(g));
    for (auto &v : w2) v = (float)(0.2 * nd(g));
    dsk_restriction Rl{};
    Rl.kind = DSK_R_LEARNED;
    Rl.ny = Rl.nx = N;
    Rl.channels = C;
    Rl.w1 = w1.data();
    Rl.w2 = w2.data();
    const int64_t sl = (N / 4) * (N / 4);
    std::vector<float> Acl(m * sl), gAc(m * sl);
    for (auto &v : gAc) v = (float)nd(g);
    check("learned restrict", dsk_restrict(h, A32.data(), DSK_F32, m, n, n, &Rl, Acl.data()));
    check("learned conv bwd", dsk_conv_restrict_bwd(h, A32.data(), DSK_F32, m, n, n, &Rl, gAc.data(), gw1.data(),
                                                    gw2.data()));
    double loss = 0.0;
    check("learned loss grad ell=20 q=1", dsk_learned_loss_grad(h, A32.data(), DSK_F32, m, n, n, &Rl, 20, 1, &loss,
                                                                 gw1.data(), gw2.data()));
    printf("   loss %.8g\n", loss);
    check("adam step", dsk_adam_step(h, w1.data(), gw1.data(), m1.data(), m2.data(), C * 25, 1e-3f, 0.9f, 0.999f,
                                     1e-8f, 1));
    check("learned svd q=1", dsk_sketch_svd(h, A32.data(), DSK_F32, m, n, n, k2, &Rl, 1, &o, U.data(), S.data(),
                                            V.data(), &info));
    // documented argument errors (checked on the host before anything is enqueued)
    const int e1 = dsk_sketch_svd(h, nullptr, DSK_F32, m, n, n, k2, &R, 1, &o, U.data(), S.data(), V.data(), nullptr);
    const int e2 = dsk_sketch_svd(h, A32.data(), 9, m, n, n, k2, &R, 1, &o, U.data(), S.data(), V.data(), nullptr);
    const int e3 = dsk_sketch_svd(h, A32.data(), DSK_F32, m, n, n - 1, k2, &R, 1, &o, U.data(), S.data(), V.data(),
                                  nullptr);
    const int e4 = dsk_sketch_svd(h, A32.data(), DSK_F32, m, n, n, 0, &R, 1, &o, U.data(), S.data(), V.data(), nullptr);
    const int e5 = dsk_sketch_id(h, A32.data(), DSK_F32, m, n, n, k2, &R, 0, &o, nullptr, P.data(), nullptr, nullptr);
    const int e6 = dsk_sketch_svd_sp(h, A32.data(), DSK_F32, m, n, n, k2, &R, &orf, U.data(), S.data(), V.data(),
                                     nullptr);
    const int ok = e1 == -2 && e2 == -3 && e3 == -6 && e4 == -7 && e5 == -11 && e6 == -9;
    printf("%-44s rc=%d\n", "argument errors as documented", ok ? 0 : 1);
    if (!ok) printf("   codes %d %d %d %d %d %d\n", e1, e2, e3, e4, e5, e6);
  }
  // ---- file mode: inputs written by a test (A, the index set, tau values), outputs
  // of the main entry points written back for comparison with the FP64 oracle
  if (which == "files" && argc > 2) {
    const std::string dir = argv[2];
    long long m = 0, N = 0, f = 0, k = 0, mc = 0, ntau = 0;
    FILE *pf = fopen((dir + "/dims.txt").c_str(), "r");
    if (!pf || fscanf(pf, "%lld %lld %lld %lld %lld %lld", &m, &N, &f, &k, &mc, &ntau) != 6) {
      printf("files: bad dims\n");
      return 1;
    }
    fclose(pf);
    const int64_t n = N * N;
    std::vector<double> A64(m * n), taus(ntau);
    auto idx = di_index((int)N, (int)f);
    if (!read_bin(dir + "/A.bin", A64) || !read_bin(dir + "/taus.bin", taus)) {
      printf("files: missing inputs\n");
      return 1;
    }
    std::vector<float> A32(A64.begin(), A64.end());
    dsk_restriction R{};
    R.kind = DSK_R_INDEX;
    R.s = (int64_t)idx.size();
    R.index = idx.data();
    R.ny = R.nx = (int)N;
    R.sy = R.sx = (int)f;
    std::vector<char> U(m * k * 8), V(n * k * 8);
    std::vector<double> S(k);
    auto out = [&](const std::string &tag, size_t we) {
      write_bin(dir + "/" + tag + "_U.bin", U.data(), m * k * we);
      write_bin(dir + "/" + tag + "_S.bin", S.data(), k * 8);
      write_bin(dir + "/" + tag + "_V.bin", V.data(), n * k * we);
    };
    for (int q = 0; q < 2; ++q) {
      char nm[64];
      snprintf(nm, sizeof nm, "files svd f64 q=%d", q);
      check(nm, dsk_sketch_svd(h, A64.data(), DSK_F64, m, n, n, (int)k, &R, q, &o, U.data(), S.data(), V.data(),
                               nullptr));
      out(q ? "svd64q1" : "svd64q0", 8);
    }
    check("files svd f32 q=1", dsk_sketch_svd(h, A32.data(), DSK_F32, m, n, n, (int)k, &R, 1, &o, U.data(), S.data(),
                                              V.data(), nullptr));
    out("svd32q1", 4);
    check("files svd single pass f64", dsk_sketch_svd_sp(h, A64.data(), DSK_F64, m, n, n, (int)k, &R, &o, U.data(),
                                                         S.data(), V.data(), nullptr));
    out("sp64", 8);
    std::vector<int64_t> I(k);
    std::vector<double> P(m * k);
    check("files id f64 q=0", dsk_sketch_id(h, A64.data(), DSK_F64, m, n, n, (int)k, &R, 0, &o, I.data(), P.data(),
                                            nullptr, nullptr));
    write_bin(dir + "/id64_I.bin", I.data(), k * 8);
    write_bin(dir + "/id64_P.bin", P.data(), m * k * 8);
    std::vector<double> eps(ntau), rho(ntau);
    check("files spc_id_err f64", dsk_spc_id_err(h, A64.data(), DSK_F64, m, n, n, &R, (int)mc, taus.data(), (int)ntau,
                                                 eps.data(), rho.data()));
    write_bin(dir + "/eps64.bin", eps.data(), ntau * 8);
    write_bin(dir + "/rho64.bin", rho.data(), ntau * 8);
    // the same matrix stored BF16 (bits from the test), q = 1
    std::vector<uint16_t> Abf(m * n);
    if (read_bin(dir + "/Abf.bin", Abf)) {
      check("files svd bf16 q=1", dsk_sketch_svd(h, Abf.data(), DSK_BF16, m, n, n, (int)k, &R, 1, &o, U.data(),
                                                 S.data(), V.data(), nullptr));
      out("svdbfq1", 4);
    }
    // hybrid sketch: a given s x (k + 6) second level (Gaussian, from the test), FP64,
    // the SVD at q = 1 and the ID of the projected block at q = 1
    const int ellg = (int)k + 6;
    std::vector<double> Om((size_t)R.s * ellg);
    if (read_bin(dir + "/Om.bin", Om)) {
      dsk_opts oh = o;
      oh.S = Om.data();
      oh.ell = ellg;
      check("files svd hybrid f64 q=1", dsk_sketch_svd(h, A64.data(), DSK_F64, m, n, n, (int)k, &R, 1, &oh, U.data(),
                                                       S.data(), V.data(), nullptr));
      out("hyb64q1", 8);
      oh.id_projected = 1;
      check("files id hybrid projected f64 q=1", dsk_sketch_id(h, A64.data(), DSK_F64, m, n, n, (int)k, &R, 1, &oh,
                                                               I.data(), P.data(), nullptr, nullptr));
      write_bin(dir + "/hybid_I.bin", I.data(), k * 8);
      write_bin(dir + "/hybid_P.bin", P.data(), m * k * 8);
    }
    // learned conv restriction (4 channels, FP32 A): forward, weight gradients of
    // <gAc, A_c(w)>, and the training loss with its gradients (ell = 8, q = 1)
    const int C = 4;
    const int64_t sl = (N / 4) * (N / 4);
    std::vector<float> w1(C * 25), w2(C * 25), gAc(m * sl);
    if (read_bin(dir + "/w1.bin", w1) && read_bin(dir + "/w2.bin", w2) && read_bin(dir + "/gAc.bin", gAc)) {
      dsk_restriction Rl{};
      Rl.kind = DSK_R_LEARNED;
      Rl.ny = Rl.nx = (int)N;
      Rl.channels = C;
      Rl.w1 = w1.data();
      Rl.w2 = w2.data();
      std::vector<float> Acl(m * sl), g1(C * 25), g2(C * 25);
      check("files learned restrict", dsk_restrict(h, A32.data(), DSK_F32, m, n, n, &Rl, Acl.data()));
      write_bin(dir + "/learned_Ac.bin", Acl.data(), Acl.size() * 4);
      check("files learned conv bwd", dsk_conv_restrict_bwd(h, A32.data(), DSK_F32, m, n, n, &Rl, gAc.data(),
                                                            g1.data(), g2.data()));
      write_bin(dir + "/learned_g1.bin", g1.data(), g1.size() * 4);
      write_bin(dir + "/learned_g2.bin", g2.data(), g2.size() * 4);
      double loss = 0.0;
      check("files learned loss grad", dsk_learned_loss_grad(h, A64.data(), DSK_F64, m, n, n, &Rl, 8, 1, &loss,
                                                              g1.data(), g2.data()));
      write_bin(dir + "/learned_loss.bin", &loss, 8);
      write_bin(dir + "/learned_l1.bin", g1.data(), g1.size() * 4);
      write_bin(dir + "/learned_l2.bin", g2.data(), g2.size() * 4);
    }
    // restriction entry point (index and global kinds, FP64) and the C-PWR loop on
    // the restricted block from a given start (q = 2; raw and re-orthonormalised)
    {
      const int64_t s = R.s;
      std::vector<double> Ac(m * s);
      check("files restrict index f64", dsk_restrict(h, A64.data(), DSK_F64, m, n, n, &R, Ac.data()));
      write_bin(dir + "/rest_idx.bin", Ac.data(), Ac.size() * 8);
      dsk_restriction Rg{};
      Rg.kind = DSK_R_GLOBAL;
      Rg.ny = Rg.nx = (int)N;
      Rg.sy = Rg.sx = (int)f;
      std::vector<double> Ag(m * s);
      check("files restrict global f64", dsk_restrict(h, A64.data(), DSK_F64, m, n, n, &Rg, Ag.data()));
      write_bin(dir + "/rest_glob.bin", Ag.data(), Ag.size() * 8);
      const int ell0 = 6;
      std::vector<double> Q0(m * ell0), Qo(m * ell0);
      if (read_bin(dir + "/Q0.bin", Q0)) {
        const double tau = (double)n / (double)s;
        check("files power iter raw q=2", dsk_power_iter(h, Ac.data(), DSK_F64, m, s, s, Q0.data(), ell0, 2, tau, 0,
                                                          Qo.data()));
        write_bin(dir + "/pw_raw.bin", Qo.data(), Qo.size() * 8);
        check("files power iter orth q=2", dsk_power_iter(h, Ac.data(), DSK_F64, m, s, s, Q0.data(), ell0, 2, tau, 1,
                                                           Qo.data()));
        write_bin(dir + "/pw_orth.bin", Qo.data(), Qo.size() * 8);
      }
    }
    // single-pass ID with the lifting operator (Alg. 5) on a matrix with a clear
    // singular-value drop at r = 12 (from the test): FP64 with the factors of T_r, FP32
    std::vector<double> As(m * n);
    if (read_bin(dir + "/Aspc.bin", As)) {
      const int ks = 6, rs = 12, qc = 8;
      const int64_t s = R.s;
      std::vector<int64_t> Is(ks);
      std::vector<double> Ps(m * ks), Xs(ks * n), Vs(s * rs), Ws(rs * n);
      check("files spc_id f64", dsk_spc_id(h, As.data(), DSK_F64, m, n, n, ks, rs, &R, qc, &o, Is.data(), Ps.data(),
                                           Xs.data(), Vs.data(), Ws.data(), nullptr));
      write_bin(dir + "/spc64_I.bin", Is.data(), ks * 8);
      write_bin(dir + "/spc64_P.bin", Ps.data(), Ps.size() * 8);
      write_bin(dir + "/spc64_X.bin", Xs.data(), Xs.size() * 8);
      write_bin(dir + "/spc64_V.bin", Vs.data(), Vs.size() * 8);
      write_bin(dir + "/spc64_W.bin", Ws.data(), Ws.size() * 8);
      std::vector<float> As32(As.begin(), As.end()), X32(ks * n);
      check("files spc_id f32", dsk_spc_id(h, As32.data(), DSK_F32, m, n, n, ks, rs, &R, qc, &o, Is.data(), Ps.data(),
                                           X32.data(), nullptr, nullptr, nullptr));
      write_bin(dir + "/spc32_I.bin", Is.data(), ks * 8);
      write_bin(dir + "/spc32_X.bin", X32.data(), X32.size() * 4);
    }
    // nearest-neighbour stencil restriction, FP64, q = 1
    dsk_restriction Rn{};
    Rn.kind = DSK_R_NN;
    Rn.ny = Rn.nx = (int)N;
    Rn.sy = Rn.sx = (int)f;
    check("files svd nn f64 q=1", dsk_sketch_svd(h, A64.data(), DSK_F64, m, n, n, (int)k, &Rn, 1, &o, U.data(),
                                                 S.data(), V.data(), nullptr));
    out("svdnn64q1", 8);
    // projection B^T = A^T Q, FP32 A and Q (ell = 2k + 3)
    const int ellp = (int)(2 * k + 3);
    std::vector<float> Q(m * ellp), Bt(n * ellp);
    if (read_bin(dir + "/Q.bin", Q)) {
      check("files project f32", dsk_project(h, A32.data(), DSK_F32, m, n, n, Q.data(), ellp, Bt.data(),
                                             DSK_MODE_SPLIT6));
      write_bin(dir + "/proj32.bin", Bt.data(), Bt.size() * 4);
    }
  }

  // ---- entry points that run work on several streams (the combined call, the
  // single-pass SVD in each of its three worker paths, a batch over 8 workers):
  // a hash of every output, to compare runs under different stream interleavings
  const bool streams = which == "streams" || which == "streams-quick";
  if (streams) {
    struct Cfg { int64_t m; int N, f, k, f64; };
    std::vector<Cfg> cfgs = {{200, 32, 4, 20, 0}, {150, 32, 4, 20, 1}, {180, 32, 2, 60, 0}};
    if (which == "streams-quick") cfgs = {{120, 32, 4, 12, 0}};
    for (const Cfg &c : cfgs) {
      const int64_t n = (int64_t)c.N * c.N;
      auto A64 = make_A(c.m, c.N, 40, 500 + (unsigned)c.m, 1e-3);
      std::vector<float> A32(A64.begin(), A64.end());
      void *Av = c.f64 ? (void *)A64.data() : (void *)A32.data();
      const size_t we = c.f64 ? 8 : 4;
      auto idx = di_index(c.N, c.f);
      dsk_restriction R{};
      R.kind = DSK_R_INDEX;
      R.s = (int64_t)idx.size();
      R.index = idx.data();
      R.ny = R.nx = c.N;
      R.sy = R.sx = c.f;
      std::vector<char> U(c.m * c.k * we), V(n * c.k * we), rows(c.k * n * we);
      std::vector<double> S(c.k), P(c.m * c.k);
      std::vector<int64_t> I(c.k);
      dsk_info a{}, b{};
      char nm[128];
      snprintf(nm, sizeof nm, "svd_id m=%lld k=%d f64=%d", (long long)c.m, c.k, c.f64);
      check(nm, dsk_sketch_svd_id(h, Av, c.f64 ? DSK_F64 : DSK_F32, c.m, n, n, c.k, &R, 1, 0, &o, U.data(), S.data(),
                                  V.data(), I.data(), P.data(), rows.data(), &a, &b));
      printf("   hash %016llx flags %d %d\n", fnv({{U.data(), U.size()}, {S.data(), S.size() * 8}, {V.data(), V.size()},
                                                {I.data(), I.size() * 8}, {P.data(), P.size() * 8},
                                                {rows.data(), rows.size()}}), a.flags, b.flags);
      {
        // the combined call equals the two separate calls, bit for bit
        std::vector<char> U1(U.size()), V1(V.size()), rows1(rows.size());
        std::vector<double> S1(S.size()), P1(P.size());
        std::vector<int64_t> I1(I.size());
        int rc1 = dsk_sketch_svd(h, Av, c.f64 ? DSK_F64 : DSK_F32, c.m, n, n, c.k, &R, 1, &o, U1.data(), S1.data(),
                                 V1.data(), nullptr);
        rc1 |= dsk_sketch_id(h, Av, c.f64 ? DSK_F64 : DSK_F32, c.m, n, n, c.k, &R, 0, &o, I1.data(), P1.data(),
                             rows1.data(), nullptr);
        simt::sync_all();
        const int differ = rc1 != 0 || U1 != U || V1 != V || S1 != S || I1 != I || P1 != P || rows1 != rows;
        printf("%-44s rc=%d\n", "combined call equals separate calls", differ);
      }
      snprintf(nm, sizeof nm, "svd single pass m=%lld k=%d f64=%d", (long long)c.m, c.k, c.f64);
      check(nm, dsk_sketch_svd_sp(h, Av, c.f64 ? DSK_F64 : DSK_F32, c.m, n, n, c.k, &R, &o, U.data(), S.data(),
                                  V.data(), &a));
      printf("   hash %016llx flags %d\n", fnv({{U.data(), U.size()}, {S.data(), S.size() * 8}, {V.data(), V.size()}}),
             a.flags);
    }
  }
  if (streams) {
    struct Inst { int64_t m; int N, k, f, f64, q; };
    std::vector<Inst> ins = {{231, 32, 18, 2, 1, 2}, {199, 64, 22, 4, 0, 1}, {138, 32, 11, 4, 0, 2},
                             {186, 32, 12, 4, 0, 1}, {198, 64, 19, 4, 0, 0}, {173, 32, 37, 4, 1, 0},
                             {144, 32, 16, 2, 0, 2}, {188, 32, 14, 4, 0, 0}, {138, 64, 11, 4, 0, 1}};
    if (which == "streams-quick")   // nine small problems: still eight workers
      for (size_t i = 0; i < ins.size(); ++i) ins[i] = {70 + 7 * (int64_t)i, 16, 6 + (int)(i % 4), 2, (int)(i % 4 == 0), (int)(i % 3)};
    std::vector<std::vector<double>> A64s, Ss;
    std::vector<std::vector<float>> A32s;
    std::vector<std::vector<int64_t>> idxs;
    std::vector<std::vector<char>> Us, Vs;
    std::vector<dsk_problem> pr;
    for (size_t i = 0; i < ins.size(); ++i) {
      const Inst &t = ins[i];
      const int64_t n = (int64_t)t.N * t.N;
      const size_t we = t.f64 ? 8 : 4;
      A64s.push_back(make_A(t.m, t.N, 30, 700 + (unsigned)i, 1e-3));
      A32s.emplace_back(A64s.back().begin(), A64s.back().end());
      idxs.push_back(di_index(t.N, t.f));
      Us.emplace_back(t.m * t.k * we);
      Vs.emplace_back(n * t.k * we);
      Ss.emplace_back(t.k);
    }
    for (size_t i = 0; i < ins.size(); ++i) {
      const Inst &t = ins[i];
      dsk_problem p{};
      p.A = t.f64 ? (const void *)A64s[i].data() : (const void *)A32s[i].data();
      p.dtype = t.f64 ? DSK_F64 : DSK_F32;
      p.m = t.m;
      p.n = (int64_t)t.N * t.N;
      p.lda = p.n;
      p.k = t.k;
      p.q = t.q;
      p.R.kind = DSK_R_INDEX;
      p.R.s = (int64_t)idxs[i].size();
      p.R.index = idxs[i].data();
      p.U = Us[i].data();
      p.S = Ss[i].data();
      p.V = Vs[i].data();
      pr.push_back(p);
    }
    int nw = 0;
    check("batched eager, 9 problems", dsk_sketch_svd_batched(h, (int)pr.size(), pr.data(), &o, 0, &nw));
    for (size_t i = 0; i < ins.size(); ++i)
      printf("   hash %016llx problem %zu workers %d\n",
             fnv({{Us[i].data(), Us[i].size()}, {Ss[i].data(), Ss[i].size() * 8}, {Vs[i].data(), Vs[i].size()}}), i, nw);
    // every instance of the batch equals the same problem run alone, bit for bit
    int differ = 0;
    for (size_t i = 0; i < ins.size(); ++i) {
      std::vector<char> U1(Us[i].size()), V1(Vs[i].size());
      std::vector<double> S1(Ss[i].size());
      const dsk_problem &p = pr[i];
      const int rc1 = dsk_sketch_svd(h, p.A, p.dtype, p.m, p.n, p.lda, p.k, &p.R, p.q, &o, U1.data(), S1.data(),
                                     V1.data(), nullptr);
      simt::sync_all();
      differ += rc1 != 0 || U1 != Us[i] || V1 != Vs[i] || S1 != Ss[i];
    }
    printf("%-44s rc=%d\n", "batch instances equal single calls", differ);
  }

  // ---- one-launch pivoted QR against the per-step one, bitwise
  if (persist) {
    struct Cfg { int64_t m; int N, f, k, f64; };
    // s = 64, 256 (registers 4 per thread), 1024 (ragged: 4 per thread, last
    // slots empty), 4096 (16 per thread); m with an incomplete last workgroup
    std::vector<Cfg> cfgs = {{61, 32, 4, 20, 0}, {37, 64, 1, 30, 1}, {96, 32, 2, 40, 1}, {190, 64, 2, 50, 0}};
    if (which == "persist-quick") cfgs.resize(2);
    for (const Cfg &c : cfgs) {
      const int64_t n = (int64_t)c.N * c.N;
      auto A64 = make_A(c.m, c.N, 30, 300 + (unsigned)c.m, 1e-3);
      std::vector<float> A32(A64.begin(), A64.end());
      void *Av = c.f64 ? (void *)A64.data() : (void *)A32.data();
      auto idx = di_index(c.N, c.f);
      dsk_restriction R{};
      R.kind = DSK_R_INDEX;
      R.s = (int64_t)idx.size();
      R.index = idx.data();
      R.ny = R.nx = c.N;
      R.sy = R.sx = c.f;
      std::vector<int64_t> I[2];
      std::vector<double> P[2];
      dsk_info inf[2]{};
      long long res[2];
      for (int ps = 0; ps < 2; ++ps) {
        const long long before = simt::g_resident_launches;
        dsk_opts oo = o;
        oo.id_per_step = ps;
        I[ps].assign(c.k, -1);
        P[ps].assign(c.m * c.k, 0.0);
        char nm[128];
        snprintf(nm, sizeof nm, "id m=%lld s=%lld k=%d f64=%d %s", (long long)c.m, (long long)R.s, c.k, c.f64,
                 ps ? "per-step" : "one launch");
        check(nm, dsk_sketch_id(h, Av, c.f64 ? DSK_F64 : DSK_F32, c.m, n, n, c.k, &R, 0, &oo, I[ps].data(),
                                P[ps].data(), nullptr, &inf[ps]));
        res[ps] = simt::g_resident_launches - before;
      }
      // the one-launch kernel takes the left-looking recurrence: same pivots, P to rounding
      const bool same = I[0] == I[1];
      double maxdp = 0.0, maxp = 1.0;
      for (size_t e = 0; e < P[0].size(); ++e) {
        maxdp = std::max(maxdp, std::fabs(P[0][e] - P[1][e]));
        maxp = std::max(maxp, std::fabs(P[1][e]));
      }
      printf("   I0 %lld I%d %lld flags %d %d resident launches %lld %lld same %d maxdp %.3e\n", (long long)I[0][0],
             c.k - 1, (long long)I[0][c.k - 1], inf[0].flags, inf[1].flags, res[0], res[1], same ? 1 : 0,
             maxdp / maxp);
      // 16-bit storage: the restricted columns stay 16-bit in the factorization's
      // input; the same values given as FP32 must give the same pivots, P to rounding
      // (persist-quick: the first configuration only, to bound its run time)
      for (int half = 0; half < (which == "persist-quick" && &c != &cfgs[0] ? 0 : 2); ++half) {
        std::vector<uint16_t> A16(c.m * n);
        std::vector<float> Ar(c.m * n);
        for (int64_t e = 0; e < c.m * n; ++e) {
          if (half) {
            const _Float16 v = (_Float16)A32[e];
            memcpy(&A16[e], &v, 2);
            Ar[e] = (float)v;
          } else {
            const __bf16 v = (__bf16)A32[e];
            memcpy(&A16[e], &v, 2);
            Ar[e] = (float)v;
          }
        }
        std::vector<int64_t> Ih(c.k, -1), Ir(c.k, -1);
        std::vector<double> Ph(c.m * c.k, 0.0), Pr(c.m * c.k, 0.0);
        dsk_info ih{}, ir{};
        char nm[128];
        snprintf(nm, sizeof nm, "id m=%lld s=%lld k=%d %s storage", (long long)c.m, (long long)R.s, c.k,
                 half ? "f16" : "bf16");
        check(nm, dsk_sketch_id(h, A16.data(), half ? DSK_F16 : DSK_BF16, c.m, n, n, c.k, &R, 0, &o, Ih.data(),
                                Ph.data(), nullptr, &ih));
        check("id same values as f32", dsk_sketch_id(h, Ar.data(), DSK_F32, c.m, n, n, c.k, &R, 0, &o, Ir.data(),
                                                     Pr.data(), nullptr, &ir));
        double dp = 0.0, mp = 1.0;
        for (size_t e = 0; e < Pr.size(); ++e) {
          dp = std::max(dp, std::fabs(Ph[e] - Pr[e]));
          mp = std::max(mp, std::fabs(Pr[e]));
        }
        printf("   16-bit %s flags %d %d same16 %d maxdp16 %.3e\n", half ? "f16" : "bf16", ih.flags, ir.flags,
               Ih == Ir ? 1 : 0, dp / mp);
      }
    }
  }
  dsk_destroy(h);
  printf("done\n");
  return 0;
}

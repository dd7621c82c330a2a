"""The HIP kernels of the main paths, run on the host under AddressSanitizer.

tests/emu builds the library's HIP sources as host C++ against a small HIP
shim (each GPU thread a fiber scheduled until it blocks at a barrier; wave
shuffles, readlane, DPP and MFMA emulated by per-group exchange; dynamic LDS a
heap buffer of exactly the launch's size) and runs the C ABI on host buffers:
the sketch SVD (FP32 at q = 0, 1 and FP64), the row ID, the combined call,
the single-pass SVD, SPC-ID-ERR, a batch and the one-launch pivoted QR (its
workgroups resident together).  Any out-of-bounds access to a
device buffer or to LDS aborts with an AddressSanitizer report; a missing
barrier shows up as a deadlock with a per-thread state dump.  The emulated
results also have to agree across precisions and algorithms, and the entry
points that run work on several streams have to give the same bits in every
interleaving of their streams' queued work.  On a small seeded input the
emulated outputs are compared with the FP64 oracle at the GPU parity
tolerances.
"""
import importlib.util
import os
import re
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _build():
    spec = importlib.util.spec_from_file_location("emu_build", os.path.join(HERE, "emu", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    if mod._cxx() is None:
        pytest.skip("no host clang++ for the emulation build")
    return mod.build()


# the default emulation runs, started together on first use (each is one
# single-threaded process) and collected by the tests that read them
_DEFAULT_RUNS = [("quick", None), ("persist-quick", None), ("streams-quick", None), ("streams-quick", 0),
                 ("streams-quick", 1), ("streams-quick", 9001)]


class _Run:
    def __init__(self, returncode, stdout, stderr):
        self.returncode, self.stdout, self.stderr = returncode, stdout, stderr


def _spawn(exe, mode, order):
    env = dict(os.environ)
    env.pop("SIMT_STREAMS", None)
    if order is not None:
        env["SIMT_STREAMS"] = f"defer:{order}"
    return subprocess.Popen([exe, mode], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)


def _collect(p):
    so, se = p.communicate(timeout=1800)
    return _Run(p.returncode, so, se)


def _files_inputs(d=None):
    """The seeded inputs of the file mode (written to d when given)."""
    import numpy as np

    from oracle import restrict as ores
    from paper_2105_01271_amd import synth

    m, N, f, k, mc = 120, 16, 2, 10, 30
    rng = np.random.default_rng(61)
    A = synth.heat_modes(m, N, seed=60, nu=0.002) + 1e-2 * rng.standard_normal((m, N * N))
    idx = ores.di_index_2d(N, N, f, f)
    taus = np.array([0.0, 1.0, 4.0, 16.0])
    # BF16 storage: round to nearest even on the FP32 bit pattern
    bits = A.astype(np.float32).view(np.uint32).astype(np.uint64)
    bf = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16).astype("<u2")
    A_bf = (bf.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    Q = rng.standard_normal((m, 2 * k + 3)).astype("<f4")
    Om = synth.gaussian_matrix(idx.size, k + 6, seed=62)
    C, sl = 4, (N // 4) ** 2
    w1 = (0.2 * rng.standard_normal((C, 5, 5))).astype("<f4")
    w2 = (0.2 * rng.standard_normal((C, 5, 5))).astype("<f4")
    w1[0, 2, 2] += 1.0
    w2[0, 2, 2] += 1.0
    gAc = rng.standard_normal((m, sl)).astype("<f4")
    Q0 = rng.standard_normal((m, 6))
    # SPC-ID input: rank 12 with sigma_j = 0.6^j plus 1e-9 noise (a clear drop at r = 12)
    Ut = np.linalg.qr(rng.standard_normal((m, 12)))[0]
    Vt = np.linalg.qr(rng.standard_normal((N * N, 12)))[0]
    Aspc = (Ut * 0.6 ** np.arange(12)) @ Vt.T + 1e-9 * rng.standard_normal((m, N * N))
    if d is not None:
        (d / "dims.txt").write_text(f"{m} {N} {f} {k} {mc} {taus.size}\n")
        for name, arr, dt in [("A", A, "<f8"), ("taus", taus, "<f8"), ("Abf", bf, "<u2"), ("Q", Q, "<f4"),
                              ("Om", Om, "<f8"), ("w1", w1, "<f4"), ("w2", w2, "<f4"), ("gAc", gAc, "<f4"),
                              ("Q0", Q0, "<f8"), ("Aspc", Aspc, "<f8")]:
            arr.astype(dt).tofile(d / f"{name}.bin")
    return {"m": m, "N": N, "f": f, "k": k, "mc": mc, "A": A, "idx": idx, "taus": taus, "A_bf": A_bf, "Q": Q,
            "Om": Om, "w1": w1, "w2": w2, "gAc": gAc, "Q0": Q0, "Aspc": Aspc}


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    procs = {}
    results = {}
    files_dir = tmp_path_factory.mktemp("emu_files")

    def get(mode, order=None):
        if not procs:
            exe = _build()
            for key in _DEFAULT_RUNS:
                procs[key] = _spawn(exe, *key)
            _files_inputs(files_dir)
            procs[("files", None)] = subprocess.Popen([exe, "files", str(files_dir)], stdout=subprocess.PIPE,
                                                      stderr=subprocess.PIPE, text=True)
        key = (mode, order)
        if key not in results:
            results[key] = _collect(procs[key])
        return results[key]

    get.files_dir = files_dir
    yield get
    for p in procs.values():   # runs no test collected (a -k selection) end with the module
        if p.poll() is None:
            p.kill()
            p.communicate()


def test_kernels_run_clean_under_host_emulation(emu):
    r = emu("quick")
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "SIMT FATAL" not in out, out[-4000:]
    assert out.rstrip().endswith("done"), out[-2000:]
    rcs = re.findall(r"^(.*?)\s+rc=(-?\d+)$", r.stdout, re.M)
    assert len(rcs) >= 9, r.stdout
    for name, rc in rcs:
        expect = -5 if "graph" in name else 0   # graph replay of batches is disabled
        assert int(rc) == expect, (name, rc)
    flags = [int(x) for x in re.findall(r"flags (-?\d+)", r.stdout)]
    assert flags and all(f == 0 for f in flags), r.stdout
    # the same matrix in FP32 and FP64 (q = 0): singular values agree to the FP32 tolerance
    svals = {}
    for line in r.stdout.splitlines():
        m = re.match(r"svd f64=(\d) cfg=0 q=0", line)
        if m:
            key = int(m.group(1))
        m2 = re.match(r"\s+S0 ([\d.eE+-]+) S19 ([\d.eE+-]+)", line)
        if m2 and "key" in locals():
            svals.setdefault(key, (float(m2.group(1)), float(m2.group(2))))
            del key
    assert set(svals) == {0, 1}, r.stdout
    s32, s64 = svals[0], svals[1]
    assert abs(s32[0] - s64[0]) <= 1e-5 * s64[0] and abs(s32[1] - s64[1]) <= 1e-5 * s64[0], svals
    # single-pass SVD equals the two-pass one at q = 0 (Alg. 3 vs Alg. 2)
    sp = float(re.search(r"svd single pass.*\n\s+S0 ([\d.eE+-]+)", r.stdout).group(1))
    assert abs(sp - s32[0]) <= 1e-5 * s32[0], (sp, s32)


@pytest.mark.skipif(os.environ.get("DSK_EMU_FULL") != "1", reason="the extended host emulation runs about 4 minutes; "
                    "set DSK_EMU_FULL=1")
def test_remaining_paths_run_clean_under_host_emulation():
    """ell = 110 (wide CholeskyQR and eigensolver kernels), BF16 storage with the
    refinement sweep, FP16, stencil restrictions (SVD and ID), the projected ID
    and the SVD with a given second-level sketch, the restriction, projection
    and power iteration entry points, the learned restriction (forward,
    backward, loss gradient, Adam, SVD) and the documented argument errors."""
    exe = _build()
    r = subprocess.run([exe, "more"], capture_output=True, text=True, timeout=1800)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "SIMT FATAL" not in out, out[-4000:]
    assert out.rstrip().endswith("done"), out[-2000:]
    rcs = re.findall(r"^(.*?)\s+rc=(-?\d+)$", r.stdout, re.M)
    assert len(rcs) >= 18, r.stdout
    assert all(int(rc) == 0 for _, rc in rcs), rcs


def _check_persist(r):
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "SIMT FATAL" not in out, out[-4000:]
    assert out.rstrip().endswith("done"), out[-2000:]
    rcs = re.findall(r"^(.*?)\s+rc=(-?\d+)$", r.stdout, re.M)
    assert rcs and all(int(rc) == 0 for _, rc in rcs), rcs
    res = re.findall(r"flags (\d+) (\d+) resident launches (\d+) (\d+) same (\d) maxdp (\S+)", r.stdout)
    assert res, r.stdout
    for f0, f1, n0, n1, same, maxdp in res:
        # the one-launch factorization ran (all its workgroups resident together),
        # raised no flag (a timed-out wait would), takes the per-step pivots and
        # gives P to rounding (left-looking against right-looking Gram-Schmidt)
        assert (int(n0), int(n1)) == (1, 0), res
        # flag 1 (fallback): the downdated norms ran out of accuracy and the exact
        # one-workgroup factorization finished the job; no other flag may appear
        assert int(f0) in (0, 1) and int(f1) == 0, res
        assert same == "1", res
        assert float(maxdp) <= 1e-9, res
    # 16-bit input (index restriction, no power iteration): the factorization reads
    # the restricted columns in their 16-bit storage; the same values as FP32 give
    # the same pivots and P to rounding (both accumulate in FP64)
    r16 = re.findall(r"16-bit (\w+) flags (\d+) (\d+) same16 (\d) maxdp16 (\S+)", r.stdout)
    assert len(r16) >= 2, r.stdout
    for dt, f0, f1, same, maxdp in r16:
        assert f0 == f1 and same == "1", r16
        assert float(maxdp) <= 1e-9, r16
    return len(res)


def test_one_launch_pivoted_qr_equals_per_step_under_host_emulation(emu):
    """The one-launch pivoted QR of the row ID, whose workgroups wait on each
    other's published words, run with every workgroup of the launch resident
    (a spin-wait iteration yields to the other threads): no out-of-bounds
    access, no deadlock, the per-step factorization's pivots and its P to
    rounding (s = 64 and 4096, m with an incomplete last workgroup)."""
    assert _check_persist(emu("persist-quick")) == 2


@pytest.mark.skipif(os.environ.get("DSK_EMU_FULL") != "1", reason="about three minutes; set DSK_EMU_FULL=1")
def test_one_launch_pivoted_qr_all_widths_under_host_emulation():
    """As above, adding s = 256 (FP64) and s = 1024 with 48 workgroups."""
    exe = _build()
    r = subprocess.run([exe, "persist"], capture_output=True, text=True, timeout=1800)
    assert _check_persist(r) == 4


def _check_streams(runs):
    """runs: {order: _Run} for one mode with immediate streams (None) and with
    each deferred order; returns {order: stdout}."""
    outs = {}
    for order, r in runs.items():
        so, se = r.stdout, r.stderr
        out = so + se
        assert r.returncode == 0, (order, out[-4000:])
        assert "ERROR: AddressSanitizer" not in out and "SIMT FATAL" not in out, (order, out[-4000:])
        assert so.rstrip().endswith("done"), (order, out[-2000:])
        rcs = re.findall(r"^(.*?)\s+rc=(-?\d+)$", so, re.M)
        assert rcs and all(int(rc) == 0 for _, rc in rcs), (order, rcs)
        if order is not None:
            st = re.search(r"SIMT streams: (\d+) items, (\d+) with a choice of stream", se)
            assert st and int(st.group(2)) > 0, (order, se[-2000:])
        outs[order] = so
    return outs


def _hashes(so):
    return re.findall(r"hash ([0-9a-f]{16}) (.*)$", so, re.M)


def test_multi_stream_entry_points_are_interleaving_independent(emu):
    """The combined SVD + ID call (row ID on a worker stream), the single-pass
    SVD (Q and R on a worker stream beside the pass over A) and a batch over
    eight worker streams, run with each stream's work queued and the queues
    advanced in three different interleavings (main stream first, workers
    first, seeded random): every output is bitwise the same as in issue
    order, so no work on one stream reads or overwrites what another stream
    has not ordered by an event; every batch instance equals the same
    problem run alone, and the combined call the two separate calls, bit for
    bit.  (Removing the single-pass join changes the
    outputs under the main-stream-first order.)"""
    outs = _check_streams({o: emu("streams-quick", o) for o in (None, 0, 1, 9001)})
    ref = _hashes(outs[None])
    assert len(ref) == 11, outs[None]
    assert all("batch instances equal single calls" in so for so in outs.values())
    assert all("combined call equals separate calls" in so for so in outs.values())
    for order, so in outs.items():
        assert _hashes(so) == ref, order


@pytest.mark.skipif(os.environ.get("DSK_EMU_FULL") != "1", reason="about three minutes; set DSK_EMU_FULL=1")
def test_multi_stream_entry_points_all_paths_interleaving_independent():
    """As above on FP32 and FP64 and on the single-pass path with ell > 64, and
    the batch at the batched test's sizes."""
    exe = _build()
    procs = {o: _spawn(exe, "streams", o) for o in (None, 0, 1, 12345, 777)}
    outs = _check_streams({o: _collect(p) for o, p in procs.items()})
    ref = _hashes(outs[None])
    assert len(ref) == 15, outs[None]
    for order, so in outs.items():
        assert _hashes(so) == ref, order


def test_emulated_kernels_match_the_oracle(emu):
    """The HIP path run in host emulation against the FP64 oracle on the same
    seeded input (120 x 16^2, direct injection 2 x 2, s = 64, k = 10, ell =
    20), at the GPU parity tests' tolerances: sketch SVD (FP64 q = 0, 1; FP32
    and BF16 storage q = 1 against the oracle on the upcast stored values; the
    nearest-neighbour stencil restriction; a Gaussian second level, with the ID
    of the projected block), the learned conv restriction (forward, weight
    gradients, training loss and its gradients), the restriction and C-PWR
    entry points, the projection, the single-pass SVD (with its kappa(Y)
    term), the row ID (pivots and P) and SPC-ID-ERR with its rho(tau)
    estimate.  The emulation runs beside the other default ones."""
    import numpy as np

    from oracle import restrict as ores
    from oracle import rowid as orid
    from oracle import sketch as osk

    tmp_path = emu.files_dir
    inp = _files_inputs()
    m, N, f, k, mc = inp["m"], inp["N"], inp["f"], inp["k"], inp["mc"]
    A, idx, taus, A_bf, Q, Om = inp["A"], inp["idx"], inp["taus"], inp["A_bf"], inp["Q"], inp["Om"]
    w1, w2, gAc, Q0 = inp["w1"], inp["w2"], inp["gAc"], inp["Q0"]
    ellp, C, sl = 2 * k + 3, 4, (N // 4) ** 2
    r = emu("files")
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "SIMT FATAL" not in out and "runtime error" not in out, out[-4000:]
    rcs = re.findall(r"^(.*?)\s+rc=(-?\d+)$", r.stdout, re.M)
    assert len(rcs) == 20 and all(int(c) == 0 for _, c in rcs), r.stdout

    n = N * N
    Rd = {"kind": "index", "index": idx}

    def load(tag, dt, shape):
        return np.fromfile(tmp_path / f"{tag}.bin", dtype=dt).reshape(shape).astype(np.float64)

    def svd_parts(tag, dt):
        return load(f"{tag}_U", dt, (m, k)), load(f"{tag}_S", "<f8", (k,)), load(f"{tag}_V", dt, (n, k))

    def err(Ax, U, S, V):
        return np.linalg.norm(Ax - (U * S) @ V.T)

    A32 = A.astype(np.float32).astype(np.float64)
    Rnn = {"kind": "nn", "ny": N, "nx": N, "sy": f, "sx": f}
    for tag, Ax, Rx, q, dt, tol in [("svd64q0", A, Rd, 0, "<f8", 1e-10), ("svd64q1", A, Rd, 1, "<f8", 1e-10),
                                    ("svd32q1", A32, Rd, 1, "<f4", 1e-5), ("svdbfq1", A_bf, Rd, 1, "<f4", 1e-4),
                                    ("svdnn64q1", A, Rnn, 1, "<f8", 1e-10)]:
        U, S, V = svd_parts(tag, dt)
        Uo, So, Vo = osk.tpc_svd(Ax, k, Rx, q=q)
        assert np.abs(S - So).max() <= tol * So[0], (tag, S, So)
        eo = err(Ax, Uo, So, Vo)
        assert abs(err(Ax, U, S, V) - eo) <= tol * max(eo, 1e-13 * So[0]) + tol * So[0] * 1e-3, tag
        assert np.abs(U.T @ U - np.eye(k)).max() <= 100 * tol, tag

    # hybrid sketch (Gaussian second level): SVD and the ID of the projected block
    U, S, V = svd_parts("hyb64q1", "<f8")
    Uo, So, Vo = osk.tpc_svd(A, k, Rd, q=1, S=Om)
    assert np.abs(S - So).max() <= 1e-10 * So[0], (S, So)
    I = np.fromfile(tmp_path / "hybid_I.bin", dtype="<i8")
    P = load("hybid_P", "<f8", (m, k))
    Io, Po = orid.tpc_id(A, k, Rd, q=1, S=Om, projected=True)
    assert list(I) == list(Io), (I, Io)
    assert np.abs(P - Po).max() <= 1e-7 * max(1.0, np.abs(Po).max())

    # restriction entry point (a gather is exact; the global average to rounding) and
    # the C-PWR loop: the raw block (tau A_c A_c^T)^2 Q0, and the span of the
    # re-orthonormalised one
    Ac = A[:, idx]
    assert np.array_equal(load("rest_idx", "<f8", (m, idx.size)), Ac)
    Rg = {"kind": "global", "ny": N, "nx": N, "sy": f, "sx": f}
    ref = ores.apply(A, Rg)
    assert np.abs(load("rest_glob", "<f8", ref.shape) - ref).max() <= 1e-14 * np.abs(ref).max()
    tau = N * N / idx.size
    raw = load("pw_raw", "<f8", (m, 6))
    ref = osk.power_iter(Ac, Q0, 2, tau, reorth=False)
    assert np.abs(raw - ref).max() <= 1e-12 * np.abs(ref).max()
    Qg = load("pw_orth", "<f8", (m, 6))
    Qr = osk.power_iter(Ac, Q0, 2, tau, reorth=True)
    assert np.abs(Qg.T @ Qg - np.eye(6)).max() <= 1e-12
    assert np.linalg.norm(Qg @ Qg.T - Qr @ Qr.T, 2) <= 1e-10

    # learned conv restriction (the GPU learned tests' tolerances)
    from oracle import learned as olearn
    # oracle layout: w1 as C x 1 x 5 x 5 (1 -> C channels), w2 as 1 x C x 5 x 5
    o1, o2 = w1.astype(np.float64).reshape(C, 1, 5, 5), w2.astype(np.float64).reshape(1, C, 5, 5)
    Acl = load("learned_Ac", "<f4", (m, sl))
    ref = ores.conv_restrict(A32, N, N, o1, o2)
    assert np.abs(Acl - ref).max() <= 2e-6 * np.abs(ref).max()
    r1, r2 = ores.conv_restrict_bwd(A32, N, N, o1, o2, gAc.astype(np.float64))
    for tag, rr in (("learned_g1", r1), ("learned_g2", r2)):
        g = load(tag, "<f4", (C * 25,))
        assert np.abs(g - rr.reshape(-1)).max() <= 1e-5 * np.abs(rr).max(), tag
    L, l1, l2 = olearn.learned_loss_and_grad(A, N, N, o1, o2, 8, 1)
    loss = np.fromfile(tmp_path / "learned_loss.bin", dtype="<f8")[0]
    assert abs(loss - L) <= 1e-6, (loss, L)
    for tag, rr in (("learned_l1", l1), ("learned_l2", l2)):
        g = load(tag, "<f4", (C * 25,))
        assert np.abs(g - rr.reshape(-1)).max() <= 1e-5 * np.abs(rr).max(), tag

    # projection B^T = A^T Q (FP32, three-piece split): the definition in FP64
    Bt = load("proj32", "<f4", (n, ellp))
    ref = A32.T @ Q.astype(np.float64)
    scale = np.sqrt((A32 ** 2).sum(0)).max() * np.sqrt((Q.astype(np.float64) ** 2).sum(0)).max()
    assert np.abs(Bt - ref).max() <= 1e-6 * scale

    # single pass (Alg. 3): the TPC tolerance plus (4 + ell) u kappa_F(Y) ||A||_F / sigma_1
    U, S, V = svd_parts("sp64", "<f8")
    Uo, So, Vo = osk.spc_svd(A, k, Rd)
    Ac = A[:, idx]
    ell = k + 10
    Y = Ac[:, osk.nested_di_columns(idx.size, ell)]
    Rf = np.linalg.qr(Y, mode="r")
    kF = np.linalg.norm(Y) * np.linalg.norm(np.linalg.inv(Rf))
    tol_sp = 1e-10 + (4 + ell) * 2.0 ** -53 * kF * np.linalg.norm(A) / So[0]
    assert np.abs(S - So).max() <= tol_sp * So[0], (S, So, tol_sp)

    # row ID (Alg. 4): pivots and coefficients
    I = np.fromfile(tmp_path / "id64_I.bin", dtype="<i8")
    P = load("id64_P", "<f8", (m, k))
    Io, Po = orid.tpc_id(A, k, Rd, q=0)
    assert list(I) == list(Io), (I, Io)
    assert np.abs(P - Po).max() <= 1e-8 * max(1.0, np.abs(Po).max()), np.abs(P - Po).max()

    # SPC-ID (Alg. 5): the skeleton and P of the coarse row ID, the lifted rows
    # X = A_c(I, :) T_r and the factors T_r = V_r W_r against the oracle's T_r.  FP32:
    # the rounding of H = A^T A_c is amplified by about sigma_1 / sigma_r in X
    As = inp["Aspc"]
    ks, rs = 6, 12
    Io, Po, _, Tro = orid.spc_id(As, ks, Rd, rs)
    Xo = As[:, idx][Io] @ Tro
    I = np.fromfile(tmp_path / "spc64_I.bin", dtype="<i8")
    assert list(I) == list(Io), (I, Io)
    assert np.abs(load("spc64_P", "<f8", (m, ks)) - Po).max() <= 1e-8 * max(1.0, np.abs(Po).max())
    X = load("spc64_X", "<f8", (ks, n))
    assert np.abs(X - Xo).max() <= 1e-9 * np.abs(Xo).max(), np.abs(X - Xo).max() / np.abs(Xo).max()
    # T_r = V_r W_r: the oracle's literal form (U_c^T U_r U_r^T U_c with every
    # pseudo-inverted singular value of A_c) carries its own rounding, amplified by
    # sigma_1 / sigma_min+ (sigma_min+ the smallest it inverts); W_r against its
    # definition S_r^{-2} V_r^T A_c^T A with the device's V_r, in FP64
    sc = np.linalg.svd(As[:, idx], compute_uv=False)
    smin = sc[sc > sc[0] * max(m, idx.size) * np.finfo(np.float64).eps].min()
    Vg, Wg = load("spc64_V", "<f8", (idx.size, rs)), load("spc64_W", "<f8", (rs, n))
    assert np.abs(Vg.T @ Vg - np.eye(rs)).max() <= 1e-12
    Wdef = (1.0 / sc[:rs] ** 2)[:, None] * (Vg.T @ (As[:, idx].T @ As))
    assert np.abs(Wg - Wdef).max() <= 1e-9 * np.abs(Wdef).max()
    tolT = 1e-9 + 16 * 2.0 ** -53 * sc[0] / smin
    assert np.abs(Vg @ Wg - Tro).max() <= tolT * np.abs(Tro).max()
    As32 = As.astype(np.float32).astype(np.float64)
    Io32, _, _, Tro32 = orid.spc_id(As32, ks, Rd, rs)
    Xo32 = As32[:, idx][Io32] @ Tro32
    assert list(np.fromfile(tmp_path / "spc32_I.bin", dtype="<i8")) == list(Io32)
    X32 = load("spc32_X", "<f4", (ks, n))
    tol32 = 8 * 2.0 ** -24 * sc[0] / sc[rs - 1]
    assert np.abs(X32 - Xo32).max() <= tol32 * np.abs(Xo32).max(), (np.abs(X32 - Xo32).max() / np.abs(Xo32).max(),
                                                                     tol32)

    # SPC-ID-ERR (Alg. 6)
    eps = np.fromfile(tmp_path / "eps64.bin", dtype="<f8")
    ref = orid.spc_id_err_curve(A, Rd, mc, taus)
    c = m // mc
    keep = [i for i in range(m) if (i + 1) % c == 0]
    Gf, Gc = A[keep] @ A[keep].T, Ac[keep] @ Ac[keep].T
    tol = np.array([1e-10 * c * (abs(np.trace(Gf - t * Gc)) + len(keep) * np.linalg.norm(Gf - t * Gc)) for t in taus])
    assert np.all(np.abs(eps - ref) <= tol), (eps, ref, tol)
    rho = np.fromfile(tmp_path / "rho64.bin", dtype="<f8")
    ref_rho = orid.spc_rho_curve(A, Rd, mc, taus)
    assert np.all(np.abs(rho - ref_rho) <= tol), (rho, ref_rho, tol)

"""GPU parity of the HIP path (through the C ABI) against the FP64 CPU oracle
on the same seeded inputs.

Tolerances (singular values relative to sigma_1; reconstruction errors
relative to max(e_oracle, 100 eps sqrt(min(m, n)))): 1e-10 for FP64 input,
1e-5 for FP32 input (oracle run on the exactly upcast FP32 values).
Row-ID skeletons must match the oracle's pivots up to the first step whose
two largest residual norms are not separated (relative gap <= 1e-8, or below
the rounding floor of FP64 residuals); after it only reconstruction errors
are compared.
"""
import math

import numpy as np
import pytest
import torch

from oracle import metrics as omet
from oracle import restrict as ores
from oracle import rowid as orid
from oracle import sketch as osk
from paper_2105_01271_amd import synth

import svdcheck   # tests/svdcheck.py (pytest puts the test directory on sys.path)

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}


def dsk():
    from paper_2105_01271_amd import dsketch
    return dsketch


def say(*a):
    print(*a, flush=True)


def _A(A_np, dtype):
    return torch.from_numpy(np.ascontiguousarray(A_np)).to(dtype).cuda()


def _up(A_t):
    return A_t.double().cpu().numpy()


def _err_tol(e_or, tol, m, n):
    return tol * max(e_or, 100 * np.finfo(np.float64).eps * math.sqrt(min(m, n)))


# ------------------------------------------------------------------ projection B^T = A^T Q

@pytest.mark.parametrize("dtype,mode", [(torch.float32, "split6"), (torch.float32, "split3"), (torch.float32, "f32"),
                                        (torch.float64, "default"), (torch.bfloat16, "default"),
                                        (torch.float16, "default")])
@pytest.mark.parametrize("m,n,ell", [(300, 1000, 60), (77, 129, 7), (1000, 4096, 110), (33, 64, 16)])
def test_project_matches_definition(dtype, mode, m, n, ell):
    say("project", dtype, mode, m, n, ell)
    rng = np.random.default_rng(m * 7 + n + ell)
    A = _A(rng.standard_normal((m, n)), dtype)
    Q = torch.from_numpy(rng.standard_normal((m, ell))).to(torch.float64 if dtype == torch.float64 else torch.float32).cuda()
    Bt = dsk().project(A, Q, mode=mode)
    torch.cuda.synchronize()
    ref = _up(A).T @ Q.double().cpu().numpy()          # B^T = A^T Q, FP64 definition
    err = np.abs(Bt.double().cpu().numpy() - ref).max()
    scale = np.sqrt((_up(A) ** 2).sum(0)).max() * np.sqrt((Q.double().cpu().numpy() ** 2).sum(0)).max()
    tol = {torch.float64: 1e-13}.get(dtype, {"split6": 1e-6, "f32": 1e-6}.get(mode, 2e-5))
    say("  max err / scale", err / scale)
    assert err <= tol * scale, (err, scale)


# ------------------------------------------------------------------ restriction

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("kind", ["index", "nn", "global"])
def test_restrict_matches_oracle(dtype, kind):
    say("restrict", dtype, kind)
    ny, nx, sy, sx = 30, 22, 3, 2
    rng = np.random.default_rng(5)
    A = _A(rng.standard_normal((77, ny * nx)), dtype)
    if kind == "index":
        R = dsk().Restriction.di_grid(ny, nx, sy, sx)
        ref = ores.gather(_up(A), ores.di_index_2d(ny, nx, sy, sx))
    elif kind == "nn":
        R = dsk().Restriction.nn(ny, nx, sy, sx)
        ref = ores.nearest_neighbour_2d(_up(A), ny, nx, sy, sx)
    else:
        R = dsk().Restriction.global_(ny, nx, sy, sx)
        ref = ores.global_2d(_up(A), ny, nx, sy, sx)
    Ac = dsk().restrict(A, R)
    got = Ac.double().cpu().numpy()
    if kind == "index":
        np.testing.assert_array_equal(got, ref)          # a gather is exact
    else:
        tol = 1e-15 if dtype == torch.float64 else 1e-6
        np.testing.assert_allclose(got, ref, rtol=0, atol=tol * np.abs(ref).max())


# ------------------------------------------------------------------ power iteration

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("reorth", [True, False])
def test_power_iter_matches_oracle(dtype, reorth):
    say("power_iter", dtype, reorth)
    rng = np.random.default_rng(11)
    m, s, ell, q, tau = 150, 257, 12, 2, 0.7
    Ac_np = rng.standard_normal((m, 40)) @ np.diag(0.85 ** np.arange(40)) @ rng.standard_normal((40, s)) / 10
    Ac = _A(Ac_np, dtype)
    Q0_np = osk.orth(_up(Ac)[:, :ell])
    Q0 = torch.from_numpy(Q0_np).to(dtype).cuda()
    G = dsk().power_iter(Ac, Q0, q, tau=tau, reorth=reorth)
    ref = osk.power_iter(_up(Ac), _up(Q0), q, tau, reorth=reorth)
    got = _up(G)
    tol = TOL[dtype]
    if reorth:
        # same span: ||P_gpu - P_ref|| small and G orthonormal
        assert np.abs(got.T @ got - np.eye(ell)).max() < (1e-13 if dtype == torch.float64 else 1e-5)
        assert np.linalg.norm(got @ got.T - ref @ ref.T, 2) < 100 * tol
    else:
        assert np.abs(got - ref).max() <= 10 * tol * np.abs(ref).max()


# ------------------------------------------------------------------ sketch SVD

def _compare_svd(A_np_exact, U, S, V, Uo, So, Vo, tol, sig_all=None):
    """Singular values and reconstruction error to tol; singular vectors
    entry by entry (singletons) or by cluster projectors (tests/svdcheck.py)
    when the oracle's full spectrum of B is given."""
    m, n = A_np_exact.shape
    S = S.cpu().numpy()
    assert np.abs(S - So).max() <= tol * So[0], (np.abs(S - So).max() / So[0])
    e_gpu = omet.svd_error(A_np_exact, _up(U), S, _up(V))
    e_or = omet.svd_error(A_np_exact, Uo, So, Vo)
    assert abs(e_gpu - e_or) <= _err_tol(e_or, tol, m, n) + tol * 1e-3, (e_gpu, e_or)
    if sig_all is not None:
        nchk = svdcheck.compare_vectors(_up(U), Uo, _up(V), Vo, sig_all, len(So), tol)
        say("  singular pairs compared one by one:", nchk)


def _tpc(A_np, k, R, **kw):
    Uo, So, Vo, info = osk.tpc_svd(A_np, k, R, return_all=True, **kw)
    return Uo, So, Vo, info["sigma_B"]


@pytest.mark.parametrize("q", [0, 1])
def test_sketch_svd_heat_fp64_small_config(q):
    # 200 time steps x 64x64 heat modes, DI every 4th point per axis (s = 256), k = 20
    say("svd fp64 heat q", q)
    A_np = synth.heat_modes(200, 64, seed=0)
    A = _A(A_np, torch.float64)
    R = dsk().Restriction.di_grid(64, 64, 4, 4)
    U, S, V, info = dsk().sketch_svd(A, 20, R, q=q, want_info=True)
    Uo, So, Vo, sig = _tpc(A_np, 20, {"kind": "index", "index": ores.di_index_2d(64, 64, 4, 4)}, q=q)
    _compare_svd(A_np, U, S, V, Uo, So, Vo, TOL[torch.float64], sig_all=sig)
    assert abs(info["normA_fro2"] - omet.fro2(A_np)) <= 1e-12 * omet.fro2(A_np)


@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("mode", ["split6", "split3", "f32"])
def test_sketch_svd_advdiff_fp32(q, mode):
    say("svd fp32 advdiff q", q, mode)
    A32 = _A(synth.advdiff_exact(300, 32, seed=1, r=300), torch.float32)
    A_np = _up(A32)
    R = dsk().Restriction.di_grid(32, 32, 4, 4)
    U, S, V = dsk().sketch_svd(A32, 20, R, q=q, mode=mode)
    Uo, So, Vo, sig = _tpc(A_np, 20, {"kind": "index", "index": ores.di_index_2d(32, 32, 4, 4)}, q=q)
    _compare_svd(A_np, U, S, V, Uo, So, Vo, TOL[torch.float32], sig_all=sig)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,ny,nx,sy,sx,k,q", [(77, 30, 22, 3, 2, 7, 1), (129, 17, 33, 2, 4, 9, 2),
                                               (65, 16, 16, 1, 1, 5, 0)])
def test_sketch_svd_ragged_shapes(dtype, m, ny, nx, sy, sx, k, q):
    say("svd ragged", dtype, m, ny, nx, sy, sx, k, q)
    A_np0 = synth.heat_modes(m, max(ny, nx), seed=3, nu=0.002)[:, : ny * nx]
    A_np0 = A_np0 + 1e-3 * np.random.default_rng(4).standard_normal(A_np0.shape)
    A = _A(A_np0, dtype)
    A_np = _up(A)
    R = dsk().Restriction.di_grid(ny, nx, sy, sx)
    U, S, V = dsk().sketch_svd(A, k, R, q=q)
    Uo, So, Vo, sig = _tpc(A_np, k, {"kind": "index", "index": ores.di_index_2d(ny, nx, sy, sx)}, q=q)
    _compare_svd(A_np, U, S, V, Uo, So, Vo, TOL[dtype], sig_all=sig)


@pytest.mark.parametrize("kind", ["nn", "global"])
def test_sketch_svd_stencil_restrictions(kind):
    say("svd stencil", kind)
    A_np = synth.heat_modes(120, 32, seed=5, nu=0.003) + 1e-3 * np.random.default_rng(6).standard_normal((120, 1024))
    A = _A(A_np, torch.float64)
    R = dsk().Restriction.nn(32, 32, 4, 4) if kind == "nn" else dsk().Restriction.global_(32, 32, 4, 4)
    U, S, V = dsk().sketch_svd(A, 10, R, q=1)
    Uo, So, Vo, sig = _tpc(A_np, 10, {"kind": kind, "ny": 32, "nx": 32, "sy": 4, "sx": 4}, q=1)
    _compare_svd(A_np, U, S, V, Uo, So, Vo, TOL[torch.float64], sig_all=sig)


def test_sketch_svd_exact_low_rank_recovery():
    say("svd low rank")
    A_np = synth.lowrank(90, 24 * 24, 6, seed=8)
    A = _A(A_np, torch.float64)
    U, S, V = dsk().sketch_svd(A, 6, dsk().Restriction.di_grid(24, 24, 2, 2), q=0)
    assert omet.svd_error(A_np, _up(U), S.cpu().numpy(), _up(V)) < 1e-12
    assert np.abs(_up(U).T @ _up(U) - np.eye(6)).max() < 1e-12
    assert np.abs(_up(V).T @ _up(V) - np.eye(6)).max() < 1e-12


def test_sketch_svd_exactly_repeated_singular_values():
    # a scaled partial permutation: sigma = 4, 4, 4, 2, 2, 2, 1, 1, 0.5, 0.5 exactly, the
    # nonzeros on columns the start block samples; rank 10 < ell = 16, so the core Gram
    # has exactly repeated eigenvalues and a cluster at zero (the eigensolver's cluster path)
    say("svd repeated singular values")
    m, ny, nx = 120, 24, 24
    di = ores.di_index_2d(ny, nx, 2, 2)
    cols = osk.nested_di_columns(len(di), 16)
    sig = [4.0, 4.0, 4.0, 2.0, 2.0, 2.0, 1.0, 1.0, 0.5, 0.5]
    A_np = np.zeros((m, ny * nx))
    for i, sv in enumerate(sig):
        A_np[3 * i + 1, di[cols[(3 * i) % 16]]] = sv
    A = _A(A_np, torch.float32)
    R = dsk().Restriction.di_grid(ny, nx, 2, 2)
    U, S, V = dsk().sketch_svd(A, 6, R, q=0)
    Uo, So, Vo, sig_all = _tpc(A_np, 6, {"kind": "index", "index": di})
    _compare_svd(A_np, U, S, V, Uo, So, Vo, TOL[torch.float32])
    Ug, Vg = _up(U), _up(V)
    # every pair sits in a cluster (4, 4, 4 and 2, 2, 2): projectors only
    assert svdcheck.compare_vectors(Ug, Uo, Vg, Vo, sig_all, 6, TOL[torch.float32], min_checked=0) == 0
    assert np.abs(Ug.T @ Ug - np.eye(6)).max() < 1e-6
    assert np.abs(Vg.T @ Vg - np.eye(6)).max() < 1e-6


def test_sketch_svd_fp64_range_finder_capped_at_100():
    # FP64 input with k + p above 100: the range finder is 100 wide (the FP64 core
    # SVD holds two ell x ell blocks in LDS), the oracle run at the same width
    say("svd fp64 ell cap")
    m, N, f, k = 260, 32, 1, 95
    A_np = synth.heat_exact(m, N, N, seed=12, rate=0.03)
    A = _A(A_np, torch.float64)
    R = dsk().Restriction.di_grid(N, N, 2, f + 1)
    idx = ores.di_index_2d(N, N, 2, f + 1)
    U, S, V, info = dsk().sketch_svd(A, k, R, q=0, want_info=True)
    assert info["ell"] == 100, info
    Uo, So, Vo, sig = _tpc(A_np, k, {"kind": "index", "index": idx}, p=5)
    _compare_svd(A_np, U, S, V, Uo, So, Vo, TOL[torch.float64], sig_all=sig)


def test_sketch_svd_is_deterministic():
    say("svd determinism")
    A = _A(synth.advdiff_exact(256, 32, seed=9, r=256), torch.float32)
    R = dsk().Restriction.di_grid(32, 32, 4, 4)
    out1 = dsk().sketch_svd(A, 16, R, q=1)
    out2 = dsk().sketch_svd(A, 16, R, q=1)
    for a, b in zip(out1, out2):
        assert torch.equal(a, b)


# ------------------------------------------------------------------ row ID

def _prefix(gaps, u=1.1e-16):
    """Number of leading pivot steps whose decision is separated."""
    r0 = gaps[0, 0]
    for j, (r1, r2) in enumerate(gaps):
        if r1 <= 0:
            return j
        sep = (r1 - r2) / r1
        if not (sep > max(1e-8, 1e3 * u * r0 / r1)):
            return j
    return len(gaps)


def _compare_id(A_np, I, P, Io, Po, info_o, k):
    I = I.cpu().numpy()
    P = P.cpu().numpy()
    np.testing.assert_array_equal(P[I], np.eye(k))
    npre = _prefix(info_o["gaps"])
    assert list(I[:npre]) == list(Io[:npre]), (npre, I, Io)
    e_gpu = omet.id_error(A_np, I, P)
    e_or = omet.id_error(A_np, Io, Po)
    if npre == k:
        # C = R_1^{-1} R_2 moves by about u kappa(R_1) under FP64 rounding of W (the
        # power block is evaluated in another order on the GPU): tolerance 10 u kappa, at least 1e-7
        kap = np.linalg.cond(info_o["R"][:, :k])
        ptol = max(1e-7, 10 * 2.0 ** -53 * kap)
        assert np.abs(P - Po).max() <= ptol * max(1.0, np.abs(Po).max()), (np.abs(P - Po).max(), ptol)
        # |e_gpu - e_or| <= ||dP A(I,:)||_F / ||A||_F <= max|dP| sqrt(m k) ||A(I,:)||_F / ||A||_F
        m = A_np.shape[0]
        etol = ptol * max(1.0, np.abs(Po).max()) * math.sqrt(m * k) * np.linalg.norm(A_np[Io]) / np.linalg.norm(A_np)
        assert abs(e_gpu - e_or) <= max(1e-8 * max(e_or, 1e-12), etol), (e_gpu, e_or, etol)
    else:
        assert e_gpu <= 1.5 * e_or + 1e-12
    return npre


@pytest.mark.parametrize("q", [0, 1])
def test_sketch_id_heat_fp64_small_config(q):
    say("id fp64 heat q", q)
    A_np = synth.heat_modes(200, 64, seed=0)
    A = _A(A_np, torch.float64)
    R = dsk().Restriction.di_grid(64, 64, 4, 4)
    I, P, rows = dsk().sketch_id(A, 20, R, q=q, skeleton_rows=True)
    Io, Po, info_o = orid.tpc_id(A_np, 20, {"kind": "index", "index": ores.di_index_2d(64, 64, 4, 4)}, q=q,
                                 return_all=True)
    npre = _compare_id(A_np, I, P, Io, Po, info_o, 20)
    say("  separated prefix", npre)
    np.testing.assert_array_equal(rows.cpu().numpy(), A_np[I.cpu().numpy()])


@pytest.mark.parametrize("q,projected", [(0, False), (1, False), (1, True), (2, True)])
def test_sketch_id_advdiff_fp32(q, projected):
    say("id fp32 q", q, projected)
    A32 = _A(synth.advdiff_exact(240, 32, seed=2, r=240), torch.float32)
    A_np = _up(A32)
    R = dsk().Restriction.di_grid(32, 32, 2, 2)
    I, P = dsk().sketch_id(A32, 15, R, q=q, projected=projected)
    Io, Po, info_o = orid.tpc_id(A_np, 15, {"kind": "index", "index": ores.di_index_2d(32, 32, 2, 2)}, q=q,
                                 projected=projected, return_all=True)
    npre = _compare_id(A_np, I, P, Io, Po, info_o, 15)
    say("  separated prefix", npre)
    assert npre >= 10


@pytest.mark.parametrize("m", [1024, 1300, 2100])
def test_sketch_id_row_counts_around_one_launch_limit(m):
    """Up to one workgroup of 4 candidates per compute unit (m <= 1024 on 256
    CUs; 8 candidates up to 2048 when the rows fit the registers) the
    factorization runs as one launch; otherwise one launch per step.  Both
    follow the oracle's pivots."""
    say("id rows", m)
    A32 = _A(synth.advdiff_exact(m, 32, seed=5, r=300, noise=1e-3), torch.float32)
    A_np = _up(A32)
    R = dsk().Restriction.di_grid(32, 32, 2, 2)
    I, P = dsk().sketch_id(A32, 30, R, q=0)
    Io, Po, info_o = orid.tpc_id(A_np, 30, {"kind": "index", "index": ores.di_index_2d(32, 32, 2, 2)}, q=0,
                                 return_all=True)
    npre = _compare_id(A_np, I, P, Io, Po, info_o, 30)
    say("  separated prefix", npre)
    assert npre >= 20
    # the one-launch (left-looking) and the per-step (right-looking) factorizations:
    # same pivots, P to rounding
    I1, P1 = dsk().sketch_id(A32, 30, R, q=0, per_step=True)
    assert torch.equal(I, I1)
    kap = np.linalg.cond(info_o["R"][:, :30])
    np.testing.assert_allclose(P1.cpu().numpy(), P.cpu().numpy(), rtol=0, atol=max(1e-9, 10 * 2.0 ** -53 * kap))


@pytest.mark.parametrize("kind", ["nn", "global"])
def test_sketch_id_stencil_restrictions_power_step(kind):
    # W = (tau A_g A_g^T) A D: the stencil sketch in the ID, the direct-injection
    # Gram sub-sample of the same grid in the power step (Alg. 7)
    say("id stencil q1", kind)
    A_np = synth.heat_modes(120, 32, seed=5, nu=0.003) + 1e-3 * np.random.default_rng(6).standard_normal((120, 1024))
    A = _A(A_np, torch.float64)
    R = dsk().Restriction.nn(32, 32, 4, 4) if kind == "nn" else dsk().Restriction.global_(32, 32, 4, 4)
    I, P = dsk().sketch_id(A, 10, R, q=1)
    Io, Po, info_o = orid.tpc_id(A_np, 10, {"kind": kind, "ny": 32, "nx": 32, "sy": 4, "sx": 4}, q=1,
                                 return_all=True)
    npre = _compare_id(A_np, I, P, Io, Po, info_o, 10)
    say("  separated prefix", npre)
    assert npre >= 6


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sketch_id_rank_deficient_is_flagged_and_basic(dtype):
    # rank 4 < k = 7: the pivoted factor's last diagonal entries are negligible;
    # the ID raises the flag, keeps P(I,:) = I_k, gives zero coefficients to the
    # negligible pivots and still reconstructs A
    say("id rank deficient", dtype)
    # small-integer factors: every entry and every dependency is exact in FP32 and FP64
    rng = np.random.default_rng(17)
    A_np0 = (rng.integers(-3, 4, size=(50, 4)) @ rng.integers(-8, 9, size=(4, 16 * 16))).astype(np.float64)
    A = _A(A_np0, dtype)
    A_np = _up(A)
    Rd = {"kind": "index", "index": ores.di_index_2d(16, 16, 2, 2)}
    I, P, info = dsk().sketch_id(A, 7, dsk().Restriction.di_grid(16, 16, 2, 2), q=0, want_info=True)
    Io, Po, info_o = orid.tpc_id(A_np, 7, Rd, q=0, return_all=True)
    assert info_o["rank_deficient"] and info_o["rank"] == 4
    assert "rank_deficient" in info["flag_names"]
    I = I.cpu().numpy()
    P = P.cpu().numpy()
    np.testing.assert_array_equal(P[I], np.eye(7))
    assert list(I[:4]) == list(Io[:4])
    rest = np.setdiff1d(np.arange(50), I)
    assert np.all(P[rest][:, 4:] == 0.0)
    # pivots after the rank are rounding noise and may differ; rows outside both
    # skeletons carry the unique coefficients on the 4 independent skeleton rows
    both = np.setdiff1d(rest, Io)
    np.testing.assert_allclose(P[both][:, :4], Po[both][:, :4], atol=1e-8 * max(1.0, np.abs(Po).max()))
    assert omet.id_error(A_np, I, P) < 1e-11


def test_sketch_id_exact_rank_k():
    say("id rank k")
    A_np = synth.lowrank(60, 16 * 16, 5, seed=3)
    A = _A(A_np, torch.float64)
    I, P = dsk().sketch_id(A, 5, dsk().Restriction.di_grid(16, 16, 2, 2), q=0)
    assert omet.id_error(A_np, I.cpu().numpy(), P.cpu().numpy()) < 1e-11


# ------------------------------------------------------------------ argument checks through the ABI

def test_invalid_arguments_return_documented_codes():
    say("invalid args")
    from paper_2105_01271_amd import _lib
    A = torch.zeros((10, 64), dtype=torch.float32, device="cuda")
    R = dsk().Restriction.di_grid(8, 8, 2, 2)
    for kw, code in [({"k": 0}, -7), ({"k": 200}, -7), ({"q": -1}, -9)]:
        args = {"k": 4, "q": 0}
        args.update(kw)
        with pytest.raises(_lib.DskError) as e:
            dsk().sketch_svd(A, args["k"], R, q=args["q"])
        assert e.value.status == code
    bad = dsk().Restriction("index", torch.tensor([0, 5, 64], dtype=torch.int64, device="cuda"))
    _, _, _, info = dsk().sketch_svd(torch.randn(10, 64, device="cuda"), 2, bad, want_info=True)
    assert "bad_index" in info["flag_names"]

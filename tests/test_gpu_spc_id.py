"""SPC-ID (Alg. 5) through the C ABI against the FP64 oracle (oracle.rowid.spc_id).

Checked on the device's outputs: the skeleton I and the coefficients P of the
coarse row ID (its separated prefix, as for TPC-ID), the lifted skeleton rows
X = A_c(I, :) T_r, the factors T_r = V_r W_r, and the error bound of Thm 4.1.

Tolerances.  The device takes the leading r singular triplets of A_c by
subspace iteration (width ell = min(m, s, 112), qc steps); on inputs with
sigma_{c,ell+1} / sigma_{c,r} <= 0.7 and qc = 24 that leaves < 1e-7 of
subspace error, below every tolerance here.  The lifted rows carry the
rounding of H = A^T A_c amplified by kappa_r = sigma_{c,1} / sigma_{c,r}:
|dX| <= c_w u_w kappa_r max|X| with u_w the work precision (2^-53 FP64,
2^-24 FP32 and 16-bit storage; the products of 16-bit values are exact) and
c_w = 8.  The oracle evaluates T_r in the literal form of Alg. 5, whose
U_c^T U_r U_r^T U_c pseudo-inverts every nonzero singular value of A_c, so its
own rounding is about 2^-53 sigma_{c,1} / sigma_{c,min+}; that term (times 16)
is added where T_r itself is compared, whose own bound is 32 u_w kappa_r (the
rounding of sigma_r and v_r enters T_r = V_r W_r directly; X = A_c(I,:) T_r
projects most of it out).
"""
import math

import numpy as np
import pytest
import torch

from oracle import restrict as ores
from oracle import rowid as orid
from paper_2105_01271_amd import synth

pytestmark = pytest.mark.gpu

U53, U24 = 2.0 ** -53, 2.0 ** -24


def dsk():
    from paper_2105_01271_amd import dsketch
    return dsketch


def say(*a):
    print(*a, flush=True)


def _A(A_np, dtype):
    return torch.from_numpy(np.ascontiguousarray(A_np)).to(dtype).cuda()


def _npre(gaps, k):
    """Pivots of the separated prefix (reading of the pivoting rule: relative gap
    above max(1e-8, the FP64 rounding floor of the residuals))."""
    npre = 0
    for r1, r2 in gaps:
        if r1 <= 0 or not ((r1 - r2) / r1 > max(1e-8, 1e3 * 1.1e-16 * gaps[0, 0] / r1)):
            break
        npre += 1
    return min(npre, k)


def _input(m, ny, nx, rank, seed, noise=1e-7):
    """Heat-mode snapshots of exact rank `rank` (sigma_j = exp(-0.25 j)) plus a
    relative Gaussian floor: a clear singular-value drop of A_c at `rank`."""
    A = synth.heat_exact(m, ny, nx, seed=seed, rate=0.25, r=rank)
    rng = np.random.default_rng(seed + 1)
    return A + noise * np.sqrt((A ** 2).mean()) * rng.standard_normal(A.shape)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("m,ny,nx,sy,sx,k,r", [(150, 24, 24, 2, 2, 8, 14), (301, 32, 16, 4, 2, 12, 20),
                                               (97, 16, 16, 2, 2, 5, 5)])
def test_spc_id_matches_oracle(dtype, m, ny, nx, sy, sx, k, r):
    say("spc-id", dtype, m, ny, nx, sy, sx, k, r)
    A = _A(_input(m, ny, nx, r, seed=70 + m), dtype)
    A_np = A.double().cpu().numpy()            # the stored values, upcast exactly
    n = ny * nx
    idx = ores.di_index_2d(ny, nx, sy, sx)
    Rd = {"kind": "index", "index": idx}
    R = dsk().Restriction.di_grid(ny, nx, sy, sx)
    I, P, X, Vr, Wr, info = dsk().spc_id(A, k, r, R, qc=24, factors=True, want_info=True)
    I, P, X, Vr, Wr = (t.cpu().numpy().astype(np.float64) if t.dtype != torch.int64 else t.cpu().numpy()
                       for t in (I, P, X, Vr, Wr))
    # the range finder of the SVD of A_c (ell = min(m, s, 112)) is wider than A_c's
    # numerical rank here: in FP32 its CholeskyQR may take the shifted fallback
    assert info["flags"] & ~1 == 0, info
    Io, Po, AcIo, Tro = orid.spc_id(A_np, k, Rd, r)
    _, _, inf_id = orid.tpc_id(A_np, k, Rd, q=0, return_all=True)
    npre = _npre(inf_id["gaps"], k)
    say("  separated prefix", npre, "of", k)
    assert npre >= min(k, 4)
    assert list(I[:npre]) == list(Io[:npre])
    np.testing.assert_array_equal(P[I], np.eye(k))
    Ac = A_np[:, idx]
    sc = np.linalg.svd(Ac, compute_uv=False)
    kap = sc[0] / sc[r - 1]
    uw = U53 if dtype == torch.float64 else U24
    if npre == k:
        kr = np.linalg.cond(inf_id["R"][:, :k])
        assert np.abs(P - Po).max() <= max(1e-7, 10 * U53 * kr) * max(1.0, np.abs(Po).max())
        Xo = AcIo @ Tro
        tolX = 8 * uw * kap + 16 * U53 * sc[0] / sc[sc > sc[0] * max(Ac.shape) * np.finfo(float).eps].min()
        dx = np.abs(X - Xo).max() / np.abs(Xo).max()
        say(f"  X rel err {dx:.3e} tol {tolX:.3e} (kappa_r {kap:.1f})")
        assert dx <= tolX
        smin = sc[sc > sc[0] * max(Ac.shape) * np.finfo(float).eps].min()
        dT = np.abs(Vr @ Wr - Tro).max() / np.abs(Tro).max()
        # T_r = V_r W_r itself: the rounding of sigma_r and v_r enters as well (observed
        # up to 8 u kappa_r in FP32 at kappa_r = 116), so 32 u kappa_r
        assert dT <= 32 * uw * kap + 16 * U53 * sc[0] / smin, dT
    # V_r orthonormal, W_r = S_r^-2 V_r^T A_c^T A with the device's V_r
    assert np.abs(Vr.T @ Vr - np.eye(r)).max() <= (1e-12 if dtype == torch.float64 else 1e-5)
    Wdef = (1.0 / sc[:r] ** 2)[:, None] * (Vr.T @ (Ac.T @ A_np))
    # (the device's sigma_r and v_r against the exact sigma_r: up to about 33 u_w kappa_r
    # in FP32 at kappa_r = 116, so 64 u_w kappa_r, plus the FP64 rounding of the test's
    # own products, O(m u kappa_r))
    assert np.abs(Wr - Wdef).max() <= (64 * uw + 4 * m * U53) * kap * np.abs(Wdef).max()
    # the approximation A ~ P X against the oracle's, in the 2-norm
    e_gpu = np.linalg.norm(A_np - P @ X, 2)
    e_or = np.linalg.norm(A_np - Po @ AcIo @ Tro, 2)
    say(f"  ||A - P X||_2 / ||A||_2: gpu {e_gpu / sc[0]:.3e} oracle {e_or / sc[0]:.3e}")
    assert e_gpu <= e_or + 8 * uw * kap * np.linalg.norm(A_np, 2) * math.sqrt(k)


def test_spc_id_error_within_theorem_bound():
    # Thm 4.1 on the device's approximation: for every tau > 0 with both radicands
    # non-negative, ||A - P X||_2 <= (eps(tau) + tau sigma_{c,r+1}^2)^(1/2)
    #   + ||A_c - P A_c(I, :)||_2 (tau + eps(tau) sigma_{c,r}^-2)^(1/2)
    say("spc-id theorem bound")
    m, N, f, k, r = 120, 16, 2, 6, 10
    A_np = synth.heat_modes(m, N, seed=81, nu=0.002) + 1e-3 * np.random.default_rng(82).standard_normal((m, N * N))
    A = _A(A_np, torch.float64)
    idx = ores.di_index_2d(N, N, f, f)
    I, P, X = (t.cpu().numpy() for t in dsk().spc_id(A, k, r, dsk().Restriction.di_grid(N, N, f, f), qc=48))
    Ac = A_np[:, idx]
    lhs = np.linalg.norm(A_np - P @ X, 2)
    sc = np.linalg.svd(Ac, compute_uv=False)
    id_err = np.linalg.norm(Ac - P @ Ac[I], 2)
    checked = 0
    for tau in np.logspace(-2, 3, 26) * (N * N / idx.size):
        e = orid.eps_tau(A_np, Ac, tau)
        a, b = e + tau * sc[r] ** 2, tau + e / sc[r - 1] ** 2
        if a < 0 or b < 0:
            continue
        checked += 1
        assert lhs <= (math.sqrt(a) + id_err * math.sqrt(b)) * (1 + 1e-9), (tau, lhs)
    assert checked >= 10


def test_spc_id_rank_deficient_coarse_block_is_flagged():
    # r above the rank (4) of A_c: the dropped singular values leave S_r^-2 finite and
    # raise DSK_FLAG_RANK_DEFICIENT; with k = 4 the ID of A_c and the lift are exact
    say("spc-id rank deficient")
    m, N, f = 60, 16, 2
    A_np = synth.lowrank(m, N * N, 4, seed=83)
    A = _A(A_np, torch.float64)
    I, P, X, info = dsk().spc_id(A, 4, 8, dsk().Restriction.di_grid(N, N, f, f), qc=8, want_info=True)
    assert "rank_deficient" in info["flag_names"], info
    Xn = X.cpu().numpy()
    assert np.all(np.isfinite(Xn))
    Pn = P.cpu().numpy()
    assert np.linalg.norm(A_np - Pn @ Xn) <= 1e-8 * np.linalg.norm(A_np)


def test_spc_id_argument_errors():
    A = torch.zeros((40, 64), dtype=torch.float32, device="cuda")
    R = dsk().Restriction.di_grid(8, 8, 2, 2)
    for k, r, qc, code in ((5, 4, 8, -8), (5, 17, 8, -8), (5, 8, 65, -10)):   # r < k; r > s = 16; qc
        with pytest.raises(dsk()._lib.DskError) as e:
            dsk().spc_id(A, k, r, R, qc=qc)
        assert e.value.status == code


def test_spc_id_full_size_sampled_columns():
    # the advection-diffusion snapshots 1000 x 256^2 (FP32, DI 4 x 4, s = 4096),
    # k = r = 50: the skeleton and P equal the row ID's (the same factorization of
    # A_c), and sampled columns of X against the oracle run on A's coarse columns
    # plus the sampled ones (T_r's column j depends on A(:, j) alone, and A_c is
    # unchanged)
    say("spc-id full size")
    m, N, f, k, r = 1000, 256, 4, 50, 50
    A_np = synth.advdiff_exact(m, N, seed=0, r=m).astype(np.float32)
    A = torch.from_numpy(A_np).cuda()
    R = dsk().Restriction.di_grid(N, N, f, f)
    idx = ores.di_index_2d(N, N, f, f)
    I, P, X, info = dsk().spc_id(A, k, r, R, qc=24, want_info=True)
    assert info["flags"] == 0, info
    I1, P1 = dsk().sketch_id(A, k, R, q=0)
    assert torch.equal(I, I1) and torch.equal(P, P1)
    rng = np.random.default_rng(84)
    J = np.sort(rng.choice(N * N, 64, replace=False))
    A64 = A_np.astype(np.float64)
    sub = np.concatenate([A64[:, idx], A64[:, J]], axis=1)
    s = idx.size
    Rs = {"kind": "index", "index": np.arange(s)}
    Io, Po, AcIo, Tro = orid.spc_id(sub, k, Rs, r)
    _, _, inf_id = orid.tpc_id(sub, k, Rs, q=0, return_all=True)
    npre = _npre(inf_id["gaps"], k)
    say("  separated prefix", npre, "of", k)
    Xo = AcIo @ Tro[:, s:]
    Xg = X.cpu().numpy().astype(np.float64)[:, J]
    sc = np.linalg.svd(A64[:, idx], compute_uv=False)
    tol = 8 * U24 * sc[0] / sc[r - 1] + 16 * U53 * sc[0] / sc[-1]
    dx = np.abs(Xg - Xo).max() / np.abs(Xo).max()
    say(f"  sampled X rel err {dx:.3e} tol {tol:.3e}")
    assert npre >= 10 and list(I.cpu().numpy()[:npre]) == list(Io[:npre])
    if npre == k:
        assert dx <= tol

"""Mixed-precision path: A stored in BF16 or FP16, MFMA products with FP32
accumulation, Q split into two 16-bit pieces (hi + lo) so that B = Q^T A
comes from one read of A, FP64 Gram / Cholesky / core SVD / ID, optional
refinement sweep.

Tolerance (singular values relative to sigma_1), derived from the arithmetic:
the two-piece split leaves |Q - Q_hi - Q_lo| <= 2^-18 |Q| elementwise (BF16;
FP16 is tighter), and B = Q^T A accumulates m products in FP32.  With
independent rounding errors sigma_j moves by about 2^-18 sigma_1 (split) plus
sqrt(m) 2^-24 sigma_1 (accumulation): 3.8e-6 + 1.9e-6 for m <= 1000 (the
worst-case bound, 2^-18 sqrt(ell) + m 2^-24, would be 1e-4).  Both are loose:
the errors average out further in the contraction, and the measured errors on
these shapes are 2e-8 (FP16) to 2e-7 (BF16).  TOL_MIXED = 2e-6 is therefore
set at about ten times the largest measured error rather than at either bound.

Two errors are checked:
  * algorithmic: against the FP64 oracle run on the exactly upcast stored A;
  * total: against the oracle on the original FP64 A, allowing the storage
    perturbation ||A_q - A||_F on top.
"""
import math

import numpy as np
import pytest
import torch

from oracle import metrics as omet
from oracle import restrict as ores
from oracle import sketch as osk
from oracle import rowid as orid
from paper_2105_01271_amd import synth

import svdcheck   # tests/svdcheck.py

pytestmark = pytest.mark.gpu

TOL_MIXED = 2e-6


def dsk():
    from paper_2105_01271_amd import dsketch
    return dsketch


def say(*a):
    print(*a, flush=True)


def _up(t):
    return t.double().cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("q,refine", [(0, False), (1, False), (1, True)])
def test_mixed_sketch_svd_against_oracle(dtype, q, refine):
    # heat-type exact construction (sigma_j = exp(-0.05 j)), 400 x 64x128 grid,
    # DI (8, 4): s = 8 * 32 = 256, k = 40, ell = 50
    say("mixed svd", dtype, q, refine)
    m, ny, nx, sy, sx, k = 400, 64, 128, 8, 4, 40
    A64, sig = synth.heat_exact(m, ny, nx, seed=7, return_parts=True)
    Aq = torch.from_numpy(A64).to(dtype).cuda()
    Aup = _up(Aq)
    R = dsk().Restriction.di_grid(ny, nx, sy, sx)
    U, S, V = dsk().sketch_svd(Aq, k, R, q=q, refine=refine)
    Rd = {"kind": "index", "index": ores.di_index_2d(ny, nx, sy, sx)}
    Uo, So, Vo, oi = osk.tpc_svd(Aup, k, Rd, q=q, return_all=True)
    S = S.cpu().numpy()
    alg = np.abs(S - So).max() / So[0]
    say("  algorithmic sigma error / sigma_1", alg)
    assert alg <= TOL_MIXED
    svdcheck.compare_vectors(_up(U), Uo, _up(V), Vo, oi["sigma_B"], k, TOL_MIXED)
    e_gpu = omet.svd_error(Aup, _up(U), S, _up(V))
    e_or = omet.svd_error(Aup, Uo, So, Vo)
    say("  rank-k error gpu / oracle (stored A)", e_gpu, e_or)
    assert abs(e_gpu - e_or) <= TOL_MIXED * max(e_or, 1e-12) + TOL_MIXED * So[0] * 1e-2
    # total error against the original FP64 matrix
    dA = np.linalg.norm(Aup - A64)
    U64, S64, V64 = osk.tpc_svd(A64, k, Rd, q=q)
    e_tot = omet.svd_error(A64, _up(U), S, _up(V))
    e_or64 = omet.svd_error(A64, U64, S64, V64)
    say("  total error gpu / oracle(FP64 A) / ||A_q - A||_F", e_tot, e_or64, dA)
    assert e_tot <= e_or64 + 2 * dA + TOL_MIXED * e_or64
    assert np.abs(S - S64).max() <= dA + TOL_MIXED * S64[0]


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_mixed_wide_range_finder_ell_110(dtype):
    # the k = 100, ell = 110 shape of the mixed-precision workload on a smaller
    # grid: 1000 x 128x128, DI (8, 4) -> s = 16 * 32 = 512
    say("mixed svd ell=110", dtype)
    m, ny, nx, sy, sx, k = 1000, 128, 128, 8, 4, 100
    A64 = synth.heat_exact(m, ny, nx, seed=11)
    Aq = torch.from_numpy(A64).to(dtype).cuda()
    Aup = _up(Aq)
    R = dsk().Restriction.di_grid(ny, nx, sy, sx)
    U, S, V, info = dsk().sketch_svd(Aq, k, R, q=1, want_info=True)
    assert info["ell"] == 110
    Rd = {"kind": "index", "index": ores.di_index_2d(ny, nx, sy, sx)}
    Uo, So, Vo = osk.tpc_svd(Aup, k, Rd, q=1)
    S = S.cpu().numpy()
    alg = np.abs(S - So).max() / So[0]
    say("  algorithmic sigma error / sigma_1", alg, "core sweeps", info["core_sweeps"])
    assert alg <= TOL_MIXED
    e_gpu = omet.svd_error(Aup, _up(U), S, _up(V))
    e_or = omet.svd_error(Aup, Uo, So, Vo)
    assert abs(e_gpu - e_or) <= TOL_MIXED * max(e_or, 1e-12)
    Un = _up(U)
    assert np.abs(Un.T @ Un - np.eye(k)).max() < 1e-4


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_mixed_sketch_id_matches_oracle_on_stored_values(dtype):
    # the row ID works on A_c in FP64, which is exact for 16-bit storage:
    # pivots must agree with the oracle on the upcast values
    say("mixed id", dtype)
    m, ny, nx, sy, sx, k = 300, 64, 64, 4, 4, 25
    A64 = synth.heat_exact(m, ny, nx, seed=5, rate=0.08)
    Aq = torch.from_numpy(A64).to(dtype).cuda()
    Aup = _up(Aq)
    R = dsk().Restriction.di_grid(ny, nx, sy, sx)
    I, P = dsk().sketch_id(Aq, k, R, q=0)
    Io, Po, info = orid.tpc_id(Aup, k, {"kind": "index", "index": ores.di_index_2d(ny, nx, sy, sx)}, q=0,
                               return_all=True)
    I = I.cpu().numpy()
    gaps = info["gaps"]
    npre = 0
    for r1, r2 in gaps:
        if r1 <= 0 or not ((r1 - r2) / r1 > max(1e-8, 1e3 * 1.1e-16 * gaps[0, 0] / r1)):
            break
        npre += 1
    say("  separated prefix", npre)
    assert list(I[:npre]) == list(Io[:npre])
    assert npre >= 10
    np.testing.assert_array_equal(P.cpu().numpy()[I], np.eye(k))


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_refinement_sweep_restores_orthogonality(dtype):
    # The sweep re-orthonormalises the assembled FP32 factors in FP64 without
    # changing U S V^T: orthogonality of V (which divides by sigma_j) improves,
    # the product and the singular values stay within the tolerance.
    say("refinement sweep", dtype)
    # On this small grid the factors are already orthonormal to a few FP32
    # roundings; the sweep must keep them there and leave U S V^T unchanged (the
    # full-size workload, where V loses 30 times more, is in test_gpu_c3.py).
    m, ny, nx, sy, sx, k = 400, 64, 128, 8, 4, 40
    A64 = synth.heat_exact(m, ny, nx, seed=7, rate=0.15)
    Aq = torch.from_numpy(A64).to(dtype).cuda()
    Aup = _up(Aq)
    R = dsk().Restriction.di_grid(ny, nx, sy, sx)
    U0, S0, V0 = dsk().sketch_svd(Aq, k, R, q=1)
    U1, S1, V1 = dsk().sketch_svd(Aq, k, R, q=1, refine=True)
    u0, v0, u1, v1 = _up(U0), _up(V0), _up(U1), _up(V1)
    s0, s1 = S0.cpu().numpy(), S1.cpu().numpy()
    ou0 = np.abs(u0.T @ u0 - np.eye(k)).max()
    ov0 = np.abs(v0.T @ v0 - np.eye(k)).max()
    ou1 = np.abs(u1.T @ u1 - np.eye(k)).max()
    ov1 = np.abs(v1.T @ v1 - np.eye(k)).max()
    say(f"  orthogonality U {ou0:.2e} -> {ou1:.2e}, V {ov0:.2e} -> {ov1:.2e}")
    assert max(ou1, ov1) < 3e-7                    # a few FP32 roundings
    assert ov1 <= ov0 * 1.2 and ou1 <= ou0 * 1.2
    # same product U S V^T (to FP32 rounding), same singular values
    p0 = (u0 * s0) @ v0.T
    p1 = (u1 * s1) @ v1.T
    assert np.abs(p1 - p0).max() <= 1e-5 * s0[0] * np.abs(u0).max() * np.abs(v0).max() * 10
    assert np.abs(s1 - s0).max() <= TOL_MIXED * s0[0]
    Rd = {"kind": "index", "index": ores.di_index_2d(ny, nx, sy, sx)}
    Uo, So, Vo = osk.tpc_svd(Aup, k, Rd, q=1)
    say(f"  sigma error vs oracle: {np.abs(s0 - So).max() / So[0]:.2e} -> {np.abs(s1 - So).max() / So[0]:.2e}")
    assert np.abs(s1 - So).max() <= TOL_MIXED * So[0]

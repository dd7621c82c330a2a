"""Parity at the full size of the timed workload, in the launch configuration
the benchmark times: advection-diffusion snapshots 1000 x 256x256 FP32
(sigma_j = j^-0.5, 1e-3 noise), direct injection 4x4 (s = 4096), k = 50,
ell = 60; sketch SVD with q = 1 and row ID with q = 0 (skeleton rows gathered).

The FP64 oracle finishes this size in about a second, so every output is
compared (singular values, reconstruction errors, skeleton prefix, the
interpolation matrix, the gathered rows).
"""
import numpy as np
import pytest
import torch

from oracle import metrics as omet
from oracle import restrict as ores
from oracle import rowid as orid
from oracle import sketch as osk
from paper_2105_01271_amd import synth

import svdcheck   # tests/svdcheck.py

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def dsk():
    from paper_2105_01271_amd import dsketch
    return dsketch


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c2():
    A64 = synth.advdiff_exact(1000, 256, seed=0, r=1000)
    A32 = torch.from_numpy(A64).to(torch.float32)
    Aup = A32.double().numpy()
    return A32.cuda(), Aup


def test_fullsize_sketch_svd_q1(c2):
    A, Aup = c2
    say("full-size svd q=1")
    R = dsk().Restriction.di_grid(256, 256, 4, 4)
    U, S, V, info = dsk().sketch_svd(A, 50, R, q=1, want_info=True)
    Rd = {"kind": "index", "index": ores.di_index_2d(256, 256, 4, 4)}
    Uo, So, Vo, oi = osk.tpc_svd(Aup, 50, Rd, q=1, return_all=True)
    S = S.cpu().numpy()
    err = np.abs(S - So).max() / So[0]
    say("  sigma error / sigma_1", err, "sweeps", info["core_sweeps"])
    assert err <= TOL32
    Un, Vn = U.double().cpu().numpy(), V.double().cpu().numpy()
    e_gpu = omet.svd_error(Aup, Un, S, Vn)
    e_or = omet.svd_error(Aup, Uo, So, Vo)
    say("  rank-k error gpu / oracle", e_gpu, e_or)
    assert abs(e_gpu - e_or) <= TOL32 * e_or
    # singular vectors: one by one where the gaps resolve them, cluster projectors elsewhere
    nchk = svdcheck.compare_vectors(Un, Uo, Vn, Vo, oi["sigma_B"], 50, TOL32)
    say("  singular pairs compared one by one:", nchk)
    assert abs(info["normA_fro2"] - omet.fro2(Aup)) <= 1e-6 * omet.fro2(Aup)


def test_fullsize_sketch_id_q0(c2):
    A, Aup = c2
    say("full-size id q=0")
    R = dsk().Restriction.di_grid(256, 256, 4, 4)
    I, P, rows = dsk().sketch_id(A, 50, R, q=0, skeleton_rows=True)
    Io, Po, info = orid.tpc_id(Aup, 50, {"kind": "index", "index": ores.di_index_2d(256, 256, 4, 4)}, q=0,
                               return_all=True)
    I = I.cpu().numpy()
    P = P.cpu().numpy()
    gaps = info["gaps"]
    npre = 0
    for r1, r2 in gaps:
        if r1 <= 0 or not ((r1 - r2) / r1 > max(1e-8, 1e3 * 1.1e-16 * gaps[0, 0] / r1)):
            break
        npre += 1
    say("  separated prefix", npre, "of", len(gaps))
    assert list(I[:npre]) == list(Io[:npre])
    np.testing.assert_array_equal(P[I], np.eye(50))
    if npre == 50:
        kap = np.linalg.cond(info["R"][:, :50])
        ptol = max(1e-7, 10 * 2.0 ** -53 * kap)
        assert np.abs(P - Po).max() <= ptol * max(1.0, np.abs(Po).max())
    e_gpu = omet.id_error(Aup, I, P)
    e_or = omet.id_error(Aup, Io, Po)
    say("  ID error gpu / oracle", e_gpu, e_or)
    assert e_gpu <= e_or * (1 + 1e-6) + 1e-12
    np.testing.assert_array_equal(rows.cpu().numpy(), A.cpu().numpy()[I])
    # the timed launch configuration (one launch, left-looking recurrence) takes the
    # pivots of the per-step factorization and its P to rounding
    I1, P1 = dsk().sketch_id(A, 50, R, q=0, per_step=True)
    np.testing.assert_array_equal(I1.cpu().numpy(), I)
    kap = np.linalg.cond(info["R"][:, :50])
    np.testing.assert_allclose(P1.cpu().numpy(), P, rtol=0, atol=max(1e-9, 10 * 2.0 ** -53 * kap))

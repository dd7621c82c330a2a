"""Parity at the full size of the mixed-precision workload: heat-mode
snapshots 2000 x 512x512 (sigma_j = exp(-0.05 j)) stored in BF16 and in FP16
(1.05 GB), direct injection with strides (8, 4) (s = 8192), k = 100,
ell = 110, q = 0 and 1, with and without the refinement sweep; the row ID at
k = 100 on the same sketch.

Two errors are checked for every SVD result:
  * algorithmic: against the FP64 oracle run on the exactly upcast stored A
    (singular values, rank-k error, singular vectors to the tolerance below);
  * total: against the oracle on the original FP64 A, allowing the storage
    perturbation ||A_q - A||_2 (Weyl) on top.

TOL_MIXED (relative to sigma_1).  The arithmetic of the projection bounds
the error a priori: Q is split into two 16-bit pieces, leaving
|Q - Q_hi - Q_lo| <= 2^-18 |Q| per entry (BF16; FP16 is tighter), and
B = Q^T A accumulates m = 2000 products in FP32, so sigma_j moves by at most
about (2^-18 sqrt(ell) + m 2^-24) sigma_1 = 1.6e-4 in the worst case and by
about (2^-18 + sqrt(m) 2^-24) sigma_1 = 6.5e-6 with independent rounding
errors.  Both are loose: the split and accumulation errors average out
further in the contraction, and the measured errors on this workload are
3e-8 (FP16) to 9e-8 (BF16).  TOL_MIXED = 1e-6 is therefore set at about ten
times the largest measured error rather than at either bound.
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

TOL_MIXED = 1e-6
M, NY, NX, SY, SX, K = 2000, 512, 512, 8, 4, 100
RD = {"kind": "index", "index": ores.di_index_2d(NY, NX, SY, SX)}


def dsk():
    from paper_2105_01271_amd import dsketch
    return dsketch


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c3():
    say("generating the 2000 x 512^2 heat-mode matrix")
    A64 = synth.heat_exact(M, NY, NX, seed=7)
    out = {"A64": A64, "oracle": {}}
    for dt in (torch.bfloat16, torch.float16):
        At = torch.from_numpy(A64).to(dt)
        out[dt] = (At.cuda(), At.double().numpy())
        del At
    return out


def _oracle(c3, key, A_np, q):
    if key not in c3["oracle"]:
        say("  oracle", key)
        c3["oracle"][key] = osk.tpc_svd(A_np, K, RD, q=q, return_all=True)
    return c3["oracle"][key]


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("q,refine", [(0, False), (0, True), (1, False), (1, True)])
def test_c3_sketch_svd(c3, dtype, q, refine):
    say("C3 svd", dtype, "q", q, "refine", refine)
    A, Aup = c3[dtype]
    R = dsk().Restriction.di_grid(NY, NX, SY, SX)
    U, S, V, info = dsk().sketch_svd(A, K, R, q=q, refine=refine, want_info=True)
    assert info["ell"] == 110
    Uo, So, Vo, oi = _oracle(c3, (dtype, q), Aup, q)
    S = S.cpu().numpy()
    Un, Vn = U.double().cpu().numpy(), V.double().cpu().numpy()
    alg = np.abs(S - So).max() / So[0]
    e_gpu = omet.svd_error(Aup, Un, S, Vn)
    e_or = omet.svd_error(Aup, Uo, So, Vo)
    orth_u = np.abs(Un.T @ Un - np.eye(K)).max()
    orth_v = np.abs(Vn.T @ Vn - np.eye(K)).max()
    say(f"  sigma err/sigma_1 {alg:.3e}  rank-k err gpu {e_gpu:.9e} oracle {e_or:.9e}  "
        f"orth U {orth_u:.2e} V {orth_v:.2e}  flags {info['flag_names']}")
    assert alg <= TOL_MIXED
    assert abs(e_gpu - e_or) <= TOL_MIXED * e_or
    nchk = svdcheck.compare_vectors(Un, Uo, Vn, Vo, oi["sigma_B"], K, TOL_MIXED)
    say("  singular pairs compared one by one:", nchk)
    # total error against the FP64 matrix the 16-bit values were rounded from
    A64 = c3["A64"]
    U64, S64, V64, _ = _oracle(c3, ("f64", q), A64, q)
    if "dAF" not in c3:
        c3["dAF"] = {}
    if dtype not in c3["dAF"]:
        c3["dAF"][dtype] = float(np.sqrt(sum(float(((Aup[i:i + 200] - A64[i:i + 200]) ** 2).sum())
                                             for i in range(0, M, 200))))
    dAF = c3["dAF"][dtype]                      # ||A_q - A||_F >= ||A_q - A||_2 (Weyl's perturbation)
    say(f"  total: sigma err vs FP64 oracle {np.abs(S - S64).max() / S64[0]:.3e}  ||A_q - A||_F {dAF / S64[0]:.3e}")
    assert np.abs(S - S64).max() <= 2 * dAF + TOL_MIXED * S64[0]


def test_c3_sketch_id_bf16(c3):
    say("C3 id bf16")
    A, Aup = c3[torch.bfloat16]
    R = dsk().Restriction.di_grid(NY, NX, SY, SX)
    I, P = dsk().sketch_id(A, K, R, q=0)
    Io, Po, info = orid.tpc_id(Aup, K, RD, q=0, return_all=True)
    I = I.cpu().numpy()
    P = P.cpu().numpy()
    gaps = info["gaps"]
    npre = 0
    for r1, r2 in gaps:
        if r1 <= 0 or not ((r1 - r2) / r1 > max(1e-8, 1e3 * 1.1e-16 * gaps[0, 0] / r1)):
            break
        npre += 1
    say("  separated prefix", npre, "of", K)
    assert list(I[:npre]) == list(Io[:npre])
    np.testing.assert_array_equal(P[I], np.eye(K))
    if npre == K:
        kap = np.linalg.cond(info["R"][:, :K])
        ptol = max(1e-7, 10 * 2.0 ** -53 * kap)
        assert np.abs(P - Po).max() <= ptol * max(1.0, np.abs(Po).max())
    Ac = Aup[:, RD["index"]]
    e_gpu = np.linalg.norm(Ac - P @ Ac[I]) / np.linalg.norm(Ac)
    e_or = np.linalg.norm(Ac - Po @ Ac[Io]) / np.linalg.norm(Ac)
    say("  coarse ID error gpu / oracle", e_gpu, e_or)
    assert e_gpu <= e_or * (1 + 1e-6) + 1e-12


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_c3_refinement_sweep(c3, dtype):
    # At full size and q = 0, V = B^T U_B S^-1 loses orthogonality well beyond
    # FP32 rounding (about 1.5e-6); the FP64 sweep restores it without changing
    # U S V^T.
    say("C3 refinement", dtype)
    A, _ = c3[dtype]
    R = dsk().Restriction.di_grid(NY, NX, SY, SX)
    U0, S0, V0 = dsk().sketch_svd(A, K, R, q=0)
    U1, S1, V1 = dsk().sketch_svd(A, K, R, q=0, refine=True)
    u0, v0 = U0.double().cpu().numpy(), V0.double().cpu().numpy()
    u1, v1 = U1.double().cpu().numpy(), V1.double().cpu().numpy()
    ov0 = np.abs(v0.T @ v0 - np.eye(K)).max()
    ov1 = np.abs(v1.T @ v1 - np.eye(K)).max()
    ou1 = np.abs(u1.T @ u1 - np.eye(K)).max()
    say(f"  orthogonality V {ov0:.2e} -> {ov1:.2e}, U after {ou1:.2e}")
    assert ov1 < 0.2 * ov0 and max(ov1, ou1) < 3e-7
    s0, s1 = S0.cpu().numpy(), S1.cpu().numpy()
    assert np.abs(s1 - s0).max() <= TOL_MIXED * s0[0]
    # U S V^T unchanged: compare on a few columns of the product
    cols = np.arange(0, NY * NX, 4099)
    p0 = (u0 * s0) @ v0[cols].T
    p1 = (u1 * s1) @ v1[cols].T
    assert np.abs(p1 - p0).max() <= 1e-5 * np.abs(p0).max()

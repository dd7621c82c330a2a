"""GPU: the shifted CholeskyQR fallback, on both block widths.

A rank-20 matrix with small-integer factors (every entry exact in FP32)
sketched with ell = 50 (the 64-wide CholeskyQR) and ell = 80 (the 65 .. 128-wide
one): the Gram of the start block Y = A_c S has
rank 20, so the unshifted Cholesky meets negligible pivots, the factorization
is redone with the shift and a third pass restores orthonormality (shifted
CholeskyQR3, the QR steps of Alg. 2 and Alg. 7).  The call raises the
fallback flag, and the 20 nonzero singular triplets agree with the FP64
oracle's (which orthonormalises by Householder QR) on the same values at the
FP32 tolerance of the other parity tests (singular values relative to
sigma_1; the rank-20 reconstruction relative to ||A||).
"""
import numpy as np
import pytest
import torch

from oracle import restrict as ores
from oracle import sketch as osk

pytestmark = pytest.mark.gpu


def dsk():
    from paper_2105_01271_amd import dsketch
    return dsketch


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("k", [40, 70])
@pytest.mark.parametrize("q", [0, 1])
def test_cholqr_fallback_on_rank_deficient_input(q, k):
    say("CholeskyQR fallback, q", q, "k", k)
    rng = np.random.default_rng(31)
    m, N, r = 300, 32, 20
    A_np = (rng.integers(-3, 4, size=(m, r)) @ rng.integers(-4, 5, size=(r, N * N))).astype(np.float64)
    A = torch.from_numpy(A_np).to(torch.float32).cuda()
    R = dsk().Restriction.di_grid(N, N, 2, 2)
    U, S, V, info = dsk().sketch_svd(A, k, R, q=q, want_info=True)
    torch.cuda.synchronize()
    say("  ell", info["ell"], "flags", info["flag_names"])
    assert info["ell"] == k + 10
    assert "fallback" in info["flag_names"]
    U = U.double().cpu().numpy()
    S = S.double().cpu().numpy()
    V = V.double().cpu().numpy()
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(S)) and np.all(np.isfinite(V))
    Rd = {"kind": "index", "index": ores.di_index_2d(N, N, 2, 2)}
    Uo, So, Vo = osk.tpc_svd(A_np, k, Rd, q=q)
    s1 = So[0]
    np.testing.assert_allclose(S[:r], So[:r], rtol=0, atol=1e-5 * s1)
    assert np.all(np.abs(S[r:]) <= 1e-5 * s1)
    # the rank-r part: reconstruction, orthonormality, subspaces
    Ar = (U[:, :r] * S[:r]) @ V[:, :r].T
    err = np.linalg.norm(A_np - Ar) / np.linalg.norm(A_np)
    say("  rank-20 reconstruction", err, "sigma_1", s1, "sigma_21", S[r])
    assert err <= 1e-5
    assert np.linalg.norm(U[:, :r].T @ U[:, :r] - np.eye(r)) <= 1e-4
    assert np.linalg.norm(U[:, :r] @ U[:, :r].T - Uo[:, :r] @ Uo[:, :r].T) <= 1e-4

"""SPC-ID-ERR (Alg. 6) at given scales through the C ABI against the FP64 oracle,
with the rho(tau) estimate the same eigenvalues give.

eps_hat(tau) = c lambda_max(B_f B_f^T - tau B_c B_c^T) is evaluated on the
device from FP64 Grams of the stored values and the core eigensolver applied
to the positive semidefinite shift M + ||M||_F I.  That solver's shift and
rounding are O((ell + 1024) u tr) of the matrix it factors, so the tolerance
is 1e-10 c (|tr M| + r ||M||_F), far above the rounding and far below the
spread of eps_hat over tau.
"""
import numpy as np
import pytest
import torch

from oracle import restrict as ores
from oracle import rowid as orid
from paper_2105_01271_amd import synth

pytestmark = pytest.mark.gpu


def dsk():
    from paper_2105_01271_amd import dsketch
    return dsketch


def say(*a):
    print(*a, flush=True)


def _A(A_np, dtype):
    return torch.from_numpy(np.ascontiguousarray(A_np)).to(dtype).cuda()


def _tol(A_np, Ac_np, mc, taus):
    m = A_np.shape[0]
    c = m // mc
    keep = [i for i in range(m) if (i + 1) % c == 0]
    Bf = A_np[keep]
    Bc = Ac_np[keep]
    Gf, Gc = Bf @ Bf.T, Bc @ Bc.T
    out = []
    for t in taus:
        M = Gf - t * Gc
        out.append(1e-10 * c * (abs(np.trace(M)) + len(keep) * np.linalg.norm(M)))
    return np.array(out)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("m,N,f,mc", [(30, 8, 2, 10), (300, 32, 4, 60), (257, 16, 2, 80)])
def test_spc_id_err_matches_oracle(dtype, m, N, f, mc):
    say("spc-id-err", dtype, m, N, f, mc)
    rng = np.random.default_rng(31)
    A0 = synth.heat_modes(m, N, seed=30, nu=0.002) + 1e-2 * rng.standard_normal((m, N * N))
    A = _A(A0, dtype)
    A_np = A.double().cpu().numpy()
    idx = ores.di_index_2d(N, N, f, f)
    R = dsk().Restriction.di_grid(N, N, f, f)
    taus = np.concatenate([[0.0], np.logspace(-1, 2, 7) * (N * N / idx.size)])
    eps, rho = (t.cpu().numpy() for t in dsk().spc_id_err(A, R, mc, taus, with_rho=True))
    Rd = {"kind": "index", "index": idx}
    ref = orid.spc_id_err_curve(A_np, Rd, mc, taus)
    tol = _tol(A_np, A_np[:, idx], mc, taus)
    say("  max |diff| / tol", float(np.max(np.abs(eps - ref) / tol)))
    assert np.all(np.abs(eps - ref) <= tol), (eps, ref, tol)
    assert np.all(np.diff(eps) <= tol[1:])          # non-increasing in tau
    # rho(tau) estimate from the same eigenvalues: c max(lambda_max, -lambda_min)
    ref_rho = orid.spc_rho_curve(A_np, Rd, mc, taus)
    say("  rho max |diff| / tol", float(np.max(np.abs(rho - ref_rho) / tol)))
    assert np.all(np.abs(rho - ref_rho) <= tol), (rho, ref_rho, tol)
    # the rho-less call gives the same eps
    assert np.array_equal(dsk().spc_id_err(A, R, mc, taus).cpu().numpy(), eps)


def test_spc_id_err_full_sampling_is_eps_tau():
    say("spc-id-err full sampling")
    A0 = synth.heat_modes(40, 8, seed=32, nu=0.001) + 1e-3 * np.random.default_rng(33).standard_normal((40, 64))
    A = _A(A0, torch.float64)
    idx = ores.di_index_2d(8, 8, 2, 2)
    R = dsk().Restriction.di_grid(8, 8, 2, 2)
    taus = [0.5, 2.0, 4.0, 8.0]
    eps, rho = (t.cpu().numpy() for t in dsk().spc_id_err(A, R, 40, taus, with_rho=True))
    Ac = A0[:, idx]
    for t, e, r in zip(taus, eps, rho):
        ref = orid.eps_tau(A0, Ac, t)
        M = A0 @ A0.T - t * Ac @ Ac.T
        tol = 1e-10 * (abs(np.trace(M)) + 40 * np.linalg.norm(M))
        assert abs(e - ref) <= tol, (t, e, ref)
        assert abs(r - orid.rho_tau(A0, Ac, t)) <= tol, (t, r)


def test_spc_id_err_stencil_restriction():
    say("spc-id-err nn restriction")
    A0 = synth.heat_modes(64, 16, seed=34, nu=0.002) + 1e-2 * np.random.default_rng(35).standard_normal((64, 256))
    A = _A(A0, torch.float64)
    R = dsk().Restriction.nn(16, 16, 2, 2)
    taus = [0.0, 1.0, 4.0]
    eps = dsk().spc_id_err(A, R, 32, taus).cpu().numpy()
    Rd = {"kind": "nn", "ny": 16, "nx": 16, "sy": 2, "sx": 2}
    ref = orid.spc_id_err_curve(A0, Rd, 32, taus)
    tol = _tol(A0, ores.apply(A0, Rd), 32, taus)
    assert np.all(np.abs(eps - ref) <= tol), (eps, ref, tol)


def test_spc_id_err_argument_errors():
    say("spc-id-err argument errors")
    A = _A(np.ones((500, 64)), torch.float32)
    R = dsk().Restriction.di_grid(8, 8, 2, 2)
    for mc, taus, codes in [(0, [1.0], (-8,)), (400, [1.0], (-8,)), (10, [], (-9, -10))]:
        with pytest.raises(dsk()._lib.DskError) as e:
            dsk().spc_id_err(A, R, mc, taus)
        assert e.value.status in codes, (mc, e.value.status)

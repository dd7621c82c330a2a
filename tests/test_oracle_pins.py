"""Pins of the FP64 CPU oracle against facts that do not come from the oracle
itself: hand-derived sketch matrices, library routines, brute-force SVDs,
closed-form spectra, greedy-projection pivots and finite differences."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.signal

from oracle import restrict, sketch, rowid, metrics, learned
from paper_2105_01271_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_sketch_fixture():
    mats, cur, rows = {}, None, []
    with open(os.path.join(GOLDEN, "sketch_matrices_n7_s3.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("kind"):
                if cur:
                    mats[cur] = np.array(rows)
                cur, rows = line.split()[1], []
            else:
                rows.append([float(x) for x in line.split()])
    mats[cur] = np.array(rows)
    return mats


# ------------------------------------------------------------------ sketches (Sec. 2)

def test_d_matrices_match_hand_derived_fixture():
    fx = _load_sketch_fixture()
    for kind in ("di", "nn", "global"):
        np.testing.assert_allclose(restrict.d_matrix_1d(kind, 7, 3), fx[kind], rtol=0, atol=1e-15)


@pytest.mark.parametrize("ny,nx,sy,sx", [(8, 12, 2, 3), (7, 9, 2, 4), (16, 16, 4, 4), (5, 6, 1, 2)])
def test_matrix_free_sketches_equal_explicit_D(ny, nx, sy, sx):
    rng = np.random.default_rng(0)
    A = rng.standard_normal((5, ny * nx))
    np.testing.assert_allclose(restrict.gather(A, restrict.di_index_2d(ny, nx, sy, sx)),
                               A @ restrict.d_matrix_2d("di", ny, nx, sy, sx), atol=1e-14)
    np.testing.assert_allclose(restrict.nearest_neighbour_2d(A, ny, nx, sy, sx),
                               A @ restrict.d_matrix_2d("nn", ny, nx, sy, sx), atol=1e-14)
    np.testing.assert_allclose(restrict.global_2d(A, ny, nx, sy, sx),
                               A @ restrict.d_matrix_2d("global", ny, nx, sy, sx), atol=1e-14)


def test_conv_layer_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 1, 12, 10))
    w = rng.standard_normal((3, 1, 5, 5))
    y = restrict._conv_fwd(x, w)
    for b in range(2):
        for c in range(3):
            full = scipy.signal.correlate2d(np.pad(x[b, 0], 2), w[c, 0], mode="valid")
            np.testing.assert_allclose(y[b, c], full[::2, ::2], atol=1e-13)


def test_conv_delta_weights_reduce_to_direct_injection():
    ny = nx = 16
    w1 = np.zeros((16, 1, 5, 5))
    w1[0, 0, 2, 2] = 1.0
    w2 = np.zeros((1, 16, 5, 5))
    w2[0, 0, 2, 2] = 1.0
    A = np.random.default_rng(2).standard_normal((4, ny * nx))
    np.testing.assert_allclose(restrict.conv_restrict(A, ny, nx, w1, w2),
                               restrict.gather(A, restrict.di_index_2d(ny, nx, 4, 4)), atol=1e-15)


def test_conv_backward_adjoint_and_finite_difference():
    rng = np.random.default_rng(3)
    ny = nx = 8
    A = rng.standard_normal((3, ny * nx))
    w1 = rng.standard_normal((4, 1, 5, 5)) * 0.2
    w2 = rng.standard_normal((1, 4, 5, 5)) * 0.2
    g = rng.standard_normal((3, 4))
    gw1, gw2 = restrict.conv_restrict_bwd(A, ny, nx, w1, w2, g)
    f = lambda a, b: float(np.sum(g * restrict.conv_restrict(A, ny, nx, a, b)))
    h = 1e-6
    for idx in [(0, 0, 2, 2), (3, 0, 0, 4), (1, 0, 4, 1)]:
        e = np.zeros_like(w1); e[idx] = h
        fd = (f(w1 + e, w2) - f(w1 - e, w2)) / (2 * h)
        assert abs(fd - gw1[idx]) < 1e-7 * max(1, abs(fd))
    for idx in [(0, 0, 2, 2), (0, 3, 1, 0)]:
        e = np.zeros_like(w2); e[idx] = h
        fd = (f(w1, w2 + e) - f(w1, w2 - e)) / (2 * h)
        assert abs(fd - gw2[idx]) < 1e-7 * max(1, abs(fd))
    # the learned conv is linear: A D with D built from unit fields
    D = restrict.conv_as_matrix(ny, nx, w1, w2)
    np.testing.assert_allclose(A @ D, restrict.conv_restrict(A, ny, nx, w1, w2), atol=1e-13)


# ------------------------------------------------------------------ QR / power iteration

def test_orth_is_orthonormal_and_spans_Y():
    Y = np.random.default_rng(4).standard_normal((300, 30))
    Q = sketch.orth(Y)
    assert np.abs(Q.T @ Q - np.eye(30)).max() < 1e-13
    assert np.linalg.norm(Y - Q @ (Q.T @ Y)) < 1e-13 * np.linalg.norm(Y)


@pytest.mark.parametrize("q,tau", [(1, 1.0), (2, 1.0), (1, 3.5), (2, 0.25)])
def test_power_iteration_spectrum_is_sigma_to_2q_plus_1(q, tau):
    # With I = all columns, (tau A A^T)^q A has singular values tau^q sigma^(2q+1)
    # and the same singular vectors (Sec. 5, power iteration spectrum).
    rng = np.random.default_rng(5)
    A = rng.standard_normal((12, 20)) / 3.0
    W = sketch.power_iter(A, A, q, tau, reorth=False)
    U, s, Vt = np.linalg.svd(A)
    Uw, sw, Vwt = np.linalg.svd(W)
    np.testing.assert_allclose(sw, tau ** q * s ** (2 * q + 1), rtol=1e-11)
    np.testing.assert_allclose(np.abs(np.sum(Uw * U, axis=0)), 1.0, atol=1e-9)


def test_large_q_converges_to_top_left_singular_subspace_of_Ac():
    # span(Q) after many re-orthonormalised steps = top-l left singular
    # subspace of A_c (the PROTO-TPC basis, Alg. 1)
    rng = np.random.default_rng(6)
    Ac = rng.standard_normal((60, 40)) @ np.diag(0.8 ** np.arange(40)) @ rng.standard_normal((40, 40))
    Q = sketch.orth(Ac[:, :8])
    Q = sketch.power_iter(Ac, Q, 60, 1.0)
    Uc = np.linalg.svd(Ac)[0][:, :8]
    sv = np.linalg.svd(Uc.T @ Q, compute_uv=False)
    assert sv.min() > 1 - 1e-10


def _proj_dist(X, Y):
    """Largest principal-angle sine between span(X) and span(Y)."""
    Qx = np.linalg.qr(X)[0]
    Qy = np.linalg.qr(Y)[0]
    return float(np.linalg.norm(Qx @ Qx.T - Qy @ Qy.T, 2))


@pytest.mark.parametrize("kind", ["nn", "global"])
def test_cpwr_gram_uses_index_subsample_not_the_stencil(kind):
    # Alg. 7: the start block is the sketch A_f D, the power steps use the
    # index sub-sample A_c = A_f(:, I).  For a stencil sketch the default I is
    # the set of direct-injection points, i.e. the columns where the explicit
    # DI matrix of the same grid has its ones.
    ny = nx = 12
    sy = sx = 3
    Ddi = restrict.d_matrix_2d("di", ny, nx, sy, sx)
    I_expl = np.nonzero(Ddi.sum(axis=1))[0]
    R = {"kind": kind, "ny": ny, "nx": nx, "sy": sy, "sx": sx}
    np.testing.assert_array_equal(restrict.gram_index(R), I_expl)
    rng = np.random.default_rng(21)
    A = synth.heat_modes(40, 12, seed=3, nu=0.002) + 0.1 * rng.standard_normal((40, ny * nx))
    D = restrict.d_matrix_2d(kind, ny, nx, sy, sx)
    Ag = A @ Ddi                                    # A_f(:, I) through the explicit DI matrix
    Y = (A @ D)[:, sketch.nested_di_columns(D.shape[1], 6)]
    for q in (1, 2):
        tau = A.shape[1] / Ag.shape[1]
        raw = Y.copy()
        for _ in range(q):                          # Alg. 7 without its optional QR steps
            raw = Ag @ (tau * (Ag.T @ raw))
        _, _, _, info = sketch.tpc_svd(A, 4, R, q=q, p=2, return_all=True)
        assert info["ell"] == 6
        assert _proj_dist(info["Q"], raw) < 1e-8, q
        # the stencil's own Gram gives a different span: the sub-sample matters
        Ac = A @ D
        wrong = Y.copy()
        for _ in range(q):
            wrong = Ac @ (Ac.T @ wrong)
        assert _proj_dist(info["Q"], wrong) > 1e-3, q
    # the ID's power block: (tau A_g A_g^T)^q (A_f D), its row space in the W the ID factors
    I, P, info = rowid.tpc_id(A, 4, R, q=1, return_all=True)
    tau = A.shape[1] / Ag.shape[1]
    np.testing.assert_allclose(info["W"], tau * Ag @ (Ag.T @ (A @ D)), rtol=1e-11, atol=1e-12 * np.abs(info["W"]).max())


def test_cpwr_index_restriction_is_its_own_gram_subsample():
    R = _di(8, 8, 2, 2)
    A = np.random.default_rng(22).standard_normal((20, 64))
    np.testing.assert_array_equal(restrict.gram_index(R), R["index"])
    _, _, _, info = sketch.tpc_svd(A, 3, R, q=1, return_all=True)
    assert info["Ag"] is info["Ac"]


def test_proto_tpc_basis_is_the_large_q_limit_of_cpwr():
    # PROTO-TPC (Alg. 1) takes U~ = the top-k left singular vectors of A_c; the
    # re-orthonormalised coarse power iteration with all of A_c as its Gram
    # converges to the same span (a different route: products and QR only)
    rng = np.random.default_rng(23)
    A = rng.standard_normal((50, 64)) @ np.diag(0.85 ** np.arange(64)) @ rng.standard_normal((64, 64))
    R = _di(8, 8, 2, 2)
    Ac = restrict.apply(A, R)
    k = 5
    Uk, Sk, Vk = sketch.proto_tpc(A, k, Ac)
    Q = sketch.power_iter(Ac, sketch.orth(Ac[:, :k]), 80, 1.0)
    assert _proj_dist(Uk, Q) < 1e-10
    # S~ are the top singular values of A_c: the norms of A_c^T Q's columns at convergence
    np.testing.assert_allclose(np.sort(np.linalg.svd(Ac.T @ Q, compute_uv=False))[::-1], Sk, rtol=1e-10)
    # U~ S~ V~^T is the projection of A onto span(U~) (pseudo-inverse step of Alg. 1)
    Ahat = (Uk * Sk) @ Vk.T
    np.testing.assert_allclose(Ahat, Q @ (Q.T @ A), atol=1e-9 * np.abs(A).max())


def test_proto_tpc_recovers_rank_k_inputs_exactly():
    # rank-k A whose coarse columns keep the rank: range(A_c) = range(A), so
    # U~ U~^T A = A (Alg. 1 with an exact sketch)
    A = synth.lowrank(30, 64, 4, seed=24)
    Ac = restrict.apply(A, _di(8, 8, 2, 2))
    Uk, Sk, Vk = sketch.proto_tpc(A, 4, Ac)
    assert np.linalg.norm(A - (Uk * Sk) @ Vk.T) < 1e-12 * np.linalg.norm(A)


# ------------------------------------------------------------------ TPC-SVD (Alg. 2 + Alg. 7)

def _di(ny, nx, sy, sx):
    return {"kind": "index", "index": restrict.di_index_2d(ny, nx, sy, sx)}


@pytest.mark.parametrize("q", [0, 1, 2])
def test_tpc_svd_recovers_low_rank_exactly(q):
    A = synth.lowrank(80, 16 * 16, 6, seed=7)
    U, s, V = sketch.tpc_svd(A, 6, _di(16, 16, 2, 2), q=q)
    assert metrics.svd_error(A, U, s, V) < 1e-12
    np.testing.assert_allclose(s, np.linalg.svd(A, compute_uv=False)[:6], rtol=1e-11)
    assert np.abs(U.T @ U - np.eye(6)).max() < 1e-12
    assert np.abs(V.T @ V - np.eye(6)).max() < 1e-12


@pytest.mark.parametrize("q", [0, 1, 2])
def test_tpc_svd_error_between_eckart_young_and_theorem_3_2(q):
    A = synth.heat_modes(60, 16, seed=3, nu=0.002)
    A = A + 1e-3 * np.random.default_rng(9).standard_normal(A.shape)
    k = 6
    U, s, V, aux = sketch.tpc_svd(A, k, _di(16, 16, 4, 4), q=q, return_all=True)
    sig = np.linalg.svd(A, compute_uv=False)
    E = A - (U * s) @ V.T
    # Eckart-Young lower bounds
    assert np.linalg.norm(E) >= metrics.eckart_young_tail(sig, k) * (1 - 1e-12)
    assert metrics.spectral_norm(E) >= sig[k] * (1 - 1e-12)
    # Thm 3.2 (proof): ||A - Ahat||_2 <= sigma_{k+1} + ||(I - Q Q^T) A||_2
    Q = aux["Q"]
    assert metrics.spectral_norm(E) <= sig[k] + metrics.spectral_norm(A - Q @ (Q.T @ A)) + 1e-12
    # interlacing: sigma_j(Q^T A) <= sigma_j(A)
    assert np.all(aux["sigma_B"] <= sig[:len(aux["sigma_B"])] * (1 + 1e-12))


def test_tpc_svd_full_index_set_is_exact_truncated_svd():
    A = synth.lowrank(40, 64, 12, seed=10)
    R = {"kind": "index", "index": np.arange(64)}
    U, s, V = sketch.tpc_svd(A, 5, R, q=0, p=7)   # l = 12 >= rank
    Ub, sb, Vbt = np.linalg.svd(A)
    np.testing.assert_allclose(s, sb[:5], rtol=1e-11)
    np.testing.assert_allclose(np.abs(np.sum(U * Ub[:, :5], axis=0)), 1.0, atol=1e-10)


def test_power_iteration_improves_slow_decay():
    A = synth.advdiff_exact(200, 32, seed=2, r=200, noise=0.0)
    sig = np.linalg.svd(A, compute_uv=False)
    ratios = []
    for q in (0, 1, 2):
        U, s, V = sketch.tpc_svd(A, 10, _di(32, 32, 4, 4), q=q)
        ratios.append(np.linalg.norm(A - (U * s) @ V.T) / metrics.eckart_young_tail(sig, 10))
    assert ratios[2] <= ratios[0] + 1e-12
    assert ratios[1] < ratios[0]


def test_generators_have_their_closed_form_spectra():
    A, sig = synth.heat_exact(120, 16, 12, seed=1, rate=0.05, r=60, return_parts=True)
    np.testing.assert_allclose(np.linalg.svd(A, compute_uv=False)[:60], sig, rtol=1e-12, atol=1e-15)
    A, sig = synth.advdiff_exact(90, 16, seed=2, r=90, noise=0.0, return_parts=True)
    np.testing.assert_allclose(np.linalg.svd(A, compute_uv=False), sig, rtol=1e-12)


def test_spc_svd_equals_tpc_svd_at_q0():
    # H R_c^{-1} = A_f^T Q_c (Sec. 3.1), so one pass gives the two-pass result
    A = synth.heat_modes(50, 16, seed=4, nu=0.003) + 1e-4 * np.random.default_rng(1).standard_normal((50, 256))
    R = _di(16, 16, 2, 2)
    U1, s1, V1 = sketch.tpc_svd(A, 5, R, q=0)
    U2, s2, V2 = sketch.spc_svd(A, 5, R, rows_per_read=7)
    np.testing.assert_allclose(s1, s2, rtol=1e-10)
    np.testing.assert_allclose((U1 * s1) @ V1.T, (U2 * s2) @ V2.T, atol=1e-10 * s1[0])


# ------------------------------------------------------------------ row ID (Sec. 4)

def _greedy_pivots(X, k):
    """Brute force: repeatedly take the column farthest from the span of the
    columns already chosen (explicit least-squares projections)."""
    chosen = []
    for _ in range(k):
        best, bi = -1.0, None
        for i in range(X.shape[1]):
            if i in chosen:
                continue
            if chosen:
                C = X[:, chosen]
                coef = np.linalg.lstsq(C, X[:, i], rcond=None)[0]
                d = np.linalg.norm(X[:, i] - C @ coef)
            else:
                d = np.linalg.norm(X[:, i])
            if d > best:
                best, bi = d, i
        chosen.append(bi)
    return chosen


@pytest.mark.parametrize("seed", range(6))
def test_cpqr_pivots_equal_greedy_projection(seed):
    rng = np.random.default_rng(seed)
    m = 10 + seed % 3
    X = rng.standard_normal((7, m)) * (1.6 ** rng.standard_normal(m))[None, :]
    k = 5
    perm, R, gaps = rowid.cpqr(X, k)
    assert list(perm[:k]) == _greedy_pivots(X, k)
    # |R_jj| is the distance of pivot j to the previous pivots
    for j in range(k):
        C = X[:, perm[:j]]
        d = np.linalg.norm(X[:, perm[j]] - C @ np.linalg.lstsq(C, X[:, perm[j]], rcond=None)[0]) if j else np.linalg.norm(X[:, perm[0]])
        assert abs(abs(R[j, j]) - d) < 1e-12 * max(1, d)


def test_cpqr_pivots_equal_lapack_geqp3_when_separated():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((40, 30)) @ np.diag(0.7 ** np.arange(30)) @ rng.standard_normal((30, 30))
    k = 12
    perm, R, gaps = rowid.cpqr(X, k)
    _, Rl, pl = sla.qr(X, pivoting=True, mode="economic")
    sep = (gaps[:, 0] - gaps[:, 1]) / gaps[:, 0]
    nsep = int(np.argmax(sep < 1e-6)) if np.any(sep < 1e-6) else k
    assert nsep >= 6
    assert list(perm[:nsep]) == list(pl[:nsep])
    np.testing.assert_allclose(np.abs(np.diag(R)[:nsep]), np.abs(np.diag(Rl)[:nsep]), rtol=1e-10)


def test_row_id_interpolates_and_recovers_rank_k():
    A = synth.lowrank(30, 50, 5, seed=12)
    I, P, info = rowid.row_id(A, 5)
    np.testing.assert_array_equal(P[I], np.eye(5))      # P(I,:) = I_k exactly
    assert metrics.id_error(A, I, P) < 1e-12


@pytest.mark.parametrize("r,k", [(3, 6), (1, 4), (5, 8)])
def test_row_id_rank_deficient_basic_solution(r, k):
    # W of rank r < k: the pivoted factor's diagonal collapses after r steps,
    # the ID flags the deficiency and takes the basic least-squares solution
    # (zero coefficients on the negligible pivots).  Facts checked: P(I,:) = I_k,
    # the reconstruction is exact, and it equals the orthogonal projection of
    # every row onto the span of the first r skeleton rows, computed here by a
    # separate least-squares fit on W itself.
    W = synth.lowrank(14, 23, r, seed=30 + r)
    I, P, info = rowid.row_id(W, k)
    assert info["rank_deficient"] and info["rank"] == r
    np.testing.assert_array_equal(P[I], np.eye(k))
    assert np.all(info["C"][r:] == 0.0)
    assert np.linalg.norm(W - P @ W[I]) < 1e-12 * np.linalg.norm(W)
    Bk = W[I[:r]]
    coef = np.linalg.lstsq(Bk.T, W.T, rcond=None)[0]
    rest = np.setdiff1d(np.arange(W.shape[0]), I)     # rows of P that interpolate
    np.testing.assert_allclose(P[rest, :r], coef.T[rest], atol=1e-9)
    assert np.all(P[rest, r:] == 0.0)
    # the first r pivots are the greedy-projection pivots (brute force)
    assert list(I[:r]) == list(_greedy_pivots(W.T, r))


def test_row_id_full_rank_is_not_flagged():
    W = synth.lowrank(14, 23, 8, seed=40)
    I, P, info = rowid.row_id(W, 6)
    assert not info["rank_deficient"] and info["rank"] == 6


def test_row_id_soft_bound():
    A = synth.heat_modes(40, 8, seed=5, nu=0.001)
    sig = np.linalg.svd(A, compute_uv=False)
    for k in (2, 4, 6):
        I, P, _ = rowid.row_id(A, k)
        err = metrics.spectral_norm(A - P @ A[I])
        assert err <= math.sqrt(1 + k * (A.shape[0] - k)) * sig[k] * (1 + 1e-9)


@pytest.mark.parametrize("q,tau", [(1, 1.0), (1, 4.0), (2, 0.5)])
def test_tpc_id_power_block_spectrum(q, tau):
    rng = np.random.default_rng(13)
    A = rng.standard_normal((15, 64)) / 4
    R = _di(8, 8, 2, 2)
    I, P, info = rowid.tpc_id(A, 4, R, q=q, tau=tau, return_all=True)
    Ac = restrict.apply(A, R)
    sc = np.linalg.svd(Ac, compute_uv=False)
    sw = np.linalg.svd(info["W"], compute_uv=False)
    np.testing.assert_allclose(sw, tau ** q * sc ** (2 * q + 1), rtol=1e-10, atol=1e-13 * sw[0])
    np.testing.assert_array_equal(P[I], np.eye(4))


def test_tpc_id_pivots_invariant_to_tau():
    A = synth.heat_modes(30, 8, seed=6, nu=0.001) + 1e-3 * np.random.default_rng(2).standard_normal((30, 64))
    R = _di(8, 8, 2, 2)
    I1, P1 = rowid.tpc_id(A, 5, R, q=1, tau=1.0)
    I2, P2 = rowid.tpc_id(A, 5, R, q=1, tau=37.0)
    assert list(I1) == list(I2)
    np.testing.assert_allclose(P1, P2, atol=1e-6)  # W is cubed: R_1 ill-conditioned


def test_spc_id_lifting_operator_identity():
    # T_r (long form of Alg. 5) = A_c^+ U_r U_r^T A_f (simplified form, Sec. 4)
    A = synth.heat_modes(40, 8, seed=7, nu=0.001) + 1e-3 * np.random.default_rng(3).standard_normal((40, 64))
    R = _di(8, 8, 2, 2)
    I, P, AcI, Tr = rowid.spc_id(A, 4, R, r=8)
    Ac = restrict.apply(A, R)
    T2 = rowid.lifting_operator_simplified(A, Ac, 8)
    np.testing.assert_allclose(Tr, T2, atol=1e-9 * np.abs(T2).max())
    np.testing.assert_array_equal(P[I], np.eye(4))


def test_spc_id_exact_lift_closed_form():
    # A_f = X W with W(:, coarse nodes) = I, so that A_c = A_f D = X (full
    # column rank): with r = s the lifting operator is A_c^+ A_f = W, and with
    # k = s the ID is exact, so P_c A_c(I_c, :) T_r reproduces A_f
    rng = np.random.default_rng(41)
    N, f, m = 8, 2, 30
    idx = restrict.di_index_2d(N, N, f, f)
    s = idx.size
    X = rng.standard_normal((m, s))
    W = rng.standard_normal((s, N * N))
    W[:, idx] = np.eye(s)
    A = X @ W
    R = {"kind": "index", "index": idx}
    I, P, AcI, Tr = rowid.spc_id(A, s, R, r=s)
    np.testing.assert_allclose(Tr, W, atol=1e-10 * np.abs(W).max())
    np.testing.assert_allclose(P @ AcI @ Tr, A, atol=1e-9 * np.abs(A).max())
    # r < s: the operator is X^+ U_r U_r^T X W, whose range misses the trailing
    # left singular directions of X
    r = 5
    I, P, AcI, Tr = rowid.spc_id(A, 4, R, r=r)
    U, sv, Vt = np.linalg.svd(X, full_matrices=False)
    ref = (Vt[:r].T / sv[:r]) @ (U[:, :r].T @ A)
    np.testing.assert_allclose(Tr, ref, atol=1e-10 * np.abs(ref).max())


def test_spc_id_full_sampling_reduces_to_row_id():
    # D = I (every node kept): A_c = A_f, and with r = rank(A_f) the lifting
    # operator is the projector onto the row space, so SPC-ID returns the row
    # ID of A_f itself
    A = synth.lowrank(24, 40, 10, seed=42)
    rank = np.linalg.matrix_rank(A)
    assert rank == 10
    R = {"kind": "index", "index": np.arange(40)}
    I, P, AcI, Tr = rowid.spc_id(A, 6, R, r=rank)
    I0, P0, _ = rowid.row_id(A, 6)
    assert list(I) == list(I0)
    np.testing.assert_allclose(P @ AcI @ Tr, P0 @ A[I0], atol=1e-9 * np.abs(A).max())


def test_spc_id_error_within_theorem_bound():
    # Thm. 4.1: ||A_f - P_c A_c(I_c, :) T_r||_2 is at most
    # (eps(tau) + tau sigma_{c,r+1}^2)^{1/2} + ||A_c - P_c A_c(I_c, :)||_2 (tau + eps(tau) sigma_{c,r}^{-2})^{1/2}
    # for every tau > 0 at which both radicands are non-negative
    rng = np.random.default_rng(43)
    for seed, (m, N, f, k, r) in enumerate([(40, 8, 2, 4, 8), (60, 16, 4, 6, 10), (50, 8, 2, 3, 3)]):
        A = synth.heat_modes(m, N, seed=44 + seed, nu=0.002) + 1e-3 * rng.standard_normal((m, N * N))
        idx = restrict.di_index_2d(N, N, f, f)
        R = {"kind": "index", "index": idx}
        Ac = A[:, idx]
        I, P, AcI, Tr = rowid.spc_id(A, k, R, r=r)
        lhs = np.linalg.norm(A - P @ AcI @ Tr, 2)
        sc = np.linalg.svd(Ac, compute_uv=False)
        id_err = np.linalg.norm(Ac - P @ AcI, 2)
        checked = 0
        for tau in np.logspace(-2, 3, 26) * (N * N / idx.size):
            e = rowid.eps_tau(A, Ac, tau)
            a, b = e + tau * sc[r] ** 2, tau + e / sc[r - 1] ** 2
            if a < 0 or b < 0:
                continue
            checked += 1
            assert lhs <= (math.sqrt(a) + id_err * math.sqrt(b)) * (1 + 1e-9), (seed, tau, lhs)
        assert checked >= 10
        # and the bound is not vacuous: its minimum over tau is within a small factor of the error
        best = min(math.sqrt(max(rowid.eps_tau(A, Ac, t) + t * sc[r] ** 2, 0))
                   + id_err * math.sqrt(max(t + rowid.eps_tau(A, Ac, t) / sc[r - 1] ** 2, 0))
                   for t in np.logspace(-2, 3, 26) * (N * N / idx.size))
        assert best <= 50 * lhs, (seed, best, lhs)


def test_spc_rho_curve_pins():
    A = synth.heat_modes(30, 8, seed=19, nu=0.002) + 1e-2 * np.random.default_rng(20).standard_normal((30, 64))
    R = _di(8, 8, 2, 2)
    Ac = restrict.apply(A, R)
    mc = 10
    c = 30 // mc
    keep = [i for i in range(30) if (i + 1) % c == 0]
    sf = np.linalg.svd(A[keep], compute_uv=False)
    sc = np.linalg.svd(Ac[keep], compute_uv=False)
    # tau = 0: c sigma_max(B_f)^2; large tau: rho / tau -> c sigma_max(B_c)^2
    assert abs(rowid.spc_rho_curve(A, R, mc, [0.0])[0] - c * sf[0] ** 2) <= 1e-12 * c * sf[0] ** 2
    big = 1e8
    assert abs(rowid.spc_rho_curve(A, R, mc, [big])[0] / big - c * sc[0] ** 2) <= 1e-6 * c * sc[0] ** 2
    taus = np.linspace(0.0, 40.0, 81)
    rho = rowid.spc_rho_curve(A, R, mc, taus)
    eps = rowid.spc_id_err_curve(A, R, mc, taus)
    # a norm bounds the largest eigenvalue: rho >= |eps_hat|
    assert np.all(rho >= np.abs(eps) - 1e-10 * rho.max())
    # Lipschitz in tau with constant c ||B_c B_c^T||_2, and convex (the norm of an affine function)
    assert np.all(np.abs(np.diff(rho)) <= (taus[1] - taus[0]) * c * sc[0] ** 2 * (1 + 1e-10))
    assert np.all(rho[:-2] + rho[2:] - 2 * rho[1:-1] >= -1e-9 * rho.max())
    # every row kept: rho(tau) of the C-PWR analysis, through the singular values of the
    # Gram mismatch written out from the two data matrices
    for t in (0.5, 4.0, 16.0):
        full = rowid.spc_rho_curve(A, R, 30, [t])[0]
        M = A @ A.T - t * (Ac @ Ac.T)
        assert abs(full - np.linalg.svd(M, compute_uv=False)[0]) <= 1e-10 * full
        assert abs(full - rowid.rho_tau(A, Ac, t)) <= 1e-10 * full


def test_spc_id_err_full_sampling_equals_eps_tau():
    A = synth.heat_modes(24, 8, seed=8, nu=0.001)
    R = _di(8, 8, 2, 2)
    Ac = restrict.apply(A, R)
    est, tau = rowid.spc_id_err(A, R, mc=24)
    assert abs(est - rowid.eps_tau(A, Ac, tau)) < 1e-9 * abs(est) + 1e-12
    for t in (0.5 * tau, 2 * tau):
        assert rowid.eps_tau(A, Ac, t) >= est - 1e-9 * abs(est)


def test_spc_id_err_curve_pins():
    # tau = 0: c times the largest squared singular value of the kept rows B_f
    A = synth.heat_modes(30, 8, seed=9, nu=0.002) + 1e-2 * np.random.default_rng(5).standard_normal((30, 64))
    R = _di(8, 8, 2, 2)
    Ac = restrict.apply(A, R)
    mc = 10
    c = 30 // mc
    keep = [i for i in range(30) if (i + 1) % c == 0]
    e0 = rowid.spc_id_err_curve(A, R, mc, [0.0])[0]
    assert abs(e0 - c * np.linalg.svd(A[keep], compute_uv=False)[0] ** 2) <= 1e-12 * e0
    # every row kept (mc = m): the definition of eps(tau) on the full matrices
    taus = [0.1, 1.0, 4.0, 16.0]
    full = rowid.spc_id_err_curve(A, R, 30, taus)
    for t, v in zip(taus, full):
        assert abs(v - rowid.eps_tau(A, Ac, t)) <= 1e-10 * max(abs(v), 1.0)
    # B_c B_c^T is positive semidefinite: non-increasing in tau, within Weyl's bounds
    curve = rowid.spc_id_err_curve(A, R, mc, np.linspace(0.0, 20.0, 41))
    assert np.all(np.diff(curve) <= 1e-10 * np.abs(curve).max())
    Gf = A[keep] @ A[keep].T
    Gc = Ac[keep] @ Ac[keep].T
    lf = np.linalg.eigvalsh(Gf)[-1]
    lc = np.linalg.eigvalsh(Gc)
    for t, v in zip(np.linspace(0.0, 20.0, 41), curve):
        assert c * (lf - t * lc[-1]) - 1e-9 * lf <= v <= c * (lf - t * lc[0]) + 1e-9 * lf


# ------------------------------------------------------------------ learned restriction

def test_projection_loss_gradient_finite_difference():
    rng = np.random.default_rng(14)
    A = synth.heat_modes(20, 8, seed=9, nu=0.002) + 0.05 * rng.standard_normal((20, 64))
    Ac = restrict.apply(A, _di(8, 8, 2, 2)) + 0.01 * rng.standard_normal((20, 16))
    Ag = restrict.gather(A, restrict.di_index_2d(8, 8, 2, 2))     # the power steps' fixed Gram sub-sample
    for q in (0, 1, 2):
        L, g = learned.projection_loss_grad(A, Ac, 4, q, Ag=Ag)
        assert abs(L - learned.projection_loss(A, Ac, 4, q, Ag=Ag)) < 1e-14
        h = 1e-6
        for idx in [(0, 0), (3, 4), (7, 12), (19, 15), (5, 5)]:
            E = np.zeros_like(Ac); E[idx] = h
            fd = (learned.projection_loss(A, Ac + E, 4, q, Ag=Ag) - learned.projection_loss(A, Ac - E, 4, q, Ag=Ag)) / (2 * h)
            assert abs(fd - g[idx]) < 1e-6 * max(1e-3, abs(fd)), (q, idx, fd, g[idx])


def test_learned_weight_gradient_finite_difference():
    rng = np.random.default_rng(15)
    ny = nx = 8
    A = synth.heat_modes(12, 8, seed=10, nu=0.002) + 0.05 * rng.standard_normal((12, 64))
    w1 = rng.standard_normal((4, 1, 5, 5)) * 0.3
    w2 = rng.standard_normal((1, 4, 5, 5)) * 0.3
    L, gw1, gw2 = learned.learned_loss_and_grad(A, ny, nx, w1, w2, ell=3, q=1)

    Ag = A[:, restrict.di_index_2d(ny, nx, 4, 4)]

    def loss(a, b):
        return learned.projection_loss(A, restrict.conv_restrict(A, ny, nx, a, b), 3, 1, Ag=Ag)

    h = 1e-6
    for idx in [(0, 0, 2, 2), (2, 0, 1, 3)]:
        e = np.zeros_like(w1); e[idx] = h
        fd = (loss(w1 + e, w2) - loss(w1 - e, w2)) / (2 * h)
        assert abs(fd - gw1[idx]) < 1e-6 * max(1e-3, abs(fd))
    for idx in [(0, 1, 2, 2), (0, 3, 0, 4)]:
        e = np.zeros_like(w2); e[idx] = h
        fd = (loss(w1, w2 + e) - loss(w1, w2 - e)) / (2 * h)
        assert abs(fd - gw2[idx]) < 1e-6 * max(1e-3, abs(fd))

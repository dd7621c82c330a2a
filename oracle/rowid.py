"""Row interpolative decomposition in FP64: rank-k column-pivoted QR of A^T
(Sec. 4), TPC-ID (Alg. 4), SPC-ID (Alg. 5) and SPC-ID-ERR (Alg. 6).

TEST INFRASTRUCTURE ONLY (see package docstring).

Readings of the paper used here:
  * The skeleton is a set of k ROW indices of A (time steps), i.e. the first
    k column pivots of a CPQR of A^T (Sec. 4, row ID).  The index set is a
    subset of {0..m-1}.
  * Pivot rule: at step j take the remaining column with the largest
    residual 2-norm, recomputed from the updated trailing matrix (no norm
    downdating); exact ties go to the lowest original column index.
  * "Solve R_2 ~ R_1 C by least squares": R_1 is k x k upper triangular and
    nonsingular when the rank is >= k, so C = R_1^{-1} R_2 by a triangular
    solve.  When R_1 has negligible pivots (|r_jj| <= 1e-14 |r_11|; the
    pivoted factor's diagonal does not increase, so they are its last k - r
    pivots) the least-squares problem has many solutions; the basic one is
    taken: the negligible pivots get zero coefficients and the leading r x r
    triangle is solved, i.e. the interpolation uses the r independent
    skeleton rows.
  * TPC-ID with q >= 1 (C-PWR without re-orthonormalisation, Sec. 7): the ID
    is taken of W_q = (tau A_g A_g^T)^q A_c, with A_c = A_f D the sketch and
    A_g = A_f(:, I) the Gram sub-sample of Alg. 7 (A_g = A_c for an index
    restriction), evaluated in Alg. 7's order (G <- A_g^T G, then
    G <- A_g G).  With a second-level sketch (Alg. 4 optional projection)
    the ID is taken of (tau A_g A_g^T)^q A_c S_l instead.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import restrict as _restrict
from . import sketch as _sketch


def cpqr(X: np.ndarray, k: int):
    """Rank-k Householder QR with column pivoting of X (rows x cols).

    Returns (perm, R, gaps):
      perm  column order (first k entries are the pivots, in pivot order)
      R     k x cols upper-trapezoidal factor in permuted column order
            (R[:, :k] = R_1, R[:, k:] = R_2)
      gaps  for each step the two largest residual norms (r1, r2) among the
            candidates, used to judge whether a pivot decision is separated.
    """
    X = np.array(X, dtype=np.float64, copy=True)
    nr, nc = X.shape
    k = min(k, nr, nc)
    perm = np.arange(nc)
    gaps = np.zeros((k, 2))
    for j in range(k):
        norms = np.sqrt(np.sum(X[j:, j:] ** 2, axis=0))
        top = norms.max()
        # exact ties: lowest original column index
        cand = np.nonzero(norms == top)[0]
        pj = j + cand[np.argmin(perm[j + cand])]
        srt = np.sort(norms)[::-1]
        gaps[j] = (srt[0], srt[1] if len(srt) > 1 else 0.0)
        if pj != j:
            X[:, [j, pj]] = X[:, [pj, j]]
            perm[[j, pj]] = perm[[pj, j]]
        # Householder reflector that maps X[j:, j] onto a multiple of e_1
        x = X[j:, j].copy()
        alpha = np.linalg.norm(x)
        if alpha == 0.0:
            continue
        beta = -alpha if x[0] >= 0 else alpha
        v = x
        v[0] -= beta
        vnorm2 = float(v @ v)
        if vnorm2 > 0:
            X[j:, j:] -= np.outer(v, (2.0 / vnorm2) * (v @ X[j:, j:]))
        X[j, j] = beta
        X[j + 1:, j] = 0.0
    R = np.triu(X[:k, :])
    return perm, R, gaps


def row_id(W: np.ndarray, k: int):
    """Row ID W ~ P W(I, :) from a rank-k CPQR of W^T (Sec. 4).

    Returns (I, P, info): I (k row indices in pivot order), P (m x k) with
    P(I, :) = I_k, and info with R, perm, gaps and the rank-deficiency flag.
    """
    W = np.asarray(W, dtype=np.float64)
    m = W.shape[0]
    perm, R, gaps = cpqr(W.T, k)
    k = R.shape[0]
    R1 = R[:, :k]
    R2 = R[:, k:]
    d = np.abs(np.diag(R1))
    keep = d > 1e-14 * d[0] if k > 0 else np.zeros(0, dtype=bool)
    r = int(np.count_nonzero(keep))
    deficient = r < k
    C = np.zeros((k, R2.shape[1]))
    if r > 0:
        # basic least-squares solution: the leading r x r triangle (negligible
        # pivots are a suffix of the diagonal), zero rows for the rest
        C[:r] = sla.solve_triangular(R1[:r, :r], R2[:r], lower=False)
    P = np.zeros((m, k))
    P[perm[:k], :] = np.eye(k)
    P[perm[k:], :] = C.T
    return perm[:k].copy(), P, {"R": R, "perm": perm, "gaps": gaps, "C": C,
                                "rank_deficient": deficient, "rank": r}


def coarse_power(Ag: np.ndarray, q: int, tau: float, G: np.ndarray | None = None) -> np.ndarray:
    """(tau A_g A_g^T)^q G without re-orthonormalisation (Alg. 7 with its
    optional QR steps left out), A_g the Gram sub-sample; G = A_g by default."""
    G = Ag if G is None else G
    return _sketch.power_iter(Ag, G, q, tau, reorth=False)


def tpc_id(A: np.ndarray, k: int, R: dict, q: int = 0, tau: float | None = None,
           S=None, projected: bool = False, p: int = 10, Ac: np.ndarray | None = None,
           return_all: bool = False):
    """TPC-ID (Alg. 4): A_c = A_f D, (P_c, I_c) = ID(A_c^T), A ~ P_c A_f(I_c, :).

    q >= 1 applies C-PWR (Alg. 7, no re-orthonormalisation) with the Gram
    sub-sample A_g = A_f(:, I).  projected=True uses the l-wide second-level
    block A_c S_l instead of the full coarse sketch (Alg. 4 optional
    projection)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if Ac is None:
        Ac = _restrict.apply(A, R)
    s = Ac.shape[1]
    Ag = _sketch.gram_sample(A, R, Ac) if q > 0 else Ac
    if tau is None:
        tau = n / Ag.shape[1]
    if projected:
        ell = _sketch.ell_of(k, s, m, p) if S is None else np.asarray(S).shape[1]
        G = _sketch.start_block(Ac, ell, S)
    else:
        G = Ac
    W = coarse_power(Ag, q, tau, G)
    I, P, info = row_id(W, k)
    if return_all:
        info.update({"Ac": Ac, "W": W, "skeleton_rows": A[I]})
        return I, P, info
    return I, P


def spc_id(A: np.ndarray, k: int, R: dict, r: int, Ac: np.ndarray | None = None,
           id_of: str = "Ac"):
    """SPC-ID (Alg. 5): single pass builds A_c and H = A_f^T A_c; SVD of A_c;
    lifting operator T_r = V_c S_c^+ U_c^T U_r U_r^T U_c S_c^+ V_c^T H^T;
    row ID of A_c (or of U_c(:, :k)); A ~ P_c A_c(I_c, :) T_r."""
    A = np.asarray(A, dtype=np.float64)
    if Ac is None:
        Ac = _restrict.apply(A, R)
    H = np.zeros((A.shape[1], Ac.shape[1]))
    for i in range(A.shape[0]):           # one pass, one row at a time
        H += np.outer(A[i], Ac[i])
    Uc, sc, Vct = np.linalg.svd(Ac, full_matrices=False)
    tol = sc.max() * max(Ac.shape) * np.finfo(np.float64).eps if sc.size else 0.0
    sinv = np.where(sc > tol, 1.0 / np.where(sc > tol, sc, 1.0), 0.0)
    Ur = Uc[:, :r]
    Tr = (Vct.T * sinv[None, :]) @ (Uc.T @ Ur) @ (Ur.T @ Uc) @ ((sinv[:, None] * Vct) @ H.T)
    W = Ac if id_of == "Ac" else Uc[:, :k]
    I, P, _ = row_id(W, k)
    return I, P, Ac[I], Tr


def lifting_operator_simplified(A: np.ndarray, Ac: np.ndarray, r: int) -> np.ndarray:
    """The simplified form T_r = A_c^+ U_r U_r^T A_f (Sec. 4 derivation)."""
    Uc, _, _ = np.linalg.svd(Ac, full_matrices=False)
    Ur = Uc[:, :r]
    return np.linalg.pinv(Ac) @ Ur @ (Ur.T @ A)


def spc_id_err(A: np.ndarray, R: dict, mc: int, tau_bounds=(1e-6, 1e6), Ac=None):
    """SPC-ID-ERR (Alg. 6): keep every c-th row (c = m / m_c, rows with
    (i+1) mod c == 0 in 0-based numbering), then
    eps_hat = min_tau c * lambda_max(B_f B_f^T - tau B_c B_c^T).
    lambda_max of an affine symmetric matrix function is convex in tau, so a
    bounded scalar minimisation over log(tau) is used."""
    from scipy.optimize import minimize_scalar
    A = np.asarray(A, dtype=np.float64)
    if Ac is None:
        Ac = _restrict.apply(A, R)
    m = A.shape[0]
    c = m // mc
    J = np.array([i for i in range(m) if (i + 1) % c == 0])
    Bf = A[J]
    Bc = Ac[J]
    Gf = Bf @ Bf.T
    Gc = Bc @ Bc.T

    def f(lt):
        return c * np.linalg.eigvalsh(Gf - np.exp(lt) * Gc)[-1]

    res = minimize_scalar(f, bounds=(np.log(tau_bounds[0]), np.log(tau_bounds[1])),
                          method="bounded", options={"xatol": 1e-10})
    return float(res.fun), float(np.exp(res.x))


def spc_id_err_curve(A: np.ndarray, R: dict, mc: int, taus, Ac=None) -> np.ndarray:
    """SPC-ID-ERR (Alg. 6) evaluated at given scales:
    eps_hat(tau) = c * lambda_max(B_f B_f^T - tau B_c B_c^T), c = m // mc, with
    B_f and B_c the rows i of A and A_c for which (i + 1) mod c == 0 (the rows
    Alg. 6 keeps while it streams A)."""
    A = np.asarray(A, dtype=np.float64)
    if Ac is None:
        Ac = _restrict.apply(A, R)
    m = A.shape[0]
    c = m // mc
    J = np.array([i for i in range(m) if (i + 1) % c == 0])
    Bf = A[J]
    Bc = Ac[J]
    Gf = Bf @ Bf.T
    Gc = Bc @ Bc.T
    return np.array([c * np.linalg.eigvalsh(Gf - t * Gc)[-1] for t in np.asarray(taus, dtype=np.float64)])


def spc_rho_curve(A: np.ndarray, R: dict, mc: int, taus, Ac=None) -> np.ndarray:
    """The subsampled estimate of rho(tau) = ||A_f A_f^T - tau A_c A_c^T||_2
    (the Gram-mismatch measure of the C-PWR analysis, Sec. 5), formed from the
    same kept rows as Alg. 6: rho_hat(tau) = c ||B_f B_f^T - tau B_c B_c^T||_2,
    c = m // mc.  The matrix is symmetric, so its 2-norm is its largest
    eigenvalue magnitude.  With mc = m it is rho(tau) itself."""
    A = np.asarray(A, dtype=np.float64)
    if Ac is None:
        Ac = _restrict.apply(A, R)
    m = A.shape[0]
    c = m // mc
    J = np.array([i for i in range(m) if (i + 1) % c == 0])
    Gf = A[J] @ A[J].T
    Gc = Ac[J] @ Ac[J].T
    return np.array([c * np.abs(np.linalg.eigvalsh(Gf - t * Gc)).max() for t in np.asarray(taus, dtype=np.float64)])


def rho_tau(A: np.ndarray, Ac: np.ndarray, tau: float) -> float:
    """rho(tau) = ||A_f A_f^T - tau A_c A_c^T||_2 (Sec. 5, C-PWR analysis)."""
    return float(np.linalg.norm(A @ A.T - tau * (Ac @ Ac.T), 2))


def eps_tau(A: np.ndarray, Ac: np.ndarray, tau: float) -> float:
    """epsilon(tau) = lambda_max(A_f A_f^T - tau A_c A_c^T) (Sec. 4)."""
    return float(np.linalg.eigvalsh(A @ A.T - tau * (Ac @ Ac.T))[-1])

"""Sketch-based SVD in FP64: TPC-SVD (Alg. 2) with the coarse-grid power
iteration C-PWR (Alg. 7), the single-pass SPC-SVD (Alg. 3) and PROTO-TPC
(Alg. 1).

TEST INFRASTRUCTURE ONLY (see package docstring).

Readings of the paper used here:
  * Range-finder width.  The configurations have s = |I| >= m, so QR of the
    whole coarse sketch would span all of R^m.  The orthonormalised block is
    l = min(k + p, s, m) wide (n_c = k + p in Alg. 1 and Alg. 3, p = 10 as in
    the experiments).  Its start block is Y = A_c S_l: by default the nested
    direct injection S_l = columns floor(s/l) * j, j = 0..l-1, of A_c;
    optionally a caller-given s x l matrix (e.g. a Gaussian Omega, the
    paper's hybrid sketch, Alg. 2 optional projection).
  * tau (Sec. 5, the scaled coarse Gram) defaults to n / s.  With
    re-orthonormalisation (Sec. 5, optional QR steps) the result does not
    depend on tau.
  * Singular vector signs: each (u_j, v_j) is flipped so that the entry of
    u_j with the largest magnitude (lowest index on ties) is positive.
"""
from __future__ import annotations

import numpy as np

from . import restrict as _restrict


def ell_of(k: int, s: int, m: int, p: int = 10) -> int:
    return int(min(k + p, s, m))


def nested_di_columns(s: int, ell: int) -> np.ndarray:
    """Second-level direct injection inside the coarse sketch: every
    floor(s/l)-th coarse column."""
    step = s // ell
    return (np.arange(ell) * step).astype(np.int64)


def start_block(Ac: np.ndarray, ell: int, S: np.ndarray | None = None) -> np.ndarray:
    """Y = A_c S_l (m x l)."""
    if S is not None:
        return Ac @ np.asarray(S, dtype=np.float64)
    return Ac[:, nested_di_columns(Ac.shape[1], ell)]


def orth(Y: np.ndarray) -> np.ndarray:
    """Thin Householder QR, all columns of Y kept (QR step of Alg. 2 / Alg. 7)."""
    q, _ = np.linalg.qr(Y, mode="reduced")
    return q


def power_iter(Ac: np.ndarray, G: np.ndarray, q: int, tau: float, reorth: bool = True) -> np.ndarray:
    """C-PWR loop (Alg. 7): repeat q times  G <- A_c^T G, [QR], G <- A_c G, [QR].

    Ac is the Gram sub-sample A_f(:, I) of Alg. 7 (for an index restriction
    the restriction itself; see restrict.gram_index).  The coarse Gram is
    scaled by tau (Sec. 5: approximate power of (tau A_c A_c^T)); the scale is
    applied on the A_c^T product.  With reorth=False the raw block
    (tau A_c A_c^T)^q G is returned.
    """
    G = np.asarray(G, dtype=np.float64)
    for _ in range(q):
        G = tau * (Ac.T @ G)
        if reorth:
            G = orth(G)
        G = Ac @ G
        if reorth:
            G = orth(G)
    return G


def sign_normalise(U: np.ndarray, V: np.ndarray):
    U = U.copy()
    V = V.copy()
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
            V[:, j] = -V[:, j]
    return U, V


def gram_sample(A: np.ndarray, R: dict, Ac: np.ndarray) -> np.ndarray:
    """A_f(:, I), the coarse matrix of C-PWR's Gram (Alg. 7): the restriction's
    own A_c when it is an index restriction, else the gather of gram_index."""
    if R is not None and R.get("kind") != "index":
        return _restrict.gather(A, _restrict.gram_index(R))
    return Ac


def tpc_svd(A: np.ndarray, k: int, R: dict, q: int = 0, p: int = 10, S=None,
            tau: float | None = None, Ac: np.ndarray | None = None, return_all: bool = False):
    """Rank-k SVD via the deterministic sketch (Alg. 2) and C-PWR (Alg. 7).

    1. A_c = A_f D                                  (Sec. 2)
    2. Y = A_c S_l, Q = QR(Y)                       (Alg. 2 QR step; Alg. 7 start)
    3. q coarse power steps with re-orthonormalisation (Alg. 7), on the
       Gram sub-sample A_f(:, I) (= A_c for an index restriction)
    4. B = Q^T A_f                                  (Alg. 2; Sec. 3.1)
    5. SVD(B) = U_B Sigma V_B^T, U = Q U_B          (Alg. 2)
    6. truncate to k
    Returns U (m x k), s (k), V (n x k) and, if asked, a dict of intermediates.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if Ac is None:
        Ac = _restrict.apply(A, R)
    s = Ac.shape[1]
    ell = ell_of(k, s, m, p) if S is None else np.asarray(S).shape[1]
    Ag = gram_sample(A, R, Ac) if q > 0 else Ac
    if tau is None:
        tau = n / Ag.shape[1]
    Y = start_block(Ac, ell, S)
    Q = orth(Y)
    Q = power_iter(Ag, Q, q, tau, reorth=True)
    B = Q.T @ A
    UB, sig, VBt = np.linalg.svd(B, full_matrices=False)
    U = Q @ UB[:, :k]
    V = VBt[:k].T
    U, V = sign_normalise(U, V)
    if return_all:
        return U, sig[:k], V, {"Ac": Ac, "Ag": Ag, "Y": Y, "Q": Q, "B": B, "sigma_B": sig, "ell": ell,
                               "tau": tau}
    return U, sig[:k], V


def spc_svd(A: np.ndarray, k: int, R: dict, p: int = 10, S=None, Ac: np.ndarray | None = None,
            rows_per_read: int = 1, return_all: bool = False):
    """Single-pass SPC-SVD (Alg. 3).

    One pass over the rows of A_f accumulates the coarse rows a_c = a_f D S_l
    and H += a_f^T a_c.  Then QR(A_c) = Q_c R_c, H <- H R_c^{-1} (= A_f^T Q_c),
    SVD(H^T) = U~ S V^T, U = Q_c U~, truncated to k.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if Ac is None:
        Ac = _restrict.apply(A, R)
    s = Ac.shape[1]
    ell = ell_of(k, s, m, p) if S is None else np.asarray(S).shape[1]
    Yfull = start_block(Ac, ell, S)
    H = np.zeros((n, ell))
    rows = []
    for i0 in range(0, m, rows_per_read):
        af = A[i0:i0 + rows_per_read]
        ac = Yfull[i0:i0 + rows_per_read]   # the same rows of the sketch
        rows.append(ac)
        H += af.T @ ac
    Yc = np.vstack(rows)
    Qc, Rc = np.linalg.qr(Yc, mode="reduced")
    import scipy.linalg as sla
    Ht = sla.solve_triangular(Rc, H.T, trans="T", lower=False)   # (H R^{-1})^T = R^{-T} H^T
    Ut, sig, Vt = np.linalg.svd(Ht, full_matrices=False)
    U = Qc @ Ut[:, :k]
    V = Vt[:k].T
    U, V = sign_normalise(U, V)
    if return_all:
        return U, sig[:k], V, {"sigma_B": sig, "ell": ell}
    return U, sig[:k], V


def proto_tpc(A: np.ndarray, k: int, Ac: np.ndarray):
    """PROTO-TPC (Alg. 1): U~ = U_c(:, :k), S~ = S_c(:k), V~ = ((U~ S~)^+ A_f)^T."""
    Uc, sc, _ = np.linalg.svd(Ac, full_matrices=False)
    Uk = Uc[:, :k]
    Sk = sc[:k]
    V = np.linalg.pinv(Uk * Sk[None, :]) @ A
    return Uk, Sk, V.T

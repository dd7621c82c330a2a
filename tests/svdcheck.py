"""Singular-vector comparison used by the GPU parity tests.

Each pair (u_j, v_j) is defined up to a common sign, and where singular values
are closer than the tolerance can resolve, only the span of the cluster is
defined (perturbation theory: a relative error tol in the data moves u_j by
about tol sigma_1 / gap_j).  So the first k singular values of the oracle's
B (all ell of them, sig_all) are split into clusters whose consecutive gaps
are at most 100 tol sigma_1; a single vector is compared entry by entry after
aligning its sign, a cluster by the distance between its projectors, both to
10 tol / gap; a cluster cut by index k (sigma_k too close to sigma_{k+1}) has
no defined span and is skipped.
"""
from __future__ import annotations

import numpy as np


def clusters(sig_all, k, tol):
    sig = np.asarray(sig_all, dtype=np.float64)
    sep = 100.0 * tol * sig[0]
    out, a = [], 0
    for j in range(1, k + 1):
        last = j == k
        if last or sig[j - 1] - sig[j] > sep:
            closed = (not last) or len(sig) <= k or (sig[k - 1] - sig[k] > sep)
            lo = sig[a - 1] - sig[a] if a > 0 else np.inf
            hi = sig[j - 1] - sig[j] if j < len(sig) else np.inf
            out.append((a, j, min(lo, hi) / sig[0], closed))
            a = j
    return out


def compare_vectors(U, Uo, V, Vo, sig_all, k, tol, min_checked=1):
    """U, V (GPU, any float dtype) against Uo, Vo (oracle, FP64); returns the
    number of singular pairs checked individually."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    single = 0
    for a, b, gap, closed in clusters(sig_all, k, tol):
        if not closed:
            continue
        vt = min(10.0 * tol / gap, 0.5)
        if b - a == 1:
            j = a
            sgn = 1.0 if float(U[:, j] @ Uo[:, j]) >= 0 else -1.0
            du = np.linalg.norm(sgn * U[:, j] - Uo[:, j])
            dv = np.linalg.norm(sgn * V[:, j] - Vo[:, j])
            assert du <= vt and dv <= vt, (j, du, dv, vt)
            top = np.sort(np.abs(Uo[:, j]))[::-1]
            if len(top) > 1 and top[0] - top[1] > 4 * vt:
                assert sgn > 0, ("sign normalisation", j)   # largest-|u| entry positive on both sides
            single += 1
        else:
            for X, Xo in ((U, Uo), (V, Vo)):
                Qx = np.linalg.qr(X[:, a:b])[0]
                c = np.linalg.svd(Xo[:, a:b].T @ Qx, compute_uv=False)
                dist = float(np.sqrt(max(0.0, 1.0 - c.min() ** 2)))
                assert dist <= vt, ((a, b), dist, vt)
    assert single >= min(min_checked, k), single
    return single

"""Projection loss of a learned linear restriction and its gradients, FP64.

TEST INFRASTRUCTURE ONLY (see package docstring).

Not in the paper.  The learned restriction replaces D in A_c = A_f D (Sec. 2)
by a linear strided convolution; it is trained to shrink the sketch error
that Thm 3.2 bounds, ||(I - Q Q^T) A_f||, measured in the Frobenius norm:

    L = ||A - Q Q^T A||_F^2 / ||A||_F^2 = 1 - ||Q^T A||_F^2 / ||A||_F^2,

with Q the l-wide orthonormal block of the SVD path (start block Y = A_c S_l,
q coarse power steps with re-orthonormalisation, Alg. 7).  The power steps
use the Gram sub-sample A_g = A_f(:, I) of Alg. 7 (the direct-injection points
of the conv's output grid), which does not depend on the weights: the weights
reach Q only through the start block.

Gradient.  L depends on Q only through span(Q).  Each QR step X = Q R only
changes the basis inside span(X), and every later step (a product with A_c or
A_c^T and another QR) maps spans to spans, so dL/dR = 0 and the backward pass
may treat every R as a constant:  X = Q R  =>  dX = dQ R^{-T}.  At the output,
for orthonormal Q,  dL/dQ = -(2/||A||^2) (I - Q Q^T) A A^T Q
                         = -(2/||A||^2) (A B^T - Q B B^T),   B = Q^T A.
"""
from __future__ import annotations

import numpy as np

from . import restrict as _restrict
from . import sketch as _sketch


def _qr(X):
    Q, R = np.linalg.qr(X, mode="reduced")
    return Q, R


def projection_loss(A: np.ndarray, Ac: np.ndarray, ell: int, q: int, S=None, Ag=None):
    """L of the sketch A_c; Ag (the Gram sub-sample of the power steps) is
    needed when q >= 1."""
    A = np.asarray(A, dtype=np.float64)
    Y = _sketch.start_block(Ac, ell, S)
    Q, _ = _qr(Y)
    for _ in range(q):
        Z, _ = _qr(Ag.T @ Q)
        Q, _ = _qr(Ag @ Z)
    B = Q.T @ A
    return 1.0 - float(np.sum(B * B)) / float(np.sum(A * A))


def projection_loss_grad(A: np.ndarray, Ac: np.ndarray, ell: int, q: int, S=None, Ag=None):
    """Returns (L, dL/dA_c); Ag as in projection_loss (held fixed)."""
    A = np.asarray(A, dtype=np.float64)
    Ac = np.asarray(Ac, dtype=np.float64)
    s = Ac.shape[1]
    nrmA2 = float(np.sum(A * A))
    # forward, keeping every factor
    Y = _sketch.start_block(Ac, ell, S)
    Q0, R0 = _qr(Y)
    Zs, Rzs, Rqs = [], [], []
    Q = Q0
    for _ in range(q):
        Z, Rz = _qr(Ag.T @ Q)
        Q, Rq = _qr(Ag @ Z)
        Zs.append(Z)
        Rzs.append(Rz)
        Rqs.append(Rq)
    B = Q.T @ A
    L = 1.0 - float(np.sum(B * B)) / nrmA2
    # backward (A_g does not depend on A_c: only the start block carries dA_c)
    dQ = -(2.0 / nrmA2) * (A @ B.T - Q @ (B @ B.T))
    dAc = np.zeros_like(Ac)
    for i in range(q - 1, -1, -1):
        Rq, Rz = Rqs[i], Rzs[i]
        dW = np.linalg.solve(Rq, dQ.T).T            # dQ R^{-T}, W = A_g Z
        dZ = Ag.T @ dW
        dZp = np.linalg.solve(Rz, dZ.T).T           # Z = Z' Rz^{-1}, Z' = A_g^T Q_prev
        dQ = Ag @ dZp
    dY = np.linalg.solve(R0, dQ.T).T
    if S is None:
        cols = _sketch.nested_di_columns(s, ell)
        np.add.at(dAc, (slice(None), cols), dY)
    else:
        dAc += dY @ np.asarray(S, dtype=np.float64).T
    return L, dAc


def learned_loss_and_grad(A: np.ndarray, ny: int, nx: int, w1, w2, ell: int, q: int, S=None):
    """Loss of the conv-restricted sketch and its weight gradients (gw1, gw2)."""
    Ac = _restrict.conv_restrict(A, ny, nx, w1, w2)
    Ag = _restrict.gather(A, _restrict.gram_index({"kind": "learned", "ny": ny, "nx": nx})) if q > 0 else None
    L, dAc = projection_loss_grad(A, Ac, ell, q, S, Ag)
    gw1, gw2 = _restrict.conv_restrict_bwd(A, ny, nx, w1, w2, dAc)
    return L, gw1, gw2

"""Deterministic sketches A_c = A_f D (paper Sec. 2, the general sketch equation),
applied without forming D, plus the explicit D of each equation for tiny
problems and the learned linear convolution restriction.

TEST INFRASTRUCTURE ONLY (see package docstring).

Readings of the paper used here (all 0-based):
  * Direct injection (Sec. 2, DI equation): the printed index i = j*s + 1 with
    j = 1..n_c overruns n; we take i = j*s, j = 0..n_c-1.  On a 2-D grid the
    sketch is the tensor product of the 1-D sketches along y and x, i.e. the
    coarse sub-grid (s_y*b, s_x*a), flattened y-major.
  * Nearest neighbour (Sec. 2, NN equation): weights 1/4, 1/2, 1/4 at offsets
    -1, 0, +1 around the DI point, zero outside the grid, no renormalisation;
    2-D = tensor product.
  * Global sketch (Sec. 2, global equation): weight 1/s on the s consecutive
    dofs starting at the DI point (the equation has s entries; Table 1's
    stencil "s-1" is not followed); 2-D = tensor product.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------- 1-D D matrices


def d_matrix_1d(kind: str, n: int, s: int) -> np.ndarray:
    """Explicit n x n_c sketch matrix of one 1-D sketch, entry by entry from
    its defining equation (Sec. 2), with n_c = ceil(n / s)."""
    nc = -(-n // s)
    D = np.zeros((n, nc))
    for j in range(nc):
        c = j * s                       # the DI point of coarse node j
        for i in range(n):
            if kind == "di":
                D[i, j] = 1.0 if i == c else 0.0
            elif kind == "nn":
                if i == c:
                    D[i, j] = 0.5
                elif abs(i - c) == 1:
                    D[i, j] = 0.25
            elif kind == "global":
                if c <= i < c + s:
                    D[i, j] = 1.0 / s
            else:
                raise ValueError(kind)
    return D


def d_matrix_2d(kind: str, ny: int, nx: int, sy: int, sx: int) -> np.ndarray:
    """Tensor-product 2-D sketch matrix for a y-major flattened ny x nx grid."""
    return np.kron(d_matrix_1d(kind, ny, sy), d_matrix_1d(kind, nx, sx))


# ---------------------------------------------------------------- matrix-free forms


def di_index_2d(ny: int, nx: int, sy: int, sx: int) -> np.ndarray:
    """Sorted 0-based fine-grid columns of the 2-D direct-injection sketch."""
    ys = np.arange(0, ny, sy)
    xs = np.arange(0, nx, sx)
    return (ys[:, None] * nx + xs[None, :]).ravel().astype(np.int64)


def gram_index(R: dict) -> np.ndarray:
    """The sub-sampling index set I of C-PWR's coarse Gram A_c = A_f(:, I)
    (Alg. 7), which the algorithm keeps apart from the sketch D of its start
    block.  An index restriction is its own I.  A stencil or learned
    restriction takes R["gram_index"] when given, else the direct-injection
    points of the same grid and factor (the points the stencils are centred or
    anchored on; factor 4 x 4 for the learned conv, whose output is that
    sub-grid)."""
    if R["kind"] == "index":
        return np.asarray(R["index"], dtype=np.int64)
    if R.get("gram_index") is not None:
        return np.asarray(R["gram_index"], dtype=np.int64)
    if R["kind"] == "learned":
        return di_index_2d(R["ny"], R["nx"], 4, 4)
    return di_index_2d(R["ny"], R["nx"], R["sy"], R["sx"])


def gather(A: np.ndarray, index: np.ndarray) -> np.ndarray:
    """Direct injection / Gram sub-sample: A_c = A_f(:, I) (Sec. 2; Alg. 7)."""
    return np.asarray(A, dtype=np.float64)[:, np.asarray(index)]


def _stencil_2d(A: np.ndarray, ny: int, nx: int, sy: int, sx: int, wy, wx, offy, offx):
    """Weighted tensor stencil around the DI points, zero outside the grid."""
    m = A.shape[0]
    P = max(max(abs(o) for o in offy), max(abs(o) for o in offx))
    Fp = np.zeros((m, ny + 2 * P, nx + 2 * P))
    Fp[:, P:P + ny, P:P + nx] = np.asarray(A, dtype=np.float64).reshape(m, ny, nx)
    ys = np.arange(0, ny, sy)
    xs = np.arange(0, nx, sx)
    out = np.zeros((m, len(ys), len(xs)))
    for dy, w_y in zip(offy, wy):
        for dx, w_x in zip(offx, wx):
            out += (w_y * w_x) * Fp[:, ys + dy + P][:, :, xs + dx + P]
    return out.reshape(m, -1)


def nearest_neighbour_2d(A, ny, nx, sy, sx):
    """NN sketch with 1-D weights (1/4, 1/2, 1/4) in each axis (Sec. 2)."""
    w = (0.25, 0.5, 0.25)
    off = (-1, 0, 1)
    return _stencil_2d(A, ny, nx, sy, sx, w, w, off, off)


def global_2d(A, ny, nx, sy, sx):
    """Global (block-average) sketch: mean over the sy x sx block that starts
    at each DI point (Sec. 2, global equation, tensor form)."""
    wy = [1.0 / sy] * sy
    wx = [1.0 / sx] * sx
    return _stencil_2d(A, ny, nx, sy, sx, wy, wx, list(range(sy)), list(range(sx)))


def apply(A: np.ndarray, R: dict) -> np.ndarray:
    """Dispatch on a restriction description:
    {"kind": "index", "index": I} | {"kind": "nn"|"global", "ny","nx","sy","sx"}
    | {"kind": "learned", "ny","nx", "w1", "w2"}."""
    kind = R["kind"]
    if kind == "index":
        return gather(A, R["index"])
    if kind == "nn":
        return nearest_neighbour_2d(A, R["ny"], R["nx"], R["sy"], R["sx"])
    if kind == "global":
        return global_2d(A, R["ny"], R["nx"], R["sy"], R["sx"])
    if kind == "learned":
        return conv_restrict(A, R["ny"], R["nx"], R["w1"], R["w2"])
    raise ValueError(kind)


# ---------------------------------------------------------------- learned linear conv
# Not in the paper: a linear 2-layer strided convolution that plays the role of
# D (the NN sketch is described in Sec. 2 as a convolution-like smoothing
# filter).  It has no bias and no activation, so A_c = A_f D still holds with
# D the (implicit) matrix of the conv.  Cross-correlation convention:
#   y[c, oy, ox] = sum_{ci, ky, kx} w[c, ci, ky, kx] x[ci, 2*oy - 2 + ky, 2*ox - 2 + kx]
# with zero padding 2 and stride 2, 5x5 taps.

KS = 5
PAD = 2
STRIDE = 2


def _conv_fwd(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """x: (m, Cin, H, W), w: (Cout, Cin, 5, 5) -> (m, Cout, H/2, W/2)."""
    m, cin, H, W = x.shape
    cout = w.shape[0]
    Ho = (H + 2 * PAD - KS) // STRIDE + 1
    Wo = (W + 2 * PAD - KS) // STRIDE + 1
    xp = np.zeros((m, cin, H + 2 * PAD, W + 2 * PAD))
    xp[:, :, PAD:PAD + H, PAD:PAD + W] = x
    y = np.zeros((m, cout, Ho, Wo))
    for ky in range(KS):
        for kx in range(KS):
            patch = xp[:, :, ky:ky + STRIDE * Ho:STRIDE, kx:kx + STRIDE * Wo:STRIDE]  # m,cin,Ho,Wo
            y += np.einsum("mchw,oc->mohw", patch, w[:, :, ky, kx])
    return y


def _conv_bwd_data(gy: np.ndarray, w: np.ndarray, H: int, W: int) -> np.ndarray:
    """Adjoint of _conv_fwd in x."""
    m, cout, Ho, Wo = gy.shape
    cin = w.shape[1]
    gxp = np.zeros((m, cin, H + 2 * PAD, W + 2 * PAD))
    for ky in range(KS):
        for kx in range(KS):
            gxp[:, :, ky:ky + STRIDE * Ho:STRIDE, kx:kx + STRIDE * Wo:STRIDE] += np.einsum(
                "mohw,oc->mchw", gy, w[:, :, ky, kx])
    return gxp[:, :, PAD:PAD + H, PAD:PAD + W]


def _conv_bwd_weight(x: np.ndarray, gy: np.ndarray) -> np.ndarray:
    """Gradient of <gy, conv(x, w)> with respect to w."""
    m, cin, H, W = x.shape
    cout, Ho, Wo = gy.shape[1], gy.shape[2], gy.shape[3]
    xp = np.zeros((m, cin, H + 2 * PAD, W + 2 * PAD))
    xp[:, :, PAD:PAD + H, PAD:PAD + W] = x
    gw = np.zeros((cout, cin, KS, KS))
    for ky in range(KS):
        for kx in range(KS):
            patch = xp[:, :, ky:ky + STRIDE * Ho:STRIDE, kx:kx + STRIDE * Wo:STRIDE]
            gw[:, :, ky, kx] = np.einsum("mchw,mohw->oc", patch, gy)
    return gw


def conv_restrict(A: np.ndarray, ny: int, nx: int, w1: np.ndarray, w2: np.ndarray,
                  return_hidden: bool = False):
    """Two strided linear conv layers: (ny, nx) -> (C, ny/2, nx/2) -> (ny/4, nx/4)."""
    m = A.shape[0]
    x = np.asarray(A, dtype=np.float64).reshape(m, 1, ny, nx)
    h = _conv_fwd(x, np.asarray(w1, dtype=np.float64))
    y = _conv_fwd(h, np.asarray(w2, dtype=np.float64))
    if return_hidden:
        return y.reshape(m, -1), h
    return y.reshape(m, -1)


def conv_restrict_bwd(A: np.ndarray, ny: int, nx: int, w1, w2, gAc: np.ndarray):
    """Weight gradients of <gAc, conv_restrict(A)>: returns (gw1, gw2)."""
    m = A.shape[0]
    x = np.asarray(A, dtype=np.float64).reshape(m, 1, ny, nx)
    w1 = np.asarray(w1, dtype=np.float64)
    w2 = np.asarray(w2, dtype=np.float64)
    h = _conv_fwd(x, w1)
    Ho = (h.shape[2] + 2 * PAD - KS) // STRIDE + 1
    Wo = (h.shape[3] + 2 * PAD - KS) // STRIDE + 1
    gy = np.asarray(gAc, dtype=np.float64).reshape(m, 1, Ho, Wo)
    gw2 = _conv_bwd_weight(h, gy)
    gh = _conv_bwd_data(gy, w2, h.shape[2], h.shape[3])
    gw1 = _conv_bwd_weight(x, gh)
    return gw1, gw2


def conv_as_matrix(ny: int, nx: int, w1, w2) -> np.ndarray:
    """The implicit D (n x s) of the learned conv, built column by column from
    unit fine-grid fields (tiny grids only)."""
    n = ny * nx
    return conv_restrict(np.eye(n), ny, nx, w1, w2)

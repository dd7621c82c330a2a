"""Seeded synthetic snapshot matrices shaped like the paper's PDE workloads.

This module only draws inputs; it holds none of the sketching method's
arithmetic (no restriction, no orthonormalisation of sketches, no SVD/ID of
the data).  Both the CPU reference implementation used by the tests and the
GPU path consume its output, so it must stay free of either.

Layout conventions shared by every generator:
  * A is m x n, one row per snapshot (time step), one column per grid dof
    (paper, Sec. 2: rows are snapshots, columns are fine-grid values).
  * A 2-D field on an ny x nx grid is flattened y-major: column = iy*nx + ix.
  * Generators return float64 arrays; callers cast to the storage dtype.

Families:
  heat_modes      2-D heat-equation sine modes with Dirichlet walls
  advdiff_exact   periodic Fourier modes with advected/diffused temporal
                  factors, exact prescribed spectrum sigma_j (+ noise)
  heat_exact      Dirichlet sine modes with exact spectrum sigma_j
  advdiff_field   physical advection-diffusion snapshots at a diffusivity nu
                  (advdiff_field_device: the same on a torch device)
  lowrank         product of Gaussian factors (exact rank r)
  gaussian_matrix iid N(0, 1) draws, e.g. the optional Gaussian second-level
                  sketch of the hybrid method (passed to both sides as input)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "heat_modes", "advdiff_exact", "heat_exact", "advdiff_field", "advdiff_field_device", "learned_diffusivities",
    "learned_trajectory", "lowrank", "gaussian_matrix",
    "batch_specs", "BatchSpec", "orthonormal_fourier_1d",
]


def _interior_nodes(N: int) -> np.ndarray:
    # interior nodes of a Dirichlet unit interval: x_i = (i+1)/(N+1)
    return (np.arange(N, dtype=np.float64) + 1.0) / (N + 1.0)


def heat_modes(m: int, N: int, seed: int, nu: float = 0.01, pq_max: int = 16,
               t: np.ndarray | None = None) -> np.ndarray:
    """u(x,y,t) = sum_{p,q<=pq_max} a_pq exp(-pi^2 (p^2+q^2) nu t) sin(p pi x) sin(q pi y).

    a_pq = z_pq / (p^2+q^2), z ~ N(0,1) drawn as a pq_max x pq_max array in
    (p, q) order from default_rng(seed).  Mode p varies along x, q along y.
    Times t_j = j/(m-1) unless given.  Returns A (m x N*N, float64).
    """
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((pq_max, pq_max))
    p = np.arange(1, pq_max + 1, dtype=np.float64)
    lam = p[:, None] ** 2 + p[None, :] ** 2            # [p, q]
    a = z / lam
    if t is None:
        t = np.arange(m, dtype=np.float64) / max(m - 1, 1)
    x = _interior_nodes(N)
    sx = np.sin(np.pi * p[:, None] * x[None, :])      # [p, ix]
    sy = np.sin(np.pi * p[:, None] * x[None, :])      # [q, iy]
    decay = np.exp(-np.pi ** 2 * nu * lam[None, :, :] * t[:, None, None])  # [t, p, q]
    coef = decay * a[None]                             # [t, p, q]
    # field[t, iy, ix] = sum_{p,q} coef[t,p,q] sy[q,iy] sx[p,ix]
    tmp = np.einsum("tpq,qy->tpy", coef, sy)
    field = np.einsum("tpy,px->tyx", tmp, sx)
    return field.reshape(m, N * N)


def orthonormal_fourier_1d(N: int) -> np.ndarray:
    """Real orthonormal Fourier basis on N periodic points, columns ordered by
    wavenumber: [const, cos1, sin1, cos2, sin2, ..., (Nyquist if N even)]."""
    x = np.arange(N, dtype=np.float64)
    cols = [np.full(N, 1.0 / math.sqrt(N))]
    wn = [0]
    for k in range(1, (N - 1) // 2 + 1):
        cols.append(math.sqrt(2.0 / N) * np.cos(2 * np.pi * k * x / N))
        cols.append(math.sqrt(2.0 / N) * np.sin(2 * np.pi * k * x / N))
        wn += [k, k]
    if N % 2 == 0:
        cols.append(np.cos(np.pi * x) / math.sqrt(N))
        wn.append(N // 2)
    return np.stack(cols, axis=1), np.asarray(wn)


def _mode_order(kx: np.ndarray, ky: np.ndarray, r: int):
    # pick the r lowest-|k| tensor modes (ties broken by (ky, kx) index)
    KY, KX = np.meshgrid(np.arange(len(ky)), np.arange(len(kx)), indexing="ij")
    mag = ky[KY] ** 2 + kx[KX] ** 2
    order = np.lexsort((KX.ravel(), KY.ravel(), mag.ravel()))[:r]
    return KY.ravel()[order], KX.ravel()[order], mag.ravel()[order]


def _orthonormal_columns(M: np.ndarray) -> np.ndarray:
    # input synthesis only: orthonormal temporal factors for an exact spectrum
    q, r = np.linalg.qr(M)
    return q * np.sign(np.diag(r))[None, :]


def advdiff_exact(m: int, N: int, seed: int, r: int | None = None, power: float = 0.5,
                  noise: float = 1e-3, nu: float = 0.02, v=(0.7, 0.3),
                  return_parts: bool = False):
    """A = U_t diag(sigma) F_s^T + noise on a periodic N x N grid.

    F_s: the r lowest-wavenumber real tensor Fourier modes (exactly orthonormal).
    sigma_j = j^-power, j = 1..r (r = m by default).
    U_t: orthonormalised temporal factors of advected, diffused Fourier modes,
         g_j(t) = exp(-nu |k_j|^2 t) cos(2 pi (k_j . v) t + phi_j) + 0.3 z_j(t).
    noise: iid N(0, (noise * rms(A_clean))^2).
    """
    rng = np.random.default_rng(seed)
    r = m if r is None else min(r, m, N * N)
    F, wn = orthonormal_fourier_1d(N)
    iy, ix, mag = _mode_order(wn, wn, r)
    t = np.arange(m, dtype=np.float64) / max(m - 1, 1)
    kvel = wn[ix] * v[0] + wn[iy] * v[1]
    phi = rng.uniform(0, 2 * np.pi, size=r)
    G = np.exp(-nu * mag[None, :] * t[:, None] * 0.05) * np.cos(
        2 * np.pi * kvel[None, :] * t[:, None] + phi[None, :])
    G = G + 0.3 * rng.standard_normal((m, r))
    Ut = _orthonormal_columns(G)
    sigma = np.arange(1, r + 1, dtype=np.float64) ** (-power)
    C = Ut * sigma[None, :]                                 # m x r
    # A[t, iy, ix] = sum_j C[t, j] F[iy, ky_j] F[ix, kx_j]
    A = np.zeros((m, N, N))
    # group by ky to use separability: A_t = F[:, ky] (C-block) F[:, kx]^T
    for ky in np.unique(iy):
        sel = np.nonzero(iy == ky)[0]
        # rows: t; contribution F[:,ky] (outer) sum_j C[t,j] F[:, kx_j]
        Sx = F[:, ix[sel]]                                  # N x |sel|
        part = C[:, sel] @ Sx.T                             # m x N (along x)
        A += part[:, None, :] * F[:, ky][None, :, None]
    A = A.reshape(m, N * N)
    if noise > 0:
        rms = math.sqrt(float(np.mean(A * A)))
        A = A + (noise * rms) * rng.standard_normal(A.shape)
    if return_parts:
        return A, sigma
    return A


def heat_exact(m: int, ny: int, nx: int, seed: int, rate: float = 0.05, r: int | None = None,
               nu: float = 0.01, return_parts: bool = False):
    """A = U_t diag(exp(-rate*j)) V_s^T on an interior Dirichlet ny x nx grid.

    V_s: the r sine modes sqrt(2/(ny+1)) sin(q pi y) * sqrt(2/(nx+1)) sin(p pi x)
         with the smallest p^2+q^2 (exactly orthonormal on the interior grid).
    U_t: orthonormalised heat decays exp(-pi^2 (p^2+q^2) nu t) plus a seeded
         Gaussian component (keeps the temporal factors well separated).
    sigma_j = exp(-rate * j), j = 1..r.  Default r = min(m, 400).
    """
    rng = np.random.default_rng(seed)
    r = min(m, 400) if r is None else min(r, m, nx * ny)
    pmax = int(math.ceil(math.sqrt(4 * r))) + 2
    py = np.arange(1, min(pmax, ny) + 1, dtype=np.float64)
    px = np.arange(1, min(pmax, nx) + 1, dtype=np.float64)
    iy, ix, mag = _mode_order(px, py, r)     # indices into py (rows) / px (cols)
    xg = _interior_nodes(nx)
    yg = _interior_nodes(ny)
    Sx = math.sqrt(2.0 / (nx + 1)) * np.sin(np.pi * px[None, :] * xg[:, None])   # nx x P
    Sy = math.sqrt(2.0 / (ny + 1)) * np.sin(np.pi * py[None, :] * yg[:, None])   # ny x Q
    t = np.arange(m, dtype=np.float64) / max(m - 1, 1)
    lam = py[iy] ** 2 + px[ix] ** 2
    G = np.exp(-np.pi ** 2 * nu * lam[None, :] * t[:, None]) + rng.standard_normal((m, r))
    Ut = _orthonormal_columns(G)
    sigma = np.exp(-rate * np.arange(1, r + 1, dtype=np.float64))
    C = Ut * sigma[None, :]
    # A[t, y, x] = sum_j C[t, j] Sy[y, iy_j] Sx[x, ix_j], as two products over the
    # (q, p) mode grid: M[t, q, p] = sum_j C[t, j] [iy_j = q][ix_j = p]
    nq, npx = Sy.shape[1], Sx.shape[1]
    M = np.zeros((m, nq, npx))
    np.add.at(M, (slice(None), iy, ix), C)
    T1 = M.reshape(m * nq, npx) @ Sx.T                       # (m q) x nx
    A = np.empty((m, ny, nx))
    step = max(1, (1 << 27) // max(1, ny * nx))             # rows per block (bounded temporaries)
    T1 = T1.reshape(m, nq, nx)
    for t0 in range(0, m, step):
        A[t0:t0 + step] = np.einsum("yq,tqx->tyx", Sy, T1[t0:t0 + step], optimize=True)
    A = A.reshape(m, ny * nx)
    if return_parts:
        return A, sigma
    return A


def advdiff_field(m: int, N: int, seed: int, nu: float, kmax: int = 24, alpha: float = 1.0,
                  v=(0.6, 0.35), T: float = 1.0) -> np.ndarray:
    """Physical advection-diffusion snapshots on a periodic N x N grid.

    u(x,y,t) = sum_{|k|<=kmax} c_k exp(-4 pi^2 nu |k|^2 t) cos(2 pi k.(x - v t) + phi_k),
    c_k ~ N(0,1) / (1+|k|)^alpha, phi_k ~ U[0, 2 pi), x on the grid i/N, t_j = T j/(m-1).
    Returns A (m x N*N, float64).
    """
    rng = np.random.default_rng(seed)
    ks = [(kx, ky) for ky in range(-kmax, kmax + 1) for kx in range(0, kmax + 1)
          if (kx > 0 or ky > 0) and kx * kx + ky * ky <= kmax * kmax]
    ks = np.asarray(ks, dtype=np.float64)
    kk = np.sqrt((ks ** 2).sum(1))
    c = rng.standard_normal(len(ks)) / (1.0 + kk) ** alpha
    phi = rng.uniform(0, 2 * np.pi, size=len(ks))
    t = T * np.arange(m, dtype=np.float64) / max(m - 1, 1)
    x = np.arange(N, dtype=np.float64) / N
    # cos(a + b) with a = 2 pi (kx x + ky y), b = phi - 2 pi k.v t
    amp = c[None, :] * np.exp(-4 * np.pi ** 2 * nu * (kk ** 2)[None, :] * t[:, None])
    b = phi[None, :] - 2 * np.pi * (ks @ np.asarray(v, dtype=np.float64))[None, :] * t[:, None]
    # cos(a_x + a_y + b) = Re(z e^{i a_y} e^{i a_x}) with z = amp e^{i b}, a_x = 2 pi kx x,
    # a_y = 2 pi ky y: one grid row y at a time, A(:, y, :) = Re((z * e^{i a_y}) E_x)
    z = amp * np.exp(1j * b)                                  # m x K
    ex = np.exp(2j * np.pi * ks[:, 0][:, None] * x[None, :])  # K x N (x)
    ey = np.exp(2j * np.pi * ks[:, 1][:, None] * x[None, :])  # K x N (y)
    exr, exi = np.ascontiguousarray(ex.real), np.ascontiguousarray(ex.imag)
    zr, zi = np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)
    A = np.empty((m, N, N))
    for y in range(N):
        cr, ci = ey[:, y].real[None, :], ey[:, y].imag[None, :]
        wr = zr * cr - zi * ci                                # Re(z e^{i a_y}), contiguous for BLAS
        wi = zr * ci + zi * cr
        A[:, y, :] = wr @ exr - wi @ exi
    return A.reshape(m, N * N)


def advdiff_field_device(m: int, N: int, seed: int, nu: float, device, kmax: int = 24, alpha: float = 1.0,
                         v=(0.6, 0.35), T: float = 1.0, dtype=None):
    """advdiff_field's snapshots formed on a torch device (the same seeded modes,
    amplitudes and phases, drawn on the host; the sums in FP64 on the device):
    equal to advdiff_field up to rounding.  Returns an m x N*N torch tensor of
    `dtype` (default float64) on `device`."""
    import torch
    rng = np.random.default_rng(seed)
    ks = [(kx, ky) for ky in range(-kmax, kmax + 1) for kx in range(0, kmax + 1)
          if (kx > 0 or ky > 0) and kx * kx + ky * ky <= kmax * kmax]
    ks = np.asarray(ks, dtype=np.float64)
    kk = np.sqrt((ks ** 2).sum(1))
    c = rng.standard_normal(len(ks)) / (1.0 + kk) ** alpha
    phi = rng.uniform(0, 2 * np.pi, size=len(ks))
    f64 = torch.float64
    t = torch.arange(m, dtype=f64, device=device) * (T / max(m - 1, 1))
    x = torch.arange(N, dtype=f64, device=device) / N
    ks_t = torch.from_numpy(ks).to(device)
    kk_t = torch.from_numpy(kk).to(device)
    amp = torch.from_numpy(c).to(device)[None, :] * torch.exp(-4 * np.pi ** 2 * nu * (kk_t ** 2)[None, :] * t[:, None])
    kv = ks_t @ torch.tensor(v, dtype=f64, device=device)
    b = torch.from_numpy(phi).to(device)[None, :] - 2 * np.pi * kv[None, :] * t[:, None]
    zr, zi = amp * torch.cos(b), amp * torch.sin(b)
    ax = 2 * np.pi * ks_t[:, 0][:, None] * x[None, :]
    ay = 2 * np.pi * ks_t[:, 1][:, None] * x[None, :]
    exr, exi = torch.cos(ax).contiguous(), torch.sin(ax).contiguous()
    eyr, eyi = torch.cos(ay), torch.sin(ay)
    out = torch.empty((m, N, N), dtype=dtype or f64, device=device)
    for y in range(N):
        cr, ci = eyr[:, y][None, :], eyi[:, y][None, :]
        wr = zr * cr - zi * ci
        wi = zr * ci + zi * cr
        out[:, y, :] = (wr @ exr - wi @ exi).to(out.dtype)
    return out.reshape(m, N * N)


# The learned-restriction workload: advection-diffusion trajectories (1000
# snapshots of 256 x 256 each) at diffusivities drawn log-uniformly from
# [0.005, 0.05] with a fixed seed for training, and held-out diffusivities for
# validation (the judge) and test.  The velocity (6, 3.5) makes the temporal
# content rich enough that a rank-50 approximation leaves a visible tail
# (about 0.11 of ||A||_F at nu = 0.006, 3e-4 at nu = 0.04).
LEARNED_GRID = 256
LEARNED_ROWS = 1000
LEARNED_VELOCITY = (6.0, 3.5)


def learned_diffusivities(n_train: int = 20, seed: int = 500):
    """(train, validation, test) diffusivity lists of the learned-restriction
    workload; validation and test values are not in the training list."""
    rng = np.random.default_rng(seed)
    train = np.sort(np.exp(rng.uniform(np.log(0.005), np.log(0.05), n_train)))
    return [float(v) for v in train], [0.0083, 0.031], [0.0061, 0.0187, 0.042]


def learned_trajectory(nu: float, seed: int, device, dtype=None, rows: int = LEARNED_ROWS):
    """One trajectory of the learned-restriction workload on a torch device
    (rows x 256^2, FP32 unless dtype is given)."""
    import torch
    return advdiff_field_device(rows, LEARNED_GRID, seed=seed, nu=nu, device=device, kmax=24, alpha=1.0,
                                v=LEARNED_VELOCITY, dtype=dtype or torch.float32)


def lowrank(m: int, n: int, r: int, seed: int) -> np.ndarray:
    """Exact rank-r matrix X Z^T with iid Gaussian factors."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, r)) @ rng.standard_normal((r, n))


def gaussian_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    """rows x cols iid standard normal values from numpy's default_rng(seed)."""
    return np.random.default_rng(seed).standard_normal((rows, cols))


@dataclass
class BatchSpec:
    seed: int
    m: int
    N: int          # grid side, n = N*N
    k: int
    factor: int     # coarse factor per axis
    family: str     # "heat" or "advdiff"


def batch_specs(count: int = 64, base_seed: int = 1000) -> list[BatchSpec]:
    """Ragged batch of snapshot problems, instance i drawn from seed base_seed+i:
    m ~ U[100, 2000], n in {64^2, 128^2, 256^2}, k ~ U[10, 64], factor in {2, 4}."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        m = int(rng.integers(100, 2001))
        N = int(rng.choice([64, 128, 256]))
        k = int(rng.integers(10, 65))
        f = int(rng.choice([2, 4]))
        fam = "heat" if rng.random() < 0.5 else "advdiff"
        out.append(BatchSpec(base_seed + i, m, N, k, f, fam))
    return out


def batch_matrix(spec: BatchSpec) -> np.ndarray:
    """Draw the snapshot matrix of one ragged instance (float64)."""
    if spec.family == "heat":
        return heat_exact(spec.m, spec.N, spec.N, spec.seed, rate=0.05, r=min(spec.m, 200))
    return advdiff_exact(spec.m, spec.N, spec.seed, r=min(spec.m, 400), noise=1e-3)

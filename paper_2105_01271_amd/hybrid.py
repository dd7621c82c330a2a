"""Hybrid deterministic-randomized sketch and the MREO trial harness (Sec. 6).

The hybrid sketch applies a seeded Gaussian s x ell second level to the
deterministic coarse sketch, Y = A_c Omega (the optional random projection of
Alg. 3 and Alg. 5); the sketch entry points take Omega as the S option, so
the random numbers are an input like A.  MREO, the max ratio of error to
oracle over independent trials (Sec. 6), is
    max_t ||A - U_t S_t V_t^T||_F / ||A - A_k||_F,
with A_k the truncated SVD.  For the rank-k outputs of the SVD entry points
U is orthonormal and V S = A^T U (V = B^T U_B S^-1 with B^T = A^T Q, U = Q
U_B), so ||A - U S V^T||_F^2 = ||A||_F^2 - sum_j S_j^2, evaluated from the
device's FP64 ||A||_F^2 and S.  That identity loses accuracy when the error
is below about sqrt(u) ||A||_F (u of the input type); the harness is for the
regime the paper measures, errors well above it.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import dsketch, synth


def gaussian_second_level(s: int, ell: int, seed: int, dtype=torch.float32, device="cuda") -> torch.Tensor:
    """Omega (s x ell) with iid N(0, 1) entries from synth.gaussian_matrix(s, ell, seed)."""
    return torch.from_numpy(synth.gaussian_matrix(s, ell, seed)).to(dtype=dtype, device=device)


def trial_errors(A: torch.Tensor, k: int, R: dsketch.Restriction, trials: int = 100, q: int = 0, seed0: int = 0,
                 single_pass: bool = False, p: int = 10, mode="default") -> np.ndarray:
    """Rank-k Frobenius errors ||A - U S V^T||_F of `trials` hybrid sketch SVDs,
    trial t drawing Omega with seed seed0 + t (TPC-SVD with q power steps, or
    SPC-SVD when single_pass)."""
    m = A.shape[0]
    s = R.coarse_size()
    ell = min(k + p, s, m)
    wd = torch.float64 if A.dtype == torch.float64 else torch.float32
    out = np.empty(trials)
    for t in range(trials):
        S = gaussian_second_level(s, ell, seed0 + t, dtype=wd, device=A.device)
        if single_pass:
            _, Sv, _, info = dsketch.sketch_svd_sp(A, k, R, S=S, mode=mode, want_info=True)
        else:
            _, Sv, _, info = dsketch.sketch_svd(A, k, R, q=q, S=S, mode=mode, want_info=True)
        s2 = float((Sv * Sv).sum().item())
        out[t] = math.sqrt(max(info["normA_fro2"] - s2, 0.0))
    return out


def mreo(errors: np.ndarray, tail_fro: float) -> float:
    """Max ratio of error to oracle: max_t errors[t] / ||A - A_k||_F."""
    return float(np.max(np.asarray(errors)) / tail_fro)

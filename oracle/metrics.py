"""Error metrics of Sec. 6 in FP64.  TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import numpy as np


def fro2(A: np.ndarray) -> float:
    A = np.asarray(A, dtype=np.float64)
    return float(np.sum(A * A))


def rel_fro_error(A: np.ndarray, Ahat: np.ndarray) -> float:
    """||A - Ahat||_F / ||A||_F (Sec. 6, relative Frobenius error)."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A - Ahat) / np.linalg.norm(A))


def svd_error(A, U, s, V) -> float:
    return rel_fro_error(A, (np.asarray(U, np.float64) * np.asarray(s, np.float64)[None, :])
                         @ np.asarray(V, np.float64).T)


def id_error(A, I, P) -> float:
    A = np.asarray(A, dtype=np.float64)
    return rel_fro_error(A, np.asarray(P, np.float64) @ A[np.asarray(I)])


def eckart_young_tail(sigma: np.ndarray, k: int) -> float:
    """||A - A_k||_F = (sum_{i>k} sigma_i^2)^{1/2} (Eckart-Young, Sec. 6)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    return float(np.sqrt(np.sum(sigma[k:] ** 2)))


def ratio_to_oracle(A, Ahat, sigma_full, k) -> float:
    """One trial of MREO (Sec. 6): ||A - Ahat||_F / ||A - A_k||_F."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A - Ahat) / eckart_young_tail(sigma_full, k))


def spectral_norm(M: np.ndarray) -> float:
    return float(np.linalg.norm(np.asarray(M, dtype=np.float64), 2))

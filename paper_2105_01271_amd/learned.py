"""Training loop of the learned linear restriction (extension; not in the paper).

The restriction is two 5x5 stride-2 linear convolutions (1 -> C -> 1 channels)
that map an ny x nx snapshot to ny/4 x nx/4 coarse values, A_c = A D with D
the conv (Sec. 2 with a learned D).  It is trained to shrink the sketch error
that Thm 3.2 bounds, L = ||A - Q Q^T A||_F^2 / ||A||_F^2, with Q the ell-wide
block of the SVD path (start block + q coarse power steps, Alg. 7).  Every
step runs in the library: the loss and its weight gradients
(dsk_learned_loss_grad) and the Adam update (dsk_adam_step); this module only
draws minibatches and loops, and compares the result with direct injection
(the fallback) on validation data.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dsketch


def direct_injection_weights(C: int, noise: float = 0.0, seed: int = 0, device="cuda"):
    """Weights whose conv equals direct injection on the (4, 4) sub-grid:
    centre taps of channel 0 set to one (plus optional seeded noise elsewhere)."""
    rng = np.random.default_rng(seed)
    w1 = noise * rng.standard_normal((C, 5, 5))
    w2 = noise * rng.standard_normal((C, 5, 5))
    w1[0, 2, 2] = 1.0
    w2[0, 2, 2] = 1.0
    return (torch.from_numpy(w1).to(torch.float32).to(device), torch.from_numpy(w2).to(torch.float32).to(device))


def train(A, ny: int, nx: int, C: int = 16, ell: int = 60, q: int = 0, steps: int = 100,
          batch: int = 500, lr: float = 2e-3, seed: int = 0, w1=None, w2=None, log=None, val=None,
          val_every: int = 100):
    """Adam on the projection loss over random row minibatches (rows = snapshots).
    A is one matrix or a list of matrices (e.g. one trajectory per diffusivity):
    each minibatch is a sorted random subset of the rows of one of them, chosen
    at random.  With validation matrices `val`, the projection loss on them is
    taken every val_every steps and the weights with the lowest one are
    returned.  Returns (w1, w2, history of minibatch losses)."""
    mats = list(A) if isinstance(A, (list, tuple)) else [A]
    dev = mats[0].device
    if w1 is None or w2 is None:
        w1, w2 = direct_injection_weights(C, noise=1e-3, seed=seed, device=dev)
    w1 = w1.clone().contiguous()
    w2 = w2.clone().contiguous()
    m1a, m2a = torch.zeros_like(w1), torch.zeros_like(w1)
    m1b, m2b = torch.zeros_like(w2), torch.zeros_like(w2)
    rng = np.random.default_rng(seed)
    hist = []
    vals = (list(val) if isinstance(val, (list, tuple)) else [val]) if val is not None else None
    best = None
    for t in range(1, steps + 1):
        X = mats[int(rng.integers(len(mats)))] if len(mats) > 1 else mats[0]
        m = X.shape[0]
        rows = np.sort(rng.choice(m, size=min(batch, m), replace=False))
        Ab = X[torch.from_numpy(rows).to(dev)].contiguous()
        R = dsketch.Restriction.learned(ny, nx, w1, w2)
        loss, g1, g2 = dsketch.learned_loss_grad(Ab, R, ell, q)
        dsketch.adam_step(w1, g1, m1a, m2a, t, lr=lr)
        dsketch.adam_step(w2, g2, m1b, m2b, t, lr=lr)
        hist.append(loss)
        if log is not None:
            log(t, loss)
        if vals is not None and (t % val_every == 0 or t == steps):
            lv = sum(projection_loss(V, ny, nx, w1, w2, ell, q) for V in vals) / len(vals)
            if best is None or lv < best[0]:
                best = (lv, w1.clone(), w2.clone())
    if best is not None:
        return best[1], best[2], hist
    return w1, w2, hist


def projection_loss(A: torch.Tensor, ny: int, nx: int, w1, w2, ell: int = 60, q: int = 0) -> float:
    """The training loss ||A - Q Q^T A||_F^2 / ||A||_F^2 of the restriction with
    weights (w1, w2) on A (dsk_learned_loss_grad; its gradient is discarded)."""
    loss, _, _ = dsketch.learned_loss_grad(A.contiguous(), dsketch.Restriction.learned(ny, nx, w1, w2), ell, q)
    return float(loss)


def judge(A_val, ny: int, nx: int, w1, w2, ell: int = 60, q: int = 0):
    """Direct injection as fallback and judge: the projection loss of the learned
    restriction and of direct injection on the same (4, 4) coarse grid (the conv
    with only the centre taps of channel 0, i.e. the same s), averaged over the
    validation matrices.  Returns (choice, learned_loss, di_loss), choice
    "learned" only when its loss is strictly lower."""
    mats = list(A_val) if isinstance(A_val, (list, tuple)) else [A_val]
    C = w1.shape[0]
    d1, d2 = direct_injection_weights(C, noise=0.0, device=mats[0].device)
    ll = sum(projection_loss(X, ny, nx, w1, w2, ell, q) for X in mats) / len(mats)
    ld = sum(projection_loss(X, ny, nx, d1, d2, ell, q) for X in mats) / len(mats)
    return ("learned" if ll < ld else "direct_injection"), ll, ld


def restriction_for(choice: str, ny: int, nx: int, w1, w2, device="cuda"):
    """The restriction the judge chose: the learned conv, or direct injection on
    the (4, 4) sub-grid as an index restriction."""
    if choice == "learned":
        return dsketch.Restriction.learned(ny, nx, w1, w2)
    return dsketch.Restriction.di_grid(ny, nx, 4, 4, device=device)

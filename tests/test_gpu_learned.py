"""Learned linear restriction (extension): conv forward / backward, the
projection-loss gradient and a few Adam steps on the GPU against the FP64
oracle (oracle.restrict conv, oracle.learned loss and gradients).

Tolerances: the HIP conv accumulates in FP32 (relative 1e-6 of the output
scale).  The loss gradient runs its coarse algebra in FP64 but takes A_c from
the FP32 conv and, for FP32 input, the two passes over A at FP32 accuracy.
Its sensitivity to such perturbations depends on the conditioning of the
power blocks (every R^{-1} of the chain amplifies them), so the gradient test
uses the slowly decaying advection-diffusion spectrum, where an FP32-level
perturbation of A_c moves the oracle's own gradient by ~2e-6 of its largest
entry: gradients are compared at 1e-5 (FP64 input) and 1e-4 (FP32 input) of
their largest entry, the loss (a number in [0, 1]) at 1e-6 / 1e-5 absolute.
"""
import numpy as np
import pytest
import torch

from oracle import learned as olearn
from oracle import restrict as ores
from oracle import rowid as orid
from oracle import sketch as osk
from paper_2105_01271_amd import synth

pytestmark = pytest.mark.gpu


def dsk():
    from paper_2105_01271_amd import dsketch
    return dsketch


def say(*a):
    print(*a, flush=True)


def _w(C, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((C, 5, 5)) * 0.2, rng.standard_normal((C, 5, 5)) * 0.2


def _R(ny, nx, w1, w2):
    return dsk().Restriction.learned(ny, nx, torch.from_numpy(w1).float().cuda(), torch.from_numpy(w2).float().cuda())


def _oracle_w(w1, w2):
    C = w1.shape[0]
    # the device weights are FP32: the oracle takes exactly those values
    w1 = w1.astype(np.float32).astype(np.float64)
    w2 = w2.astype(np.float32).astype(np.float64)
    return w1.reshape(C, 1, 5, 5), w2.reshape(1, C, 5, 5)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64, torch.bfloat16, torch.float16])
@pytest.mark.parametrize("m,ny,nx,C", [(5, 32, 32, 4), (3, 40, 24, 3), (4, 256, 256, 16), (2, 72, 136, 32)])
def test_conv_forward_matches_oracle(dtype, m, ny, nx, C):
    say("conv fwd", dtype, m, ny, nx, C)
    rng = np.random.default_rng(ny * 3 + nx + C)
    A = torch.from_numpy(rng.standard_normal((m, ny * nx))).to(dtype).cuda()
    w1, w2 = _w(C, C)
    Ac = dsk().restrict(A, _R(ny, nx, w1, w2))
    o1, o2 = _oracle_w(w1, w2)
    ref = ores.conv_restrict(A.double().cpu().numpy(), ny, nx, o1, o2)
    got = Ac.double().cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say("  max rel err", err)
    assert got.shape == ref.shape
    assert err <= 2e-6


@pytest.mark.parametrize("m,ny,nx,C", [(3, 48, 40, 5), (2, 64, 64, 16), (1, 36, 20, 2)])
def test_conv_backward_matches_oracle(m, ny, nx, C):
    say("conv bwd", m, ny, nx, C)
    rng = np.random.default_rng(m + ny + nx + C)
    A = torch.from_numpy(rng.standard_normal((m, ny * nx))).float().cuda()
    w1, w2 = _w(C, C + 1)
    s = (ny // 4) * (nx // 4)
    g = torch.from_numpy(rng.standard_normal((m, s))).float().cuda()
    gw1, gw2 = dsk().conv_restrict_bwd(A, _R(ny, nx, w1, w2), g)
    o1, o2 = _oracle_w(w1, w2)
    r1, r2 = ores.conv_restrict_bwd(A.double().cpu().numpy(), ny, nx, o1, o2, g.double().cpu().numpy())
    e1 = np.abs(gw1.double().cpu().numpy() - r1.reshape(C, 5, 5)).max() / np.abs(r1).max()
    e2 = np.abs(gw2.double().cpu().numpy() - r2.reshape(C, 5, 5)).max() / np.abs(r2).max()
    say("  rel err gw1 / gw2", e1, e2)
    assert e1 <= 1e-5 and e2 <= 1e-5


@pytest.mark.parametrize("dtype,tol,ltol", [(torch.float64, 1e-5, 1e-6), (torch.float32, 1e-4, 1e-5)])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_learned_loss_gradient_matches_oracle(dtype, tol, ltol, q):
    say("learned loss grad", dtype, q)
    m, ny, nx, C, ell = 60, 32, 32, 4, 8
    A_np = synth.advdiff_exact(m, 32, seed=4, r=m)
    A = torch.from_numpy(A_np).to(dtype).cuda()
    w1, w2 = _w(C, 7)
    w1[0, 2, 2] += 1.0
    w2[0, 2, 2] += 1.0
    loss, g1, g2 = dsk().learned_loss_grad(A, _R(ny, nx, w1, w2), ell, q)
    o1, o2 = _oracle_w(w1, w2)
    L, r1, r2 = olearn.learned_loss_and_grad(A.double().cpu().numpy(), ny, nx, o1, o2, ell, q)
    say("  loss gpu / oracle", loss, L)
    assert abs(loss - L) <= ltol
    e1 = np.abs(g1.double().cpu().numpy() - r1.reshape(C, 5, 5)).max() / np.abs(r1).max()
    e2 = np.abs(g2.double().cpu().numpy() - r2.reshape(C, 5, 5)).max() / np.abs(r2).max()
    say("  rel err gw1 / gw2", e1, e2)
    assert e1 <= tol and e2 <= tol


def test_learned_sketch_svd_and_id_match_oracle():
    say("learned sketch svd / id")
    m, ny, nx, C = 80, 64, 64, 4
    A_np = synth.heat_modes(m, 64, seed=9, nu=0.003) + 1e-3 * np.random.default_rng(2).standard_normal((m, 4096))
    A = torch.from_numpy(A_np).cuda()
    w1, w2 = _w(C, 11)
    w1[0, 2, 2] += 1.0
    w2[0, 2, 2] += 1.0
    R = _R(ny, nx, w1, w2)
    o1, o2 = _oracle_w(w1, w2)
    Ro = {"kind": "learned", "ny": ny, "nx": nx, "w1": o1, "w2": o2}
    U, S, V = dsk().sketch_svd(A, 10, R, q=1)
    Uo, So, Vo = osk.tpc_svd(A_np, 10, Ro, q=1)
    err = np.abs(S.cpu().numpy() - So).max() / So[0]
    say("  sigma err", err)
    assert err <= 1e-6
    I, P = dsk().sketch_id(A, 10, R, q=0)
    Io, Po, info = orid.tpc_id(A_np, 10, Ro, q=0, return_all=True)
    gaps = info["gaps"]
    npre = 0
    for r1, r2 in gaps:   # the FP32 conv perturbs A_c at ~1e-7 relative: pivots must agree while separated by more
        if r1 <= 0 or not ((r1 - r2) / r1 > 1e-5):
            break
        npre += 1
    say("  separated prefix", npre)
    assert list(I.cpu().numpy()[:npre]) == list(Io[:npre])


def test_adam_training_tracks_oracle_and_reduces_loss():
    say("learned training")
    m, ny, nx, C, ell, q = 64, 32, 32, 4, 8, 0
    A_np = synth.advdiff_exact(m, 32, seed=6, r=m)
    A = torch.from_numpy(A_np).float().cuda()
    A_up = A.double().cpu().numpy()
    from paper_2105_01271_amd import learned
    w1, w2 = learned.direct_injection_weights(C, noise=1e-2, seed=5)
    # CPU reference: oracle gradients + Adam written out here, same hyper-parameters
    r1 = w1.double().cpu().numpy()
    r2 = w2.double().cpu().numpy()
    mo = [np.zeros_like(r1), np.zeros_like(r1), np.zeros_like(r2), np.zeros_like(r2)]
    lr, b1, b2, eps = 2e-3, 0.9, 0.999, 1e-8
    ref_hist = []
    for t in range(1, 6):
        L, g1, g2 = olearn.learned_loss_and_grad(A_up, ny, nx, r1.reshape(C, 1, 5, 5), r2.reshape(1, C, 5, 5), ell, q)
        ref_hist.append(L)
        for i, (p, g) in enumerate(((r1, g1.reshape(C, 5, 5)), (r2, g2.reshape(C, 5, 5)))):
            mo[2 * i] = b1 * mo[2 * i] + (1 - b1) * g
            mo[2 * i + 1] = b2 * mo[2 * i + 1] + (1 - b2) * g * g
            p -= lr * (mo[2 * i] / (1 - b1 ** t)) / (np.sqrt(mo[2 * i + 1] / (1 - b2 ** t)) + eps)
    _, _, hist = learned.train(A, ny, nx, C=C, ell=ell, q=q, steps=5, batch=m, lr=lr, w1=w1, w2=w2)
    say("  gpu", hist)
    say("  ref", ref_hist)
    for a, b in zip(hist, ref_hist):
        assert abs(a - b) <= 1e-5
    _, _, hist30 = learned.train(A, ny, nx, C=C, ell=ell, q=q, steps=30, batch=m, lr=1e-2, w1=w1, w2=w2)
    say("  30 steps", hist30[0], hist30[-1])
    assert hist30[-1] < hist30[0]


def test_learned_restriction_against_direct_injection_at_held_out_diffusivities():
    # The learned-restriction workload: training on 20 trajectories (20000 rows of
    # 256^2) at seeded diffusivities in [0.005, 0.05], 600 Adam steps, each on one
    # whole trajectory (ell = 60, q = 1), keeping the weights with the lowest
    # loss on two held-out validation trajectories (checked every 100 steps);
    # direct injection on the same (4, 4) grid (s = 4096) is the judge on those
    # trajectories and the fallback; then the rank-50 sketch SVD (q = 1) at three
    # held-out test diffusivities.  Measured: training lowers the projection loss
    # on the validation trajectories by a quarter to a third against direct
    # injection's, so the judge keeps the learned conv; the rank-50 error at the
    # held-out diffusivities moves between 1% worse and 7% better than direct
    # injection's depending on the training run (0.1128 to 0.1220 against
    # 0.1209 at nu = 0.0061; optimum 0.1098; rounding-level changes in the
    # library's reductions are enough to move a run within that range): no
    # robust gain on this workload, and no loss beyond a few percent.  The
    # assertions keep to what held in every run.
    from paper_2105_01271_amd import learned
    say("learned vs direct injection")
    dev = torch.device("cuda")
    N, k, ell, q = synth.LEARNED_GRID, 50, 60, 1
    tr, va, te = synth.learned_diffusivities()
    train = [synth.learned_trajectory(nu, 1000 + i, dev) for i, nu in enumerate(tr)]
    val = [synth.learned_trajectory(nu, 2000 + i, dev) for i, nu in enumerate(va)]
    w1, w2, hist = learned.train(train, N, N, C=16, ell=ell, q=q, steps=600, batch=1000, lr=2e-3, seed=0, val=val)
    say(f"  minibatch loss first 20 {np.mean(hist[:20]):.3e} last 20 {np.mean(hist[-20:]):.3e}")
    del train
    choice, ll, ld = learned.judge(val, N, N, w1, w2, ell, q)
    say(f"  judge: {choice} (validation loss learned {ll:.4e}, direct injection {ld:.4e})")
    assert (choice == "learned") == (ll < ld)
    R = learned.restriction_for(choice, N, N, w1, w2)
    Rdi = dsk().Restriction.di_grid(N, N, 4, 4)

    def err(A, R):
        U, S, V = dsk().sketch_svd(A, k, R, q=q)
        A64 = A.double()
        E = A64 - (U.double() * S.double()[None, :]) @ V.double().T
        return float(torch.linalg.norm(E) / torch.linalg.norm(A64))

    e_sel, e_di = [], []
    for i, nu in enumerate(te):
        A = synth.learned_trajectory(nu, 3000 + i, dev)
        s = torch.linalg.svdvals(A.double())
        opt = float(torch.sqrt((s[k:] ** 2).sum() / (s ** 2).sum()))
        e_sel.append(err(A, R))
        e_di.append(err(A, Rdi))
        say(f"  test nu {nu}: optimal {opt:.4e} direct injection {e_di[-1]:.4e} chosen {e_sel[-1]:.4e}")
        assert e_sel[-1] >= opt * (1 - 1e-6)
    assert ll < ld and choice == "learned"
    gains = [1.0 - a / b for a, b in zip(e_sel, e_di)]
    say("  relative change of the rank-50 error against direct injection:", [f"{g:+.4f}" for g in gains])
    assert all(g >= -0.03 for g in gains)

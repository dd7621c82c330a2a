"""Python binding of libdsketch: argument marshalling only.

Each function has the name of a C entry point of include/dsketch.h and passes
torch tensors to it as raw device pointers together with torch's current HIP
stream.  Every step of the computation runs in the library's HIP kernels;
torch provides device memory and streams.  There is no CPU path: without a
GPU and the built library every call raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

_DT = {torch.float64: _lib.DSK_F64, torch.float32: _lib.DSK_F32,
       torch.bfloat16: _lib.DSK_BF16, torch.float16: _lib.DSK_F16}
_MODES = {"default": _lib.DSK_MODE_DEFAULT, "split3": _lib.DSK_MODE_SPLIT3, "f32": _lib.DSK_MODE_F32,
          "split6": _lib.DSK_MODE_SPLIT6}

_handles: dict = {}
DSK_ERR_SCRATCH = 90   # dsk_project_noalloc: size beyond its fixed scratch


def _handle(device: torch.device):
    lib = _lib.load()
    idx = device.index if device.index is not None else torch.cuda.current_device()
    h = _handles.get(idx)
    if h is None:
        hp = ctypes.c_void_p()
        _lib.check("dsk_create", lib.dsk_create(ctypes.byref(hp), idx, None))
        h = hp
        _handles[idx] = h
    stream = torch.cuda.current_stream(idx).cuda_stream
    _lib.check("dsk_set_stream", lib.dsk_set_stream(h, ctypes.c_void_p(stream)))
    return h


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _work_dtype(dt: torch.dtype) -> torch.dtype:
    return torch.float64 if dt == torch.float64 else torch.float32


def _check_second_level(S, A: torch.Tensor, R: "Restriction"):
    """S (s x ell) must be a contiguous device tensor in A's work dtype: the
    library reads it through a plain pointer with that element size."""
    if S is None:
        return
    if not isinstance(S, torch.Tensor) or not S.is_cuda or S.dim() != 2 or not S.is_contiguous():
        raise ValueError("S must be a contiguous 2-D device tensor")
    if S.dtype != _work_dtype(A.dtype):
        raise ValueError(f"S must have dtype {_work_dtype(A.dtype)} (the work dtype of A)")
    if S.shape[0] != R.coarse_size():
        raise ValueError(f"S must have {R.coarse_size()} rows (the coarse size)")


def _check_matrix(A: torch.Tensor):
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D row-major tensor (unit column stride)")
    if A.dtype not in _DT:
        raise ValueError(f"unsupported dtype {A.dtype}")


@dataclass
class Restriction:
    """Host description of the sketch D of A_c = A D (paper Sec. 2).

    kind: "index" (direct injection / Gram sub-sample), "nn", "global",
    "learned" (two 5x5 stride-2 linear conv layers, w1 and w2 of shape (C, 5, 5)).
    """
    kind: str
    index: torch.Tensor | None = None      # device int64 (s,)
    ny: int = 0
    nx: int = 0
    sy: int = 1
    sx: int = 1
    w1: torch.Tensor | None = None         # learned: device float32 (C, 5, 5)
    w2: torch.Tensor | None = None         # learned: device float32 (C, 5, 5)

    @staticmethod
    def di_grid(ny: int, nx: int, sy: int, sx: int, device="cuda") -> "Restriction":
        """Direct injection on a y-major ny x nx grid: coarse nodes (sy*b, sx*a)."""
        ys = np.arange(0, ny, sy, dtype=np.int64)
        xs = np.arange(0, nx, sx, dtype=np.int64)
        idx = (ys[:, None] * nx + xs[None, :]).reshape(-1)
        return Restriction("index", torch.from_numpy(idx).to(device), ny, nx, sy, sx)

    @staticmethod
    def from_index(index, device="cuda") -> "Restriction":
        t = torch.as_tensor(index, dtype=torch.int64).to(device)
        return Restriction("index", t)

    @staticmethod
    def nn(ny, nx, sy, sx) -> "Restriction":
        return Restriction("nn", None, ny, nx, sy, sx)

    @staticmethod
    def global_(ny, nx, sy, sx) -> "Restriction":
        return Restriction("global", None, ny, nx, sy, sx)

    @staticmethod
    def learned(ny, nx, w1: torch.Tensor, w2: torch.Tensor) -> "Restriction":
        """Learned linear conv restriction (ny/4 x nx/4 coarse values per row)."""
        w1 = w1.detach().to(torch.float32).contiguous()
        w2 = w2.detach().to(torch.float32).contiguous()
        if w1.shape != w2.shape or w1.dim() != 3 or tuple(w1.shape[1:]) != (5, 5) or not w1.is_cuda:
            raise ValueError("w1, w2 must be device tensors of shape (C, 5, 5)")
        return Restriction("learned", None, ny, nx, 4, 4, w1, w2)

    def coarse_size(self) -> int:
        if self.kind == "index":
            return int(self.index.numel())
        if self.kind == "learned":
            return (self.ny // 4) * (self.nx // 4)
        return (-(-self.ny // self.sy)) * (-(-self.nx // self.sx))

    def to_c(self) -> _lib.Restriction:
        r = _lib.Restriction()
        r.kind = {"index": _lib.DSK_R_INDEX, "nn": _lib.DSK_R_NN, "global": _lib.DSK_R_GLOBAL,
                  "learned": _lib.DSK_R_LEARNED}[self.kind]
        if self.kind == "index":
            r.s = int(self.index.numel())
            r.index = self.index.data_ptr()
        r.ny, r.nx, r.sy, r.sx = self.ny, self.nx, self.sy, self.sx
        if self.kind == "learned":
            r.channels = int(self.w1.shape[0])
            r.w1 = self.w1.data_ptr()
            r.w2 = self.w2.data_ptr()
        return r


def _opts(p=10, S=None, tau=None, id_projected=False, mode="default", refine=False, id_per_step=False):
    lib = _lib.load()
    o = _lib.Opts()
    lib.dsk_opts_default(ctypes.byref(o))
    o.p = int(p)
    if S is not None:
        o.S = S.data_ptr()
        o.ell = int(S.shape[1])
    o.tau = float(tau) if tau is not None else 0.0
    o.id_projected = int(bool(id_projected))
    o.mode = _MODES[mode] if isinstance(mode, str) else int(mode)
    o.refine = int(bool(refine))
    o.id_per_step = int(bool(id_per_step))
    return o


def _info_dict(info: _lib.Info) -> dict:
    return {"ell": info.ell, "flags": info.flags,
            "flag_names": [v for b, v in _lib.FLAG_NAMES.items() if info.flags & b],
            "normA_fro2": info.normA_fro2, "normB_fro2": info.normB_fro2, "sigma_tail": info.sigma_tail,
            "core_sweeps": info.core_sweeps}


def restrict(A: torch.Tensor, R: Restriction) -> torch.Tensor:
    """A_c = A D (dsk_restrict)."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    s = R.coarse_size()
    Ac = torch.empty((m, s), dtype=_work_dtype(A.dtype), device=A.device)
    rc = R.to_c()
    _lib.check("dsk_restrict", lib.dsk_restrict(_handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0),
                                                ctypes.byref(rc), _ptr(Ac)))
    return Ac


def project(A: torch.Tensor, Q: torch.Tensor, mode="default") -> torch.Tensor:
    """B^T = A^T Q (dsk_project); returns the n x ell matrix B^T."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    Q = Q.contiguous()
    ell = Q.shape[1]
    Bt = torch.empty((n, ell), dtype=_work_dtype(A.dtype), device=A.device)
    _lib.check("dsk_project", lib.dsk_project(_handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0), _ptr(Q),
                                              ell, _ptr(Bt), _MODES[mode] if isinstance(mode, str) else int(mode)))
    return Bt


def project_noalloc(A: torch.Tensor, Q: torch.Tensor, Bt: torch.Tensor, mode="default") -> int:
    """B^T = A^T Q into the caller's Bt (n x ell, work dtype) by dsk_project_noalloc:
    no device allocation in the call (the handle must exist: create it beforehand with
    handle(device)).  Returns the status (0, or DSK_ERR_SCRATCH when the size's plan
    exceeds the fixed scratch); argument errors raise."""
    lib = _lib.load()
    m, n = A.shape
    st = lib.dsk_project_noalloc(_handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0), _ptr(Q),
                                 Q.shape[1], _ptr(Bt), _MODES[mode] if isinstance(mode, str) else int(mode))
    if st not in (0, DSK_ERR_SCRATCH):
        _lib.check("dsk_project_noalloc", st)
    return st


def handle(device: torch.device):
    """The library handle of `device` (created on first use; creating it is the
    set-up the allocation-free entry point relies on)."""
    return _handle(device)


def sketch_svd(A: torch.Tensor, k: int, R: Restriction, q: int = 0, p: int = 10, S=None, tau=None,
               mode="default", refine=False, want_info: bool = False):
    """Rank-k SVD by TPC-SVD + C-PWR (dsk_sketch_svd).  Returns U (m x k), S (k, f64), V (n x k)[, info]."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    wd = _work_dtype(A.dtype)
    U = torch.empty((m, k), dtype=wd, device=A.device)
    Sv = torch.empty((k,), dtype=torch.float64, device=A.device)
    V = torch.empty((n, k), dtype=wd, device=A.device)
    _check_second_level(S, A, R)
    o = _opts(p=p, S=S, tau=tau, mode=mode, refine=refine)
    rc = R.to_c()
    info = _lib.Info()
    st = lib.dsk_sketch_svd(_handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0), int(k), ctypes.byref(rc),
                            int(q), ctypes.byref(o), _ptr(U), _ptr(Sv), _ptr(V),
                            ctypes.byref(info) if want_info else None)
    _lib.check("dsk_sketch_svd", st)
    if want_info:
        return U, Sv, V, _info_dict(info)
    return U, Sv, V


def sketch_svd_sp(A: torch.Tensor, k: int, R: Restriction, p: int = 10, S=None, mode="default",
                  want_info: bool = False):
    """Rank-k SVD by the single-pass SPC-SVD (dsk_sketch_svd_sp, Alg. 3).
    Returns U (m x k), S (k, f64), V (n x k)[, info]."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    wd = _work_dtype(A.dtype)
    U = torch.empty((m, k), dtype=wd, device=A.device)
    Sv = torch.empty((k,), dtype=torch.float64, device=A.device)
    V = torch.empty((n, k), dtype=wd, device=A.device)
    _check_second_level(S, A, R)
    o = _opts(p=p, S=S, mode=mode)
    rc = R.to_c()
    info = _lib.Info()
    st = lib.dsk_sketch_svd_sp(_handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0), int(k),
                               ctypes.byref(rc), ctypes.byref(o), _ptr(U), _ptr(Sv), _ptr(V),
                               ctypes.byref(info) if want_info else None)
    _lib.check("dsk_sketch_svd_sp", st)
    if want_info:
        return U, Sv, V, _info_dict(info)
    return U, Sv, V


def spc_id_err(A: torch.Tensor, R: Restriction, mc: int, taus, with_rho: bool = False):
    """SPC-ID-ERR (dsk_spc_id_err, Alg. 6) at the given scales: eps_hat(tau) for
    each tau (float64 device tensor); with_rho=True also returns the estimate of
    rho(tau) = ||A_f A_f^T - tau A_c A_c^T||_2 from the same kept rows."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    t = torch.as_tensor(taus, dtype=torch.float64).to(A.device).contiguous()
    eps = torch.empty_like(t)
    rho = torch.empty_like(t) if with_rho else None
    rc = R.to_c()
    _lib.check("dsk_spc_id_err", lib.dsk_spc_id_err(_handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0),
                                                    ctypes.byref(rc), int(mc), _ptr(t), int(t.numel()), _ptr(eps),
                                                    _ptr(rho)))
    return (eps, rho) if with_rho else eps


def sketch_id(A: torch.Tensor, k: int, R: Restriction, q: int = 0, p: int = 10, S=None, tau=None,
              projected=False, skeleton_rows=False, want_info: bool = False, per_step: bool = False):
    """Rank-k row ID by TPC-ID (dsk_sketch_id).  Returns I (k, int64), P (m x k, f64)[, A(I,:)][, info].
    per_step: run the pivoted QR as one launch per pivot step even where the one-launch form fits."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    I = torch.empty((k,), dtype=torch.int64, device=A.device)
    P = torch.empty((m, k), dtype=torch.float64, device=A.device)
    rows = torch.empty((k, n), dtype=A.dtype, device=A.device) if skeleton_rows else None
    _check_second_level(S, A, R)
    o = _opts(p=p, S=S, tau=tau, id_projected=projected, id_per_step=per_step)
    rc = R.to_c()
    info = _lib.Info()
    st = lib.dsk_sketch_id(_handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0), int(k), ctypes.byref(rc),
                           int(q), ctypes.byref(o), _ptr(I), _ptr(P), _ptr(rows),
                           ctypes.byref(info) if want_info else None)
    _lib.check("dsk_sketch_id", st)
    out = [I, P]
    if skeleton_rows:
        out.append(rows)
    if want_info:
        out.append(_info_dict(info))
    return tuple(out)


def spc_id(A: torch.Tensor, k: int, r: int, R: Restriction, qc: int = 24, factors: bool = False,
           want_info: bool = False):
    """Rank-k row ID by the single-pass SPC-ID (dsk_spc_id, Alg. 5): A ~ P X with
    X = A_c(I, :) T_r the lifted skeleton rows (k x n, work dtype).  Returns I, P, X
    [, V_r (s x r), W_r (r x n) with T_r = V_r W_r][, info]."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    wdt = torch.float64 if A.dtype == torch.float64 else torch.float32
    s = R.coarse_size()
    I = torch.empty((k,), dtype=torch.int64, device=A.device)
    P = torch.empty((m, k), dtype=torch.float64, device=A.device)
    X = torch.empty((k, n), dtype=wdt, device=A.device)
    Vr = torch.empty((s, r), dtype=wdt, device=A.device) if factors else None
    Wr = torch.empty((r, n), dtype=wdt, device=A.device) if factors else None
    o = _opts()
    rc = R.to_c()
    info = _lib.Info()
    st = lib.dsk_spc_id(_handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0), int(k), int(r),
                        ctypes.byref(rc), int(qc), ctypes.byref(o), _ptr(I), _ptr(P), _ptr(X), _ptr(Vr), _ptr(Wr),
                        ctypes.byref(info) if want_info else None)
    _lib.check("dsk_spc_id", st)
    out = [I, P, X]
    if factors:
        out += [Vr, Wr]
    if want_info:
        out.append(_info_dict(info))
    return tuple(out)


def timing_enable(enable: bool = True, device="cuda"):
    """Bracket each projection kernel (B^T = A^T Q) with HIP events (dsk_timing_enable)."""
    lib = _lib.load()
    _lib.check("dsk_timing_enable", lib.dsk_timing_enable(_handle(torch.device(device)), int(bool(enable))))


def timing_read(device="cuda"):
    """(launches, total milliseconds) of the timed projection kernels since the last read."""
    lib = _lib.load()
    cnt = ctypes.c_int()
    ms = ctypes.c_double()
    _lib.check("dsk_timing_read", lib.dsk_timing_read(_handle(torch.device(device)), ctypes.byref(cnt),
                                                      ctypes.byref(ms)))
    return cnt.value, ms.value


def power_iter(Ac: torch.Tensor, Q0: torch.Tensor, q: int, tau: float = 1.0, reorth: bool = True) -> torch.Tensor:
    """C-PWR loop alone (dsk_power_iter)."""
    _check_matrix(Ac)
    lib = _lib.load()
    m, s = Ac.shape
    Q0 = Q0.contiguous().to(Ac.dtype)
    ell = Q0.shape[1]
    Qout = torch.empty_like(Q0)
    st = lib.dsk_power_iter(_handle(Ac.device), _ptr(Ac), _DT[Ac.dtype], m, s, Ac.stride(0), _ptr(Q0), ell, int(q),
                            float(tau), int(bool(reorth)), _ptr(Qout))
    _lib.check("dsk_power_iter", st)
    return Qout


def conv_restrict_bwd(A: torch.Tensor, R: Restriction, gAc: torch.Tensor):
    """Weight gradients (gw1, gw2) of sum(gAc * restrict(A, R)) for a learned R (dsk_conv_restrict_bwd)."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    gAc = gAc.contiguous()
    if gAc.dtype != torch.float32 or tuple(gAc.shape) != (m, R.coarse_size()):
        raise ValueError("gAc must be float32 of shape (m, s)")
    gw1 = torch.empty_like(R.w1)
    gw2 = torch.empty_like(R.w2)
    rc = R.to_c()
    _lib.check("dsk_conv_restrict_bwd", lib.dsk_conv_restrict_bwd(
        _handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0), ctypes.byref(rc), _ptr(gAc), _ptr(gw1),
        _ptr(gw2)))
    return gw1, gw2


def learned_loss_grad(A: torch.Tensor, R: Restriction, ell: int, q: int = 0):
    """Projection loss ||A - Q Q^T A||_F^2 / ||A||_F^2 of the learned sketch and its weight
    gradients (dsk_learned_loss_grad).  Returns (loss: float, gw1, gw2)."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    gw1 = torch.empty_like(R.w1)
    gw2 = torch.empty_like(R.w2)
    loss = ctypes.c_double()
    rc = R.to_c()
    _lib.check("dsk_learned_loss_grad", lib.dsk_learned_loss_grad(
        _handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0), ctypes.byref(rc), int(ell), int(q),
        ctypes.byref(loss), _ptr(gw1), _ptr(gw2)))
    return loss.value, gw1, gw2


def adam_step(param: torch.Tensor, grad: torch.Tensor, m1: torch.Tensor, m2: torch.Tensor, step: int,
              lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One in-place Adam update of a float32 device tensor (dsk_adam_step)."""
    lib = _lib.load()
    for t in (param, grad, m1, m2):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != param.numel():
            raise ValueError("adam_step needs contiguous float32 tensors of equal size")
    _lib.check("dsk_adam_step", lib.dsk_adam_step(_handle(param.device), _ptr(param), _ptr(grad), _ptr(m1), _ptr(m2),
                                                  param.numel(), float(lr), float(beta1), float(beta2), float(eps),
                                                  int(step)))


def sketch_svd_batched(problems, p: int = 10, mode="default", graph: bool = False):
    """dsk_sketch_svd for a list of (A, k, R, q) problems in one call (dsk_sketch_svd_batched):
    concurrent worker streams, optionally captured into a HIP graph and replayed on later calls
    with the same tensors.  Returns [(U, S, V), ...]."""
    lib = _lib.load()
    if not problems:
        return []
    dev = problems[0][0].device
    arr = (_lib.Problem * len(problems))()
    outs = []
    keep = []
    for i, (A, k, R, q) in enumerate(problems):
        _check_matrix(A)
        m, n = A.shape
        wd = _work_dtype(A.dtype)
        U = torch.empty((m, k), dtype=wd, device=dev)
        Sv = torch.empty((k,), dtype=torch.float64, device=dev)
        V = torch.empty((n, k), dtype=wd, device=dev)
        pr = arr[i]
        pr.A, pr.dtype, pr.m, pr.n, pr.lda = _ptr(A), _DT[A.dtype], m, n, A.stride(0)
        pr.k, pr.q = int(k), int(q)
        pr.R = R.to_c()
        pr.U, pr.S, pr.V = _ptr(U), _ptr(Sv), _ptr(V)
        outs.append((U, Sv, V))
        keep.append(R)
    o = _opts(p=p, mode=mode)
    nw = ctypes.c_int32()
    st = lib.dsk_sketch_svd_batched(_handle(dev), len(problems), arr, ctypes.byref(o),
                                    _lib.DSK_BATCH_GRAPH if graph else 0, ctypes.byref(nw))
    _lib.check("dsk_sketch_svd_batched", st)
    return outs


class BatchedSVD:
    """A fixed batch whose outputs are allocated once, so that repeated calls replay
    one captured HIP graph (dsk_sketch_svd_batched with DSK_BATCH_GRAPH)."""

    def __init__(self, problems, p: int = 10, mode="default"):
        self._lib = _lib.load()
        self.dev = problems[0][0].device
        self.arr = (_lib.Problem * len(problems))()
        self.outs = []
        self._keep = []
        for i, (A, k, R, q) in enumerate(problems):
            _check_matrix(A)
            m, n = A.shape
            wd = _work_dtype(A.dtype)
            U = torch.empty((m, k), dtype=wd, device=self.dev)
            Sv = torch.empty((k,), dtype=torch.float64, device=self.dev)
            V = torch.empty((n, k), dtype=wd, device=self.dev)
            pr = self.arr[i]
            pr.A, pr.dtype, pr.m, pr.n, pr.lda = _ptr(A), _DT[A.dtype], m, n, A.stride(0)
            pr.k, pr.q = int(k), int(q)
            pr.R = R.to_c()
            pr.U, pr.S, pr.V = _ptr(U), _ptr(Sv), _ptr(V)
            self.outs.append((U, Sv, V))
            self._keep.append((A, R))
        self.opts = _opts(p=p, mode=mode)
        self.nworkers = 0

    def __call__(self, graph: bool = True):
        nw = ctypes.c_int32()
        st = self._lib.dsk_sketch_svd_batched(_handle(self.dev), len(self.outs), self.arr, ctypes.byref(self.opts),
                                              _lib.DSK_BATCH_GRAPH if graph else 0, ctypes.byref(nw))
        _lib.check("dsk_sketch_svd_batched", st)
        self.nworkers = nw.value
        return self.outs


def autotune(A: torch.Tensor, ell: int, mode="default"):
    """Tune the K-split of the projection B^T = A^T Q for A's shape (dsk_autotune).
    Returns (nsplit, milliseconds per projection)."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    ns = ctypes.c_int32()
    ms = ctypes.c_float()
    _lib.check("dsk_autotune", lib.dsk_autotune(_handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0), int(ell),
                                                _MODES[mode] if isinstance(mode, str) else int(mode),
                                                ctypes.byref(ns), ctypes.byref(ms)))
    return ns.value, ms.value


def sketch_svd_id(A: torch.Tensor, k: int, R: Restriction, q_svd: int = 1, q_id: int = 0, p: int = 10,
                  skeleton_rows: bool = False, mode="default"):
    """Sketch SVD and row ID of the same matrix in one call (dsk_sketch_svd_id): the ID runs on a
    worker stream concurrently with the SVD.  Returns (U, S, V, I, P[, A(I,:)])."""
    _check_matrix(A)
    lib = _lib.load()
    m, n = A.shape
    wd = _work_dtype(A.dtype)
    U = torch.empty((m, k), dtype=wd, device=A.device)
    Sv = torch.empty((k,), dtype=torch.float64, device=A.device)
    V = torch.empty((n, k), dtype=wd, device=A.device)
    I = torch.empty((k,), dtype=torch.int64, device=A.device)
    P = torch.empty((m, k), dtype=torch.float64, device=A.device)
    rows = torch.empty((k, n), dtype=A.dtype, device=A.device) if skeleton_rows else None
    o = _opts(p=p, mode=mode)
    rc = R.to_c()
    st = lib.dsk_sketch_svd_id(_handle(A.device), _ptr(A), _DT[A.dtype], m, n, A.stride(0), int(k), ctypes.byref(rc),
                               int(q_svd), int(q_id), ctypes.byref(o), _ptr(U), _ptr(Sv), _ptr(V), _ptr(I), _ptr(P),
                               _ptr(rows), None, None)
    _lib.check("dsk_sketch_svd_id", st)
    out = [U, Sv, V, I, P]
    if skeleton_rows:
        out.append(rows)
    return tuple(out)

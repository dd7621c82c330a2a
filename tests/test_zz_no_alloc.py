"""dsk_project_noalloc, the allocation-free variant of dsk_project (B^T = A^T Q,
the one full pass of Alg. 2): through the C ABI it gives the same bytes as
dsk_project (same kernels, same launch plan) on two calls in a row, the second
smaller and ragged, for every work path (16-bit and FP32 inputs on the packed-Q
MFMA kernel, FP64 with the pass split over the rows of A, whose partials then
sit in the fixed scratch); a size whose plan exceeds the fixed scratch is
refused before anything is enqueued; the call changes no device allocation."""
import pytest
import torch

from paper_2105_01271_amd import dsketch

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")

# (m, n, ell): the full-size projection of each path first, then a smaller, ragged one
CASES = {
    torch.bfloat16: [(2000, 262144, 110), (333, 10007, 37)],
    torch.float32: [(1000, 65536, 60), (257, 4099, 21)],
    torch.float64: [(200, 4096, 30), (61, 1031, 9)],
}


def _inputs(m, n, ell, dtype, seed):
    g = torch.Generator().manual_seed(seed)
    wd = torch.float64 if dtype == torch.float64 else torch.float32
    A = torch.randn(m, n, generator=g, dtype=torch.float32).to(dtype).to(DEV)
    Q = torch.randn(m, ell, generator=g, dtype=torch.float64).to(wd).to(DEV)
    return A, Q


@pytest.mark.parametrize("dtype", list(CASES), ids=lambda d: str(d).split(".")[-1])
def test_noalloc_projection_equals_dsk_project(dtype):
    dsketch.handle(DEV)
    for i, (m, n, ell) in enumerate(CASES[dtype]):
        print(f"noalloc {dtype} m={m} n={n} ell={ell}", flush=True)
        A, Q = _inputs(m, n, ell, dtype, 11 + i)
        ref = dsketch.project(A, Q)
        out = torch.full_like(ref, float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info(DEV)[0]
        st = dsketch.project_noalloc(A, Q, out)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info(DEV)[0]
        assert st == 0
        assert free1 == free0, "the allocation-free projection changed free device memory"
        assert torch.equal(out, ref), (out - ref).abs().max().item()


def test_noalloc_projection_refuses_sizes_beyond_its_scratch():
    dsketch.handle(DEV)
    # F32, m = 50000, ell = 112: the packed Q alone is 1563 * 7 * 3 KiB > 32 MiB
    A, Q = _inputs(50000, 64, 112, torch.float32, 5)
    out = torch.full((64, 112), float("nan"), device=DEV)
    st = dsketch.project_noalloc(A, Q, out)
    torch.cuda.synchronize()
    assert st == dsketch.DSK_ERR_SCRATCH
    assert torch.isnan(out).all()
    # dsk_project itself takes the size (its arena grows)
    ref = dsketch.project(A, Q)
    torch.cuda.synchronize()
    assert torch.isfinite(ref).all()

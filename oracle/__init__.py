"""Plain FP64 CPU reference of the deterministic-sketch low-rank method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package; the
product path never does, and it shares no code with the HIP implementation.

Source: Dunton & Doostan, "Deterministic matrix sketches for low-rank
compression of high-dimensional simulation data" (arXiv 2105.01271).
Each function cites the section / algorithm / equation it follows.  Every
step is written out in float64 NumPy; LAPACK is used only for small dense
primitives (thin QR, SVD, triangular solve, symmetric eigenvalues), exactly
as the algorithms name them.

Modules
  restrict   deterministic sketches D (Sec. 2) and the learned linear conv
  sketch     TPC-SVD (Alg. 2), C-PWR (Alg. 7), SPC-SVD (Alg. 3), PROTO-TPC (Alg. 1)
  rowid      column-pivoted QR row ID (Sec. 4), TPC-ID (Alg. 4),
             SPC-ID (Alg. 5), SPC-ID-ERR (Alg. 6)
  metrics    relative Frobenius error, Eckart-Young tail, MREO ratio (Sec. 6)
  learned    projection loss of a learned restriction and its gradients

Parity status: every function here is pinned by a `-m "not gpu"` test
against an independent fact (brute-force SVD, closed-form spectra, explicit
sketch matrices from the equations, greedy-projection pivots, finite
differences).  None is "parity unpinned".
"""
from . import restrict, sketch, rowid, metrics, learned  # noqa: F401

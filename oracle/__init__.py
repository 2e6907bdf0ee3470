"""FP64 CPU oracle for the MMGKS-OF hot path (test infrastructure only).

This package is the checker, not the product.  Only the test-suite, the smoke
check of the package entry file and the ``cpu_baseline`` leg of the benchmark
may import it.  It shares no code with the HIP library: every operator below is
written out from the paper's definitions (or from the stated reading where the
paper is silent), in float64, with library primitives (sparse matrices, QR,
dense solves) used only as single steps.

Modules
-------
forward   H: parallel-beam Radon (hat model) and 9x9 Gaussian blur   (Sec. 2.1)
regops    Psi from eq. (L); motion matrices M(s), M-bar, M-bar' (Sec. 3, eq. m_matrix)
          and the derivative of the bilinear warp with respect to the flow
optflow   App. C image derivatives, Horn-Schunck flow update (eq. of_reg, p=q=2),
          reverse flow (Remark on estimating the reverse optical flow)
mmgks     MM weights, Golub-Kahan start, discrepancy principle, MMGKS-OF (Alg. 1)
"""
from . import forward, regops, optflow, mmgks  # noqa: F401

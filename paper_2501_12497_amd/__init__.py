"""MI355X (gfx950) implementation of the MMGKS-OF hot path.

The compute lives in the HIP library libmmof.so (sources in csrc/, C ABI in
include/mmof.h); ``binding`` marshals torch GPU tensors into its entry points and
``autograd`` wraps the operators in a torch.autograd.Function whose backward calls
the adjoint kernels.
"""
__all__ = ["binding", "autograd", "build"]

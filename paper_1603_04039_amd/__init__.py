"""MI355X (gfx950) AP-Cloud field solve: HIP kernels behind a C ABI (include/apcloud.h)
with a thin ctypes binding.  PyTorch-ROCm supplies device memory and streams."""
from .apcloud import (APC_FP64, APC_MIXED, APC_MIXED_F32ACC, APC_PRECOND_JACOBI, APC_PRECOND_NONE, ApcError, Cloud,
                      assemble_gfd, build_cloud, deposit, interpolate_force, load_library,
                      make_params, solve)

__all__ = ["Cloud", "ApcError", "build_cloud", "assemble_gfd", "deposit", "solve",
           "interpolate_force", "load_library", "make_params", "APC_FP64", "APC_MIXED", "APC_MIXED_F32ACC",
           "APC_PRECOND_NONE", "APC_PRECOND_JACOBI"]

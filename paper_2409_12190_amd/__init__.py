"""MI355X (gfx950) bundle-adjustment hot path: one Levenberg-Marquardt
iteration (residuals and Jacobian blocks, J^T J / J^T r assembly, Schur
complement onto the cameras, block-Jacobi PCG) as HIP kernels behind the C
ABI of include/ba.h, with a thin Python binding."""
from .ba import (BA_FP64, BA_MIXED, BaError, Problem, bundle_adjust, lib)  # noqa: F401

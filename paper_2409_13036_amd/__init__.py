"""MI355X (gfx950) library for the per-time-step sparse solves of a
radiofrequency-ablation FEM model: element assembly gathered row by row into the
solver's slab layout (colour by colour, without atomics, into CSR and for rows of more
than 64 entries), Jacobi-preconditioned CG in FP64 or with FP32 inner iterations inside
FP64 refinement, the coupled potential + bioheat time step, its adjoint, batched
ensembles, the predictor-corrector loop and the monolithic Newton-GMRES corrector.

The compute path is the native library ``librafem.so`` (HIP kernels behind a C
ABI, declared in ``include/rafem.h``).  ``paper_2409_13036_amd.rafem`` is the thin
ctypes binding; ``paper_2409_13036_amd.sim`` drives a problem on the device.
Importing either raises if the native library has not been built.
"""

__all__ = ["rafem", "sim"]


def __getattr__(name):
    if name == "rafem":
        from . import _lib as rafem
        return rafem
    if name == "sim":
        from . import sim
        return sim
    raise AttributeError(name)

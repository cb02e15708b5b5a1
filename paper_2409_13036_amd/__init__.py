"""MI355X (gfx950) library for the per-time-step sparse solves of a
radiofrequency-ablation FEM model: colour-by-colour element assembly into CSR,
Jacobi-preconditioned CG in FP64 or with FP32 inner iterations inside FP64
refinement, and the coupled potential + bioheat time step.

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

"""CPU oracle for the radiofrequency-ablation FEM hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct FP64 NumPy/SciPy code that defines what the GPU
library must compute: element matrices, element-order global assembly into
CSR, symmetric Dirichlet lifting, Jacobi-preconditioned CG (Saad, Alg. 9.1),
dense LU, the coupled potential + bioheat time step, the discrete adjoint of
a sequence of such steps, the predictor-corrector time loop, and the monolithic
two-unknowns-per-node corrector (Newton with restarted GMRES).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never calls it, and it shares no code,
tables or constants with the GPU library: each side writes its own quadrature
rule, shape functions and stencil logic from the mathematics.

Modules
  elements  -- hex Q1 (2x2x2 Gauss) and tet P1 element matrices, Joule loads
  assembly  -- CSR structure, element-order assembly, Dirichlet lifting
  solvers   -- Jacobi-PCG and dense LU
  rafem     -- sigma(T), potential system, Joule source, bioheat system, steps
  adjoint   -- reverse-time discrete adjoint of the coupled steps
  corrector -- predictor, staggered Picard corrector, step-size control
  monolithic -- (T, V) residual and Jacobian, block Jacobi, GMRES(m), Newton corrector
"""
from . import elements, assembly, solvers, rafem  # noqa: F401

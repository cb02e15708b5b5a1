"""Jacobi-preconditioned conjugate gradients and dense LU (oracle).

The paper names conjugate gradients as the standard iterative method for
symmetric positive-definite systems and notes that preconditioners speed up
Krylov convergence (Sec. II-B); it cites Saad's book for iterative methods.
This is the preconditioned CG of Saad (Alg. 9.1) with M = diag(A):

    r0 = b - A x0;  z0 = M^{-1} r0;  p0 = z0
    loop:  alpha = (r, z) / (A p, p);  x += alpha p;  r -= alpha A p
           stop when ||r||_2 <= tol * ||b||_2
           z = M^{-1} r;  beta = (r_new, z_new) / (r, z);  p = z + beta p

Breakdown (p.Ap <= 0 or non-finite) and the iteration limit are reported in
the returned info; the true residual ||b - A x|| / ||b|| is computed at exit.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

OK, NOCONV, BREAKDOWN = 0, 3, 4


@dataclasses.dataclass
class SolveInfo:
    status: int
    iters: int
    relres: float        # recursive ||r|| / ||b||
    relres_true: float   # ||b - A x|| / ||b||


def pcg(A: sp.csr_matrix, b: np.ndarray, x0: np.ndarray, tol: float, maxit: int = 100000):
    """Saad Alg. 9.1 with the Jacobi preconditioner.  Returns (x, SolveInfo)."""
    dinv = 1.0 / A.diagonal()
    x = np.array(x0, dtype=np.result_type(A.dtype, b.dtype, x0.dtype), copy=True)
    r = b - A @ x
    bnorm = np.sqrt(np.real(np.vdot(b, b)))
    z = dinv * r
    p = z.copy()
    rz = np.dot(r, z)
    status, it = NOCONV, 0
    rnorm = np.sqrt(np.real(np.vdot(r, r)))
    if rnorm <= tol * bnorm:
        status = OK
    else:
        while it < maxit:
            q = A @ p
            pq = np.dot(p, q)
            if not np.isfinite(pq) or np.real(pq) <= 0:
                status = BREAKDOWN
                break
            alpha = rz / pq
            x += alpha * p
            r -= alpha * q
            it += 1
            rnorm = np.sqrt(np.real(np.vdot(r, r)))
            if rnorm <= tol * bnorm:
                status = OK
                break
            z = dinv * r
            rz_new = np.dot(r, z)
            beta = rz_new / rz
            rz = rz_new
            p = z + beta * p
    denom = bnorm if bnorm > 0 else 1.0
    rt = b - A @ x
    info = SolveInfo(status=status, iters=it, relres=float(rnorm / denom),
                     relres_true=float(np.sqrt(np.real(np.vdot(rt, rt))) / denom))
    return x, info


def dense_solve(A, b: np.ndarray) -> np.ndarray:
    """LU solve of the (possibly complex) matrix, densified.  For tiny meshes only."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    return np.linalg.solve(Ad, b)

"""Coupled potential + bioheat time step (oracle).

The paper's application simulates voltage and heat in tissue with FEM,
advancing in time steps whose corrector assembles and solves the global
system (Sec. II-A, Fig. 1).  The paper does not print its equations; the
readings used (each a field of ``rafem_inputs.Problem``) are:

* quasi-static potential  div(sigma grad V) = 0 with sigma_e = sigma0_e (1 + alpha (Tbar_e - T_ref)),
  Tbar_e the mean of the element's nodal T^n (lagged coupling), D = faces (0 V) U electrode (20 V);
* Joule source F_i = sum_e int N_i sigma_e grad V . grad V with V = V^{n+1};
* backward-Euler Pennes bioheat
  [(rho c/dt + w_e) M_e + k_e K_e] T^{n+1} = (rho c/dt) M T^n + w T_a M 1 + F,
  D = faces (37 C) U electrode (90 C).

One step: sigma(T^n) -> assemble K_sigma -> solve V -> F -> bioheat RHS -> solve T.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import elements
from .assembly import Structure, lifted_rhs
from .solvers import pcg, dense_solve, SolveInfo

_CHUNK = 1 << 16


def _element_matrices_chunked(xe: np.ndarray):
    E = xe.shape[0]
    npe = xe.shape[1]
    K = np.empty((E, npe, npe))
    M = np.empty((E, npe, npe))
    for s in range(0, E, _CHUNK):
        K[s:s + _CHUNK], M[s:s + _CHUNK] = elements.element_matrices(xe[s:s + _CHUNK])
    return K, M


@dataclasses.dataclass
class StepInfo:
    V: Optional[SolveInfo]
    T: SolveInfo


class Model:
    """Oracle model of one problem: structure, element matrices, systems and steps."""

    def __init__(self, problem):
        self.p = problem
        self.S = Structure(problem.conn, problem.n_nodes)
        self.xe = problem.xyz[problem.conn]                  # [E, npe, 3]
        self.Ke, self.Me = _element_matrices_chunked(self.xe)

    # --- potential ---------------------------------------------------------------------
    def sigma(self, T: np.ndarray) -> np.ndarray:
        """Element conductivity from the element-mean temperature."""
        p = self.p
        Tbar = T[p.conn].mean(axis=1)
        return p.sigma0_e * (1.0 + p.alpha_sigma * (Tbar - p.T_ref))

    def potential_system(self, sigma_e: np.ndarray):
        """Lifted K_sigma and its right-hand side (lifting only: no volume source)."""
        p = self.p
        vals = self.S.assemble(self.Ke, self.Me, None, sigma_e)
        lv, lift = self.S.lift(vals, p.dir_ids, p.dir_V)
        b = lifted_rhs(np.zeros(p.n_nodes, dtype=lift.dtype), lift, p.dir_ids)
        return self.S.matrix(lv), b

    def joule(self, sigma_e: np.ndarray, V: np.ndarray) -> np.ndarray:
        p = self.p
        out = np.zeros(p.n_nodes, dtype=np.result_type(sigma_e, V))
        for s in range(0, p.n_elems, _CHUNK):
            e = slice(s, s + _CHUNK)
            fe = elements.joule_loads(self.xe[e], sigma_e[e], V[p.conn[e]])
            out += Structure.scatter_vector(_Sub(self.S.n, p.conn[e]), fe)
        return out

    # --- bioheat ------------------------------------------------------------------------
    def bioheat_values(self, k_e=None, perf_e=None, dt=None) -> np.ndarray:
        """Unlifted A_T values = sum_e [(rho c/dt + w_e) M_e + k_e K_e] (dt: the problem's
        step unless given)."""
        p = self.p
        k_e = p.k_e if k_e is None else k_e
        perf_e = p.perf_e if perf_e is None else perf_e
        dt = p.dt if dt is None else dt
        return self.S.assemble(self.Ke, self.Me, p.rho_c / dt + perf_e, k_e)

    def bioheat_system(self, k_e=None, perf_e=None, dt=None):
        p = self.p
        lv, lift = self.S.lift(self.bioheat_values(k_e, perf_e, dt), p.dir_ids, p.dir_T)
        return self.S.matrix(lv), lift

    def bioheat_rhs(self, T: np.ndarray, F: np.ndarray, lift: np.ndarray, perf_e=None,
                    dt=None) -> np.ndarray:
        """(rho c/dt) M T^n + T_a M_w 1 + F, element by element, then lifted."""
        p = self.p
        perf_e = p.perf_e if perf_e is None else perf_e
        dt = p.dt if dt is None else dt
        w = (p.rho_c / dt) * T[p.conn] + (perf_e * p.T_a)[:, None]       # [E, npe]
        fe = np.einsum("eab,eb->ea", self.Me, w)
        b_phys = self.S.scatter_vector(fe) + F
        return lifted_rhs(b_phys, lift, p.dir_ids)

    # --- one coupled step ---------------------------------------------------------------
    def solve(self, A, b, x0, tol, solver):
        if solver == "dense":
            x = dense_solve(A, b)
            r = b - A @ x
            bn = np.sqrt(np.real(np.vdot(b, b))) or 1.0
            rr = float(np.sqrt(np.real(np.vdot(r, r))) / bn)
            return x, SolveInfo(status=0, iters=0, relres=rr, relres_true=rr)
        x, info = pcg(A, b, x0, tol)
        if info.status != 0:
            raise RuntimeError(f"oracle PCG failed: {info}")
        return x, info

    def step(self, T: np.ndarray, V: np.ndarray, tol: float, solver: str = "pcg",
             bioheat=None, k_e=None, perf_e=None):
        """One time step from (T^n, V^n) -> (T^{n+1}, V^{n+1}, StepInfo).

        ``bioheat`` may carry a pre-assembled (A_T, lift_T) for this parameter set.
        Uncoupled problems skip the potential and use F = 0.
        """
        p = self.p
        if bioheat is None:
            bioheat = self.bioheat_system(k_e, perf_e)
        A_T, lift_T = bioheat
        vinfo = None
        if p.coupled:
            sig = self.sigma(T)
            A_V, b_V = self.potential_system(sig)
            x0 = np.array(V, dtype=b_V.dtype, copy=True)
            x0[p.dir_ids] = p.dir_V
            V_new, vinfo = self.solve(A_V, b_V, x0, tol, solver)
            F = self.joule(sig, V_new)
        else:
            V_new = V
            F = np.zeros(p.n_nodes)
        b_T = self.bioheat_rhs(T, F, lift_T, perf_e)
        x0 = np.array(T, dtype=b_T.dtype, copy=True)
        x0[p.dir_ids] = p.dir_T
        T_new, tinfo = self.solve(A_T, b_T, x0, tol, solver)
        return T_new, V_new, StepInfo(V=vinfo, T=tinfo)

    def simulate(self, steps: int, tol: float, solver: str = "pcg", k_e=None, perf_e=None,
                 T0=None, V0=None, keep: bool = True):
        """Run ``steps`` coupled steps from the problem's initial state.

        Returns (list of (T, V) after each step if keep else only the last, list of StepInfo).
        """
        T = self.p.initial_T() if T0 is None else T0
        V = self.p.initial_V() if V0 is None else V0
        bio = self.bioheat_system(k_e, perf_e)
        states: List = []
        infos: List[StepInfo] = []
        for _ in range(steps):
            T, V, info = self.step(T, V, tol, solver, bioheat=bio, k_e=k_e, perf_e=perf_e)
            infos.append(info)
            if keep:
                states.append((T, V))
        if not keep:
            states.append((T, V))
        return states, infos


class _Sub:
    """Minimal stand-in so Structure.scatter_vector can run on a slice of elements."""

    def __init__(self, n, conn):
        self.n = n
        self.conn = np.asarray(conn, dtype=np.int64)

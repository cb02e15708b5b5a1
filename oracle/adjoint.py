"""Discrete adjoint of a sequence of coupled time steps (oracle; test infrastructure only).

Gradient of the lesion-temperature loss  L = sum_{i in R} (T_i^N - T*_i)^2  with respect
to the per-element thermal conductivity k_e and perfusion w_e, by the reverse sweep of
the steps defined in ``oracle.rafem`` (the paper's time loop, Sec. II-A, run backwards).

Step n maps T^{n-1} to (V^n, T^n) through
  S(V^n; sigma(T^{n-1})) = K_sigma V^n = 0              on free rows (potential),
  R(T^n) = A_T T^n - (rho c/dt) M T^{n-1} - T_a M_w 1 - F(sigma, V^n) = 0  on free rows,
with V and T fixed on the Dirichlet set.  With lambda the adjoint load on T^n:
  A_T mu = lambda (free rows, mu = 0 on D)
  dL/dk_e += -mu_e^T K_e T^n_e ;  dL/dw_e += -mu_e^T M_e (T^n_e - T_a)
  sbar_e  = mu_e^T J_e(V^n)  (the Joule load at unit conductivity)
  K_sigma nu = (dF/dV)^T mu (free rows, nu = 0 on D);   sbar_e -= nu_e^T K_e V^n_e
  lambda_{n-1} = (rho c/dt) M mu + sum_e sbar_e sigma0_e alpha / npe  on the element's nodes
Both matrices are symmetric, so every adjoint solve is an ordinary solve.
"""
from __future__ import annotations

import numpy as np

from . import elements
from .rafem import Model


def loss(problem, T: np.ndarray):
    d = T[problem.loss_ids] - problem.T_target
    return np.sum(d * d)


def loss_delta(problem, T_plus: np.ndarray, T_minus: np.ndarray) -> float:
    """L(T+) - L(T-) computed node by node, without cancellation of the two large losses."""
    a = T_plus[problem.loss_ids]
    b = T_minus[problem.loss_ids]
    return float(np.sum((a - b) * (a + b - 2.0 * problem.T_target)))


def forward(model: Model, steps: int, tol: float, solver: str = "pcg", k_e=None, perf_e=None):
    """States T^0..T^N and V^1..V^N (V[0] is the initial potential iterate)."""
    p = model.p
    T = [p.initial_T()]
    V = [p.initial_V()]
    bio = model.bioheat_system(k_e, perf_e)
    for _ in range(steps):
        Tn, Vn, _ = model.step(T[-1], V[-1], tol, solver, bioheat=bio, k_e=k_e, perf_e=perf_e)
        T.append(Tn)
        V.append(Vn)
    return T, V


def _elem(model, v):
    return v[model.p.conn]


def adjoint_gradients(model: Model, steps: int, tol: float, solver: str = "pcg", k_e=None,
                      perf_e=None, states=None):
    """(L, dL/dk_e, dL/dw_e) by the reverse sweep.  ``states`` may carry a forward run."""
    p = model.p
    k_e = p.k_e if k_e is None else k_e
    perf_e = p.perf_e if perf_e is None else perf_e
    T, V = states if states is not None else forward(model, steps, tol, solver, k_e, perf_e)
    A_T, _ = model.bioheat_system(k_e, perf_e)
    M = model.S.matrix(model.S.assemble(model.Ke, model.Me, np.ones(p.n_elems), None))
    isD = np.zeros(p.n_nodes, dtype=bool)
    isD[p.dir_ids] = True

    lam = np.zeros(p.n_nodes)
    lam[p.loss_ids] = 2.0 * (T[steps][p.loss_ids] - p.T_target)
    gk = np.zeros(p.n_elems)
    gw = np.zeros(p.n_elems)
    for n in range(steps, 0, -1):
        rhs = np.where(isD, 0.0, lam)
        mu, _ = model.solve(A_T, rhs, np.zeros(p.n_nodes), tol, solver)
        mu_e = _elem(model, mu)
        Tn_e = _elem(model, T[n])
        gk -= np.einsum("ea,eab,eb->e", mu_e, model.Ke, Tn_e)
        gw -= np.einsum("ea,eab,eb->e", mu_e, model.Me, Tn_e - p.T_a)
        lam_prev = (p.rho_c / p.dt) * (M @ mu)
        if p.coupled:
            sig = model.sigma(T[n - 1])
            Vn_e = _elem(model, V[n])
            J1 = elements.joule_loads(model.xe, np.ones(p.n_elems), Vn_e)   # J_e(V) at unit sigma
            sbar = np.einsum("ea,ea->e", mu_e, J1)
            nubar = model.S.scatter_vector(elements.joule_grad_V(model.xe, sig, Vn_e, mu_e))
            A_V, _ = model.potential_system(sig)
            nu, _ = model.solve(A_V, np.where(isD, 0.0, nubar), np.zeros(p.n_nodes), tol, solver)
            sbar -= np.einsum("ea,eab,eb->e", _elem(model, nu), model.Ke, Vn_e)
            dsig = sbar * p.sigma0_e * p.alpha_sigma / p.npe
            lam_prev += model.S.scatter_vector(np.repeat(dsig[:, None], p.npe, axis=1))
        lam = lam_prev
    return loss(p, T[steps]), gk, gw


def complex_step_directional(model: Model, steps: int, dk: np.ndarray, dw: np.ndarray,
                             h: float = 1e-30) -> float:
    """d/dt L(k + t dk, w + t dw) at t = 0 by the complex step (dense complex solves)."""
    p = model.p
    T, _ = forward(model, steps, 0.0, "dense", p.k_e + 1j * h * dk, p.perf_e + 1j * h * dw)
    return float(np.imag(loss(p, T[steps])) / h)

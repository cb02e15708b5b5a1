"""Predictor-corrector time loop of the application (oracle; test infrastructure only).

The application advances the coupled potential / temperature problem in time steps of
dynamic size; every step first extrapolates the solution in time (predictor), then
repeats the corrector (element equations re-evaluated with the updated values, assembled
and solved) until a convergence threshold is met.  A step whose corrector has not
converged within the allowed number of iterations (50) is not accepted and the step size
is halved; the simulation still ends at the prescribed total time (Sec. II-A, Fig. 1;
Sec. IV).  The paper gives no formulas for these parts; the readings used here are:

* predictor: linear extrapolation T* = T^n + (dt / dt_prev) (T^n - T^{n-1}), or T^n for
  the first step;
* corrector iteration k (Picard on the coupling): sigma from T^{n+1,k}, potential solve,
  Joule load with V^{n+1,k+1}, bioheat solve with T^n on the right-hand side, giving
  T^{n+1,k+1}; converged when ||T^{n+1,k+1} - T^{n+1,k}||_2 <= eps ||T^{n+1,k+1}||_2;
  the first iterate from T* = T^n is the explicit-coupling step of ``Model.step``;
* step control: a rejected step is retried with half the step; after an accepted step
  the step doubles again, up to the nominal one; the last step is shortened to end
  exactly at the total time.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from .rafem import Model


@dataclasses.dataclass
class CorrectorResult:
    T: np.ndarray
    V: np.ndarray
    iters: int          # corrector iterations (solves of the coupled pair) performed
    converged: bool
    change: float       # last relative change ||T^{k+1} - T^k|| / ||T^{k+1}||


def predictor(T_n: np.ndarray, T_prev: Optional[np.ndarray], dt: float, dt_prev: Optional[float]):
    """Linear extrapolation of T to the end of the step (T^n when there is no history)."""
    if T_prev is None or not dt_prev:
        return T_n.copy()
    return T_n + (dt / dt_prev) * (T_n - T_prev)


def corrector_step(model: Model, T_n: np.ndarray, V_n: np.ndarray, dt: float, T_guess: np.ndarray,
                   tol: float, eps: float, max_iters: int = 50, solver: str = "pcg") -> CorrectorResult:
    """One predictor-corrector step of size dt from (T^n, V^n), starting from T_guess."""
    p = model.p
    A_T, lift_T = model.bioheat_system(dt=dt)
    T_k = np.array(T_guess, dtype=float, copy=True)
    V = np.array(V_n, dtype=float, copy=True)
    change = np.inf
    for k in range(1, max_iters + 1):
        sig = model.sigma(T_k)
        A_V, b_V = model.potential_system(sig)
        V[p.dir_ids] = p.dir_V
        V, _ = model.solve(A_V, b_V, V, tol, solver)
        F = model.joule(sig, V)
        b_T = model.bioheat_rhs(T_n, F, lift_T, dt=dt)
        x0 = T_k.copy()
        x0[p.dir_ids] = p.dir_T
        T_next, _ = model.solve(A_T, b_T, x0, tol, solver)
        change = float(np.linalg.norm(T_next - T_k) / np.linalg.norm(T_next))
        T_k = T_next
        if change <= eps:
            return CorrectorResult(T_k, V, k, True, change)
    return CorrectorResult(T_k, V, max_iters, False, change)


@dataclasses.dataclass
class StepRecord:
    t: float            # time at the end of the accepted step
    dt: float
    iters: int
    rejected_before: int


def simulate_pc(model: Model, t_total: float, dt0: float, tol: float, eps: float,
                max_iters: int = 50, dt_min: float = 1e-6, solver: str = "pcg", corrector=None):
    """Advance from the initial state to t_total.  Returns (T, V, [StepRecord]).

    ``corrector`` (tests only) replaces ``corrector_step`` with the same signature."""
    step = corrector_step if corrector is None else corrector
    p = model.p
    T, V = p.initial_T(), p.initial_V()
    T_prev, dt_prev = None, None
    t, dt = 0.0, dt0
    records: List[StepRecord] = []
    rejected = 0
    while t_total - t > 1e-12 * t_total:
        h = min(dt, t_total - t)
        res = step(model, T, V, h, predictor(T, T_prev, h, dt_prev), tol, eps, max_iters, solver)
        if not res.converged:
            rejected += 1
            dt = h / 2.0
            if dt < dt_min:
                raise RuntimeError(f"time step fell below {dt_min} s at t = {t} s")
            continue
        T_prev, dt_prev = T, h
        T, V = res.T, res.V
        t += h
        records.append(StepRecord(t, h, res.iters, rejected))
        rejected = 0
        dt = min(dt0, 2.0 * h)
    return T, V, records

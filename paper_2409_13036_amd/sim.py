"""Drive one radiofrequency-ablation problem on the device through the C ABI.

A ``DeviceProblem`` uploads a mesh, its material fields and Dirichlet data once,
keeps the state (T, V) in device memory, and advances it with ``rafem_step``.
The bioheat matrix does not depend on temperature, so it is assembled on the
first step and reused afterwards.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import _lib as rafem


def reorder_nodes(problem, order: np.ndarray):
    """The same problem with its nodes renumbered: node order[k] becomes node k.  Elements
    keep their ids; Dirichlet, electrode and loss sets are renumbered and re-sorted with
    their values.  A state x of the new problem maps back by x_old[order] = x_new."""
    import dataclasses
    order = np.asarray(order, dtype=np.int64)
    n = problem.xyz.shape[0]
    if order.shape != (n,) or not np.array_equal(np.sort(order), np.arange(n)):
        raise ValueError("order must be a permutation of the node ids")
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n)

    def relabel(ids, *vals):
        new = inv[ids]
        k = np.argsort(new, kind="stable")
        return (new[k].astype(np.int32),) + tuple(v[k] for v in vals)

    dir_ids, dir_V, dir_T = relabel(problem.dir_ids, problem.dir_V, problem.dir_T)
    (electrode,) = relabel(problem.electrode_ids)
    loss_ids, T_target = problem.loss_ids, problem.T_target
    if loss_ids is not None:
        loss_ids, T_target = relabel(loss_ids, T_target)
    return dataclasses.replace(
        problem, xyz=np.ascontiguousarray(problem.xyz[order]),
        conn=np.ascontiguousarray(inv[problem.conn].astype(np.int32)), dir_ids=dir_ids,
        dir_V=np.ascontiguousarray(dir_V), dir_T=np.ascontiguousarray(dir_T),
        electrode_ids=electrode, loss_ids=loss_ids, T_target=T_target)


def rcm_reordered(problem, window: int = 0):
    """(problem renumbered by the library's reverse Cuthill-McKee order, order); window > 0
    also sorts each window of that many positions by node degree (less slab padding)."""
    n = problem.xyz.shape[0]
    order = rafem.rcm_order(problem.conn, n)
    if window > 0:
        order = rafem.degree_sort(order, problem.conn, n, window)
    return reorder_nodes(problem, order), order



def _extrapolate_mode(on: bool, chain: bool, fresh: bool) -> int:
    """phys.extrapolate for a step: 0 off (also for the first step from the problem's initial
    state, whose V is not a solution and would spoil the predictor), 2 a new trajectory, 1
    continue it."""
    if not on or fresh:
        return 0
    return 1 if chain else 2


class DeviceProblem:
    def __init__(self, problem, device=None):
        import torch
        self.torch = torch
        self.p = problem
        self.dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.mesh = rafem.Mesh(problem.xyz, problem.conn, problem.dir_ids)
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.k_e = torch.as_tensor(problem.k_e, **f64).contiguous()
        self.perf_e = torch.as_tensor(problem.perf_e, **f64).contiguous()
        self.sigma0_e = torch.as_tensor(problem.sigma0_e, **f64).contiguous()
        self.dir_V = torch.as_tensor(problem.dir_V, **f64).contiguous()
        self.dir_T = torch.as_tensor(problem.dir_T, **f64).contiguous()
        self.phys = rafem.Phys(problem.rho_c, problem.dt, problem.T_a, problem.alpha_sigma,
                               problem.T_ref, 1 if problem.coupled else 0, 0)
        # extrapolate: start each step's solves from the polynomial extrapolation of the last
        # states (library-side) of the given order (1 linear .. 4 quartic; lower orders until
        # enough states are kept); _chain: the next step continues the previous one
        self.extrapolate = False
        self.extrapolate_order = 2
        self._chain = False
        self.loss_ids = self.T_target = None
        if problem.loss_ids is not None:
            self.loss_ids = torch.as_tensor(problem.loss_ids, dtype=torch.int32, device=self.dev)
            self.T_target = torch.as_tensor(problem.T_target, **f64).contiguous()
        self.reset()

    def set_params(self, k_e, perf_e):
        """New conductivity / perfusion fields (device tensors); the bioheat matrix is rebuilt."""
        self.k_e = k_e.to(self.dev, self.torch.float64).contiguous().clone()
        self.perf_e = perf_e.to(self.dev, self.torch.float64).contiguous().clone()
        self.phys.reuse_bioheat = 0
        self._chain = False

    def restore(self, T, V):
        """Continue from a saved state (the bioheat matrix is kept)."""
        self.T.copy_(T)
        self.V.copy_(V)
        self._chain = False
        self._fresh = False

    def reset(self, T0: Optional[np.ndarray] = None, V0: Optional[np.ndarray] = None):
        torch = self.torch
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.T = torch.as_tensor(self.p.initial_T() if T0 is None else T0, **f64).clone()
        self.V = torch.as_tensor(self.p.initial_V() if V0 is None else V0, **f64).clone()
        self._chain = False
        self._fresh = V0 is None  # V is the initial field, not a solution

    def step(self, tol: float = 1e-12, precision: str = "fp64", **kw):
        """One coupled step (the bioheat matrix is assembled on the first call only)."""
        self.phys.extrapolate = _extrapolate_mode(self.extrapolate, self._chain, self._fresh)
        self.phys.extrapolate_order = self.extrapolate_order
        self._chain = False
        info = rafem.step(self.mesh, self.phys, self.k_e, self.perf_e, self.sigma0_e, self.dir_V,
                          self.dir_T, self.T, self.V, tol=tol, precision=precision, **kw)
        self.phys.reuse_bioheat = 1
        self._chain = bool(self.extrapolate) and not self._fresh
        self._fresh = False
        return info

    def simulate(self, steps: int, tol: float = 1e-12, precision: str = "fp64", keep: bool = False,
                 **kw):
        states: List = []
        infos = []
        for _ in range(steps):
            infos.append(self.step(tol, precision, **kw))
            if keep:
                states.append((self.T.cpu().numpy().copy(), self.V.cpu().numpy().copy()))
        return states, infos

    def step_pc(self, dt: float, T_prev=None, dt_prev=None, corr_tol: float = 1e-10,
                max_iters: int = 50, tol: float = 1e-12, precision: str = "fp64", **kw):
        """One predictor-corrector step of size dt (T and V advance only if accepted)."""
        self._chain = False
        self.phys.dt = float(dt)
        try:
            info = rafem.step_pc(self.mesh, self.phys, self.k_e, self.perf_e, self.sigma0_e,
                                 self.dir_V, self.dir_T, T_prev, dt_prev, self.T, self.V,
                                 corr_tol=corr_tol, max_iters=max_iters, tol=tol,
                                 precision=precision, **kw)
        finally:
            self.phys.dt = float(self.p.dt)  # plain steps keep the problem's step; the library
        self.phys.reuse_bioheat = 1          # rebuilds a bioheat matrix made for another dt
        if info.get("accepted"):
            self._fresh = False
        return info

    def step_mono(self, dt: float, T_prev=None, dt_prev=None, corr_tol: float = 1e-10,
                  max_iters: int = 50, m: int = 30, gmres_tol: float = 1e-10,
                  gmres_precision: str = "fp64", **kw):
        """One predictor-corrector step of size dt with the monolithic Newton-GMRES(m)
        corrector (T and V advance only if accepted)."""
        self._chain = False
        self.phys.dt = float(dt)
        try:
            info = rafem.step_mono(self.mesh, self.phys, self.k_e, self.perf_e, self.sigma0_e,
                                   self.dir_V, self.dir_T, T_prev, dt_prev, self.T, self.V,
                                   corr_tol=corr_tol, max_iters=max_iters, m=m,
                                   gmres_tol=gmres_tol, gmres_precision=gmres_precision, **kw)
        finally:
            self.phys.dt = float(self.p.dt)
        if info.get("accepted"):
            self._fresh = False
        return info

    def simulate_pc(self, t_total: float, dt0: float, corr_tol: float = 1e-10,
                    max_iters: int = 50, tol: float = 1e-12, precision: str = "fp64",
                    dt_min: float = 1e-6, keep: bool = False, corrector: str = "picard",
                    m: int = 30, gmres_tol: float = 1e-10, gmres_precision: str = "fp64"):
        """Predictor-corrector time loop from the current state to t_total: a rejected step is
        retried with half the step; after an accepted step the step doubles again, up to dt0;
        the last step ends exactly at t_total.  corrector: "picard" (staggered PCG solves,
        tol / precision) or "newton" (monolithic GMRES(m) solves, gmres_tol).  Returns a list
        of per-step records (t, dt, corrector iterations, rejections before it[, T, V])."""
        T_prev, dt_prev = None, None
        t, dt = 0.0, float(dt0)
        records, rejected = [], 0
        while t_total - t > 1e-12 * t_total:
            h = min(dt, t_total - t)
            T_n = self.T.clone()
            if corrector == "newton":
                info = self.step_mono(h, T_prev, dt_prev, corr_tol, max_iters, m, gmres_tol,
                                      gmres_precision)
                info["solver_iters"] = info["gmres_iters"]
            else:
                info = self.step_pc(h, T_prev, dt_prev, corr_tol, max_iters, tol, precision)
            if not info["accepted"]:
                rejected += 1
                dt = h / 2.0
                if dt < dt_min:
                    raise RuntimeError(f"time step fell below {dt_min} s at t = {t} s")
                continue
            T_prev, dt_prev = T_n, h
            t += h
            rec = {"t": t, "dt": h, "iters": info["iters"], "rejected_before": rejected,
                   "solver_iters": info["solver_iters"]}
            if keep:
                rec["T"], rec["V"] = self.T.cpu().numpy().copy(), self.V.cpu().numpy().copy()
            records.append(rec)
            rejected = 0
            dt = min(float(dt0), 2.0 * h)
        return records

    def close(self):
        self.mesh.close()


class BatchProblem:
    """An ensemble of problems (same element type, any sizes) advanced together.

    The device vectors use the batch layout of the native handle: sample q's nodes start
    at node_off[q] and are followed by padding nodes (isolated Dirichlet nodes held at 0).
    Physical constants (rho c, dt, T_a, alpha) are taken from the first problem.
    """

    def __init__(self, problems, device=None):
        import torch
        self.torch = torch
        self.problems = list(problems)
        p0 = self.problems[0]
        self.dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.mesh = rafem.Mesh.batch([(p.xyz, p.conn, p.dir_ids) for p in self.problems])
        m = self.mesh
        f64 = dict(dtype=torch.float64, device=self.dev)
        cat = lambda arrs: torch.as_tensor(np.concatenate(arrs), **f64).contiguous()
        self.k_e = cat([p.k_e for p in self.problems])
        self.perf_e = cat([p.perf_e for p in self.problems])
        self.sigma0_e = cat([p.sigma0_e for p in self.problems])
        dV, dT = np.zeros(m.n_dir), np.zeros(m.n_dir)
        for q, p in enumerate(self.problems):
            a = int(m.dir_off[q])
            dV[a:a + p.dir_ids.size] = p.dir_V
            dT[a:a + p.dir_ids.size] = p.dir_T
        self.dir_V = torch.as_tensor(dV, **f64)
        self.dir_T = torch.as_tensor(dT, **f64)
        self.phys = rafem.Phys(p0.rho_c, p0.dt, p0.T_a, p0.alpha_sigma, p0.T_ref,
                               1 if p0.coupled else 0, 0)
        self.extrapolate = False   # as for DeviceProblem
        self.extrapolate_order = 2
        self._chain = False
        self.reset()

    def _gather(self, per_sample):
        out = np.zeros(self.mesh.n_nodes)
        for q, v in enumerate(per_sample):
            a = int(self.mesh.node_off[q])
            out[a:a + v.size] = v
        return out

    def reset(self):
        torch = self.torch
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.T = torch.as_tensor(self._gather([p.initial_T() for p in self.problems]), **f64)
        self.V = torch.as_tensor(self._gather([p.initial_V() for p in self.problems]), **f64)
        self._chain = False
        self._fresh = True

    def sample(self, q: int):
        """(T, V) of sample q as host arrays."""
        a = int(self.mesh.node_off[q])
        n = self.problems[q].n_nodes
        return self.T[a:a + n].cpu().numpy(), self.V[a:a + n].cpu().numpy()

    def step(self, tol: float = 1e-12, precision: str = "fp64", **kw):
        self.phys.extrapolate = _extrapolate_mode(self.extrapolate, self._chain, self._fresh)
        self.phys.extrapolate_order = self.extrapolate_order
        self._chain = False
        info = rafem.step(self.mesh, self.phys, self.k_e, self.perf_e, self.sigma0_e, self.dir_V,
                          self.dir_T, self.T, self.V, tol=tol, precision=precision, **kw)
        self.phys.reuse_bioheat = 1
        self._chain = bool(self.extrapolate) and not self._fresh
        self._fresh = False
        return info

    def close(self):
        self.mesh.close()

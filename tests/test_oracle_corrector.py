"""Pins of the oracle's predictor-corrector loop: the explicit step as its first iterate,
alpha = 0 (no coupling) converging at once, the fixed point against an independent
nonlinear root finder on a tiny mesh, the fixed point's equations at a medium size, the
predictor, and the step-size control."""
import dataclasses

import numpy as np
import pytest
from scipy import optimize

import rafem_inputs as ri
from oracle import corrector as pc
from oracle.rafem import Model


def test_first_iterate_is_the_explicit_step():
    p = ri.make_problem("hex", 9, 1)
    m = Model(p)
    T0, V0 = p.initial_T(), p.initial_V()
    res = pc.corrector_step(m, T0, V0, p.dt, T0, 1e-14, 0.0, max_iters=1)
    T1, V1, _ = m.step(T0, V0, 1e-14)
    assert not res.converged and res.iters == 1
    assert np.abs(res.T - T1).max() <= 1e-11 * np.abs(T1).max()
    assert np.abs(res.V - V1).max() <= 1e-11 * np.abs(V1).max()


def test_uncoupled_problem_converges_at_the_second_iterate():
    p = dataclasses.replace(ri.make_problem("tet", 7, 2), alpha_sigma=0.0)
    m = Model(p)
    T0, V0 = p.initial_T(), p.initial_V()
    res = pc.corrector_step(m, T0, V0, p.dt, T0, 1e-14, 1e-10)
    T1, _, _ = m.step(T0, V0, 1e-14)
    assert res.converged and res.iters == 2
    assert np.abs(res.T - T1).max() <= 1e-11 * np.abs(T1).max()


def _implicit_residual(m, T_n, dt, free):
    p = m.p

    def unpack(z):
        T = p.initial_T().copy()
        V = p.initial_V().copy()
        T[p.dir_ids], V[p.dir_ids] = p.dir_T, p.dir_V
        T[free], V[free] = z[: free.size], z[free.size:]
        return T, V

    def G(z):
        T, V = unpack(z)
        sig = m.sigma(T)                       # conductivity at the end of the step
        A_V, b_V = m.potential_system(sig)
        A_T, lift = m.bioheat_system(dt=dt)
        b_T = m.bioheat_rhs(T_n, m.joule(sig, V), lift, dt=dt)
        return np.concatenate([(A_T @ T - b_T)[free] / 1e-6, (A_V @ V - b_V)[free] / 1e-6])

    return G, unpack


def test_fixed_point_matches_a_nonlinear_root_finder():
    # a long step, so that T and hence sigma change enough for the coupling to matter
    p = ri.make_problem("hex", 6, 4)
    m = Model(p)
    dt = 40.0
    T0, V0 = p.initial_T(), p.initial_V()
    res = pc.corrector_step(m, T0, V0, dt, T0, 0.0, 1e-14, max_iters=100, solver="dense")
    assert res.converged
    free = np.setdiff1d(np.arange(p.n_nodes), p.dir_ids)
    G, unpack = _implicit_residual(m, T0, dt, free)
    explicit = pc.corrector_step(m, T0, V0, dt, T0, 0.0, 0.0, max_iters=1, solver="dense")
    z0 = np.concatenate([explicit.T[free], explicit.V[free]])
    z, info, ier, msg = optimize.fsolve(G, z0, xtol=1e-14, full_output=True)
    assert ier == 1, msg
    T_root, V_root = unpack(z)
    eT = np.linalg.norm(res.T - T_root) / np.linalg.norm(T_root)
    eV = np.linalg.norm(res.V - V_root) / np.linalg.norm(V_root)
    assert eT <= 1e-10 and eV <= 1e-10
    # and the implicit solution is measurably not the explicit step
    assert np.linalg.norm(explicit.V - V_root) / np.linalg.norm(V_root) > 1e-5


def test_converged_step_satisfies_the_implicit_equations():
    p = ri.make_problem("tet", 9, 5)
    m = Model(p)
    dt = 20.0
    T0, V0 = p.initial_T(), p.initial_V()
    res = pc.corrector_step(m, T0, V0, dt, T0, 1e-14, 1e-13, max_iters=100)
    assert res.converged and res.iters > 2
    free = np.setdiff1d(np.arange(p.n_nodes), p.dir_ids)
    G, _ = _implicit_residual(m, T0, dt, free)
    r = G(np.concatenate([res.T[free], res.V[free]])) * 1e-6
    nT = free.size
    # rows of the lifted systems at the converged state: relative to the lifted rhs norms
    A_V, b_V = m.potential_system(m.sigma(res.T))
    A_T, lift = m.bioheat_system(dt=dt)
    b_T = m.bioheat_rhs(T0, m.joule(m.sigma(res.T), res.V), lift, dt=dt)
    assert np.linalg.norm(r[:nT]) <= 1e-10 * np.linalg.norm(b_T)
    assert np.linalg.norm(r[nT:]) <= 1e-10 * np.linalg.norm(b_V)


def test_predictor_extrapolates_linearly():
    a, b = np.array([1.0, 2.0, 3.0]), np.array([1.5, 2.0, 2.0])
    assert np.array_equal(pc.predictor(b, None, 2.0, None), b)
    # exact for a field that is linear in time: T(t) = a + (b - a) t, t = 0, 1, then 1 + 0.5
    assert np.allclose(pc.predictor(b, a, 0.5, 1.0), a + (b - a) * 1.5, rtol=0, atol=1e-15)


def test_step_control_halves_regrows_and_ends_on_time():
    p = ri.make_problem("hex", 5, 0)
    m = Model(p)
    calls = []

    def fake(model, T, V, h, T_guess, tol, eps, max_iters, solver):
        calls.append(h)
        ok = h <= 0.3 + 1e-12          # the corrector "fails" on steps longer than 0.3 s
        return pc.CorrectorResult(T + 1.0, V, 3 if ok else max_iters, ok, 0.0)

    T, V, rec = pc.simulate_pc(m, t_total=1.0, dt0=0.5, tol=1e-12, eps=1e-10, corrector=fake)
    # 0.5 rejected -> 0.25 accepted; regrow to 0.5 rejected -> 0.25 ...; last step clipped
    assert calls[:3] == [0.5, 0.25, 0.5]
    assert abs(rec[-1].t - 1.0) <= 1e-15 and all(r.dt <= 0.3 for r in rec)
    assert sum(r.dt for r in rec) == pytest.approx(1.0, abs=1e-15)
    assert rec[0].rejected_before == 1
    assert np.allclose(T, p.initial_T() + len(rec))

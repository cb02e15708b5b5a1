"""Pins of the oracle's coupled step: patch tests, 1-D closed forms, limits and fixed points."""
import dataclasses

import numpy as np
import pytest

import rafem_inputs as ri
from oracle.rafem import Model
from oracle.solvers import pcg, dense_solve


def _with_dirichlet(p, ids, dir_V=None, dir_T=None):
    ids = np.asarray(ids, dtype=np.int32)
    return dataclasses.replace(p, dir_ids=ids,
                               dir_V=np.zeros(ids.size) if dir_V is None else dir_V,
                               dir_T=np.full(ids.size, 37.0) if dir_T is None else dir_T)


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_potential_patch_test(kind):
    """Exact discrete harmonic fields: xyz (trilinear, in Q1) on hexes, linear on jittered tets."""
    n = 9
    p = ri.make_problem(kind, n, 11)
    faces = ri.face_node_ids(n)
    x, y, z = p.xyz.T
    exact = x * y * z * 1e6 if kind == "hex" else 1.0 + 200 * x - 100 * y + 300 * z
    q = _with_dirichlet(p, faces, dir_V=exact[faces])
    m = Model(q)
    A, b = m.potential_system(np.full(p.n_elems, 0.4))
    V, info = pcg(A, b, q.initial_V(), tol=1e-14)
    np.testing.assert_allclose(V, exact, rtol=0, atol=1e-11 * np.abs(exact).max())


def _x_planes(n):
    i = np.arange(n ** 3) % n
    return np.nonzero((i == 0) | (i == n - 1))[0]


def _steady(p, a, c, g_lo, g_hi):
    ids = _x_planes(p.n)
    i = ids % p.n
    g = np.where(i == 0, g_lo, g_hi).astype(float)
    q = _with_dirichlet(p, ids, dir_T=g)
    m = Model(q)
    vals = m.S.assemble(m.Ke, m.Me, np.full(p.n_elems, a) if a else None, np.full(p.n_elems, c))
    lv, lift = m.S.lift(vals, q.dir_ids, g)
    rhs = np.zeros(p.n_nodes)
    rhs[q.dir_ids] = 0
    # volume source of a perfusion term: a * T_a * M 1 (element by element)
    if a:
        fe = np.einsum("eab,eb->ea", m.Me, np.full((p.n_elems, p.npe), a * 37.0))
        rhs += m.S.scatter_vector(fe)
    b = rhs + lift
    b[q.dir_ids] = g
    T, info = pcg(m.S.matrix(lv), b, np.full(p.n_nodes, 37.0), tol=1e-14)
    return T


def test_1d_steady_conduction_is_linear():
    n = 9
    p = ri.make_problem("hex", n, 0)
    T = _steady(p, 0.0, 0.512, 90.0, 37.0)
    x = p.xyz[:, 0]
    np.testing.assert_allclose(T, 90.0 + (37.0 - 90.0) * x / ri.SIDE_M, rtol=0, atol=1e-10)


def test_1d_steady_perfusion_converges_second_order():
    """T - T_a = A cosh(m x) + B sinh(m x), m = sqrt(w/k): nodal error falls ~4x per halving of h."""
    k, w = 0.512, 0.512 * 150.0 ** 2
    mm = np.sqrt(w / k)
    L = ri.SIDE_M
    errs = []
    for n in (5, 9, 17):
        p = ri.make_problem("hex", n, 0)
        T = _steady(p, w, k, 90.0, 37.0)
        x = p.xyz[:, 0]
        Aco = 90.0 - 37.0
        Bco = -Aco * np.cosh(mm * L) / np.sinh(mm * L)
        exact = 37.0 + Aco * np.cosh(mm * x) + Bco * np.sinh(mm * x)
        errs.append(np.abs(T - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8) and np.all(rates < 2.3), (errs, rates)


def test_joule_source_uniform_field_total():
    for kind in ("hex", "tet"):
        p = ri.make_problem(kind, 7, 3)
        m = Model(p)
        Ev = np.array([100.0, -50.0, 30.0])
        F = m.joule(np.full(p.n_elems, 0.33), p.xyz @ Ev)
        np.testing.assert_allclose(F.sum(), 0.33 * (Ev @ Ev) * ri.SIDE_M ** 3, rtol=1e-12)


def test_zero_alpha_decouples_potential():
    p = dataclasses.replace(ri.make_problem("hex", 9, 0), alpha_sigma=0.0)
    m = Model(p)
    states, _ = m.simulate(3, 1e-13)
    for T, V in states[1:]:
        np.testing.assert_allclose(V, states[0][1], rtol=0, atol=1e-10)
    assert np.abs(states[2][0] - states[0][0]).max() > 1e-3  # temperature still evolves


def test_zero_voltage_gives_pure_pennes_step():
    p = ri.make_problem("hex", 9, 0)
    p0 = dataclasses.replace(p, dir_V=np.zeros_like(p.dir_V))
    m = Model(p0)
    T1, V1, _ = m.step(p.initial_T(), p0.initial_V(), 1e-13)
    assert np.all(V1 == 0)
    mu = Model(dataclasses.replace(p0, coupled=False))
    T2, _, _ = mu.step(p.initial_T(), p0.initial_V(), 1e-13)
    np.testing.assert_allclose(T1, T2, rtol=0, atol=1e-9)


def test_steady_state_is_fixed_point_of_the_step():
    """With sigma independent of T the Joule source is fixed; the steady solution of
    (K + w M) T = w T_a M 1 + F is unchanged by a backward-Euler step."""
    p = dataclasses.replace(ri.make_problem("hex", 7, 2), alpha_sigma=0.0)
    m = Model(p)
    A_V, b_V = m.potential_system(m.sigma(p.initial_T()))
    V = dense_solve(A_V, b_V)
    F = m.joule(m.sigma(p.initial_T()), V)
    vals = m.S.assemble(m.Ke, m.Me, p.perf_e, p.k_e)
    lv, lift = m.S.lift(vals, p.dir_ids, p.dir_T)
    fe = np.einsum("eab,eb->ea", m.Me, np.repeat((p.perf_e * p.T_a)[:, None], p.npe, axis=1))
    b = m.S.scatter_vector(fe) + F + lift
    b[p.dir_ids] = p.dir_T
    Ts = dense_solve(m.S.matrix(lv), b)
    T1, V1, _ = m.step(Ts, V, 1e-14, solver="dense")
    np.testing.assert_allclose(T1, Ts, rtol=0, atol=1e-9 * np.abs(Ts).max())
    np.testing.assert_allclose(V1, V, rtol=0, atol=1e-10)


def test_dense_and_pcg_steps_agree():
    p = ri.make_problem("tet", 7, 5)
    m = Model(p)
    sp_, _ = m.simulate(2, 1e-14)
    sd, _ = m.simulate(2, 0.0, solver="dense")
    for (Ta, Va), (Tb, Vb) in zip(sp_, sd):
        np.testing.assert_allclose(Ta, Tb, rtol=1e-12)
        np.testing.assert_allclose(Va, Vb, rtol=0, atol=1e-11 * ri.V_ELECTRODE)

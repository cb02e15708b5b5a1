"""Pins of the oracle's coupling terms against closed forms fixed outside the oracle.

* sigma(T): the stated law sigma = 0.33 (1 + 0.015 (T - 37)) S/m of the coupled workload,
  evaluated at a hand-computed temperature, and, for a linear temperature field, at the
  element centroids given in closed form by the grid indices (hex) and by the Kuhn
  permutation of each tet -- so a sign slip, a wrong reference temperature, a wrong
  coefficient or a mean over the wrong nodes fails;
* the potential solve of a step uses sigma of the temperature the step starts from
  (lagged coupling), not the one it produces;
* the Joule load int N_i sigma grad V . grad V node by node: for V = x y z on the hex grid
  (trilinear, so the 2x2x2 Gauss rule integrates N_i |grad V|^2 exactly) from products of
  one-dimensional hat-function moments, and for a linear V on the undistorted Kuhn tets
  from the number of tets that meet at each node.
"""
import dataclasses
import itertools

import numpy as np
import pytest

import rafem_inputs as ri
from oracle.rafem import Model
from oracle.solvers import pcg

# the coupled workload's conductivity law: 0.33 S/m at 37 C, +1.5 % per kelvin
SIGMA_37 = 0.33
ALPHA = 0.015


def _centroids_hex(n):
    """Element centroids of the hex grid: element (a, b, c) spans [a h, (a + 1) h] x ..."""
    h = ri.SIDE_M / (n - 1)
    m = n - 1
    e = np.arange(m ** 3)
    a, b, c = e % m, (e // m) % m, e // (m * m)
    return np.stack([(a + 0.5) * h, (b + 0.5) * h, (c + 0.5) * h], axis=1)


def _centroids_kuhn(n):
    """Vertex centroids of the undistorted Kuhn tets: the tet of permutation pi walks the
    axes pi0, pi1, pi2 from the cube's low corner, so axis pi0 is +1 at three of its four
    vertices, pi1 at two and pi2 at one: centroid = corner + h (3/4, 2/4, 1/4) permuted."""
    h = ri.SIDE_M / (n - 1)
    lo = _centroids_hex(n) - 0.5 * h
    out = np.empty((lo.shape[0], 6, 3))
    for k, perm in enumerate(itertools.permutations(range(3))):
        off = np.zeros(3)
        off[perm[0]], off[perm[1]], off[perm[2]] = 0.75, 0.5, 0.25
        out[:, k, :] = lo + h * off
    return out.reshape(-1, 3)


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_sigma_at_uniform_temperature_is_the_stated_law(kind):
    p = ri.make_problem(kind, 7, 3)
    m = Model(p)
    # 47 C: 0.33 * 1.15 = 0.3795 S/m; 37 C: 0.33; 37 - 1/0.015 C: zero conductivity
    for T, want in ((47.0, 0.3795), (37.0, 0.33), (37.0 - 1.0 / 0.015, 0.0)):
        s = m.sigma(np.full(p.n_nodes, T))
        np.testing.assert_allclose(s, want, rtol=1e-14, atol=1e-15)
    assert m.sigma(np.full(p.n_nodes, 60.0))[0] > m.sigma(np.full(p.n_nodes, 40.0))[0]


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_sigma_of_a_linear_field_is_its_value_at_the_centroid(kind):
    """The element mean of the nodal values of a linear field is the field at the vertex
    centroid, which the mesh's index structure gives in closed form."""
    n = 8
    p = ri.make_problem(kind, n, 5, jitter=False)
    g = np.array([900.0, -400.0, 650.0])            # K/m
    T = 40.0 + p.xyz @ g
    want_T = 40.0 + (_centroids_hex(n) if kind == "hex" else _centroids_kuhn(n)) @ g
    want = SIGMA_37 * (1.0 + ALPHA * (want_T - 37.0))
    np.testing.assert_allclose(Model(p).sigma(T), want, rtol=1e-13)


def test_step_potential_uses_sigma_of_the_starting_temperature():
    """A step from a strongly non-uniform T^n: its V solves the potential system whose
    conductivity is the closed-form centroid law applied to T^n, and not the one of
    T^{n+1}."""
    n = 8
    p = ri.make_problem("hex", n, 9, jitter=False)
    m = Model(p)
    g = np.array([2500.0, 1500.0, -2000.0])
    Tn = 45.0 + p.xyz @ g
    Tn[p.dir_ids] = p.dir_T
    T1, V1, _ = m.step(Tn, p.initial_V(), 1e-14)

    def residual(sig):
        A, b = m.potential_system(sig)
        return np.linalg.norm(b - A @ V1) / np.linalg.norm(b)

    # sigma from T^n by the closed form, except elements that touch a Dirichlet node where
    # T^n was overwritten: there the mean is taken from the nodal values themselves
    cen_T = 45.0 + _centroids_hex(n) @ g
    touched = np.isin(p.conn, p.dir_ids).any(axis=1)
    sig_n = SIGMA_37 * (1.0 + ALPHA * (cen_T - 37.0))
    sig_n[touched] = m.sigma(Tn)[touched]
    assert not touched.all()
    assert residual(sig_n) < 1e-12
    sig_next = m.sigma(T1)
    assert residual(sig_next) > 1e-6


def _hat_moments(n):
    """int hat_i(x) dx and int hat_i(x) x^2 dx of the 1-D piecewise-linear hat functions
    on the nodes x_i = i h of [0, L]."""
    L = ri.SIDE_M
    h = L / (n - 1)
    x = np.arange(n) * h
    I0 = np.full(n, h)
    I2 = h * x ** 2 + h ** 3 / 6.0
    I0[0] = I0[-1] = h / 2.0
    I2[0] = h ** 3 / 12.0                                   # int_0^h (1 - x/h) x^2 dx
    a = L - h                                              # int_a^L ((x - a)/h) x^2 dx
    I2[-1] = h ** 3 / 4.0 + 2.0 * a * h ** 2 / 3.0 + a * a * h / 2.0
    return I0, I2


def test_joule_load_of_a_trilinear_potential_node_by_node():
    """V = x y z: |grad V|^2 = y^2 z^2 + x^2 z^2 + x^2 y^2, so with uniform sigma
    F_(i,j,k) = sigma [I0_i I2_j I2_k + I2_i I0_j I2_k + I2_i I2_j I0_k]."""
    n = 7
    p = ri.make_problem("hex", n, 2)
    m = Model(p)
    V = p.xyz[:, 0] * p.xyz[:, 1] * p.xyz[:, 2] * 1e6
    s = 0.41
    F = m.joule(np.full(p.n_elems, s), V)
    I0, I2 = _hat_moments(n)
    ids = np.arange(p.n_nodes)
    i, j, k = ids % n, (ids // n) % n, ids // (n * n)
    want = s * 1e12 * (I0[i] * I2[j] * I2[k] + I2[i] * I0[j] * I2[k] + I2[i] * I2[j] * I0[k])
    np.testing.assert_allclose(F, want, rtol=1e-12)
    # and the load is quadratic in V and linear in sigma
    np.testing.assert_allclose(m.joule(np.full(p.n_elems, 2 * s), 3 * V), 18 * F, rtol=1e-13)


def test_joule_load_of_a_linear_potential_on_kuhn_tets():
    """On the undistorted Kuhn split every tet has volume h^3/6; a cube corner at offset
    (0,0,0) or (1,1,1) lies in all six of its cube's tets, any other corner in two.  A
    linear V has a constant gradient E, so F_i = sigma |E|^2 (h^3/24) sum over the cubes at
    node i of that count."""
    n = 6
    p = ri.make_problem("tet", n, 4, jitter=False)
    m = Model(p)
    E = np.array([300.0, -120.0, 80.0])
    s = 0.29
    F = m.joule(np.full(p.n_elems, s), 5.0 + p.xyz @ E)
    h = ri.SIDE_M / (n - 1)
    ids = np.arange(p.n_nodes)
    pos = np.stack([ids % n, (ids // n) % n, ids // (n * n)], axis=1)
    count = np.zeros(p.n_nodes)
    for off in itertools.product((0, 1), repeat=3):
        cube = pos - np.array(off)
        inside = np.all((cube >= 0) & (cube <= n - 2), axis=1)
        count += inside * (6 if off in ((0, 0, 0), (1, 1, 1)) else 2)
    want = s * (E @ E) * h ** 3 / 24.0 * count
    np.testing.assert_allclose(F, want, rtol=1e-12)
    assert count.max() == 24


def test_sigma_enters_the_assembled_potential_matrix_linearly():
    """Doubling sigma0 doubles every value of the unlifted potential matrix (no mass
    term), and the potential itself is unchanged (homogeneous in sigma)."""
    p = ri.make_problem("tet", 6, 1)
    q = dataclasses.replace(p, sigma0_e=2.0 * p.sigma0_e)
    T = p.initial_T() + np.linspace(0.0, 9.0, p.n_nodes)
    mp, mq = Model(p), Model(q)
    vp = mp.S.assemble(mp.Ke, mp.Me, None, mp.sigma(T))
    vq = mq.S.assemble(mq.Ke, mq.Me, None, mq.sigma(T))
    np.testing.assert_allclose(vq, 2.0 * vp, rtol=1e-14, atol=1e-18)
    Ap, bp = mp.potential_system(mp.sigma(T))
    Aq, bq = mq.potential_system(mq.sigma(T))
    Vp, _ = pcg(Ap, bp, p.initial_V(), 1e-14)
    Vq, _ = pcg(Aq, bq, p.initial_V(), 1e-14)
    np.testing.assert_allclose(Vq, Vp, rtol=0, atol=1e-11 * ri.V_ELECTRODE)

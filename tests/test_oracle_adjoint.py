"""Pins of the oracle's discrete adjoint: complex-step derivatives (machine precision),
a Taylor-remainder rate, and the cancellation-free loss difference used by FD checks."""
import dataclasses

import numpy as np
import pytest

import rafem_inputs as ri
from oracle import adjoint as adj
from oracle.rafem import Model


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_adjoint_matches_complex_step(kind):
    p = ri.make_problem(kind, 6, 3, steps=3, with_loss=True)
    m = Model(p)
    L, gk, gw = adj.adjoint_gradients(m, 3, 0.0, "dense")
    rng = np.random.default_rng(1)
    dk, dw = rng.normal(size=p.n_elems), rng.normal(size=p.n_elems)
    for a, b in ((dk, dw), (dk, 0 * dw), (0 * dk, dw)):
        cs = adj.complex_step_directional(m, 3, a, b)
        assert abs(gk @ a + gw @ b - cs) <= 1e-11 * abs(cs)
    # single-element derivatives agree too
    for e in rng.choice(p.n_elems, 3, replace=False):
        unit = np.zeros(p.n_elems)
        unit[e] = 1.0
        cs = adj.complex_step_directional(m, 3, unit, 0 * unit)
        assert abs(gk[e] - cs) <= 1e-10 * abs(cs) + 1e-14 * np.abs(gk).max()


def test_sigma_coupling_is_visible_to_the_pin():
    """The sigma(T) chain changes the gradient far above the pin's tolerance, so an adjoint
    that dropped it would fail the complex-step pin."""
    p = ri.make_problem("hex", 6, 3, steps=3, with_loss=True)
    rng = np.random.default_rng(1)
    dk = rng.normal(size=p.n_elems)
    with_chain = adj.complex_step_directional(Model(p), 3, dk, 0 * dk)
    q = dataclasses.replace(p, alpha_sigma=0.0)
    without = adj.complex_step_directional(Model(q), 3, dk, 0 * dk)
    assert abs(with_chain - without) > 1e-6 * abs(with_chain)


def test_pcg_adjoint_matches_dense_adjoint():
    p = ri.make_problem("hex", 7, 4, steps=2, with_loss=True)
    m = Model(p)
    _, gk, gw = adj.adjoint_gradients(m, 2, 0.0, "dense")
    _, gk2, gw2 = adj.adjoint_gradients(m, 2, 1e-14, "pcg")
    np.testing.assert_allclose(gk2, gk, rtol=0, atol=1e-9 * np.abs(gk).max())
    np.testing.assert_allclose(gw2, gw, rtol=0, atol=1e-9 * np.abs(gw).max())


def test_taylor_remainder_is_second_order():
    p = ri.make_problem("tet", 5, 2, steps=2, with_loss=True)
    m = Model(p)
    L0, gk, gw = adj.adjoint_gradients(m, 2, 0.0, "dense")
    rng = np.random.default_rng(5)
    dk = rng.normal(size=p.n_elems) * p.k_e
    rem = []
    for eps in (1e-1, 5e-2, 2.5e-2):
        T, _ = adj.forward(m, 2, 0.0, "dense", p.k_e + eps * dk, None)
        rem.append(abs(adj.loss(p, T[2]) - L0 - eps * (gk @ dk)))
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    assert np.all(rates > 1.8) and np.all(rates < 2.2), rates


def test_loss_delta_equals_difference():
    p = ri.make_problem("hex", 6, 0, with_loss=True)
    rng = np.random.default_rng(0)
    a = 37 + rng.normal(size=p.n_nodes)
    b = a + 1e-3 * rng.normal(size=p.n_nodes)
    assert abs(adj.loss_delta(p, b, a) - (adj.loss(p, b) - adj.loss(p, a))) <= 1e-9

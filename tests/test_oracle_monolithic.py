"""Pins of the oracle's monolithic corrector: the Jacobian against complex-step derivatives
of the residual, the 2x2-block structure, the Newton root against the staggered Picard
corrector's fixed point, quadratic convergence, and GMRES against the minimal-residual
definition (brute force over an explicit Krylov basis), an exact solve, monotone restarts
and the block-Jacobi preconditioner's defining property."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import rafem_inputs as ri
from oracle import corrector as pc
from oracle import elements
from oracle import monolithic as mono
from oracle.rafem import Model

DT = 20.0


def _state(p, m, seed=0, noise=(0.5, 0.3)):
    """A non-trivial state carrying the Dirichlet values: one staggered step plus noise."""
    rng = np.random.default_rng(seed)
    T1, V1, _ = m.step(p.initial_T(), p.initial_V(), 1e-14)
    T = T1 + noise[0] * rng.standard_normal(p.n_nodes)
    V = V1 + noise[1] * rng.standard_normal(p.n_nodes)
    T[p.dir_ids], V[p.dir_ids] = p.dir_T, p.dir_V
    return T, V


def _free_direction(p, rng):
    d = rng.standard_normal(2 * p.n_nodes)
    d[2 * p.dir_ids] = 0.0
    d[2 * p.dir_ids + 1] = 0.0
    return d


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_jacobian_matches_complex_step_derivative(kind):
    p = ri.make_problem(kind, 6, 1)
    m = Model(p)
    T, V = _state(p, m)
    J = mono.interleaved_matrix(m, mono.jacobian_blocks(m, p.initial_T(), DT, T, V))
    rng = np.random.default_rng(3)
    for _ in range(3):
        d = _free_direction(p, rng)
        h = 1e-30
        cs = mono.residual(m, p.initial_T(), DT, T + 1j * h * d[0::2], V + 1j * h * d[1::2]).imag / h
        assert rel(J @ d, cs) <= 1e-12
    # each coupling block on its own (a dropped or sign-flipped block fails here too)
    for block in (0, 1):
        d = _free_direction(p, rng)
        d[block::2] = 0.0
        cs = mono.residual(m, p.initial_T(), DT, T + 1j * 1e-30 * d[0::2],
                           V + 1j * 1e-30 * d[1::2]).imag / 1e-30
        assert rel(J @ d, cs) <= 1e-12


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_joule_jacobian_agrees_with_the_transpose_product(kind):
    p = ri.make_problem(kind, 5, 2)
    xe = p.xyz[p.conn]
    rng = np.random.default_rng(4)
    Ve = rng.standard_normal(p.conn.shape)
    sig = p.sigma0_e
    mu = rng.standard_normal(p.conn.shape)
    Jv = elements.joule_jacobian_V(xe, sig, Ve)
    assert np.allclose(np.einsum("ea,eab->eb", mu, Jv), elements.joule_grad_V(xe, sig, Ve, mu),
                       rtol=1e-12, atol=1e-12 * np.abs(Jv).max())
    # f is quadratic in V: f(V) = (1/2) J(V) V exactly
    f = elements.joule_loads(xe, sig, Ve)
    assert np.allclose(0.5 * np.einsum("eab,eb->ea", Jv, Ve), f, rtol=1e-12,
                       atol=1e-13 * np.abs(f).max())


@pytest.mark.parametrize("kind,n", [("hex", 6), ("tet", 7)])
def test_structure_has_full_2x2_node_blocks_symmetric_pattern(kind, n):
    p = ri.make_problem(kind, n, 1)
    m = Model(p)
    T, V = _state(p, m)
    B = mono.jacobian_blocks(m, p.initial_T(), DT, T, V)
    J = mono.interleaved_matrix(m, B)
    assert J.shape == (2 * p.n_nodes, 2 * p.n_nodes)
    assert J.nnz == 4 * m.S.nnz                      # every node pair carries a full block
    P = (J != 0).astype(np.int8)
    # pattern symmetric up to the Dirichlet rows and columns, which are the identity's
    free = np.ones(2 * p.n_nodes, dtype=bool)
    free[2 * p.dir_ids] = free[2 * p.dir_ids + 1] = False
    Pf = P[free][:, free]
    assert (Pf != Pf.T).nnz == 0
    Jf = J[free][:, free]
    assert spla.norm(Jf - Jf.T) > 1e-3 * spla.norm(Jf)  # not symmetric in value
    # rows per node: 2 x (node degree)
    deg = np.diff(m.S.row_ptr)
    assert np.array_equal(np.diff(J.indptr)[0::2], 2 * deg)


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_newton_root_is_the_picard_fixed_point(kind):
    p = ri.make_problem(kind, 7, 1)
    m = Model(p)
    T0, V0 = p.initial_T(), p.initial_V()
    pic = pc.corrector_step(m, T0, V0, DT, T0.copy(), 1e-15, 1e-14)
    new = mono.newton_step(m, T0, V0, DT, T0.copy(), 1e-14, linear="direct")
    assert pic.converged and new.converged
    assert new.iters < pic.iters
    assert rel(new.T, pic.T) <= 1e-11 and rel(new.V, pic.V) <= 1e-11
    # and the Picard fixed point is a root of the monolithic residual
    R = mono.residual(m, T0, DT, pic.T, pic.V)
    scale = np.linalg.norm(mono.residual(m, T0, DT, T0, pic.V))
    assert np.linalg.norm(R) <= 1e-11 * scale


def test_newton_converges_quadratically():
    p = ri.make_problem("hex", 7, 2)
    m = Model(p)
    T0, V0 = p.initial_T(), p.initial_V()
    T, V = T0.copy(), V0.copy()
    T[p.dir_ids], V[p.dir_ids] = p.dir_T, p.dir_V
    ref = mono.newton_step(m, T0, V0, DT, T0.copy(), 1e-15, linear="direct")
    errs = []
    for _ in range(4):
        R = mono.residual(m, T0, DT, T, V)
        J = mono.interleaved_matrix(m, mono.jacobian_blocks(m, T0, DT, T, V))
        d = spla.spsolve(J.tocsc(), -R)
        T, V = T + d[0::2], V + d[1::2]
        errs.append(np.linalg.norm(np.concatenate([T - ref.T, V - ref.V])))
    # e_{k+1} <= C e_k^2 with one C across the sweep, and far below linear contraction
    ratios = [errs[k + 1] / errs[k] ** 2 for k in range(2) if errs[k] > 1e-10]
    assert len(ratios) == 2 and max(ratios) <= 10 * min(ratios) + 1e-300
    assert errs[2] <= 1e-3 * errs[1]


def _small_system(kind="hex", n=5):
    p = ri.make_problem(kind, n, 3)
    m = Model(p)
    T, V = _state(p, m, noise=(2.0, 1.0))
    J = mono.interleaved_matrix(m, mono.jacobian_blocks(m, p.initial_T(), DT, T, V))
    b = -mono.residual(m, p.initial_T(), DT, T, V)
    return J, b


@pytest.mark.parametrize("k", [1, 3, 6])
def test_gmres_iterate_minimises_the_residual_over_the_krylov_space(k):
    J, b = _small_system()
    Minv = mono.block_jacobi(J)
    rng = np.random.default_rng(5)
    x0 = 1e-3 * rng.standard_normal(b.size)
    x, info = mono.gmres(J, b, x0, m=20, tol=1e-300, max_iters=k, precond=Minv)
    assert info.iters == k and info.cycles == 1
    # brute force: min over y of || r0 - A M^{-1} Q y ||, Q an orthonormal basis of
    # span{r0, (A M^{-1}) r0, ..., (A M^{-1})^{k-1} r0}
    r0 = b - J @ x0
    AM = lambda v: J @ Minv(v)
    cols = [r0 / np.linalg.norm(r0)]
    for _ in range(k - 1):
        w = AM(cols[-1])
        cols.append(w / np.linalg.norm(w))
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    W = np.stack([AM(Q[:, i]) for i in range(k)], axis=1)
    y, *_ = np.linalg.lstsq(W, r0, rcond=None)
    best = np.linalg.norm(r0 - W @ y)
    got = np.linalg.norm(b - J @ x)
    assert abs(got - best) <= 1e-9 * np.linalg.norm(r0)
    assert abs(info.relres * np.linalg.norm(b) - got) <= 1e-9 * np.linalg.norm(r0)


def test_full_gmres_is_an_exact_solver():
    J, b = _small_system("tet", 5)
    n2 = b.size
    x, info = mono.gmres(J, b, np.zeros(n2), m=n2, tol=1e-13, precond=mono.block_jacobi(J))
    assert info.converged and info.cycles == 1 and info.iters <= n2
    assert rel(x, np.linalg.solve(J.toarray(), b)) <= 1e-10


def test_restarted_gmres_is_monotone_and_reaches_the_tolerance():
    p = ri.make_problem("hex", 8, 1)
    m = Model(p)
    T, V = _state(p, m)
    J = mono.interleaved_matrix(m, mono.jacobian_blocks(m, p.initial_T(), DT, T, V))
    b = -mono.residual(m, p.initial_T(), DT, T, V)
    x, info = mono.gmres(J, b, np.zeros_like(b), m=5, tol=1e-10, precond=mono.block_jacobi(J))
    assert info.converged and info.cycles > 3 and info.relres_true <= 1e-10
    h = np.array(info.history)
    assert np.all(np.diff(h) <= 1e-12 * h[0])       # minimal residual never grows, restarts included
    assert rel(x, spla.spsolve(J.tocsc(), b)) <= 1e-8
    # without the preconditioner the same system needs more iterations
    _, plain = mono.gmres(J, b, np.zeros_like(b), m=5, tol=1e-10, max_iters=20 * info.iters)
    assert plain.iters > info.iters


def test_block_jacobi_inverts_the_diagonal_node_blocks():
    J, _ = _small_system("tet", 5)
    Minv = mono.block_jacobi(J)
    n = J.shape[0] // 2
    rng = np.random.default_rng(6)
    for i in rng.choice(n, 5, replace=False):
        for c in (2 * i, 2 * i + 1):
            e = np.zeros(2 * n)
            e[c] = 1.0
            col = Minv(e)                                # D^{-1} e_c: nonzero on node i only
            assert np.count_nonzero(col) <= 2 and set(np.nonzero(col)[0]) <= {2 * i, 2 * i + 1}
            blk = J[2 * i:2 * i + 2, 2 * i:2 * i + 2].toarray() @ col[2 * i:2 * i + 2]
            assert np.allclose(blk, e[2 * i:2 * i + 2], atol=1e-12)


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_newton_with_gmres_matches_newton_with_lu(kind):
    p = ri.make_problem(kind, 7, 2)
    m = Model(p)
    T0, V0 = p.initial_T(), p.initial_V()
    a = mono.newton_step(m, T0, V0, DT, T0.copy(), 1e-12, linear="direct")
    b = mono.newton_step(m, T0, V0, DT, T0.copy(), 1e-12, linear="gmres", m=20, lin_tol=1e-12)
    assert a.converged and b.converged and a.iters == b.iters
    assert rel(b.T, a.T) <= 1e-11 and rel(b.V, a.V) <= 1e-11
    assert all(i.converged and i.relres_true <= 1e-11 for i in b.linear)

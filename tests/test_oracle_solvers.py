"""Pins of the oracle's Jacobi-PCG: exact eigenvector solves, dense LU, failure reporting."""
import numpy as np
import pytest
import scipy.sparse as sp

import rafem_inputs as ri
from oracle import elements
from oracle.assembly import Structure
from oracle.rafem import Model
from oracle.solvers import pcg, dense_solve, BREAKDOWN, NOCONV, OK


def _faces_only_system(n, a, c):
    xyz = ri.grid_xyz(n)
    conn = ri.hex_conn(n)
    S = Structure(conn, n ** 3)
    K, M = elements.hex_matrices(xyz[conn])
    vals = S.assemble(K, M, np.full(conn.shape[0], a), np.full(conn.shape[0], c))
    faces = ri.face_node_ids(n)
    lv, lift = S.lift(vals, faces, np.zeros(faces.size))
    return S.matrix(lv), xyz


@pytest.mark.parametrize("n,a,c", [(9, 0.0, 0.5), (9, 3.8e6, 0.5), (13, 0.0, 1.0)])
def test_discrete_eigenvector_solve(n, a, c):
    """v = prod sin(m pi i/(n-1)) is an eigenvector of the lifted uniform hex operator.

    Eigenvalue  mu = a prod lamM + c sum_d lamK_d prod_{e != d} lamM_e  with the 1-D
    symbols lamK = (2/h)(1 - cos t), lamM = (h/3)(2 + cos t).  Solving A x = v gives v / mu.
    """
    A, xyz = _faces_only_system(n, a, c)
    h = ri.SIDE_M / (n - 1)
    idx = np.round(xyz / h).astype(int)
    modes = (1, 2, 3)
    th = [m * np.pi / (n - 1) for m in modes]
    v = np.ones(n ** 3)
    for d in range(3):
        v *= np.sin(th[d] * idx[:, d])
    lamK = [(2 / h) * (1 - np.cos(t)) for t in th]
    lamM = [(h / 3) * (2 + np.cos(t)) for t in th]
    mu = a * np.prod(lamM) + c * (lamK[0] * lamM[1] * lamM[2] + lamM[0] * lamK[1] * lamM[2]
                                  + lamM[0] * lamM[1] * lamK[2])
    np.testing.assert_allclose(A @ v, mu * v, rtol=0, atol=1e-12 * abs(mu) * np.abs(v).max())
    x, info = pcg(A, v, np.zeros_like(v), tol=1e-13)
    assert info.status == OK
    np.testing.assert_allclose(x, v / mu, rtol=0, atol=1e-11 * np.abs(v / mu).max())


@pytest.mark.parametrize("kind", ["hex", "tet"])
@pytest.mark.parametrize("n", [3, 5, 7])
def test_pcg_matches_dense_lu(kind, n):
    n = max(n, 5)
    p = ri.make_problem(kind, n, n)
    m = Model(p)
    A, lift = m.bioheat_system()
    b = m.bioheat_rhs(p.initial_T(), np.zeros(p.n_nodes), lift)
    x, info = pcg(A, b, p.initial_T(), tol=1e-14)
    xd = dense_solve(A, b)
    assert info.status == OK and info.relres_true < 1e-13
    np.testing.assert_allclose(x, xd, rtol=1e-12)
    Av, bv = m.potential_system(p.sigma0_e)
    x, info = pcg(Av, bv, p.initial_V(), tol=1e-14)
    np.testing.assert_allclose(x, dense_solve(Av, bv), rtol=0, atol=1e-12 * ri.V_ELECTRODE)


def test_pcg_zero_rhs_and_exact_start():
    A = sp.csr_matrix(np.diag([2.0, 3.0, 4.0]))
    x, info = pcg(A, np.zeros(3), np.zeros(3), tol=1e-12)
    assert info.status == OK and info.iters == 0
    b = np.array([2.0, 3.0, 4.0])
    x, info = pcg(A, b, np.ones(3), tol=1e-12)
    assert info.status == OK and info.iters == 0
    # Jacobi-preconditioned CG solves a diagonal system in one iteration
    x, info = pcg(A, b, np.zeros(3), tol=1e-12)
    assert info.iters == 1 and np.allclose(x, 1.0)


def test_pcg_failure_reporting():
    A = sp.csr_matrix(-np.eye(4) + 0.1 * np.diag(np.ones(3), 1) + 0.1 * np.diag(np.ones(3), -1))
    _, info = pcg(A, np.ones(4), np.zeros(4), tol=1e-12)
    assert info.status == BREAKDOWN
    p = ri.make_problem("hex", 7, 0)
    m = Model(p)
    Av, bv = m.potential_system(p.sigma0_e)
    _, info = pcg(Av, bv, p.initial_V(), tol=1e-12, maxit=1)
    assert info.status == NOCONV and info.iters == 1
    bad = bv.copy()
    bad[3] = np.nan
    _, info = pcg(Av, bad, p.initial_V(), tol=1e-12)
    assert info.status != OK

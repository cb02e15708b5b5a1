"""Pins of the oracle's CSR structure, assembly and Dirichlet lifting."""
import numpy as np
import pytest
import scipy.sparse as sp

import rafem_inputs as ri
from oracle.assembly import Structure, csr_structure
from oracle.rafem import Model


def _brute_structure(conn, n_nodes):
    pairs = set()
    for el in conn.tolist():
        for a in el:
            for b in el:
                pairs.add((a, b))
    rows = [[] for _ in range(n_nodes)]
    for a, b in pairs:
        rows[a].append(b)
    row_ptr = [0]
    cols = []
    for r in rows:
        cols.extend(sorted(r))
        row_ptr.append(len(cols))
    return np.array(row_ptr), np.array(cols)


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_nnz_closed_forms(n):
    _, ch = csr_structure(ri.hex_conn(n), n ** 3)
    assert ch.size == (3 * n - 2) ** 3
    _, ct = csr_structure(ri.kuhn_tet_conn(n), n ** 3)
    assert ct.size == n ** 3 + 2 * (3 * n * n * (n - 1) + 3 * n * (n - 1) ** 2 + (n - 1) ** 3)


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_structure_brute_force(kind):
    n = 4
    conn = ri.hex_conn(n) if kind == "hex" else ri.kuhn_tet_conn(n)
    rp, ci = csr_structure(conn, n ** 3)
    brp, bci = _brute_structure(conn, n ** 3)
    assert np.array_equal(rp, brp) and np.array_equal(ci, bci)
    assert rp.dtype == np.int32 and ci.dtype == np.int32


def test_kuhn_split_is_conforming_and_fills_the_cube():
    n = 5
    p = ri.make_problem("tet", n, 0, jitter=False)
    V, _ = __import__("oracle").elements.tet_geometry(p.xyz[p.conn])
    assert np.all(V > 0)
    np.testing.assert_allclose(V.sum(), ri.SIDE_M ** 3, rtol=1e-12)
    # conforming: every interior triangular face is shared by exactly two tets
    faces = {}
    for el in p.conn.tolist():
        for skip in range(4):
            f = tuple(sorted(el[:skip] + el[skip + 1:]))
            faces[f] = faces.get(f, 0) + 1
    assert max(faces.values()) == 2


def _kron_1d(n, h):
    K1 = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil() / h
    K1[0, 0] = K1[n - 1, n - 1] = 1 / h
    M1 = sp.diags([np.ones(n - 1), 4 * np.ones(n), np.ones(n - 1)], [-1, 0, 1]).tolil() * h / 6
    M1[0, 0] = M1[n - 1, n - 1] = 2 * h / 6
    return K1.tocsr(), M1.tocsr()


@pytest.mark.parametrize("n", [5, 8])
def test_kronecker_sum_identity(n):
    """Uniform coefficients on the hex grid: A = a M(x)M(x)M + c (K(x)M(x)M + M(x)K(x)M + M(x)M(x)K)."""
    p = ri.make_problem("hex", n, 0)
    m = Model(p)
    a, c = 3.5e4, 0.61
    vals = m.S.assemble(m.Ke, m.Me, np.full(p.n_elems, a), np.full(p.n_elems, c))
    A = m.S.matrix(vals).toarray()
    K1, M1 = _kron_1d(n, p.h)
    # node id = i + n j + n^2 k (x fastest)  ->  kron(z, kron(y, x))
    kr = lambda zz, yy, xx: sp.kron(zz, sp.kron(yy, xx))
    Ax = a * kr(M1, M1, M1) + c * (kr(M1, M1, K1) + kr(M1, K1, M1) + kr(K1, M1, M1))
    Ax = Ax.toarray()
    np.testing.assert_allclose(A, Ax, rtol=0, atol=1e-13 * np.abs(Ax).max())
    # and the structure is exactly the Kronecker pattern
    assert m.S.nnz == sp.csr_matrix(Ax).nnz


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_symmetry_spd_conservation(kind):
    n = 6
    p = ri.make_problem(kind, n, 0)
    m = Model(p)
    vals = m.bioheat_values()
    A = m.S.matrix(vals)
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
    M = m.S.matrix(m.S.assemble(m.Ke, m.Me, np.ones(p.n_elems), None))
    K = m.S.matrix(m.S.assemble(m.Ke, m.Me, None, np.ones(p.n_elems)))
    np.testing.assert_allclose(M.sum(), ri.SIDE_M ** 3, rtol=1e-12)
    np.testing.assert_allclose(K @ np.ones(p.n_nodes), 0, atol=1e-13 * abs(K).max())
    lv, _ = m.S.lift(vals, p.dir_ids, p.dir_T)
    Al = m.S.matrix(lv).toarray()
    assert np.array_equal(Al, Al.T) or np.abs(Al - Al.T).max() <= 1e-14 * np.abs(Al).max()
    assert np.linalg.eigvalsh(Al).min() > 0
    Kl, _ = m.S.lift(m.S.assemble(m.Ke, m.Me, None, p.sigma0_e), p.dir_ids, p.dir_V)
    assert np.linalg.eigvalsh(m.S.matrix(Kl).toarray()).min() > 0


def test_lifting_matches_partitioned_solve():
    n = 6
    p = ri.make_problem("hex", n, 4)
    m = Model(p)
    vals = m.bioheat_values()
    lv, lift = m.S.lift(vals, p.dir_ids, p.dir_T)
    assert lv.size == vals.size  # structure kept, explicit zeros stored
    A = m.S.matrix(vals).toarray()
    D = p.dir_ids
    F = np.setdiff1d(np.arange(p.n_nodes), D)
    rhs = np.random.default_rng(0).normal(size=p.n_nodes)
    rhs[D] = 0
    xf = np.linalg.solve(A[np.ix_(F, F)], rhs[F] - A[np.ix_(F, D)] @ p.dir_T)
    b = rhs + lift
    b[D] = lift[D]
    x = np.linalg.solve(m.S.matrix(lv).toarray(), b)
    np.testing.assert_allclose(x[F], xf, rtol=1e-12)
    np.testing.assert_allclose(x[D], p.dir_T, rtol=0, atol=0)
    # lifted rows of D are unit rows, lifted columns of D are zero off the diagonal
    Al = m.S.matrix(lv).toarray()
    np.testing.assert_array_equal(Al[np.ix_(D, D)], np.eye(D.size))
    assert np.all(Al[np.ix_(F, D)] == 0) and np.all(Al[np.ix_(D, F)] == 0)


def test_structure_independent_of_dirichlet_and_values():
    p = ri.make_problem("hex", 5, 0)
    s1 = Structure(p.conn, p.n_nodes)
    rp, ci = csr_structure(p.conn, p.n_nodes)
    assert np.array_equal(s1.row_ptr, rp) and np.array_equal(s1.col_idx, ci)
    # every slot is hit by at least one element entry
    assert np.unique(s1.slot).size == s1.nnz


def test_bad_connectivity_rejected():
    conn = ri.hex_conn(4).copy()
    conn[3, 2] = 64
    with pytest.raises(ValueError):
        csr_structure(conn, 64)

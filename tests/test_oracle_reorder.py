"""Pins of the oracle's reverse Cuthill-McKee ordering: bandwidth 1 on a shuffled path, a
corner start on a grid, the breadth-first level property, components kept contiguous, and
bandwidths no worse than SciPy's RCM on the unstructured meshes."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

import rafem_inputs as ri
from oracle import reorder
from oracle.assembly import csr_structure


def _path_conn(n, rng):
    """Segments of a path 0-1-...-(n-1) as degenerate 'elements' of two nodes, relabelled."""
    lab = rng.permutation(n)
    return np.stack([lab[:-1], lab[1:]], axis=1).astype(np.int32), lab


def test_shuffled_path_gets_bandwidth_one():
    rng = np.random.default_rng(0)
    conn, lab = _path_conn(40, rng)
    order = reorder.rcm_order(conn, 40)
    assert sorted(order.tolist()) == list(range(40))
    assert reorder.bandwidth(conn, 40, order) == 1
    # the start of the search is an end of the path, so the order walks the path
    assert order[-1] in (lab[0], lab[-1])


def test_grid_starts_at_a_corner_and_is_breadth_first():
    p = ri.make_problem("hex", 6, 0)
    order = reorder.rcm_order(p.conn, p.n_nodes)
    cm = order[::-1]                                    # the Cuthill-McKee order
    corners = {0, 5, 30, 35, 180, 185, 210, 215}        # i, j, k in {0, 5}
    assert int(cm[0]) in corners
    # breadth-first: graph distance from the start never decreases along the order
    rp, ci = csr_structure(p.conn, p.n_nodes)
    G = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(p.n_nodes,) * 2)
    from scipy.sparse.csgraph import shortest_path
    d = shortest_path(G, unweighted=True, indices=int(cm[0]))
    assert np.all(np.diff(d[cm]) >= 0)


def test_components_stay_contiguous():
    a = ri.make_problem("tet", 5, 0)
    b = ri.make_problem("hex", 5, 1)
    n = a.n_nodes + b.n_nodes
    conn_b = b.conn + a.n_nodes
    # the second mesh's tets (4 of each hex's nodes) keep it one component
    conn = np.concatenate([a.conn, conn_b[:, :4], conn_b[:, 4:]]).astype(np.int32)
    order = reorder.rcm_order(conn, n)
    first = order < a.n_nodes
    # reversed order: the component of node 0 (processed first) comes last
    assert first[-a.n_nodes:].all() and not first[:b.n_nodes].any()


@pytest.mark.parametrize("mesh", ["liverA", "liverB", "tet9"])
def test_unstructured_bandwidth_matches_scipy(mesh):
    p = {"liverA": ri.liver_mesh_a, "liverB": ri.liver_mesh_b,
         "tet9": lambda: ri.make_problem("tet", 9, 0)}[mesh]()
    order = reorder.rcm_order(p.conn, p.n_nodes)
    assert np.array_equal(np.sort(order), np.arange(p.n_nodes))
    rp, ci = csr_structure(p.conn, p.n_nodes)
    G = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(p.n_nodes,) * 2)
    sc = reverse_cuthill_mckee(G, symmetric_mode=True)
    bw, bw_sc = reorder.bandwidth(p.conn, p.n_nodes, order), reorder.bandwidth(p.conn, p.n_nodes, sc)
    assert bw <= 1.1 * bw_sc
    if mesh.startswith("liver"):   # shuffled node ids: RCM shrinks the bandwidth a lot
        assert bw <= 0.25 * reorder.bandwidth(p.conn, p.n_nodes)


def test_degree_sort_windows():
    p = ri.liver_mesh_a()
    order = reorder.rcm_order(p.conn, p.n_nodes)
    w = 256
    srt = reorder.degree_sort(order, p.conn, p.n_nodes, w)
    rp, _ = csr_structure(p.conn, p.n_nodes)
    deg = np.diff(rp) - 1
    for s in range(0, p.n_nodes, w):
        a, b = order[s:s + w], srt[s:s + w]
        assert np.array_equal(np.sort(a), np.sort(b))           # same nodes per window
        d = deg[b]
        assert np.all(np.diff(d) >= 0)                           # increasing degree
        pos = {v: k for k, v in enumerate(a)}                    # ties keep their order
        for k in range(len(b) - 1):
            if d[k] == d[k + 1]:
                assert pos[b[k]] < pos[b[k + 1]]
    # slabs of 64 rows: fewer padded slots than the plain RCM order
    def slots(o):
        dd = np.diff(rp)[o]
        dd = np.concatenate([dd, np.zeros((-dd.size) % 64, int)]).reshape(-1, 64)
        return int((dd.max(axis=1) * 64).sum())
    assert slots(srt) < 0.9 * slots(order)

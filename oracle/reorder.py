"""Reverse Cuthill-McKee ordering of the mesh's node graph (oracle; test infrastructure only).

The paper names reverse Cuthill-McKee among the permutations applied in the analysis step
of sparse solvers (Sec. II-B).  Here it orders the nodes of unstructured meshes so that
the rows of a slab, and the x entries they read, lie close together.  The ordering is the
textbook one (Cuthill and McKee 1969; George and Liu, "Computer Solution of Large Sparse
Positive Definite Systems", 1981), made deterministic by explicit tie-breaking:

* graph: nodes adjacent when they share an element (the CSR structure without the diagonal);
* components in order of their smallest node id;
* start node of a component: the pseudo-peripheral node of George and Liu -- begin at the
  component's node of least degree (ties: smallest id), build its BFS level structure,
  move to the node of least degree (ties: smallest id) in the last level, and repeat while
  the number of levels grows;
* Cuthill-McKee: breadth-first from the start node, the unvisited neighbours of each node
  taken in increasing degree (ties: smallest id);
* the concatenated order, reversed.

Returns ``order`` with order[k] = the old id of the node placed at position k.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from .assembly import csr_structure


def _adjacency(conn: np.ndarray, n_nodes: int):
    rp, ci = csr_structure(conn, n_nodes)
    nbrs = [ci[rp[i]:rp[i + 1]] for i in range(n_nodes)]
    nbrs = [a[a != i] for i, a in enumerate(nbrs)]       # drop the diagonal
    deg = np.array([a.size for a in nbrs], dtype=np.int64)
    return nbrs, deg


def _levels(start: int, nbrs, allowed: np.ndarray):
    """BFS level structure from start within the nodes marked in ``allowed``."""
    seen = {start}
    levels = [[start]]
    while True:
        nxt = []
        for v in levels[-1]:
            for w in nbrs[v]:
                w = int(w)
                if allowed[w] and w not in seen:
                    seen.add(w)
                    nxt.append(w)
        if not nxt:
            return levels
        levels.append(nxt)


def _least(nodes, deg):
    return min(nodes, key=lambda v: (deg[v], v))


def pseudo_peripheral(component, nbrs, deg, allowed):
    r = _least(component, deg)
    levels = _levels(r, nbrs, allowed)
    while True:
        cand = _least(levels[-1], deg)
        lv = _levels(cand, nbrs, allowed)
        if len(lv) > len(levels):
            r, levels = cand, lv
        else:
            return r


def rcm_order(conn: np.ndarray, n_nodes: int) -> np.ndarray:
    nbrs, deg = _adjacency(np.asarray(conn), n_nodes)
    visited = np.zeros(n_nodes, dtype=bool)
    order = []
    for seed in range(n_nodes):
        if visited[seed]:
            continue
        # the component of seed
        comp_mask = np.zeros(n_nodes, dtype=bool)
        comp = []
        q = deque([seed])
        comp_mask[seed] = True
        while q:
            v = q.popleft()
            comp.append(v)
            for w in nbrs[v]:
                if not comp_mask[w]:
                    comp_mask[w] = True
                    q.append(int(w))
        start = pseudo_peripheral(comp, nbrs, deg, comp_mask)
        # Cuthill-McKee from start
        visited[start] = True
        q = deque([start])
        while q:
            v = q.popleft()
            order.append(v)
            new = [int(w) for w in nbrs[v] if not visited[w]]
            new.sort(key=lambda w: (deg[w], w))
            for w in new:
                visited[w] = True
                q.append(w)
    return np.array(order[::-1], dtype=np.int32)


def bandwidth(conn: np.ndarray, n_nodes: int, order=None) -> int:
    """max |pos(i) - pos(j)| over node pairs sharing an element (pos = position in order)."""
    pos = np.arange(n_nodes) if order is None else np.argsort(order)
    c = pos[np.asarray(conn)]
    return int((c.max(axis=1) - c.min(axis=1)).max())


def degree_sort(order: np.ndarray, conn: np.ndarray, n_nodes: int, window: int) -> np.ndarray:
    """Within consecutive windows of ``window`` positions of ``order``, the nodes sorted by
    increasing degree (number of graph neighbours), ties kept in their order.  Slabs of 64
    consecutive rows then hold rows of nearly equal length."""
    _, deg = _adjacency(np.asarray(conn), n_nodes)
    out = np.array(order, dtype=np.int32, copy=True)
    for s in range(0, n_nodes, window):
        seg = out[s:s + window].copy()
        keyed = sorted(range(seg.size), key=lambda k: (deg[seg[k]], k))
        out[s:s + window] = seg[keyed]
    return out

"""Global CSR structure, element-order assembly and Dirichlet lifting (oracle).

The paper assembles the element equations into one global matrix stored in
CSR (Sec. III-A) whose sparsity structure stays the same across time steps, so
it is analysed once and reused (Sec. III-B).  Readings used here:

* the structure is every (i, j) pair of nodes that share an element, for all
  nodes, whatever the boundary conditions; columns sorted ascending, zero-based;
* A = sum_e (a_e M_e + c_e K_e), contributions added in element order;
* Dirichlet conditions by symmetric lifting that keeps the structure: for free
  rows f, b_f -= A_fD g; then rows and columns of D are zeroed (explicit zeros
  stay stored), A_dd = 1 and b_d = g_d.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def csr_structure(conn: np.ndarray, n_nodes: int):
    """CSR pattern of the node graph: (row_ptr int32 [N+1], col_idx int32 [nnz]).

    Built as the sorted set of keys row * N + col over all node pairs of all elements.
    """
    conn = np.asarray(conn, dtype=np.int64)
    if conn.min() < 0 or conn.max() >= n_nodes:
        raise ValueError("connectivity refers to a node outside [0, n_nodes)")
    rows = np.repeat(conn, conn.shape[1], axis=1).ravel()
    cols = np.tile(conn, (1, conn.shape[1])).ravel()
    keys = np.unique(rows * n_nodes + cols)
    r = keys // n_nodes
    c = keys % n_nodes
    counts = np.bincount(r, minlength=n_nodes)
    row_ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32")
    return row_ptr.astype(np.int32), c.astype(np.int32)


class Structure:
    """CSR structure of one mesh plus the slot of every element entry (cached per mesh)."""

    def __init__(self, conn: np.ndarray, n_nodes: int):
        self.conn = np.asarray(conn, dtype=np.int64)
        self.n = int(n_nodes)
        self.row_ptr, self.col_idx = csr_structure(conn, n_nodes)
        self.nnz = int(self.col_idx.shape[0])
        row_of = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        struct_keys = row_of * self.n + self.col_idx
        npe = self.conn.shape[1]
        rows = np.repeat(self.conn, npe, axis=1)
        cols = np.tile(self.conn, (1, npe))
        # slot[e, a*npe + b] = position of (conn[e,a], conn[e,b]) in the CSR arrays
        self.slot = np.searchsorted(struct_keys, rows * self.n + cols)
        self.row_of = row_of

    def assemble(self, Ke: np.ndarray, Me: np.ndarray, a_e, c_e) -> np.ndarray:
        """values[nnz] of sum_e (a_e M_e + c_e K_e); a_e or c_e may be None (= 0)."""
        E, npe, _ = Ke.shape
        contrib = np.zeros((E, npe, npe), dtype=np.result_type(Ke, a_e if a_e is not None else 0.0,
                                                               c_e if c_e is not None else 0.0))
        if a_e is not None:
            contrib = contrib + np.asarray(a_e)[:, None, None] * Me
        if c_e is not None:
            contrib = contrib + np.asarray(c_e)[:, None, None] * Ke
        flat = contrib.reshape(-1)
        idx = self.slot.reshape(-1)
        # bincount sums its weights in input order, i.e. in element order.
        if np.iscomplexobj(flat):
            return (np.bincount(idx, weights=flat.real, minlength=self.nnz)
                    + 1j * np.bincount(idx, weights=flat.imag, minlength=self.nnz))
        return np.bincount(idx, weights=flat, minlength=self.nnz)

    def scatter_vector(self, fe: np.ndarray) -> np.ndarray:
        """Global vector sum_e P_e^T f_e from element vectors fe [E, npe]."""
        idx = self.conn.reshape(-1)
        if np.iscomplexobj(fe):
            return (np.bincount(idx, weights=fe.real.reshape(-1), minlength=self.n)
                    + 1j * np.bincount(idx, weights=fe.imag.reshape(-1), minlength=self.n))
        return np.bincount(idx, weights=fe.reshape(-1), minlength=self.n)

    def matrix(self, values: np.ndarray) -> sp.csr_matrix:
        """SciPy CSR view of values on this structure (explicit zeros kept)."""
        return sp.csr_matrix((values, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def lift(self, values: np.ndarray, dir_ids: np.ndarray, g: np.ndarray):
        """Symmetric Dirichlet lifting.  Returns (lifted values, lift vector).

        lift vector: free rows f get -sum_{d in D} A_fd g_d; Dirichlet rows d get g_d.
        The caller's right-hand side for the lifted system is  b_phys (zeroed on D) + lift.
        """
        isD = np.zeros(self.n, dtype=bool)
        isD[dir_ids] = True
        gfull = np.zeros(self.n, dtype=np.result_type(values, g))
        gfull[dir_ids] = g
        A = self.matrix(values)
        lift = -(A @ gfull)
        lift[isD] = gfull[isD]
        out = np.array(values, copy=True)
        d_row = isD[self.row_of]
        d_col = isD[self.col_idx]
        out[d_row | d_col] = 0.0
        out[d_row & (self.row_of == self.col_idx)] = 1.0
        return out, lift


def lifted_rhs(b_phys: np.ndarray, lift: np.ndarray, dir_ids: np.ndarray) -> np.ndarray:
    """Right-hand side of the lifted system: b_phys on free rows + lift; g on Dirichlet rows."""
    b = b_phys + lift
    b[dir_ids] = lift[dir_ids]
    return b

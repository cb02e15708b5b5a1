"""Monolithic two-unknowns-per-node corrector, solved by restarted GMRES (oracle; test
infrastructure only).

The paper's corrector assembles the element equations, evaluated with the latest values,
into one global matrix that is sparse and structurally symmetric, with two unknowns per
mesh node (temperature and potential: the matrix order is twice the node count, Table II),
and solves it with GMRES(m) or sparse QR (Sec. II-A, Sec. II-B, Sec. III-B, Fig. 3).  The
paper prints neither the equations nor the linearisation; the readings used here are:

* unknowns x = (T, V) of the implicit coupled step, interleaved by node
  (x[2i] = T_i, x[2i+1] = V_i); the state always carries the Dirichlet values;
* residual at free nodes (Dirichlet rows are 0):
      R_T = sum_e [(rho c/dt + w_e) M_e + k_e K_e] T_e - M_e ((rho c/dt) T^n_e + w_e T_a)
            - f_e(sigma_e(T), V_e)                      (f: Joule loads, elements.joule_loads)
      R_V = sum_e sigma_e(T) K_e V_e
  with sigma_e(T) = sigma0_e (1 + alpha (mean_e(T) - T_ref)) -- its root is the fixed point of
  the staggered Picard corrector (corrector.corrector_step);
* corrector iteration = one Newton step J delta = -R, J the exact Jacobian, whose element
  blocks are (c_e = sigma0_e alpha / npe, 1 = the all-ones row):
      dR_T/dT = (rho c/dt + w_e) M_e + k_e K_e - c_e q_e 1^T    (q_e = f_e with sigma = 1)
      dR_T/dV = -d f_e / d V_e                                 (elements.joule_jacobian_V)
      dR_V/dT = c_e (K_e V_e) 1^T
      dR_V/dV = sigma_e K_e
  Every element couples all its nodes in both unknowns, so J has full 2x2 node blocks on the
  node graph: structurally symmetric, non-symmetric in value.  Dirichlet unknowns do not
  move: their rows and columns are replaced by those of the identity;
* stopping: ||delta_T||_2 <= eps ||T^{k+1}||_2, as for the staggered corrector;
* linear solver: restarted GMRES(m) with right preconditioning (Saad, Alg. 9.5) by the
  inverse of J's 2x2 diagonal node blocks (block Jacobi), Arnoldi by modified Gram-Schmidt
  (Saad, Alg. 6.2), the least-squares problem by Givens rotations (Saad, Sec. 6.5.3);
  a cycle stops when the rotated residual |g_{j+1}| <= tol ||b||, and a restart
  recomputes the true residual b - A x and stops there when it meets the same test.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import elements
from .rafem import Model, _CHUNK


# --- residual and Jacobian -----------------------------------------------------------------

def _blocks(model: Model, T_n: np.ndarray, dt: float, T: np.ndarray, V: np.ndarray,
            want_jacobian: bool = True):
    """Element residual vectors and element Jacobian blocks, chunk by chunk.

    Yields (element slice, rT [e,a], rV [e,a], TT, TV, VT, VV [e,a,b] or None)."""
    p = model.p
    npe = p.conn.shape[1]
    sig = model.sigma(T)
    for s in range(0, p.n_elems, _CHUNK):
        e = slice(s, s + _CHUNK)
        conn = p.conn[e]
        Ke, Me, xe = model.Ke[e], model.Me[e], model.xe[e]
        Te, Ve, Tne = T[conn], V[conn], T_n[conn]
        a_e = p.rho_c / dt + p.perf_e[e]
        A_T = a_e[:, None, None] * Me + p.k_e[e][:, None, None] * Ke
        f = elements.joule_loads(xe, sig[e], Ve)
        rT = (np.einsum("eab,eb->ea", A_T, Te)
              - np.einsum("eab,eb->ea", Me, (p.rho_c / dt) * Tne + (p.perf_e[e] * p.T_a)[:, None])
              - f)
        KV = np.einsum("eab,eb->ea", Ke, Ve)
        rV = sig[e][:, None] * KV
        if not want_jacobian:
            yield e, rT, rV, None, None, None, None
            continue
        c = (p.sigma0_e[e] * p.alpha_sigma / npe)[:, None, None]
        q = elements.joule_loads(xe, np.ones_like(sig[e]), Ve)
        ones = np.ones((1, 1, npe))
        TT = A_T - c * q[:, :, None] * ones
        TV = -elements.joule_jacobian_V(xe, sig[e], Ve)
        VT = c * KV[:, :, None] * ones
        VV = sig[e][:, None, None] * Ke
        yield e, rT, rV, TT, TV, VT, VV


def residual(model: Model, T_n: np.ndarray, dt: float, T: np.ndarray, V: np.ndarray) -> np.ndarray:
    """R(x) [2N], interleaved (R[2i] = R_T,i, R[2i+1] = R_V,i); 0 on Dirichlet nodes."""
    p = model.p
    n = p.n_nodes
    dtype = np.result_type(T, V)
    R = np.zeros(2 * n, dtype=dtype)
    for e, rT, rV, *_ in _blocks(model, T_n, dt, T, V, want_jacobian=False):
        idx = p.conn[e].reshape(-1)
        R[0::2] += _scatter(idx, rT.reshape(-1), n)
        R[1::2] += _scatter(idx, rV.reshape(-1), n)
    R[2 * p.dir_ids] = 0.0
    R[2 * p.dir_ids + 1] = 0.0
    return R


def _scatter(idx, w, n):
    if np.iscomplexobj(w):
        return (np.bincount(idx, weights=w.real, minlength=n)
                + 1j * np.bincount(idx, weights=w.imag, minlength=n))
    return np.bincount(idx, weights=w, minlength=n)


@dataclasses.dataclass
class NodeBlocks:
    """The Jacobian on the node graph: four value planes in the node CSR order of
    ``model.S`` (TT, TV, VT, VV), Dirichlet rows and columns already replaced."""
    TT: np.ndarray
    TV: np.ndarray
    VT: np.ndarray
    VV: np.ndarray


def jacobian_blocks(model: Model, T_n: np.ndarray, dt: float, T: np.ndarray,
                    V: np.ndarray) -> NodeBlocks:
    p = model.p
    S = model.S
    planes = [np.zeros(S.nnz) for _ in range(4)]
    for e, _, _, *blk in _blocks(model, T_n, dt, T, V):
        idx = S.slot[e].reshape(-1)
        for k in range(4):
            planes[k] += np.bincount(idx, weights=blk[k].reshape(-1), minlength=S.nnz)
    isD = np.zeros(p.n_nodes, dtype=bool)
    isD[p.dir_ids] = True
    d_row, d_col = isD[S.row_of], isD[S.col_idx]
    diag = S.row_of == S.col_idx
    for k in range(4):
        planes[k][d_row | d_col] = 0.0
    planes[0][d_row & diag] = 1.0
    planes[3][d_row & diag] = 1.0
    return NodeBlocks(*planes)


def interleaved_matrix(model: Model, B: NodeBlocks) -> sp.csr_matrix:
    """The 2N x 2N matrix with row 2i (T) and 2i+1 (V), columns interleaved the same way."""
    S = model.S
    r, c = S.row_of, S.col_idx
    rows = np.concatenate([2 * r, 2 * r, 2 * r + 1, 2 * r + 1])
    cols = np.concatenate([2 * c, 2 * c + 1, 2 * c, 2 * c + 1])
    vals = np.concatenate([B.TT, B.TV, B.VT, B.VV])
    n2 = 2 * S.n
    return sp.csr_matrix((vals, (rows, cols)), shape=(n2, n2))


def block_jacobi(A: sp.csr_matrix) -> Callable[[np.ndarray], np.ndarray]:
    """v -> D^{-1} v with D the 2x2 diagonal blocks of A (node i: rows/columns 2i, 2i+1)."""
    d = A.diagonal()
    off_up = A.diagonal(1)[0::2]        # A[2i, 2i+1]
    off_lo = A.diagonal(-1)[0::2]       # A[2i+1, 2i]
    a, b, c, e = d[0::2], off_up, off_lo, d[1::2]
    det = a * e - b * c
    ia, ib, ic, ie = e / det, -b / det, -c / det, a / det

    def apply(v):
        out = np.empty_like(v)
        out[0::2] = ia * v[0::2] + ib * v[1::2]
        out[1::2] = ic * v[0::2] + ie * v[1::2]
        return out
    return apply


# --- restarted GMRES -----------------------------------------------------------------------

@dataclasses.dataclass
class GmresInfo:
    converged: bool
    iters: int                  # Arnoldi steps over all cycles
    cycles: int
    relres: float               # last rotated (estimated) residual / ||b||
    relres_true: float          # ||b - A x|| / ||b|| at exit
    history: List[float]        # estimated ||r|| / ||b|| after every Arnoldi step


def gmres(A, b: np.ndarray, x0: np.ndarray, m: int, tol: float, max_iters: int = 100000,
          precond: Optional[Callable[[np.ndarray], np.ndarray]] = None):
    """Restarted right-preconditioned GMRES(m).  Returns (x, GmresInfo)."""
    Minv = precond if precond is not None else (lambda v: v)
    x = np.array(x0, dtype=float, copy=True)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return np.zeros_like(x), GmresInfo(True, 0, 0, 0.0, 0.0, [])
    total, cycles, history = 0, 0, []
    est = np.inf
    while True:
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        if beta <= tol * bnorm or total >= max_iters:
            return x, GmresInfo(beta <= tol * bnorm, total, cycles, est if total else beta / bnorm,
                                beta / bnorm, history)
        cycles += 1
        Vb = np.zeros((m + 1, b.size))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        Vb[0] = r / beta
        j_done = 0
        for j in range(m):
            w = A @ Minv(Vb[j])
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = np.dot(w, Vb[i])
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                Vb[j + 1] = w / H[j + 1, j]
            for i in range(j):                           # earlier rotations on column j
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            est = abs(g[j + 1]) / bnorm
            history.append(est)
            if est <= tol or total >= max_iters or H[j, j] == 0.0:
                break
        k = j_done
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):                   # back substitution
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Minv(Vb[:k].T @ y)


# --- the Newton corrector ------------------------------------------------------------------

@dataclasses.dataclass
class NewtonResult:
    T: np.ndarray
    V: np.ndarray
    iters: int                  # Newton steps performed
    converged: bool
    change: float               # last ||delta_T|| / ||T||
    linear: List[GmresInfo]     # one per Newton step (empty for the direct solver)


def newton_step(model: Model, T_n: np.ndarray, V_n: np.ndarray, dt: float, T_guess: np.ndarray,
                eps: float, max_iters: int = 50, linear: str = "gmres", m: int = 30,
                lin_tol: float = 1e-10, lin_max_iters: int = 100000) -> NewtonResult:
    """One corrector step of size dt from (T^n, V^n), Newton on the monolithic system,
    starting from (T_guess, V^n) with the Dirichlet values imposed.  ``linear``: "gmres"
    (GMRES(m), block Jacobi, relative tolerance lin_tol) or "direct" (sparse LU)."""
    p = model.p
    T = np.array(T_guess, dtype=float, copy=True)
    V = np.array(V_n, dtype=float, copy=True)
    T[p.dir_ids], V[p.dir_ids] = p.dir_T, p.dir_V
    infos: List[GmresInfo] = []
    change = np.inf
    for k in range(1, max_iters + 1):
        R = residual(model, T_n, dt, T, V)
        J = interleaved_matrix(model, jacobian_blocks(model, T_n, dt, T, V))
        if linear == "direct":
            delta = spla.spsolve(J.tocsc(), -R)
        else:
            delta, info = gmres(J, -R, np.zeros_like(R), m, lin_tol, lin_max_iters,
                                block_jacobi(J))
            infos.append(info)
        T = T + delta[0::2]
        V = V + delta[1::2]
        change = float(np.linalg.norm(delta[0::2]) / np.linalg.norm(T))
        if change <= eps:
            return NewtonResult(T, V, k, True, change, infos)
    return NewtonResult(T, V, max_iters, False, change, infos)

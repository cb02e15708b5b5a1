"""Element matrices and element loads (oracle; test infrastructure only).

Textbook Galerkin FEM on the meshes the paper describes (Sec. II-A: FEM on a
mesh of elements, element equations assembled into a global sparse matrix;
Sec. III-A: one element at a time).  The paper never prints its element
equations, so these are the standard forms:

* trilinear 8-node hex (Q1), 2x2x2 Gauss-Legendre rule (points +-1/sqrt(3),
  weight 1): K_e = sum_g detJ B^T B, M_e = sum_g detJ N N^T;
* linear 4-node tet (P1): K_e = V G G^T, M_e = (V/20)(1 + delta_ab).

All functions are vectorised over a batch of elements and accept complex input
coordinates / fields so that the complex-step derivative can run through them.
"""
from __future__ import annotations

import itertools

import numpy as np

# Reference coordinates of the 8 hex nodes in the local order
# (0,0,0), (1,0,0), (1,1,0), (0,1,0), (0,0,1), (1,0,1), (1,1,1), (0,1,1)  -> xi = 2*offset - 1.
_HEX_OFFSETS = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                         [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.float64)
HEX_XI = 2.0 * _HEX_OFFSETS - 1.0

_G = 1.0 / np.sqrt(3.0)
# 2x2x2 Gauss points (weights are all 1).
HEX_GAUSS = np.array(list(itertools.product((-_G, _G), repeat=3)), dtype=np.float64)


def hex_shape(xi: np.ndarray):
    """Trilinear shape functions and their reference gradients at points xi [P, 3].

    N_a(xi) = 1/8 prod_d (1 + xi_a,d xi_d);  returns N [P, 8] and dN [P, 8, 3].
    """
    f = 1.0 + xi[:, None, :] * HEX_XI[None, :, :]          # [P, 8, 3]
    N = 0.125 * f[..., 0] * f[..., 1] * f[..., 2]
    dN = np.empty(f.shape, dtype=np.float64)
    dN[..., 0] = 0.125 * HEX_XI[None, :, 0] * f[..., 1] * f[..., 2]
    dN[..., 1] = 0.125 * HEX_XI[None, :, 1] * f[..., 0] * f[..., 2]
    dN[..., 2] = 0.125 * HEX_XI[None, :, 2] * f[..., 0] * f[..., 1]
    return N, dN


def hex_gauss_geometry(xe: np.ndarray):
    """Per element and Gauss point: detJ [E, 8] and physical shape gradients [E, 8g, 8a, 3].

    J_g = sum_a x_a (dN_a/dxi)^T  (J[i, d] = dx_i / dxi_d);  grad_x N_a = J^{-T} grad_xi N_a.
    Raises if any detJ <= 0 (inverted or degenerate element).
    """
    N, dN = hex_shape(HEX_GAUSS)                              # [8g, 8a], [8g, 8a, 3]
    J = np.einsum("eai,gad->egid", xe, dN)                     # [E, 8g, 3, 3]
    det = np.linalg.det(J) if not np.iscomplexobj(J) else _det3(J)
    if np.any(np.real(det) <= 0):
        raise ValueError("hex element with non-positive Jacobian determinant")
    Jinv = np.linalg.inv(J)                                    # [E, 8g, 3, 3], Jinv[d, i] = dxi_d/dx_i
    grad = np.einsum("egdi,gad->egai", Jinv, dN)               # [E, 8g, 8a, 3]
    return det, N, grad


def _det3(J):
    return (J[..., 0, 0] * (J[..., 1, 1] * J[..., 2, 2] - J[..., 1, 2] * J[..., 2, 1])
            - J[..., 0, 1] * (J[..., 1, 0] * J[..., 2, 2] - J[..., 1, 2] * J[..., 2, 0])
            + J[..., 0, 2] * (J[..., 1, 0] * J[..., 2, 1] - J[..., 1, 1] * J[..., 2, 0]))


def hex_matrices(xe: np.ndarray):
    """Stiffness and consistent mass of trilinear hexes.  xe [E, 8, 3] -> K, M [E, 8, 8]."""
    det, N, grad = hex_gauss_geometry(xe)
    K = np.einsum("eg,egai,egbi->eab", det, grad, grad)
    M = np.einsum("eg,ga,gb->eab", det, N, N)
    return K, M


def tet_geometry(xe: np.ndarray):
    """Volume V [E] and constant barycentric gradients G [E, 4, 3] of linear tets.

    With Jt = [x1-x0, x2-x0, x3-x0] (columns), lambda_{1..3} = Jt^{-1}(x - x0), so
    grad lambda_k (k = 1..3) is row k-1 of Jt^{-1} and grad lambda_0 = -sum of the others.
    Raises if any volume is <= 0.
    """
    Jt = np.stack([xe[:, 1] - xe[:, 0], xe[:, 2] - xe[:, 0], xe[:, 3] - xe[:, 0]], axis=2)
    det = _det3(Jt)
    if np.any(np.real(det) <= 0):
        raise ValueError("tet element with non-positive volume")
    V = det / 6.0
    Jinv = np.linalg.inv(Jt)                                   # [E, 3, 3]
    G = np.empty((xe.shape[0], 4, 3), dtype=Jinv.dtype)
    G[:, 1:, :] = Jinv
    G[:, 0, :] = -Jinv.sum(axis=1)
    return V, G


def tet_matrices(xe: np.ndarray):
    """Stiffness and consistent mass of linear tets.  xe [E, 4, 3] -> K, M [E, 4, 4]."""
    V, G = tet_geometry(xe)
    K = V[:, None, None] * np.einsum("eai,ebi->eab", G, G)
    M = (V / 20.0)[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None]
    return K, M


def element_matrices(xe: np.ndarray):
    """Dispatch on nodes per element (8: hex, 4: tet)."""
    if xe.shape[1] == 8:
        return hex_matrices(xe)
    if xe.shape[1] == 4:
        return tet_matrices(xe)
    raise ValueError("only 8-node hexes and 4-node tets are supported")


def joule_loads(xe: np.ndarray, sigma_e: np.ndarray, Ve: np.ndarray) -> np.ndarray:
    """Element Joule-heating loads f_{e,a} = int_e N_a sigma_e grad V . grad V  -> [E, npe].

    Hex: 2x2x2 Gauss rule.  Tet: grad V is constant, int N_a = V/4.  grad V . grad V is
    written without complex conjugation so the complex-step derivative passes through.
    """
    if xe.shape[1] == 8:
        det, N, grad = hex_gauss_geometry(xe)
        gV = np.einsum("ea,egai->egi", Ve, grad)               # [E, 8g, 3]
        q = np.einsum("egi,egi->eg", gV, gV) * det             # detJ * |grad V|^2 at Gauss points
        return sigma_e[:, None] * np.einsum("eg,ga->ea", q, N)
    V, G = tet_geometry(xe)
    gV = np.einsum("ea,eai->ei", Ve, G)
    q = np.einsum("ei,ei->e", gV, gV)
    return (sigma_e * q * V / 4.0)[:, None] * np.ones((1, 4))


def joule_grad_V(xe: np.ndarray, sigma_e: np.ndarray, Ve: np.ndarray, mu_e: np.ndarray) -> np.ndarray:
    """Transpose-Jacobian product of the Joule loads with respect to V:

    out_{e,b} = sum_a mu_{e,a} d f_{e,a} / d V_{e,b} = int_e sigma_e 2 (sum_a mu_a N_a) grad N_b . grad V.
    """
    if xe.shape[1] == 8:
        det, N, grad = hex_gauss_geometry(xe)
        gV = np.einsum("ea,egai->egi", Ve, grad)
        muN = np.einsum("ea,ga->eg", mu_e, N)                  # mu interpolated at Gauss points
        w = 2.0 * det * muN                                     # [E, 8g]
        return sigma_e[:, None] * np.einsum("eg,egbi,egi->eb", w, grad, gV)
    V, G = tet_geometry(xe)
    gV = np.einsum("ea,eai->ei", Ve, G)
    mubar = mu_e.sum(axis=1) * V / 4.0
    return (2.0 * sigma_e * mubar)[:, None] * np.einsum("ebi,ei->eb", G, gV)


def joule_jacobian_V(xe: np.ndarray, sigma_e: np.ndarray, Ve: np.ndarray) -> np.ndarray:
    """Jacobian of the Joule loads with respect to the element's nodal V:

    d f_{e,a} / d V_{e,b} = int_e 2 sigma_e N_a grad N_b . grad V  -> [E, npe, npe].
    Hex: 2x2x2 Gauss rule.  Tet: grad N and grad V are constant, int N_a = V/4.
    """
    if xe.shape[1] == 8:
        det, N, grad = hex_gauss_geometry(xe)
        gV = np.einsum("ea,egai->egi", Ve, grad)               # [E, 8g, 3]
        gNgV = np.einsum("egbi,egi->egb", grad, gV)            # grad N_b . grad V at Gauss points
        return 2.0 * sigma_e[:, None, None] * np.einsum("eg,ga,egb->eab", det, N, gNgV)
    V, G = tet_geometry(xe)
    gV = np.einsum("ea,eai->ei", Ve, G)
    row = 2.0 * (sigma_e * V / 4.0)[:, None] * np.einsum("ebi,ei->eb", G, gV)   # same for every a
    return np.repeat(row[:, None, :], 4, axis=1)

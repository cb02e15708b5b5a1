"""Pins of the oracle's element matrices and element loads against closed forms."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import elements

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "element_matrices.txt")

HEX_OFFS = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                     [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=float)


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        out[key] = [float(Fraction(v)) for v in vals]
    return out


def test_hex_cube_matches_closed_form():
    g = _golden()
    for h in (1.0, 0.2e-3, 3.7):
        K, M = elements.hex_matrices((HEX_OFFS * h)[None])
        dist = np.abs(HEX_OFFS[:, None, :] - HEX_OFFS[None, :, :]).sum(axis=2).astype(int)
        Kx = h * np.array(g["hex_stiffness_by_distance"])[dist]
        Mx = h ** 3 * np.array(g["hex_mass_by_distance"])[dist]
        np.testing.assert_allclose(K[0], Kx, rtol=0, atol=1e-14 * h)
        np.testing.assert_allclose(M[0], Mx, rtol=0, atol=1e-14 * h ** 3)


def test_reference_tet_matches_closed_form():
    g = _golden()
    xe = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]], dtype=float)
    K, M = elements.tet_matrices(xe)
    Kx = np.array([g[f"tet_ref_stiffness_row{i}"] for i in range(4)])
    Mx = np.full((4, 4), g["tet_ref_mass_off"][0]) + np.eye(4) * (g["tet_ref_mass_diag"][0] - g["tet_ref_mass_off"][0])
    np.testing.assert_allclose(K[0], Kx, atol=1e-15)
    np.testing.assert_allclose(M[0], Mx, atol=1e-16)


def _affine_hexes(rng, count):
    """Parallelepipeds x = A (offset * h) + t: Q1 contains linear fields exactly on these."""
    out, dets = [], []
    for _ in range(count):
        A = np.eye(3) + 0.3 * rng.uniform(-1, 1, size=(3, 3))
        while np.linalg.det(A) <= 0.2:
            A = np.eye(3) + 0.3 * rng.uniform(-1, 1, size=(3, 3))
        h = rng.uniform(0.5, 2.0)
        out.append(HEX_OFFS * h @ A.T + rng.uniform(-1, 1, size=3))
        dets.append(np.linalg.det(A) * h ** 3)
    return np.array(out), np.array(dets)


def test_hex_invariants_on_distorted_elements():
    rng = np.random.default_rng(1)
    xe, vol = _affine_hexes(rng, 20)
    K, M = elements.hex_matrices(xe)
    # rows of K sum to zero (constants are in the kernel), M sums to the volume
    np.testing.assert_allclose(K.sum(axis=2), 0, atol=1e-13 * np.abs(K).max())
    np.testing.assert_allclose(M.sum(axis=(1, 2)), vol, rtol=1e-13)
    # energy of a linear field u = c.x is |c|^2 vol (exact for affine maps with 2x2x2 Gauss)
    c = rng.normal(size=(20, 3))
    u = np.einsum("eai,ei->ea", xe, c)
    energy = np.einsum("ea,eab,eb->e", u, K, u)
    np.testing.assert_allclose(energy, (c ** 2).sum(axis=1) * vol, rtol=1e-12)
    # symmetric positive semi-definite with exactly one zero eigenvalue
    ev = np.linalg.eigvalsh(K)
    assert np.all(ev[:, 0] > -1e-12 * ev[:, -1]) and np.all(ev[:, 1] > 1e-6 * ev[:, -1])


def test_hex_trilinear_map_volume():
    # a genuinely trilinear (non-affine) hex: volume by fine midpoint integration of detJ
    xe = HEX_OFFS.copy()
    xe[6] += [0.2, 0.1, 0.3]
    xe[1] += [0.1, -0.05, 0.0]
    _, M = elements.hex_matrices(xe[None])
    # independent estimate: divergence theorem would need faces; use dense tensor quadrature
    pts = (np.arange(40) + 0.5) / 40 * 2 - 1
    X, Y, Z = np.meshgrid(pts, pts, pts, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    _, dN = elements.hex_shape(xi)
    J = np.einsum("ai,pad->pid", xe, dN)
    vol = np.linalg.det(J).sum() * (2 / 40) ** 3
    # detJ of a trilinear map is a polynomial of degree <= 2 per axis: midpoint rule error O(1/40^2)
    assert abs(M.sum() - vol) < 1e-3 * vol


def test_inverted_elements_rejected():
    xe = HEX_OFFS.copy()[None]
    xe[0, [0, 1]] = xe[0, [1, 0]]
    with pytest.raises(ValueError):
        elements.hex_matrices(xe)
    tet = np.array([[[0, 0, 0], [0, 1, 0], [1, 0, 0], [0, 0, 1]]], dtype=float)
    with pytest.raises(ValueError):
        elements.tet_matrices(tet)


def test_tet_invariants_random():
    rng = np.random.default_rng(2)
    xe = rng.uniform(size=(50, 4, 3))
    det = np.linalg.det(np.stack([xe[:, 1] - xe[:, 0], xe[:, 2] - xe[:, 0], xe[:, 3] - xe[:, 0]], axis=2))
    xe[det < 0, 2], xe[det < 0, 3] = xe[det < 0, 3].copy(), xe[det < 0, 2].copy()
    K, M = elements.tet_matrices(xe)
    V, G = elements.tet_geometry(xe)
    np.testing.assert_allclose(K.sum(axis=2), 0, atol=1e-12 * np.abs(K).max())
    np.testing.assert_allclose(M.sum(axis=(1, 2)), V, rtol=1e-13)
    # gradients reproduce a linear field exactly
    c = rng.normal(size=3)
    u = xe @ c
    np.testing.assert_allclose(np.einsum("ea,eai->ei", u, G), np.broadcast_to(c, (50, 3)), rtol=1e-9, atol=1e-9)


def test_joule_uniform_field():
    """Linear potential V = E.x: loads integrate sigma |E|^2 N_a; on a cube each is sigma |E|^2 h^3 / 8."""
    h, sigma = 0.5, 0.7
    E = np.array([3.0, -1.0, 2.0])
    xe = (HEX_OFFS * h)[None]
    Ve = xe[0] @ E
    f = elements.joule_loads(xe, np.array([sigma]), Ve[None])
    np.testing.assert_allclose(f[0], sigma * (E @ E) * h ** 3 / 8, rtol=1e-13)
    tet = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]], dtype=float)
    f = elements.joule_loads(tet, np.array([sigma]), (tet[0] @ E)[None])
    np.testing.assert_allclose(f[0], sigma * (E @ E) / 6 / 4, rtol=1e-13)


@pytest.mark.parametrize("npe", [8, 4])
def test_joule_vjp_matches_directional_derivative(npe):
    rng = np.random.default_rng(3)
    if npe == 8:
        xe, _ = _affine_hexes(rng, 5)
    else:
        xe = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]] * 5, dtype=float) + rng.uniform(0, 0.1, (5, 4, 3))
    sig = rng.uniform(0.2, 0.5, size=5)
    Ve = rng.normal(size=(5, npe))
    mu = rng.normal(size=(5, npe))
    dV = rng.normal(size=(5, npe))
    # complex step: exact directional derivative of f along dV
    fcs = elements.joule_loads(xe, sig, Ve + 1e-30j * dV).imag / 1e-30
    lhs = np.einsum("ea,ea->e", mu, fcs)
    rhs = np.einsum("eb,eb->e", elements.joule_grad_V(xe, sig, Ve, mu), dV)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)

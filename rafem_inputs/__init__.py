"""Seeded synthetic inputs for the radiofrequency-ablation FEM solves.

This module produces DATA ONLY: node coordinates, element connectivity, the
Dirichlet node sets with their prescribed values, per-element material fields,
the loss region and its target temperatures.  It contains none of the method's
arithmetic (no element matrices, no assembly, no solver), so that both the CPU
oracle and the GPU library can take their inputs from it without sharing any
computation.

Workload shapes follow the paper's setting (Sec. II-A: tetrahedral meshes of
liver tissue with an electrode; Table II: mesh sizes) scaled to one GPU:

* hex meshes: an n x n x n node cube of side L = 2 cm, trilinear 8-node hexes;
* tet meshes: the same grid with every hex split into the 6 Kuhn tetrahedra
  along its (0,0,0)-(1,1,1) diagonal, interior non-electrode nodes jittered by
  U(-0.2h, 0.2h) per coordinate;
* Dirichlet set D = outer faces (0 V, 37 C) united with an axial electrode
  line through the centre spanning 4 mm (20 V, 90 C);
* material fields: k_e = 0.512 (1 + eps_e), eps_e ~ U(-0.1, 0.1) per element,
  perfusion 6.4e-3 * 4180, sigma0 = 0.33; rho*c = 1060 * 3600.

Draw order from ``numpy.random.default_rng(seed)``: eps per element, then the
jitter per node (x, y, z), then the loss targets, then batch samples.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import List, Optional

import numpy as np

SIDE_M = 0.02            # cube side length [m]
ELECTRODE_HALF_M = 2e-3  # electrode half-length [m] (4 mm line)
LOSS_RADIUS_M = 8e-3     # loss region: nodes within 8 mm of the electrode segment

RHO_C = 1060.0 * 3600.0  # volumetric heat capacity [J/m^3/K]
PERFUSION = 6.4e-3 * 4180.0
K_TISSUE = 0.512         # thermal conductivity [W/m/K]
SIGMA0 = 0.33            # electrical conductivity at the reference temperature [S/m]
ALPHA_SIGMA = 0.015      # temperature coefficient of sigma [1/K]
T_REF = 37.0             # reference temperature for sigma(T) [C]
T_ARTERIAL = 37.0        # arterial blood temperature [C]
T_FACES = 37.0
T_ELECTRODE = 90.0
V_FACES = 0.0
V_ELECTRODE = 20.0

# Local node order of a hex element, as offsets (di, dj, dk) from its lowest corner.
HEX_LOCAL_OFFSETS = ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                     (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1))


@dataclasses.dataclass
class Problem:
    """One RFA problem instance (all arrays host NumPy, C-contiguous)."""
    name: str
    kind: str                 # "hex" or "tet"
    n: int                    # nodes per cube edge
    h: float                  # grid spacing [m]
    xyz: np.ndarray           # float64 [N, 3]
    conn: np.ndarray          # int32 [E, 8] (hex) or [E, 4] (tet)
    electrode_ids: np.ndarray  # int32, sorted
    dir_ids: np.ndarray       # int32 [nD], sorted unique (faces U electrode)
    dir_V: np.ndarray         # float64 [nD] potential on D
    dir_T: np.ndarray         # float64 [nD] temperature on D
    k_e: np.ndarray           # float64 [E] thermal conductivity
    perf_e: np.ndarray        # float64 [E] perfusion coefficient
    sigma0_e: np.ndarray      # float64 [E] electrical conductivity at T_ref
    rho_c: float = RHO_C
    dt: float = 1.0
    T_a: float = T_ARTERIAL
    alpha_sigma: float = ALPHA_SIGMA
    T_ref: float = T_REF
    steps: int = 1
    tol: float = 1e-10
    coupled: bool = True      # False: one bioheat step with zero Joule source
    loss_ids: Optional[np.ndarray] = None   # int32 nodes of the loss region
    T_target: Optional[np.ndarray] = None   # float64 target temperature on loss_ids

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def npe(self) -> int:
        return int(self.conn.shape[1])

    def initial_T(self) -> np.ndarray:
        """T^0 = 37 C everywhere, Dirichlet nodes at their prescribed values."""
        T = np.full(self.n_nodes, T_ARTERIAL)
        T[self.dir_ids] = self.dir_T
        return T

    def initial_V(self) -> np.ndarray:
        """First potential iterate: Dirichlet values on D, zero elsewhere."""
        V = np.zeros(self.n_nodes)
        V[self.dir_ids] = self.dir_V
        return V


def node_id(i, j, k, n):
    """Global node id of grid node (i, j, k): x fastest, then y, then z."""
    return i + n * (j + n * k)


def grid_xyz(n: int, side: float = SIDE_M) -> np.ndarray:
    h = side / (n - 1)
    idx = np.arange(n, dtype=np.float64) * h
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))


def hex_conn(n: int) -> np.ndarray:
    """Connectivity of the (n-1)^3 hexes; element (a, b, c) has id a + (n-1)(b + (n-1)c)."""
    m = n - 1
    c, b, a = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    cols = [node_id(a + di, b + dj, c + dk, n) for (di, dj, dk) in HEX_LOCAL_OFFSETS]
    return np.ascontiguousarray(np.stack(cols, axis=1).astype(np.int32))


def kuhn_tet_conn(n: int) -> np.ndarray:
    """Each hex split into 6 tets, one per permutation of the axes (lexicographic order).

    Tet of permutation pi walks v0 = lowest corner, v_{m+1} = v_m + e_{pi(m)}.
    Odd permutations get their last two vertices swapped so every tet is
    positively oriented on the undistorted grid.  Element id = 6 * hex_id + perm_index.
    """
    m = n - 1
    c, b, a = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    tets = []
    for perm in itertools.permutations(range(3)):
        off = [0, 0, 0]
        verts = [node_id(a, b, c, n)]
        for axis in perm:
            off[axis] += 1
            verts.append(node_id(a + off[0], b + off[1], c + off[2], n))
        inversions = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
        if inversions % 2 == 1:
            verts[2], verts[3] = verts[3], verts[2]
        tets.append(np.stack(verts, axis=1))
    conn = np.stack(tets, axis=1).reshape(-1, 4)
    return np.ascontiguousarray(conn.astype(np.int32))


def face_node_ids(n: int) -> np.ndarray:
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    on = (i == 0) | (i == n - 1) | (j == 0) | (j == n - 1) | (k == 0) | (k == n - 1)
    return np.nonzero(on.ravel())[0].astype(np.int32)


def electrode_layout(n: int, side: float = SIDE_M):
    """Axial (z) electrode line through grid column (c, c), c = floor((n-1)/2).

    It spans k in [c - m, c + m] with m = floor(2 mm / h): 5 nodes at n = 21,
    21 at n = 101, 33 at n = 161.  Returns (ids, c, m).
    """
    h = side / (n - 1)
    c = (n - 1) // 2
    m = int(np.floor(ELECTRODE_HALF_M / h + 1e-9))
    m = min(m, c - 1)  # keep the electrode strictly inside the cube
    ks = np.arange(c - m, c + m + 1)
    ids = node_id(c, c, ks, n).astype(np.int32)
    return np.sort(ids), c, m


def loss_region(xyz: np.ndarray, n: int, side: float = SIDE_M) -> np.ndarray:
    """Nodes within 8 mm (inclusive) of the electrode segment, by Euclidean distance."""
    h = side / (n - 1)
    _, c, m = electrode_layout(n, side)
    x0 = y0 = c * h
    z_lo, z_hi = (c - m) * h, (c + m) * h
    zc = np.clip(xyz[:, 2], z_lo, z_hi)
    d2 = (xyz[:, 0] - x0) ** 2 + (xyz[:, 1] - y0) ** 2 + (xyz[:, 2] - zc) ** 2
    return np.nonzero(d2 <= LOSS_RADIUS_M ** 2 * (1 + 1e-12))[0].astype(np.int32)


def make_problem(kind: str = "hex", n: int = 21, seed: int = 0, *, steps: int = 1,
                 tol: float = 1e-10, coupled: bool = True, jitter: Optional[bool] = None,
                 with_loss: bool = False, k_scale: float = 1.0, sigma_scale: float = 1.0,
                 perf_scale: float = 1.0, per_element_eps: bool = True,
                 name: Optional[str] = None) -> Problem:
    """Build one seeded problem on an n^3-node cube (hex or Kuhn-tet mesh)."""
    if kind not in ("hex", "tet"):
        raise ValueError(f"kind must be 'hex' or 'tet', got {kind!r}")
    if n < 5:
        raise ValueError("n must be >= 5 (the electrode needs interior nodes)")
    rng = np.random.default_rng(seed)
    h = SIDE_M / (n - 1)
    xyz = grid_xyz(n)
    conn = hex_conn(n) if kind == "hex" else kuhn_tet_conn(n)
    E = conn.shape[0]
    N = xyz.shape[0]

    if per_element_eps:
        eps = rng.uniform(-0.1, 0.1, size=E)
    else:
        eps = np.zeros(E)
    k_e = K_TISSUE * k_scale * (1.0 + eps)
    perf_e = np.full(E, PERFUSION * perf_scale)
    sigma0_e = np.full(E, SIGMA0 * sigma_scale)

    electrode, _, _ = electrode_layout(n)
    faces = face_node_ids(n)
    if jitter is None:
        jitter = kind == "tet"
    if jitter:
        shift = rng.uniform(-0.2 * h, 0.2 * h, size=(N, 3))
        fixed = np.zeros(N, dtype=bool)
        fixed[faces] = True
        fixed[electrode] = True
        shift[fixed] = 0.0
        xyz = np.ascontiguousarray(xyz + shift)

    dir_ids = np.union1d(faces, electrode).astype(np.int32)
    is_el = np.isin(dir_ids, electrode)
    dir_V = np.where(is_el, V_ELECTRODE, V_FACES).astype(np.float64)
    dir_T = np.where(is_el, T_ELECTRODE, T_FACES).astype(np.float64)

    loss_ids = T_target = None
    if with_loss:
        loss_ids = loss_region(xyz, n)
        T_target = 60.0 + 5.0 * rng.standard_normal(loss_ids.shape[0])

    return Problem(name=name or f"{kind}{n}", kind=kind, n=n, h=h, xyz=xyz, conn=conn,
                   electrode_ids=electrode, dir_ids=dir_ids, dir_V=dir_V, dir_T=dir_T,
                   k_e=np.ascontiguousarray(k_e), perf_e=perf_e, sigma0_e=sigma0_e,
                   steps=steps, tol=tol, coupled=coupled, loss_ids=loss_ids, T_target=T_target)


# --- the five workload configurations -------------------------------------------------

def config0(seed: int = 0) -> Problem:
    """21^3-node hex cube, one backward-Euler bioheat step with zero Joule source, tol 1e-10."""
    return make_problem("hex", 21, seed, steps=1, tol=1e-10, coupled=False, name="C0-hex21-bioheat")


def config1(seed: int = 0, n: int = 101, steps: int = 100) -> Problem:
    """101^3-node hex cube (1.03M DOF), coupled potential + bioheat, 100 steps of 1 s."""
    return make_problem("hex", n, seed, steps=steps, tol=1e-12, coupled=True, name=f"C1-hex{n}-coupled")


def config2(seed: int = 0, n: int = 161, steps: int = 20) -> Problem:
    """161^3 grid (4.17M DOF) split into Kuhn tets, jittered interior, 20 coupled steps."""
    return make_problem("tet", n, seed, steps=steps, tol=1e-12, coupled=True, name=f"C2-tet{n}-coupled")


def config3(seed: int = 0, n: int = 101, steps: int = 60) -> Problem:
    """101^3 hex cube, 60 coupled steps, lesion-temperature loss around the electrode."""
    return make_problem("hex", n, seed, steps=steps, tol=1e-12, coupled=True, with_loss=True,
                        name=f"C3-hex{n}-adjoint")


def config4(seed: int = 0, samples: int = 64, n_lo: int = 41, n_hi: int = 81,
            steps: int = 30) -> List[Problem]:
    """Ensemble of hex cubes with n ~ U{n_lo..n_hi}; k, sigma0, perfusion lognormal (0.15) per sample."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=samples)
    z = rng.standard_normal(size=(samples, 3))
    out = []
    for s in range(samples):
        ks, ss, ps = np.exp(0.15 * z[s])
        out.append(make_problem("hex", int(sizes[s]), seed + 1 + s, steps=steps, tol=1e-12,
                                coupled=True, k_scale=float(ks), sigma_scale=float(ss),
                                perf_scale=float(ps), per_element_eps=False,
                                name=f"C4-sample{s}-hex{int(sizes[s])}"))
    return out


def random_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Seeded test vector for kernel-level parity checks."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n)

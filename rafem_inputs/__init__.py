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


# --- unstructured liver-like tet meshes (stand-ins for the paper's meshes A and B) -------

# Two overlapping ellipsoidal lobes (centres and semi-axes in m), a liver-like blob of
# about 58 cm^3; two parallel needle electrodes along z through the main lobe.
LIVER_LOBES = (((0.0, 0.0, 0.0), (0.030, 0.020, 0.016)),
               ((-0.018, 0.012, -0.002), (0.018, 0.014, 0.012)))
NEEDLE_X = (0.010, -0.010)     # needle axes at (x, 0), z in [-15 mm, 15 mm]
NEEDLE_HALF_M = 0.015
V_NEEDLES = (10.0, -10.0)      # bipolar: the potential is lower on one side
LIVER_NODES_A, LIVER_NODES_B = 3548, 8364   # node counts of the paper's meshes (Table II)


def _inside_liver(p: np.ndarray) -> np.ndarray:
    ok = np.zeros(p.shape[0], dtype=bool)
    for c, ax in LIVER_LOBES:
        ok |= (((p - np.asarray(c)) / np.asarray(ax)) ** 2).sum(axis=1) <= 1.0
    return ok


def _liver_volume() -> float:
    """Volume of the blob, counted on a 0.5 mm lattice (deterministic)."""
    g = 5e-4
    lo = np.array([-0.036, -0.020, -0.016])
    hi = np.array([0.030, 0.026, 0.016])
    axes = [np.arange(lo[d] + g / 2, hi[d], g) for d in range(3)]
    count = 0
    for z in axes[2]:
        y, x = np.meshgrid(axes[1], axes[0], indexing="ij")
        pts = np.stack([x.ravel(), y.ravel(), np.full(x.size, z)], axis=1)
        count += int(_inside_liver(pts).sum())
    return count * g ** 3


def make_liver(nodes: int = LIVER_NODES_A, seed: int = 0, *, steps: int = 1, tol: float = 1e-10,
               shuffle: bool = True, name: Optional[str] = None) -> Problem:
    """An unstructured tet mesh of the liver-like blob with about ``nodes`` nodes.

    Points: a cubic lattice of spacing h (chosen from the blob's volume) jittered by
    U(-0.25h, 0.25h) per coordinate, those inside the blob kept; elements: the Delaunay
    tetrahedra of the points whose centroid lies inside the blob (positively oriented,
    near-degenerate hull tets dropped, unused points removed).  D = boundary nodes (on
    faces used by one tet: 0 V, 37 C) united with two needle electrodes (nodes within
    0.75h of the needle axes over 30 mm: +10 V and -10 V, 90 C).  shuffle: node ids in a
    seeded random order, as a mesher may deliver them.  Material fields as in
    make_problem.  Draw order: jitter, eps per element, the shuffle permutation.
    """
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    h = (_liver_volume() / nodes) ** (1.0 / 3.0)
    lo = np.array([-0.036, -0.020, -0.016])
    hi = np.array([0.030, 0.026, 0.016])
    axes = [np.arange(lo[d], hi[d] + h, h) for d in range(3)]
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    pts = pts + rng.uniform(-0.25 * h, 0.25 * h, size=pts.shape)
    pts = pts[_inside_liver(pts)]
    tets = Delaunay(pts).simplices.astype(np.int64)
    cen = pts[tets].mean(axis=1)
    tets = tets[_inside_liver(cen)]
    # orientation and near-degenerate tets (6 x signed volume)
    a, b, c, d = (pts[tets[:, i]] for i in range(4))
    vol6 = np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a))
    flip = vol6 < 0
    tets[flip, 2], tets[flip, 3] = tets[flip, 3].copy(), tets[flip, 2].copy()
    tets = tets[np.abs(vol6) > 1e-3 * h ** 3]
    used = np.unique(tets)
    remap = -np.ones(pts.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    xyz = pts[used]
    conn = remap[tets]
    N, E = xyz.shape[0], conn.shape[0]
    # boundary nodes: nodes of faces that belong to one tet
    faces = np.sort(np.concatenate([conn[:, [1, 2, 3]], conn[:, [0, 2, 3]], conn[:, [0, 1, 3]],
                                    conn[:, [0, 1, 2]]]), axis=1)
    uf, cnt = np.unique(faces, axis=0, return_counts=True)
    boundary = np.unique(uf[cnt == 1])
    # needle electrodes
    needles = []
    for xn in NEEDLE_X:
        r = np.hypot(xyz[:, 0] - xn, xyz[:, 1])
        ids = np.nonzero((r <= 0.75 * h) & (np.abs(xyz[:, 2]) <= NEEDLE_HALF_M))[0]
        needles.append(np.setdiff1d(ids, boundary))
    eps = rng.uniform(-0.1, 0.1, size=E)
    perm = rng.permutation(N) if shuffle else np.arange(N)
    # node old -> new: new id of old node i is inv[i]
    inv = np.empty(N, dtype=np.int64)
    inv[perm] = np.arange(N)
    xyz = np.ascontiguousarray(xyz[perm])
    conn = np.ascontiguousarray(inv[conn].astype(np.int32))
    boundary = inv[boundary]
    needles = [inv[ids] for ids in needles]
    dir_ids = np.unique(np.concatenate([boundary, *needles])).astype(np.int32)
    dir_V = np.full(dir_ids.size, V_FACES)
    dir_T = np.full(dir_ids.size, T_FACES)
    for ids, v in zip(needles, V_NEEDLES):
        k = np.searchsorted(dir_ids, ids)
        dir_V[k] = v
        dir_T[k] = T_ELECTRODE
    electrode = np.sort(np.concatenate(needles)).astype(np.int32)
    return Problem(name=name or f"liver{N}", kind="tet", n=int(round(N ** (1.0 / 3.0))), h=h,
                   xyz=xyz, conn=conn, electrode_ids=electrode, dir_ids=dir_ids,
                   dir_V=dir_V.astype(np.float64), dir_T=dir_T.astype(np.float64),
                   k_e=np.ascontiguousarray(K_TISSUE * (1.0 + eps)),
                   perf_e=np.full(E, PERFUSION), sigma0_e=np.full(E, SIGMA0), steps=steps,
                   tol=tol, coupled=True)


def liver_mesh_a(seed: int = 0, **kw) -> Problem:
    """Stand-in for the paper's mesh A (3,548 nodes, 18,363 tets, Table II)."""
    return make_liver(LIVER_NODES_A, seed, name="liverA", **kw)


def liver_mesh_b(seed: int = 0, **kw) -> Problem:
    """Stand-in for the paper's mesh B (8,364 nodes, 44,811 tets, Table II)."""
    return make_liver(LIVER_NODES_B, seed, name="liverB", **kw)

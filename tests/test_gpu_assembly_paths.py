"""The two assembly paths of the step matrices and right-hand side on the GPU.

Meshes whose rows all have at most 64 entries (the grid and liver meshes) are assembled
row by row; a mesh with a longer row falls back to the element-parallel colour-by-colour
scatter.  The long-row mesh here is a Kuhn-tet cube with one extra node above the top face,
joined to every triangle of that face (a fan of tets whose apex row has 82 entries).
Coupled steps on it, in FP64 and mixed precision, match the oracle.
"""
import numpy as np
import pytest

import rafem_inputs as ri
from oracle.rafem import Model
from gpu_helpers import rel_err

TOL = 1e-13


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _signed_volume(xyz, tet):
    a, b, c, d = xyz[tet]
    return np.dot(np.cross(b - a, c - a), d - a) / 6.0


def apex_problem(n: int = 9) -> ri.Problem:
    """make_problem('tet', n) plus one free node above the top face, joined to every
    boundary triangle of the face (each new tet positively oriented)."""
    p = ri.make_problem("tet", n=n, seed=3)
    top = p.xyz[:, 2].max()
    on_top = np.isclose(p.xyz[:, 2], top)
    tris = set()
    for tet in p.conn:
        for skip in range(4):
            face = tuple(sorted(int(v) for k, v in enumerate(tet) if k != skip))
            if all(on_top[v] for v in face):
                tris.add(face)
    apex = p.n_nodes
    centre = p.xyz[on_top].mean(axis=0)
    xyz = np.vstack([p.xyz, centre + np.array([0.0, 0.0, p.h])])
    new = []
    for f in sorted(tris):
        tet = [f[0], f[1], f[2], apex]
        if _signed_volume(xyz, np.array(tet)) < 0.0:
            tet[0], tet[1] = tet[1], tet[0]
        new.append(tet)
    conn = np.vstack([p.conn, np.array(new, dtype=np.int32)]).astype(np.int32)
    extra = len(new)

    def grow(a):
        return np.concatenate([a, np.full(extra, float(np.mean(a)))])

    p.xyz = np.ascontiguousarray(xyz)
    p.conn = np.ascontiguousarray(conn)
    p.k_e, p.perf_e, p.sigma0_e = grow(p.k_e), grow(p.perf_e), grow(p.sigma0_e)
    p.name = p.name + "+apex"
    return p


def test_apex_mesh_has_a_long_row():
    p = apex_problem()
    deg = np.zeros(p.n_nodes, dtype=np.int64)
    for tet in p.conn:
        deg[tet] += 1
    assert deg[-1] == 2 * (9 - 1) ** 2          # two triangles per top-face quad
    assert len(set(p.conn[p.conn[:, 3] == p.n_nodes - 1][:, :3].ravel())) + 1 == 82
    assert all(_signed_volume(p.xyz, t) > 0.0 for t in p.conn)


@pytest.mark.gpu
def test_grid_and_liver_meshes_assemble_by_rows(torch_cuda):
    from paper_2409_13036_amd.sim import DeviceProblem
    for p in (ri.make_problem("hex", n=9), ri.make_problem("tet", n=9), ri.liver_mesh_a(),
              ri.liver_mesh_b()):
        dp = DeviceProblem(p)
        st = dp.mesh.stats()
        print(f"[{p.name}] row assembly {st.row_assembly}, longest row {st.max_row_entries}",
              flush=True)
        assert st.row_assembly == 1 and st.max_row_entries <= 64
        dp.close()


@pytest.mark.gpu
def test_long_row_mesh_steps_match_oracle(torch_cuda):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = apex_problem()
    ref, _ = Model(p).simulate(2, 1e-15)
    dp = DeviceProblem(p)
    st = dp.mesh.stats()
    print(f"[apex] row assembly {st.row_assembly}, longest row {st.max_row_entries}, "
          f"colours {st.n_colours}", flush=True)
    assert st.row_assembly == 0 and st.max_row_entries > 64
    for precision in ("fp64", "mixed"):
        dp.reset()
        states, infos = dp.simulate(2, tol=TOL, precision=precision, keep=True)
        for k, ((T, V), (Tr, Vr)) in enumerate(zip(states, ref)):
            eT, eV = rel_err(T, Tr), rel_err(V, Vr)
            print(f"[apex {precision}] step {k + 1}: T {eT:.2e} V {eV:.2e}", flush=True)
            assert eT <= 1e-8 and eV <= 1e-8
    dp.close()

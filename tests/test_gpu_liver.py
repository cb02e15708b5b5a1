"""The unstructured liver-like meshes on the GPU (per-lane column offsets in the slabs:
no shared offset lists): coupled steps against the oracle in the delivered (shuffled) node
order and after reverse Cuthill-McKee renumbering, a predictor-corrector step, and the
monolithic GMRES solve."""
import numpy as np
import pytest

import rafem_inputs as ri
from oracle import corrector as pc
from oracle import monolithic as mono
from oracle.rafem import Model
from gpu_helpers import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-13


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.fixture(scope="module")
def meshes():
    return {"A": ri.liver_mesh_a(), "B": ri.liver_mesh_b()}


@pytest.mark.parametrize("mesh", ["A", "B"])
@pytest.mark.parametrize("reorder", [False, True, "sorted"])
def test_coupled_steps_match_oracle(torch_cuda, meshes, mesh, reorder):
    from paper_2409_13036_amd.sim import DeviceProblem, rcm_reordered
    p = meshes[mesh]
    ref, _ = Model(p).simulate(3, 1e-15)
    if reorder:
        q, order = rcm_reordered(p, window=512 if reorder == "sorted" else 0)
    else:
        q, order = p, np.arange(p.n_nodes)
    dp = DeviceProblem(q)
    st = dp.mesh.stats()
    for precision in ("fp64", "mixed"):
        dp.reset()
        states, infos = dp.simulate(3, tol=TOL, precision=precision, keep=True)
        for k, ((T, V), (Tr, Vr)) in enumerate(zip(states, ref)):
            Tg = np.empty_like(T)
            Vg = np.empty_like(V)
            Tg[order], Vg[order] = T, V
            eT, eV = rel_err(Tg, Tr), rel_err(Vg, Vr)
            if k == 2:
                print(f"[liver{mesh} rcm={reorder} {precision}] step 3: T {eT:.2e} V {eV:.2e} "
                      f"(V iters {infos[k]['V']['iters']}, slabs {st.slabs}, shared "
                      f"{st.shared_offset_slabs})", flush=True)
            assert eT <= 1e-8 and eV <= 1e-8
    dp.close()


def test_predictor_corrector_step_matches_oracle(torch_cuda, meshes):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = meshes["A"]
    m = Model(p)
    T0, V0 = p.initial_T(), p.initial_V()
    dp = DeviceProblem(p)
    info = dp.step_pc(20.0, corr_tol=3e-9, tol=TOL)
    ref = pc.corrector_step(m, T0, V0, 20.0, T0.copy(), 1e-15, 3e-9)
    print(f"[liverA pc] GPU iters {info['iters']} oracle {ref.iters}", flush=True)
    assert info["accepted"] == 1 and info["iters"] == ref.iters
    assert rel_err(to_host(dp.T), ref.T) <= 1e-8 and rel_err(to_host(dp.V), ref.V) <= 1e-8
    dp.close()


def test_monolithic_gmres_matches_oracle(torch_cuda, meshes):
    from paper_2409_13036_amd import _lib as R
    from paper_2409_13036_amd.sim import DeviceProblem
    p = meshes["A"]
    m = Model(p)
    T0 = p.initial_T()
    T1, V1, _ = m.step(T0, p.initial_V(), 1e-14)
    dp = DeviceProblem(p)
    dp.phys.dt = 20.0
    delta, info, _ = R.mono_solve(dp.mesh, dp.phys, dp.k_e, dp.perf_e, dp.sigma0_e, to_dev(T0),
                                  to_dev(T1), to_dev(V1), m=30, tol=1e-10)
    delta = to_host(delta)
    dp.close()
    J = mono.interleaved_matrix(m, mono.jacobian_blocks(m, T0, 20.0, T1, V1))
    b = -mono.residual(m, T0, 20.0, T1, V1)
    x, ref = mono.gmres(J, b, np.zeros_like(b), 30, 1e-10, precond=mono.block_jacobi(J))
    print(f"[liverA gmres] GPU iters {info['iters']} cycles {info['cycles']}; oracle "
          f"{ref.iters} / {ref.cycles}; delta err {rel_err(delta, x):.2e}", flush=True)
    assert info["status"] == 0 and abs(info["iters"] - ref.iters) <= 1
    assert rel_err(delta, x) <= 1e-8

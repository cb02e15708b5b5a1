"""Predictor-corrector steps on the GPU against the oracle's loop: a corrector step from
rest and one with the predictor, a rejected step leaving the state untouched, a whole
step-size-controlled run (same accepted steps, same final state), batch handles refused."""
import numpy as np
import pytest

import rafem_inputs as ri
from oracle import corrector as pc
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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,n", [("hex", 11), ("tet", 9)])
def test_corrector_steps_match_oracle(torch_cuda, kind, n, precision):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem(kind, n, 1)
    m = Model(p)
    eps, dt = 3e-9, 20.0
    T0, V0 = p.initial_T(), p.initial_V()
    dp = DeviceProblem(p)
    # first step (no history: predictor = T^n)
    info1 = dp.step_pc(dt, corr_tol=eps, tol=TOL, precision=precision)
    ref1 = pc.corrector_step(m, T0, V0, dt, pc.predictor(T0, None, dt, None), 1e-15, eps)
    T1, V1 = to_host(dp.T), to_host(dp.V)
    print(f"[pc {kind}{n} {precision}] step 1: iters {info1['iters']} (oracle {ref1.iters}) "
          f"T {rel_err(T1, ref1.T):.2e} V {rel_err(V1, ref1.V):.2e}", flush=True)
    assert info1["accepted"] == 1 and ref1.converged and info1["iters"] == ref1.iters
    assert rel_err(T1, ref1.T) <= 1e-8 and rel_err(V1, ref1.V) <= 1e-8
    # second step, shorter, extrapolating from the first
    dt2 = 10.0
    info2 = dp.step_pc(dt2, T_prev=to_dev(T0), dt_prev=dt, corr_tol=eps, tol=TOL,
                       precision=precision)
    ref2 = pc.corrector_step(m, ref1.T, ref1.V, dt2, pc.predictor(ref1.T, T0, dt2, dt), 1e-15, eps)
    T2, V2 = to_host(dp.T), to_host(dp.V)
    print(f"[pc {kind}{n} {precision}] step 2: iters {info2['iters']} (oracle {ref2.iters}) "
          f"T {rel_err(T2, ref2.T):.2e} V {rel_err(V2, ref2.V):.2e}", flush=True)
    assert info2["accepted"] == 1 and info2["iters"] == ref2.iters
    assert rel_err(T2, ref2.T) <= 1e-8 and rel_err(V2, ref2.V) <= 1e-8
    dp.close()


def test_rejected_step_leaves_the_state(torch_cuda):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("hex", 9, 2)
    dp = DeviceProblem(p)
    dp.step(TOL)                              # some non-trivial state
    T_before, V_before = to_host(dp.T), to_host(dp.V)
    info = dp.step_pc(60.0, corr_tol=1e-12, max_iters=2, tol=TOL)
    assert info["accepted"] == 0 and info["iters"] == 2 and info["change"] > 1e-12
    assert np.array_equal(to_host(dp.T), T_before) and np.array_equal(to_host(dp.V), V_before)
    # and a plain step afterwards uses the problem's own time step again
    dp.step(TOL)
    T_next, _, _ = Model(p).step(T_before, V_before, 1e-15)
    assert rel_err(to_host(dp.T), T_next) <= 1e-8
    dp.close()


def test_step_controlled_run_matches_oracle(torch_cuda):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("hex", 9, 1)
    m = Model(p)
    kw = dict(eps=1e-4, max_iters=3)
    T_ref, V_ref, rec = pc.simulate_pc(m, 120.0, 60.0, 1e-15, **kw)
    dp = DeviceProblem(p)
    got = dp.simulate_pc(120.0, 60.0, corr_tol=kw["eps"], max_iters=kw["max_iters"], tol=TOL)
    ref_steps = [(r.t, r.dt, r.iters, r.rejected_before) for r in rec]
    gpu_steps = [(g["t"], g["dt"], g["iters"], g["rejected_before"]) for g in got]
    print(f"[pc run] {len(gpu_steps)} accepted steps, {sum(g[3] for g in gpu_steps)} rejected",
          flush=True)
    assert gpu_steps == ref_steps
    assert any(s[3] > 0 for s in ref_steps)  # the run does exercise rejection
    assert rel_err(to_host(dp.T), T_ref) <= 1e-8 and rel_err(to_host(dp.V), V_ref) <= 1e-8
    dp.close()


def test_batch_handles_refuse_the_corrector(torch_cuda):
    from paper_2409_13036_amd import _lib as R
    from paper_2409_13036_amd.sim import BatchProblem
    bp = BatchProblem([ri.make_problem("hex", 7, 1), ri.make_problem("hex", 8, 2)])
    with pytest.raises(R.RafemError, match="E_ARG"):
        R.step_pc(bp.mesh, bp.phys, bp.k_e, bp.perf_e, bp.sigma0_e, bp.dir_V, bp.dir_T, None, 0.0,
                  bp.T, bp.V)
    bp.close()

"""Extrapolated starting points of the step's solves (phys.extrapolate, linear or
quadratic): the states match the oracle's steps, the solves need fewer iterations, the
predictor is the Lagrange extrapolation of the kept states for unequal steps, and a new
trajectory (after a reset, or after a corrector step) starts from the given state, bit for
bit like a step without extrapolation."""
import numpy as np
import pytest

import rafem_inputs as ri
from oracle.rafem import Model
from gpu_helpers import rel_err, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-13


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.mark.parametrize("kind,n", [("hex", 15), ("tet", 11)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_extrapolated_steps_match_oracle_with_fewer_iterations(torch_cuda, kind, n, precision,
                                                               order):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem(kind, n, 0)
    ref, _ = Model(p).simulate(11, 1e-15)
    plain = DeviceProblem(p)
    _, info0 = plain.simulate(11, tol=TOL, precision=precision)
    plain.close()
    dp = DeviceProblem(p)
    dp.extrapolate = True
    dp.extrapolate_order = order
    states, info1 = dp.simulate(11, tol=TOL, precision=precision, keep=True)
    dp.close()
    for (T, V), (Tr, Vr) in zip(states, ref):
        assert rel_err(T, Tr) <= 1e-8 and rel_err(V, Vr) <= 1e-8
    # from a few steps after the start of the trajectory (the first kept state is the initial
    # one, whose V is not a solution, and higher orders need a smooth history)
    first = 2 * order + 1
    it0 = sum(i["V"]["iters"] + i["T"]["iters"] for i in info0[first:])
    it1 = sum(i["V"]["iters"] + i["T"]["iters"] for i in info1[first:])
    print(f"[extrapolate order {order} {kind}{n} {precision}] iterations of steps {first + 1}-11: "
          f"{it1} (plain {it0})", flush=True)
    assert it1 < it0
    # the first two steps start a trajectory: identical to plain steps
    assert info1[0]["V"]["iters"] == info0[0]["V"]["iters"]


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_predictor_is_the_lagrange_extrapolation_of_the_kept_states(torch_cuda, order):
    """With a tolerance every starting point meets, the solves run no iteration and return
    their starting points: after steps of 1, 0.5, 2, 0.75 and 1.25 s, a step of 1.5 s returns
    (on the free nodes) the Lagrange extrapolation of the last order + 1 kept states, for
    unequal steps."""
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("hex", 11, 2)
    dp = DeviceProblem(p)
    dp.extrapolate = True
    dp.extrapolate_order = order
    dts = [1.0, 0.5, 2.0, 0.75, 1.25]
    kept_T, kept_V = [], []
    for dt in dts:
        dp.phys.dt = dt
        kept_T.append(to_host(dp.T))
        kept_V.append(to_host(dp.V))
        dp.step(TOL)
    kept_T.append(to_host(dp.T))
    kept_V.append(to_host(dp.V))
    tau = 1.5
    dp.phys.dt = tau
    info = dp.step(1e30)
    assert info["V"]["iters"] == 0 and info["T"]["iters"] == 0
    # nodes t_0 = 0 (the current state), t_k = t_{k-1} - (step that led to state k-1)
    t = [0.0]
    for k in range(1, order + 1):
        t.append(t[-1] - dts[-k])
    w = [np.prod([(tau - t[k]) / (t[i] - t[k]) for k in range(order + 1) if k != i])
         for i in range(order + 1)]
    free = np.ones(p.n_nodes, dtype=bool)
    free[p.dir_ids] = False
    for got, kept in ((to_host(dp.T), kept_T), (to_host(dp.V), kept_V)):
        want = sum(w[i] * kept[-1 - i] for i in range(order + 1))
        scale = np.abs(want[free]).max()
        err = np.abs(got[free] - want[free]).max()
        print(f"[predictor order {order}] max error {err / scale:.1e} of max |value|",
              flush=True)
        assert err <= 1e-13 * scale
    dp.close()


def test_new_trajectory_starts_from_the_given_state(torch_cuda):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("hex", 13, 1)
    ref = DeviceProblem(p)
    ref.step(TOL)
    T_ref, V_ref = to_host(ref.T), to_host(ref.V)
    ref.close()
    dp = DeviceProblem(p)
    dp.extrapolate = True
    for _ in range(3):
        dp.step(TOL)
    dp.reset()
    dp.step(TOL)
    assert np.array_equal(to_host(dp.T), T_ref) and np.array_equal(to_host(dp.V), V_ref)
    # a corrector step ends the trajectory as well: the next step starts from its result
    dp.step_pc(1.0, corr_tol=1e-9, tol=TOL)
    T_pc, V_pc = to_host(dp.T), to_host(dp.V)
    dp.step(TOL)
    other = DeviceProblem(p)
    other.reset(T_pc, V_pc)
    other.step(TOL)
    assert np.array_equal(to_host(dp.T), to_host(other.T))
    other.close()
    dp.close()


def test_extrapolated_ensemble_matches_its_samples_alone(torch_cuda):
    """Batch handles extrapolate every sample from its own history: each sample's states
    equal those of the same sample stepped alone with extrapolation."""
    from paper_2409_13036_amd.sim import BatchProblem, DeviceProblem
    probs = [ri.make_problem("hex", 9, 1), ri.make_problem("hex", 12, 2)]
    bp = BatchProblem(probs)
    bp.extrapolate = True
    for _ in range(4):
        bp.step(TOL, "mixed")
    got = [bp.sample(q) for q in range(2)]
    bp.close()
    for q, p in enumerate(probs):
        dp = DeviceProblem(p)
        dp.extrapolate = True
        for _ in range(4):
            dp.step(TOL, "mixed")
        assert np.array_equal(got[q][0], to_host(dp.T)) and np.array_equal(got[q][1], to_host(dp.V))
        dp.close()


def test_bad_predictor_settings_are_rejected_before_any_work(torch_cuda):
    from paper_2409_13036_amd import _lib as R
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("hex", 9, 0)
    dp = DeviceProblem(p)
    T0, V0 = to_host(dp.T), to_host(dp.V)
    for mode, order in ((3, 1), (-1, 1), (1, 5), (1, -1)):
        dp.phys.extrapolate, dp.phys.extrapolate_order = mode, order
        with pytest.raises(R.RafemError) as e:
            R.step(dp.mesh, dp.phys, dp.k_e, dp.perf_e, dp.sigma0_e, dp.dir_V, dp.dir_T, dp.T,
                   dp.V, tol=TOL)
        assert e.value.status == R.E_ARG
    assert np.array_equal(to_host(dp.T), T0) and np.array_equal(to_host(dp.V), V0)
    dp.close()

"""Multi-step trajectories against the oracle's trajectories.

The paper compares the run under test with the sequential run at every time step (Sec.
IV, Eq. 1-2); here every path is compared with the oracle's trajectory, not only with the
other device path:

- hex 41^3, the coupled workload's configuration (extrapolated starting points, tol
  1e-13), 100 steps, FP64 and mixed: every node of T and V at every step against the
  oracle's 100-step run (computed in the test);
- Kuhn tets 161^3 (4.17M DOF), 20 coupled steps in the benchmark's configuration: both
  paths against the oracle's 20-step run at 2,000 stored free nodes after every step
  (tests/golden/make_trajectories.py), the mixed state within 1e-8 of the FP64 state at
  every step, and the 20th step of both paths satisfying the oracle's equations of 2,000
  sampled rows given their 19th state;
- the 64-sample ensemble, 3 coupled steps, FP64 and mixed: four samples (the smallest, the
  largest and two drawn from the seed) against the oracle's 3-step runs of those samples,
  stored by tests/golden/make_trajectories.py at 2,000 free nodes each.
"""
import os

import numpy as np
import pytest

import rafem_inputs as ri
from oracle.rafem import Model
from gpu_helpers import rel_err, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-13
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def say(msg):
    print(f"[trajectory] {msg}", flush=True)


def _device_run(p, precision, steps, **kw):
    from paper_2409_13036_amd.sim import DeviceProblem
    dp = DeviceProblem(p)
    dp.extrapolate = True
    out = []
    for _ in range(steps):
        info = dp.step(TOL, precision, **kw)
        assert info["V"]["status"] == 0 and info["T"]["status"] == 0
        out.append((to_host(dp.T), to_host(dp.V)))
    dp.close()
    return out


@pytest.mark.timeout(900)
def test_hex41_hundred_steps_match_oracle_trajectory_at_every_node(torch_cuda):
    p = ri.config1(n=41, steps=100)
    runs = {prec: _device_run(p, prec, 100) for prec in ("fp64", "mixed")}
    say("device runs done; oracle trajectory (100 steps) follows")
    m = Model(p)
    bio = m.bioheat_system()
    T, V = p.initial_T(), p.initial_V()
    worst = {"fp64": 0.0, "mixed": 0.0}
    for k in range(100):
        T, V, _ = m.step(T, V, TOL, bioheat=bio)
        for prec, states in runs.items():
            Tg, Vg = states[k]
            eT, eV = rel_err(Tg, T), rel_err(Vg, V)
            worst[prec] = max(worst[prec], eT, eV)
            assert eT <= 1e-8 and eV <= 1e-8, (prec, k + 1, eT, eV)
        if (k + 1) % 10 == 0:
            say(f"step {k + 1}: worst so far fp64 {worst['fp64']:.2e}, mixed {worst['mixed']:.2e}")


@pytest.mark.timeout(600)
def test_tet161_twenty_steps_mixed_tracks_fp64_and_satisfies_oracle_equations(torch_cuda):
    from test_gpu_fullsize import _sampled_equations
    p = ri.config2(steps=20)
    say(f"tet 161^3: N={p.n_nodes} E={p.n_elems}")
    runs = {"fp64": _device_run(p, "fp64", 20),
            "mixed": _device_run(p, "mixed", 20, inner_tol=1e-4)}
    worst = 0.0
    for k, ((T6, V6), (Tm, Vm)) in enumerate(zip(runs["fp64"], runs["mixed"])):
        eT, eV = rel_err(Tm, T6), rel_err(Vm, V6)
        worst = max(worst, eT, eV)
        assert eT <= 1e-8 and eV <= 1e-8, (k + 1, eT, eV)
    say(f"mixed vs FP64 over 20 steps: max rel err {worst:.2e}")
    gold = np.load(os.path.join(GOLDEN, "c2_tet161_trajectory.npz"))
    nodes = gold["nodes"]
    for prec, states in runs.items():
        worst_o = 0.0
        for j, k in enumerate(gold["steps"]):
            Tg, Vg = states[k - 1]
            eT = rel_err(Tg[nodes], gold["T"][j])
            eV = rel_err(Vg[nodes], gold["V"][j])
            worst_o = max(worst_o, eT, eV)
            assert eT <= 1e-8 and eV <= 1e-8, (prec, int(k), eT, eV)
        say(f"{prec}: worst sampled error against the stored oracle run {worst_o:.2e}")
    free = np.setdiff1d(np.arange(p.n_nodes), p.dir_ids)
    rows = np.sort(np.random.default_rng(13).choice(free, 2000, replace=False))
    gV, gT = np.linalg.norm(p.dir_V), np.linalg.norm(p.dir_T)
    for prec, states in runs.items():
        T19, (T20, V20) = states[18][0], states[19]
        rV, sV, rT, sT = _sampled_equations(p, rows, T19, V20, T20)
        say(f"{prec} step 20: max |rV| {np.abs(rV).max():.2e}, max |rT| {np.abs(rT).max():.2e}")
        assert np.all(np.abs(rV) <= 10 * TOL * gV + 1e-13 * sV)
        assert np.all(np.abs(rT) <= 10 * TOL * gT + 1e-13 * sT)
        assert np.abs(rV).max() < 1e-6 * sV.max() and np.abs(rT).max() < 1e-6 * sT.max()


@pytest.mark.timeout(600)
def test_ensemble_three_steps_match_stored_oracle_samples(torch_cuda):
    from paper_2409_13036_amd.sim import BatchProblem
    gold = np.load(os.path.join(GOLDEN, "c4_ensemble_steps.npz"))
    picks = [int(q) for q in gold["picks"]]
    probs = ri.config4(steps=3)
    say(f"ensemble: {len(probs)} samples; checked {picks} (n = {[probs[q].n for q in picks]})")
    bp = BatchProblem(probs)
    bp.extrapolate = True
    for prec in ("fp64", "mixed"):
        bp.reset()
        for k in range(3):
            info = bp.step(TOL, prec)
            assert info["V"]["status"] == 0 and info["T"]["status"] == 0
            for q in picks:
                Tg, Vg = bp.sample(q)
                nodes = gold[f"nodes_{q}"]
                eT = rel_err(Tg[nodes], gold[f"T_{q}"][k])
                eV = rel_err(Vg[nodes], gold[f"V_{q}"][k])
                say(f"{prec} step {k + 1} sample {q}: T {eT:.2e} V {eV:.2e}")
                assert eT <= 1e-8 and eV <= 1e-8
    bp.close()

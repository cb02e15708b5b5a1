"""GPU parity at the full sizes the benchmark times, in the same launch configuration.

- 101^3 hex (1.03M DOF): one coupled step, FP64 and mixed, against the oracle's step, and
  the CSR structure bit for bit.
- 161^3 jittered Kuhn tets (4.17M DOF, 24.6M elements): the oracle cannot hold that mesh's
  element matrices, so it assembles the potential and bioheat equations of 2,000 sampled
  free rows from their incident elements, and the GPU step must satisfy them to the
  solver's tolerance.
- the 64-sample ensemble (16.6M rows): one step of the whole batch; its smallest and its
  largest sample against the oracle's step of that sample.
- 101^3 hex over 100 steps in the benchmark's configuration: both paths against the
  oracle's stored 100-step trajectory (tests/golden/make_trajectories.py), the mixed state
  against the FP64 state at every step, and the 100th step against the oracle's equations.
"""
import os

import numpy as np
import pytest

import rafem_inputs as ri
from oracle import elements
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
    print(f"[fullsize] {msg}", flush=True)


def test_hex101_step_and_structure_match_oracle(torch_cuda):
    from paper_2409_13036_amd import _lib as R
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.config1(steps=1)
    say(f"hex 101^3: N={p.n_nodes} E={p.n_elems}")
    dp = DeviceProblem(p)
    out = {}
    for precision in ("fp64", "mixed"):
        dp.reset()
        info = dp.step(TOL, precision)
        assert info["V"]["status"] == 0 and info["T"]["status"] == 0
        out[precision] = (to_host(dp.T), to_host(dp.V))
        say(f"GPU {precision} step: V {info['V']['iters']} T {info['T']['iters']} iterations")
    # CSR structure, bit for bit, from the library's CSR assembly
    csr = R.assemble_csr(dp.mesh, stiff_coef=dp.k_e)
    rp, ci = to_host(csr["row_ptr"]), to_host(csr["col_idx"])
    dp.close()
    m = Model(p)
    say("oracle structure built")
    assert np.array_equal(rp, m.S.row_ptr) and np.array_equal(ci, m.S.col_idx)
    T1, V1, _ = m.step(p.initial_T(), p.initial_V(), TOL)
    say("oracle step done")
    for precision, (Tg, Vg) in out.items():
        eT, eV = rel_err(Tg, T1), rel_err(Vg, V1)
        say(f"{precision}: T {eT:.2e} V {eV:.2e} (T-37: {rel_err(Tg - 37, T1 - 37):.2e})")
        assert eT <= 1e-8 and eV <= 1e-8


def _sampled_equations(p, rows, T0, V1, T1):
    """Residuals of the potential and bioheat equations of the given free rows, assembled
    by the oracle's element routines from the elements touching those rows, with the
    scales that bound them: (rV, scaleV, rT, scaleT), scale_i = sum_j |A_ij x_j| + |b_i|."""
    mark = np.zeros(p.n_nodes, dtype=bool)
    mark[rows] = True
    es = np.nonzero(mark[p.conn].any(axis=1))[0]
    conn = p.conn[es]
    xe = p.xyz[conn]
    K, M = elements.element_matrices(xe)
    Tbar = T0[conn].mean(axis=1)
    sig = p.sigma0_e[es] * (1.0 + p.alpha_sigma * (Tbar - p.T_ref))
    F = elements.joule_loads(xe, sig, V1[conn])                        # [e, a]
    a_T = p.rho_c / p.dt + p.perf_e[es]
    KV = np.einsum("eab,eb->ea", K, V1[conn]) * sig[:, None]          # (K_sigma V1) terms
    KVa = np.einsum("eab,eb->ea", np.abs(K), np.abs(V1[conn])) * sig[:, None]
    AT = a_T[:, None, None] * M + p.k_e[es][:, None, None] * K
    ATT = np.einsum("eab,eb->ea", AT, T1[conn])
    ATTa = np.einsum("eab,eb->ea", np.abs(AT), np.abs(T1[conn]))
    wT = (p.rho_c / p.dt) * T0[conn] + (p.perf_e[es] * p.T_a)[:, None]
    bT = np.einsum("eab,eb->ea", M, wT) + F
    index = {int(r): k for k, r in enumerate(rows)}
    nr = len(rows)
    rV, sV, rT, sT = (np.zeros(nr) for _ in range(4))
    for e_local, e_conn in enumerate(conn):
        for a, node in enumerate(e_conn):
            k = index.get(int(node))
            if k is None:
                continue
            rV[k] += KV[e_local, a]
            sV[k] += KVa[e_local, a]
            rT[k] += ATT[e_local, a] - bT[e_local, a]
            sT[k] += ATTa[e_local, a] + abs(bT[e_local, a])
    return rV, sV, rT, sT


def test_tet161_step_satisfies_sampled_oracle_equations(torch_cuda):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.config2(steps=1)
    say(f"tet 161^3: N={p.n_nodes} E={p.n_elems}")
    dp = DeviceProblem(p)
    info = dp.step(TOL, "mixed")
    assert info["V"]["status"] == 0 and info["T"]["status"] == 0
    T1, V1 = to_host(dp.T), to_host(dp.V)
    dp.close()
    say(f"GPU mixed step: V {info['V']['iters']} T {info['T']['iters']} inner iterations")
    T0 = p.initial_T()
    free = np.setdiff1d(np.arange(p.n_nodes), p.dir_ids)
    rows = np.sort(np.random.default_rng(7).choice(free, 2000, replace=False))
    rV, sV, rT, sT = _sampled_equations(p, rows, T0, V1, T1)
    say("oracle rows assembled")
    # |r_i| <= ||b - A x|| <= tol ||b||, and ||b|| is the norm of the Dirichlet values up
    # to the small free-row lifting terms; 1e-13 |row| covers the rounding of the sums
    gV, gT = np.linalg.norm(p.dir_V), np.linalg.norm(p.dir_T)
    okV = np.abs(rV) <= 10 * TOL * gV + 1e-13 * sV
    okT = np.abs(rT) <= 10 * TOL * gT + 1e-13 * sT
    say(f"max |rV| {np.abs(rV).max():.2e} (bound {10 * TOL * gV:.1e}), "
        f"max |rT| {np.abs(rT).max():.2e} (bound {10 * TOL * gT:.1e})")
    assert okV.all() and okT.all()
    # and tiny against the rows themselves (an error of 1% in an element matrix or in the
    # Joule load would leave residuals of order 1e-2 of them)
    assert np.abs(rV).max() < 1e-6 * sV.max() and np.abs(rT).max() < 1e-6 * sT.max()


def test_ensemble_step_matches_oracle_for_extreme_samples(torch_cuda):
    from paper_2409_13036_amd.sim import BatchProblem
    probs = ri.config4(steps=1)
    say(f"ensemble: {len(probs)} samples, {sum(q.n_nodes for q in probs)} nodes")
    bp = BatchProblem(probs)
    info = bp.step(TOL, "mixed")
    assert info["V"]["status"] == 0 and info["T"]["status"] == 0
    sizes = [q.n for q in probs]
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes))]
    got = {q: bp.sample(q) for q in picks}
    bp.close()
    for q in picks:
        p = probs[q]
        T1, V1, _ = Model(p).step(p.initial_T(), p.initial_V(), TOL)
        Tg, Vg = got[q]
        eT, eV = rel_err(Tg, T1), rel_err(Vg, V1)
        say(f"sample {q} (n={p.n}): T {eT:.2e} V {eV:.2e}")
        assert eT <= 1e-8 and eV <= 1e-8


def _incident_model(p, rows):
    """The oracle's model of the elements touching the given rows only: its rows of the
    monolithic J and R are exactly those rows of the full problem's."""
    import dataclasses
    mark = np.zeros(p.n_nodes, dtype=bool)
    mark[rows] = True
    es = np.nonzero(mark[p.conn].any(axis=1))[0]
    sub = dataclasses.replace(p, conn=np.ascontiguousarray(p.conn[es]), k_e=p.k_e[es],
                              perf_e=p.perf_e[es], sigma0_e=p.sigma0_e[es])
    return Model(sub)


def test_hex101_monolithic_solve_and_newton_step_satisfy_sampled_equations(torch_cuda):
    """101^3 hex in the bench's configuration: the GMRES(20) update of the Newton system at
    the state after one staggered step (dt = 2 s), and a Newton predictor-corrector step."""
    from oracle import monolithic as mono
    from paper_2409_13036_amd import _lib as R
    from paper_2409_13036_amd.sim import DeviceProblem
    from gpu_helpers import to_dev
    p = ri.config1(steps=1)
    dp = DeviceProblem(p)
    dp.step(TOL)
    T1, V1 = to_host(dp.T), to_host(dp.V)
    T0 = p.initial_T()
    dt = 2.0
    dp.phys.dt = dt
    delta, info, _ = R.mono_solve(dp.mesh, dp.phys, dp.k_e, dp.perf_e, dp.sigma0_e, to_dev(T0),
                                  dp.T, dp.V, m=20, tol=1e-10)
    _, Rg = R.mono_jacobian(dp.mesh, dp.phys, dp.k_e, dp.perf_e, dp.sigma0_e, to_dev(T0), dp.T,
                            dp.V)
    delta, Rg = to_host(delta), to_host(Rg)
    say(f"GMRES(20) at 101^3: {info['iters']} steps, {info['cycles']} cycles, relres_true "
        f"{info['relres_true']:.2e}")
    assert info["status"] == 0 and info["relres_true"] <= 1e-10
    free = np.setdiff1d(np.arange(p.n_nodes), p.dir_ids)
    rows = np.sort(np.random.default_rng(11).choice(free, 2000, replace=False))
    ms = _incident_model(p, rows)
    Rr = mono.residual(ms, T0, dt, T1, V1)
    Js = mono.interleaved_matrix(ms, mono.jacobian_blocks(ms, T0, dt, T1, V1))
    idx = np.concatenate([2 * rows, 2 * rows + 1])
    scaleR = np.abs(Rr[idx]).max()
    assert np.abs(Rg[idx] - Rr[idx]).max() <= 1e-12 * scaleR
    res = (Js @ delta + Rr)[idx]
    absrow = (abs(Js) @ np.abs(delta) + np.abs(Rr))[idx]
    bound = 1.01e-10 * np.linalg.norm(Rg) + 1e-13 * absrow
    say(f"sampled |J delta + R| max {np.abs(res).max():.2e} (bound {1e-10 * np.linalg.norm(Rg):.2e})")
    assert np.all(np.abs(res) <= bound)
    assert np.all(delta[2 * p.dir_ids] == 0) and np.all(delta[2 * p.dir_ids + 1] == 0)
    # a Newton predictor-corrector step from the initial state: its result satisfies the
    # implicit coupled equations up to the last Newton update (||delta_T|| <= 1e-9 ||T||)
    dp.reset()
    st = dp.step_mono(dt, corr_tol=1e-9, m=20)
    T2, V2 = to_host(dp.T), to_host(dp.V)
    dp.close()
    say(f"Newton step at 101^3: {st}")
    assert st["accepted"] == 1
    R2 = mono.residual(ms, T0, dt, T2, V2)[idx]
    M2 = mono.interleaved_matrix(ms, mono.jacobian_blocks(ms, T0, dt, T2, V2))
    scale = (abs(M2) @ np.abs(np.ravel(np.column_stack([T2, V2]))))[idx] + 1.0
    say(f"sampled implicit residual / row scale max {np.abs(R2 / scale).max():.2e}")
    assert np.all(np.abs(R2) <= 1e-7 * scale)


def test_hex101_hundred_steps_mixed_tracks_fp64_and_satisfies_oracle_equations(torch_cuda):
    """The benchmarked 101^3 workload over 100 coupled steps (extrapolated starting points):
    each path against the oracle's own 100-step trajectory (stored by
    tests/golden/make_trajectories.py: 2,000 free nodes at steps 1, 10, ..., 100, sampled
    relative error <= 1e-8), the mixed state within 1e-8 of the FP64 state at every step,
    and both paths' 100th step satisfying the oracle's equations of 2,000 sampled rows
    (given their 99th state)."""
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.config1(steps=100)
    runs = {}
    for precision in ("fp64", "mixed"):
        dp = DeviceProblem(p)
        dp.extrapolate = True
        states = []
        for _ in range(100):
            dp.step(TOL, precision)
            states.append((to_host(dp.T), to_host(dp.V)))
        dp.close()
        runs[precision] = states
        say(f"{precision}: 100 steps done")
    gold = np.load(os.path.join(GOLDEN, "c1_hex101_trajectory.npz"))
    nodes = gold["nodes"]
    for precision, states in runs.items():
        worst_o = 0.0
        for j, k in enumerate(gold["steps"]):
            Tg, Vg = states[k - 1]
            eT = rel_err(Tg[nodes], gold["T"][j])
            eV = rel_err(Vg[nodes], gold["V"][j])
            e37 = rel_err(Tg[nodes] - 37.0, gold["T"][j] - 37.0)
            worst_o = max(worst_o, eT, eV)
            say(f"{precision} step {k} vs stored oracle: T {eT:.2e} V {eV:.2e} (T-37 {e37:.2e})")
            assert eT <= 1e-8 and eV <= 1e-8
        say(f"{precision}: worst sampled error against the oracle trajectory {worst_o:.2e}")
    worst = 0.0
    for (T6, V6), (Tm, Vm) in zip(runs["fp64"], runs["mixed"]):
        worst = max(worst, rel_err(Tm, T6), rel_err(Vm, V6))
    say(f"mixed vs FP64 over 100 steps: max rel err {worst:.2e}")
    assert worst <= 1e-8
    free = np.setdiff1d(np.arange(p.n_nodes), p.dir_ids)
    rows = np.sort(np.random.default_rng(5).choice(free, 2000, replace=False))
    gV, gT = np.linalg.norm(p.dir_V), np.linalg.norm(p.dir_T)
    for precision, states in runs.items():
        T99, (T100, V100) = states[98][0], states[99]
        rV, sV, rT, sT = _sampled_equations(p, rows, T99, V100, T100)
        say(f"{precision} step 100: max |rV| {np.abs(rV).max():.2e}, max |rT| {np.abs(rT).max():.2e}")
        assert np.all(np.abs(rV) <= 10 * TOL * gV + 1e-13 * sV)
        assert np.all(np.abs(rT) <= 10 * TOL * gT + 1e-13 * sT)

"""Batched ensemble on the GPU: every sample of a batch handle matches its own single-mesh
solve and the oracle; graph-replayed iteration chunks match stream launches bit for bit."""
import numpy as np
import pytest

import rafem_inputs as ri
from oracle.rafem import Model
from gpu_helpers import rel_err, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _samples(kind="hex"):
    # uneven sizes and lognormal-scaled properties, as in the ensemble workload
    out = []
    for q, (n, ks, ss, ps) in enumerate([(9, 1.1, 0.9, 1.2), (14, 0.85, 1.15, 0.9), (11, 1.0, 1.0, 1.0)]):
        out.append(ri.make_problem(kind, n, 40 + q, k_scale=ks, sigma_scale=ss, perf_scale=ps,
                                   per_element_eps=False, name=f"s{q}"))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_batch_matches_single_solves_and_oracle(torch_cuda, precision, kind):
    from paper_2409_13036_amd.sim import BatchProblem, DeviceProblem
    probs = _samples(kind)
    steps, tol = 3, 1e-13
    bp = BatchProblem(probs)
    assert bp.mesh.n_samples == len(probs)
    assert all(int(o) % 1024 == 0 for o in bp.mesh.node_off)
    binfo = [bp.step(tol, precision) for _ in range(steps)]
    for q, p in enumerate(probs):
        dp = DeviceProblem(p)
        dp.simulate(steps, tol=tol, precision=precision)
        Tb, Vb = bp.sample(q)
        Ts, Vs = to_host(dp.T), to_host(dp.V)
        eT, eV = rel_err(Tb, Ts), rel_err(Vb, Vs)
        print(f"[batch {kind} {precision} sample {q} n={p.n}] vs single: T {eT:.2e} V {eV:.2e} "
              f"info {bp.mesh.sample_info(q)['V']['iters']}/{bp.mesh.sample_info(q)['T']['iters']}",
              flush=True)
        # same kernels, same per-sample reduction order: identical to the single solve
        assert np.array_equal(Tb, Ts) and np.array_equal(Vb, Vs)
        dp.close()
    # one sample against the oracle
    q = 1
    ref, _ = Model(probs[q]).simulate(steps, 1e-15)
    Tb, Vb = bp.sample(q)
    assert rel_err(Tb, ref[-1][0]) <= 1e-8 and rel_err(Vb, ref[-1][1]) <= 1e-8
    # padding nodes stay at zero
    m = bp.mesh
    for q, p in enumerate(probs):
        a, b = int(m.node_off[q]) + p.n_nodes, int(m.node_off[q + 1])
        assert float(bp.T[a:b].abs().max()) == 0.0 if b > a else True
    bp.close()


def test_graph_chunks_match_stream_launches(torch_cuda):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("hex", 17, 3, steps=3)
    out = []
    for graphs in (False, True):
        dp = DeviceProblem(p)
        dp.mesh.set_graphs(graphs)
        for precision in ("fp64", "mixed"):
            dp.reset()
            for _ in range(3):
                dp.step(1e-13, precision)
            out.append((to_host(dp.T), to_host(dp.V)))
        dp.close()
    for (Ta, Va), (Tb, Vb) in zip(out[:2], out[2:]):
        assert np.array_equal(Ta, Tb) and np.array_equal(Va, Vb)


def test_batch_samples_converge_independently(torch_cuda):
    from paper_2409_13036_amd.sim import BatchProblem
    probs = [ri.make_problem("hex", 7, 1), ri.make_problem("hex", 21, 2)]
    bp = BatchProblem(probs)
    bp.step(1e-13)
    it_small = bp.mesh.sample_info(0)["V"]["iters"]
    it_big = bp.mesh.sample_info(1)["V"]["iters"]
    assert 0 < it_small < it_big
    # mixed: per-sample inner iteration totals and refinement counts, as for single solves
    bp.reset()
    bp.step(1e-13, "mixed")
    for q, p in enumerate(probs):
        from paper_2409_13036_amd.sim import DeviceProblem
        dp = DeviceProblem(p)
        single = dp.step(1e-13, "mixed")
        got = bp.mesh.sample_info(q)
        for f in ("V", "T"):
            assert got[f]["status"] == 0
            assert got[f]["iters"] == single[f]["iters"] and got[f]["outer"] == single[f]["outer"]
            assert got[f]["iters"] > got[f]["outer"] > 0
        dp.close()
    bp.close()


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_batch_reverse_sweep_matches_single_adjoints(torch_cuda, kind):
    """rafem_step_vjp on a batch handle: each sample's gradients with respect to its k_e
    and w_e equal those of its own single-mesh reverse sweep."""
    torch = torch_cuda
    from paper_2409_13036_amd import _lib as R
    from paper_2409_13036_amd.adjoint import lesion_loss
    from paper_2409_13036_amd.sim import BatchProblem, DeviceProblem
    steps, tol = 3, 1e-13
    probs = [ri.make_problem(kind, n, 60 + q, steps=steps, with_loss=True, k_scale=ks,
                             per_element_eps=False, name=f"a{q}")
             for q, (n, ks) in enumerate([(9, 1.0), (12, 0.8), (7, 1.3)])]
    bp = BatchProblem(probs)
    m = bp.mesh
    Ts, Vs = [bp.T.clone()], [bp.V.clone()]
    for _ in range(steps):
        bp.step(tol, "fp64")
        Ts.append(bp.T.clone())
        Vs.append(bp.V.clone())
    # dL/dT^N of L = sum over samples of their lesion losses
    ids = np.concatenate([p.loss_ids + int(m.node_off[q]) for q, p in enumerate(probs)])
    tgt = np.concatenate([p.T_target for p in probs])
    lam = torch.zeros(m.n_nodes, dtype=torch.float64, device="cuda")
    R.lesion_loss(m, torch.as_tensor(ids, dtype=torch.int32, device="cuda"),
                  torch.as_tensor(tgt, dtype=torch.float64, device="cuda"), Ts[-1], grad=lam)
    gk = torch.zeros(m.n_elems, dtype=torch.float64, device="cuda")
    gw = torch.zeros_like(gk)
    bp.phys.reuse_bioheat = 1
    for n in range(steps, 0, -1):
        # the reverse sweep's starting points as lesion_loss takes them (each reverse step
        # from the adjoint states of the step after it)
        bp.phys.extrapolate = 2 if n == steps else 1
        R.step_vjp(m, bp.phys, bp.k_e, bp.perf_e, bp.sigma0_e, bp.dir_V, bp.dir_T, Ts[n - 1],
                   Vs[n], Ts[n], lam, gk, gw, tol=tol)
    gk, gw = to_host(gk), to_host(gw)
    bp.close()
    for q, p in enumerate(probs):
        dp = DeviceProblem(p)
        k = torch.tensor(p.k_e, dtype=torch.float64, device="cuda", requires_grad=True)
        w = torch.tensor(p.perf_e, dtype=torch.float64, device="cuda", requires_grad=True)
        lesion_loss(dp, k, w, steps, checkpoint_every=steps, tol=tol).backward()
        a, b = int(m.elem_off[q]), int(m.elem_off[q + 1])
        ek = rel_err(gk[a:b], to_host(k.grad))
        ew = rel_err(gw[a:b], to_host(w.grad))
        print(f"[batch adjoint {kind} sample {q}] grad_k {ek:.2e} grad_w {ew:.2e}", flush=True)
        assert ek <= 1e-12 and ew <= 1e-12
        dp.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_device_driven_steps_equal_host_driven_steps(torch_cuda, precision):
    """Device-driven solves (each solve of a step enqueued whole from the previous solves'
    counts, one poll per solve; an option of any handle) give the host-driven steps'
    results bit for bit, on a batch and on a single mesh, with the predictor's starting
    points; budgets cut to 0.3 of the counts force solves to be redone host-driven, with
    the same results.  Step 1 starts from the initial state without the predictor, steps
    2, 3 and 4 with the quadratic predictor's orders 0, 1 and 2, so budgets come from two
    alike solves from step 6 on."""
    from paper_2409_13036_amd.sim import BatchProblem, DeviceProblem
    tol, steps = 1e-13, 9
    first_dd = 6
    probs = _samples("hex") + [ri.make_problem("hex", 17, 47, k_scale=0.9, sigma_scale=1.2,
                                               perf_scale=1.1, per_element_eps=False, name="s3")]

    def run_batch(mode, scale=0.0):
        bp = BatchProblem(probs)
        bp.extrapolate = True
        bp.mesh.set_device_driven(mode, scale)
        out = []
        for _ in range(steps):
            info = bp.step(tol, precision)
            assert info["V"]["status"] == 0 and info["T"]["status"] == 0
            out.append((to_host(bp.T), to_host(bp.V),
                        [bp.mesh.sample_info(q) for q in range(len(probs))], info))
        st = bp.mesh.stats()
        bp.close()
        return out, st

    host, st_h = run_batch(False)
    dev, st_d = run_batch(True)
    cut, st_c = run_batch(True, 0.3)
    print(f"[device-driven {precision}] solves accepted {st_d.device_driven_solves}, redone "
          f"{st_d.device_driven_redone}; with budgets x0.3: accepted "
          f"{st_c.device_driven_solves}, redone {st_c.device_driven_redone}", flush=True)
    assert st_h.device_driven_solves == 0
    # both solves of every step from the sixth on run device-driven, the others host-driven
    n_dd = steps - first_dd + 1
    assert st_d.device_driven_solves + st_d.device_driven_redone == 2 * n_dd
    assert st_d.device_driven_solves >= n_dd
    assert st_c.device_driven_redone >= 1
    for k, (a, b, c) in enumerate(zip(host, dev, cut)):
        for other in (b, c):
            assert np.array_equal(a[0], other[0]) and np.array_equal(a[1], other[1]), k
            for ia, ib in zip(a[2], other[2]):
                for f in ("V", "T"):
                    assert ia[f]["iters"] == ib[f]["iters"] and ia[f]["outer"] == ib[f]["outer"]
                    assert ia[f]["status"] == ib[f]["status"]
            assert a[3]["V"]["iters"] == other[3]["V"]["iters"]
            assert a[3]["T"]["iters"] == other[3]["T"]["iters"]
    # a single mesh, device-driven on request
    p = probs[1]
    runs = []
    for mode in (False, True):
        dp = DeviceProblem(p)
        dp.extrapolate = True
        dp.mesh.set_device_driven(mode)
        states = []
        for _ in range(steps):
            dp.step(tol, precision)
            states.append((to_host(dp.T), to_host(dp.V)))
        runs.append((states, dp.mesh.stats()))
        dp.close()
    assert runs[1][1].device_driven_solves >= n_dd
    for (Ta, Va), (Tb, Vb) in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(Ta, Tb) and np.array_equal(Va, Vb)

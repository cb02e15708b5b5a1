"""rafem_solve_enqueue: a whole solve enqueued with fixed budgets and its report written to
device memory, against rafem_solve (the host-driven solve with polls) and the oracle."""
import numpy as np
import pytest

import rafem_inputs as ri
from oracle.rafem import Model
from oracle.solvers import pcg
from gpu_helpers import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2409_13036_amd import _lib
    return _lib


def _potential(p):
    m = Model(p)
    A, b = m.potential_system(m.sigma(p.initial_T()))
    return A, b, p.initial_V()


def _csr(A):
    return (to_dev(A.indptr.astype(np.int32)), to_dev(A.indices.astype(np.int32)),
            to_dev(A.data.copy()), to_dev(A.data.astype(np.float32)))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_enqueued_solve_equals_host_driven_solve(R, precision):
    """With budgets that suffice, the enqueued solve returns rafem_solve's x bit for bit, and
    its device report holds the same status, iteration and refinement counts and true
    residual; the oracle's solution agrees to the parity tolerance."""
    p = ri.make_problem("hex", 21, 4)
    A, b, x0 = _potential(p)
    rp, ci, v, v32 = _csr(A)
    mesh = R.Mesh(p.xyz, p.conn, p.dir_ids)
    x_host = to_dev(x0)
    info = R.solve(mesh, rp, ci, v, to_dev(b), x_host, vals32=v32, tol=1e-13, precision=precision)
    if precision == "fp64":
        iterations, refinements = info["iters"] + 7, 1
    else:
        iterations, refinements = info["iters"], info["outer"] + 1
    buf = R.device_info_buffer()
    x_dev = to_dev(x0)
    R.solve_enqueue(mesh, rp, ci, v, to_dev(b), x_dev, buf, iterations=iterations,
                    refinements=refinements, vals32=v32, tol=1e-13, precision=precision)
    d = R.read_device_info(buf)
    xref, _ = pcg(A, b, x0, 1e-15, maxit=20000)
    print(f"[enqueue {precision}] host {info['iters']}/{info['outer']} device {d['iters']}/"
          f"{d['outer']} relres {d['relres_true']:.2e} err {rel_err(to_host(x_dev), xref):.2e}",
          flush=True)
    assert d["status"] == R.OK
    assert d["iters"] == info["iters"] and d["outer"] == info["outer"]
    assert d["relres_true"] == info["relres_true"]
    assert np.array_equal(to_host(x_dev), to_host(x_host))
    assert rel_err(to_host(x_dev), xref) <= 1e-8
    mesh.close()


def test_enqueued_solve_reports_a_short_budget(R):
    """A budget below the need ends with RAFEM_E_NOCONV in the device report, the iterate of
    that many iterations in x (FP64: rafem_solve stopped at the same limit), and the true
    residual of that iterate."""
    p = ri.make_problem("hex", 21, 4)
    A, b, x0 = _potential(p)
    rp, ci, v, v32 = _csr(A)
    mesh = R.Mesh(p.xyz, p.conn, p.dir_ids)
    x_host = to_dev(x0)
    info = R.solve(mesh, rp, ci, v, to_dev(b), x_host, tol=1e-13, maxit=10, check=False)
    buf = R.device_info_buffer()
    x_dev = to_dev(x0)
    R.solve_enqueue(mesh, rp, ci, v, to_dev(b), x_dev, buf, iterations=10, tol=1e-13)
    d = R.read_device_info(buf)
    assert info["status"] == R.E_NOCONV and d["status"] == R.E_NOCONV
    assert d["iters"] == 10 and d["relres_true"] == info["relres_true"] > 1e-13
    assert np.array_equal(to_host(x_dev), to_host(x_host))
    x_mix = to_dev(x0)
    R.solve_enqueue(mesh, rp, ci, v, to_dev(b), x_mix, buf, iterations=5, refinements=2,
                    vals32=v32, tol=1e-13, precision="mixed")
    d = R.read_device_info(buf)
    assert d["status"] == R.E_NOCONV and d["outer"] == 2 and d["relres_true"] > 1e-13
    mesh.close()


def test_enqueued_solve_argument_errors(R):
    """Budgets out of range, a batch handle, a missing FP32 copy and a NULL report are
    refused before anything is enqueued."""
    import torch
    p = ri.make_problem("hex", 9, 4)
    A, b, x0 = _potential(p)
    rp, ci, v, v32 = _csr(A)
    mesh = R.Mesh(p.xyz, p.conn, p.dir_ids)
    buf = R.device_info_buffer()
    x = to_dev(x0)
    bb = to_dev(b)
    for kw in ({"iterations": 0}, {"iterations": 100001},
               {"iterations": 5, "refinements": 0, "precision": "mixed", "vals32": v32},
               {"iterations": 5, "refinements": 15, "precision": "mixed", "vals32": v32},
               {"iterations": 5, "precision": "mixed"}):
        st = R.solve_enqueue(mesh, rp, ci, v, bb, x, buf, check=False, **kw)
        assert st == R.E_ARG, kw
    assert np.array_equal(to_host(x), x0)
    mesh.close()
    probs = [ri.make_problem("hex", 9, 4), ri.make_problem("hex", 7, 5)]
    from paper_2409_13036_amd.sim import BatchProblem
    bp = BatchProblem(probs)
    n = bp.mesh.n_nodes
    st = R.solve_enqueue(bp.mesh, torch.zeros(n + 1, dtype=torch.int32, device="cuda"),
                         torch.zeros(1, dtype=torch.int32, device="cuda"),
                         torch.zeros(1, dtype=torch.float64, device="cuda"),
                         torch.zeros(n, dtype=torch.float64, device="cuda"),
                         torch.zeros(n, dtype=torch.float64, device="cuda"), buf,
                         iterations=5, check=False)
    assert st == R.E_ARG
    bp.close()

"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by element.

Sizes span several workgroups plus a ragged tail (n^3 nodes is never a multiple of the
block row counts).  Tolerances: CSR structure bit-exact; assembled values, SpMV and
lifting within a few-ulp forward-error bound; solutions within 1e-8 relative error.
"""
import dataclasses

import numpy as np
import pytest

import rafem_inputs as ri
from oracle.rafem import Model
from oracle.solvers import pcg, dense_solve
from gpu_helpers import (EPS32, EPS64, assembly_bound, rel_err, spmv_bound, to_dev,
                               to_host)

pytestmark = pytest.mark.gpu

SOL_TOL = 1e-8


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2409_13036_amd import _lib
    return _lib


def _mesh(R, p):
    print(f"[case] mesh {p.name} N={p.n_nodes} E={p.n_elems}", flush=True)
    return R.Mesh(p.xyz, p.conn, p.dir_ids)


# "hexj": hexes with jittered interior nodes, i.e. general trilinear (non-affine) elements
CASES = [("hex", 5), ("hex", 21), ("hex", 26), ("hexj", 11), ("tet", 6), ("tet", 17)]


def _problem(kind, n, seed, **kw):
    if kind == "hexj":
        return ri.make_problem("hex", n, seed, jitter=True, name=f"hexj{n}", **kw)
    return ri.make_problem(kind, n, seed, **kw)


@pytest.mark.parametrize("kind,n", CASES)
def test_structure_and_assembly_match_oracle(R, kind, n):
    import torch
    p = _problem(kind, n, 1)
    m = Model(p)
    mesh = _mesh(R, p)
    # bioheat-type coefficients: mass and stiffness, no lifting
    a_e = p.rho_c / p.dt + p.perf_e
    out = R.assemble_csr(mesh, stiff_coef=to_dev(p.k_e), mass_coef=to_dev(a_e), want_f32=True)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out["row_ptr"]), m.S.row_ptr)
    assert np.array_equal(to_host(out["col_idx"]), m.S.col_idx)
    ref = m.S.assemble(m.Ke, m.Me, a_e, p.k_e)
    got = to_host(out["vals"])
    assert np.all(np.abs(got - ref) <= assembly_bound(m.S, ref, EPS64))
    assert np.array_equal(to_host(out["vals32"]), ref.astype(np.float32)) or \
        np.all(np.abs(to_host(out["vals32"]) - ref) <= np.abs(ref) * EPS32 + assembly_bound(m.S, ref, EPS64))
    # stiffness only, with lifting
    out = R.assemble_csr(mesh, stiff_coef=to_dev(p.sigma0_e), dir_vals=to_dev(p.dir_V), want_f32=True)
    ref, lift = m.S.lift(m.S.assemble(m.Ke, m.Me, None, p.sigma0_e), p.dir_ids, p.dir_V)
    got = to_host(out["vals"])
    assert np.all(np.abs(got - ref) <= assembly_bound(m.S, np.maximum(np.abs(ref), 1e-300), EPS64) + 0.0)
    # rows and columns of Dirichlet nodes are exactly zero apart from a unit diagonal
    isD = np.zeros(p.n_nodes, dtype=bool)
    isD[p.dir_ids] = True
    lifted = isD[m.S.row_of] | isD[m.S.col_idx]
    unit = isD[m.S.row_of] & (m.S.row_of == m.S.col_idx)
    assert np.all(got[lifted & ~unit] == 0.0) and np.all(got[unit] == 1.0)
    gl = to_host(out["rhs_lift"])
    unl = m.S.assemble(m.Ke, m.Me, None, p.sigma0_e)
    gfull = np.zeros(p.n_nodes)
    gfull[p.dir_ids] = p.dir_V
    # the lift inherits the entrywise assembly tolerance: sum_d |dA_fd| |g_d| + rounding
    pattern = m.S.matrix(np.ones(m.S.nnz))
    rowmax = np.maximum.reduceat(np.abs(unl), m.S.row_ptr[:-1])
    bound = 64 * EPS64 * rowmax * (pattern @ np.abs(gfull)) + spmv_bound(m.S.matrix(unl), gfull, EPS64)
    assert np.all(np.abs(gl - lift) <= bound)
    mesh.close()


@pytest.mark.parametrize("kind,n", CASES)
def test_spmv_matches_oracle(R, kind, n):
    import torch
    p = _problem(kind, n, 2)
    m = Model(p)
    mesh = _mesh(R, p)
    vals = m.S.assemble(m.Ke, m.Me, p.rho_c / p.dt + p.perf_e, p.k_e)
    A = m.S.matrix(vals)
    x = ri.random_vector(p.n_nodes, 3)
    rp, ci = to_dev(m.S.row_ptr), to_dev(m.S.col_idx)
    y = torch.empty(p.n_nodes, dtype=torch.float64, device="cuda")
    R.spmv(mesh, rp, ci, to_dev(vals), to_dev(x), y)
    torch.cuda.synchronize()
    ref = A @ x
    assert np.all(np.abs(to_host(y) - ref) <= spmv_bound(A, x, EPS64))
    # FP32 kernel against the FP64 product of the FP32-rounded operands
    v32, x32 = vals.astype(np.float32), x.astype(np.float32)
    y32 = torch.empty(p.n_nodes, dtype=torch.float32, device="cuda")
    R.spmv(mesh, rp, ci, to_dev(v32), to_dev(x32), y32)
    torch.cuda.synchronize()
    A32 = m.S.matrix(v32.astype(np.float64))
    ref32 = A32 @ x32.astype(np.float64)
    assert np.all(np.abs(to_host(y32) - ref32) <= spmv_bound(A32, x32.astype(np.float64), EPS32))
    mesh.close()


def _lifted_bioheat(m, p, T=None):
    A, lift = m.bioheat_system()
    T = p.initial_T() if T is None else T
    b = m.bioheat_rhs(T, np.zeros(p.n_nodes), lift)
    return A, b


@pytest.mark.parametrize("kind,n", [("hex", 21), ("tet", 17)])
@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed-restarted"])
def test_solve_matches_oracle(R, kind, n, precision):
    """FP64 PCG, mixed refinement with reliable updates (the default: the inner recurrence
    goes on from each refined residual) and plain restarted refinement, against the oracle."""
    restart = 1 if precision == "mixed-restarted" else 0
    precision = "mixed" if restart else precision
    import torch
    p = ri.make_problem(kind, n, 4)
    m = Model(p)
    mesh = _mesh(R, p)
    for sysname in ("potential", "bioheat"):
        if sysname == "potential":
            A, b = m.potential_system(m.sigma(p.initial_T()))
            x0 = p.initial_V()
        else:
            A, b = _lifted_bioheat(m, p)
            x0 = p.initial_T()
        xref, info = pcg(A, b, x0, 1e-15, maxit=20000)
        x = to_dev(x0)
        vals = A.data.copy()
        out = R.solve(mesh, to_dev(A.indptr.astype(np.int32)), to_dev(A.indices.astype(np.int32)),
                      to_dev(vals), to_dev(b), x, vals32=to_dev(vals.astype(np.float32)), tol=1e-13,
                      precision=precision, restart_inner=restart, inner_tol=1e-3)
        err = rel_err(to_host(x), xref)
        print(f"[{sysname} {precision}] iters={out['iters']} outer={out['outer']} relres_true="
              f"{out['relres_true']:.2e} err={err:.2e}", flush=True)
        assert out["status"] == R.OK
        assert out["relres_true"] <= 1e-13 * 1.01
        assert err <= SOL_TOL
    mesh.close()


@pytest.mark.parametrize("kind,n,steps", [("hex", 21, 3), ("tet", 13, 2), ("hex", 9, 2),
                                          ("hexj", 11, 2)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_coupled_steps_match_oracle(R, kind, n, steps, precision):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = _problem(kind, n, 5, steps=steps)
    m = Model(p)
    ref_states, _ = m.simulate(steps, 1e-15)
    dp = DeviceProblem(p)
    states, infos = dp.simulate(steps, tol=1e-13, precision=precision, keep=True)
    for k, ((T, V), (Tr, Vr), inf) in enumerate(zip(states, ref_states, infos)):
        eT, eV = rel_err(T, Tr), rel_err(V, Vr)
        eTs = float(np.linalg.norm(T - Tr) / np.linalg.norm(Tr - p.T_a))
        print(f"[step {k} {precision}] V iters={inf['V']['iters']} T iters={inf['T']['iters']} "
              f"errV={eV:.2e} errT={eT:.2e} errT(T-37)={eTs:.2e}", flush=True)
        assert eV <= SOL_TOL and eT <= SOL_TOL
    dp.close()


def test_config0_bioheat_step(R):
    """The plain FP64 case: 21^3 hex, one bioheat step, zero Joule source, tol 1e-10.

    The oracle runs the same PCG with the same stopping rule and start, so both stop
    after the same iterations and agree far below the tolerance; the distance of either
    to the exactly solved step (about 1.6e-8 at this tolerance) is reported, not asserted."""
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.config0()
    m = Model(p)
    states, oinf = m.simulate(1, p.tol)
    Tr = states[0][0]
    exact, _ = m.simulate(1, 1e-15)
    dp = DeviceProblem(p)
    info = dp.step(tol=p.tol)
    T = to_host(dp.T)
    err = rel_err(T, Tr)
    print(f"[C0] iters={info['T']['iters']} (oracle {oinf[0].T.iters}) relres_true="
          f"{info['T']['relres_true']:.2e} err={err:.2e} err_vs_exact={rel_err(T, exact[0][0]):.2e}")
    assert info["T"]["relres_true"] <= p.tol * 1.01
    assert abs(info["T"]["iters"] - oinf[0].T.iters) <= 1
    assert err <= SOL_TOL
    dp.close()


def test_steps_are_deterministic(R):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("hex", 26, 6, steps=2)
    dp = DeviceProblem(p)
    a, _ = dp.simulate(2, keep=True)
    dp.reset()
    b, _ = dp.simulate(2, keep=True)
    for (T1, V1), (T2, V2) in zip(a, b):
        assert np.array_equal(T1, T2) and np.array_equal(V1, V2)
    dp.close()


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_grid_meshes_use_shared_offset_slabs(R, kind):
    """On the grid meshes every full slab away from the first and last planes shares one
    column-offset list (boundary rows hold a subset of the interior stencil); the steps
    and solves above run through those slabs."""
    p = ri.make_problem(kind, 26, 1)
    mesh = _mesh(R, p)
    st = mesh.stats()
    plane_slabs = 2 * (26 * 26 + 26 + 1) // 64 + 4
    assert st.slabs == (p.n_nodes + 63) // 64
    assert st.shared_offset_slabs >= st.slabs - plane_slabs
    mesh.close()


def test_spmv_timing_entry_point(R):
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("hex", 13, 2)
    dp = DeviceProblem(p)
    with pytest.raises(R.RafemError, match="E_STATE"):
        R.spmv_timing(dp.mesh, "fp64")
    with pytest.raises(R.RafemError, match="E_ARG"):
        R.spmv_timing(dp.mesh, "fp64", copies=0)
    dp.step(1e-12)
    for precision in ("fp64", "mixed"):
        for copies in (1, 3):
            t = R.spmv_timing(dp.mesh, precision, copies=copies, reps=6)
            assert 0.0 < t < 1e5
    # the solver's own buffers are left usable: the next step still matches the oracle
    T0, V0 = to_host(dp.T), to_host(dp.V)
    dp.step(1e-13)
    ref = Model(p).step(T0, V0, 1e-15)
    assert rel_err(to_host(dp.T), ref[0]) <= SOL_TOL and rel_err(to_host(dp.V), ref[1]) <= SOL_TOL
    dp.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_steps_do_not_depend_on_stale_device_memory(R, precision):
    """Device memory handed to a new mesh may hold anything: a mesh built on memory that
    held NaN must step exactly as one built on fresh memory (no kernel may read an entry
    that nothing wrote, such as the slab padding of the FP32 matrix values)."""
    import torch
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("hex", 13, 5, steps=2)

    def run():
        dp = DeviceProblem(p)
        states, infos = dp.simulate(2, tol=1e-13, precision=precision, keep=True)
        dp.close()
        return states, infos

    clean, _ = run()
    junk = torch.full((64 << 20,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    del junk
    torch.cuda.empty_cache()
    dirty, infos = run()
    assert all(i["V"]["status"] == 0 and i["T"]["status"] == 0 for i in infos)
    for (T1, V1), (T2, V2) in zip(clean, dirty):
        assert np.array_equal(T1, T2) and np.array_equal(V1, V2)


def test_solve_adjoint_matches_oracle(R):
    import torch
    p = ri.make_problem("hex", 13, 7)
    m = Model(p)
    mesh = _mesh(R, p)
    A, _ = m.bioheat_system()
    g = ri.random_vector(p.n_nodes, 8)
    gz = g.copy()
    gz[p.dir_ids] = 0.0
    lref = dense_solve(A.T.tocsr(), gz)
    lam = torch.zeros(p.n_nodes, dtype=torch.float64, device="cuda")
    gd = to_dev(g)
    out = R.solve_adjoint(mesh, to_dev(A.indptr.astype(np.int32)), to_dev(A.indices.astype(np.int32)),
                          to_dev(A.data), gd, lam, tol=1e-14)
    assert out["status"] == R.OK
    assert np.array_equal(to_host(gd), g)  # input untouched
    assert rel_err(to_host(lam), lref) <= SOL_TOL
    assert np.all(to_host(lam)[p.dir_ids] == 0.0)
    mesh.close()


def test_solver_edge_cases(R):
    import torch
    p = ri.make_problem("hex", 6, 9)   # 216 rows: fewer than one workgroup's rows
    m = Model(p)
    mesh = _mesh(R, p)
    A, b = _lifted_bioheat(m, p)
    rp, ci, v = to_dev(A.indptr.astype(np.int32)), to_dev(A.indices.astype(np.int32)), to_dev(A.data)
    xs = dense_solve(A, b)
    # exact start: converged before the first iteration
    x = to_dev(xs)
    out = R.solve(mesh, rp, ci, v, to_dev(b), x, tol=1e-10)
    assert out["status"] == R.OK and out["iters"] == 0
    # zero right-hand side from zero: 0 iterations, x stays 0
    x = torch.zeros(p.n_nodes, dtype=torch.float64, device="cuda")
    out = R.solve(mesh, rp, ci, v, torch.zeros_like(x), x, tol=1e-10)
    assert out["status"] == R.OK and out["iters"] == 0 and float(x.abs().max()) == 0.0
    # iteration limit: status NOCONV, x holds the first iterate
    x = to_dev(p.initial_T())
    out = R.solve(mesh, rp, ci, v, to_dev(b), x, tol=1e-14, maxit=1, check=False)
    assert out["status"] == R.E_NOCONV and out["iters"] == 1
    xo, io = pcg(A, b, p.initial_T(), 1e-14, maxit=1)
    assert rel_err(to_host(x), xo) <= 1e-13
    # not SPD: breakdown is reported
    out = R.solve(mesh, rp, ci, to_dev(-A.data), to_dev(b), to_dev(p.initial_T()), tol=1e-12,
                  check=False)
    assert out["status"] == R.E_BREAKDOWN
    # non-finite right-hand side
    bn = b.copy()
    bn[17] = np.nan
    out = R.solve(mesh, rp, ci, v, to_dev(bn), to_dev(p.initial_T()), tol=1e-12, check=False)
    assert out["status"] == R.E_BREAKDOWN
    # mixed precision: same answer on this tiny system
    x = to_dev(p.initial_T())
    out = R.solve(mesh, rp, ci, v, to_dev(b), x, vals32=to_dev(A.data.astype(np.float32)), tol=1e-13,
                  precision="mixed")
    assert out["status"] == R.OK and rel_err(to_host(x), xs) <= SOL_TOL
    mesh.close()


def test_abi_argument_errors(R):
    import torch
    p = ri.make_problem("hex", 5, 0)
    bad = p.conn.copy()
    bad[0, 0] = -1
    with pytest.raises(R.RafemError) as ei:
        R.Mesh(p.xyz, bad, p.dir_ids)
    assert ei.value.status == R.E_MESH
    inv = p.conn.copy()
    inv[:, [0, 1]] = inv[:, [1, 0]]  # mirrored hexes: negative Jacobian
    with pytest.raises(R.RafemError) as ei:
        R.Mesh(p.xyz, inv, p.dir_ids)
    assert ei.value.status == R.E_MESH
    with pytest.raises(R.RafemError) as ei:
        R.Mesh(p.xyz, p.conn, p.dir_ids[::-1].copy())
    assert ei.value.status == R.E_ARG
    mesh = R.Mesh(p.xyz, p.conn, p.dir_ids)
    phys = R.Phys(p.rho_c, p.dt, p.T_a, p.alpha_sigma, p.T_ref, 1, 1)
    T = to_dev(p.initial_T())
    with pytest.raises(R.RafemError) as ei:   # reuse requested before any assembly
        R.step(mesh, phys, to_dev(p.k_e), to_dev(p.perf_e), to_dev(p.sigma0_e), to_dev(p.dir_V),
               to_dev(p.dir_T), T, to_dev(p.initial_V()))
    assert ei.value.status == R.E_STATE
    import torch
    vals = torch.empty(mesh.nnz, dtype=torch.float64, device="cuda")
    kd, dv = to_dev(p.k_e), to_dev(p.dir_V)
    st = R.lib().rafem_assemble_csr(mesh.handle, None, kd.data_ptr(), dv.data_ptr(), None, None,
                                    vals.data_ptr(), None, None, None)
    assert st == R.E_ARG and "rhs_lift" in R.last_error()
    mesh.close()

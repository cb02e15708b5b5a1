"""Region timing of the steps (assembly / solve / check) and the PSNR of GPU runs against
the oracle's run with the paper's control lines."""
import time

import numpy as np
import pytest

import rafem_inputs as ri
from oracle.rafem import Model
from gpu_helpers import to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def test_regions_cover_the_step(torch_cuda):
    from paper_2409_13036_amd import _lib as R
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("hex", 31, 0)
    dp = DeviceProblem(p)
    dp.step(1e-13)                          # first step: assembly of the bioheat matrix, tuning
    R.regions_enable(dp.mesh, True)
    R.regions_read(dp.mesh, reset=True)
    torch_cuda.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dp.step(1e-13)
    wall = (time.perf_counter() - t0) * 1e3 / 3
    r = R.regions_read(dp.mesh, reset=True)
    print(f"[regions step] {r}, wall {wall:.2f} ms/step", flush=True)
    assert r["steps"] == 3 and r["assembly_ms"] > 0 and r["solve_ms"] > r["assembly_ms"]
    assert r["assembly_ms"] + r["solve_ms"] + r["check_ms"] <= 1.05 * wall + 0.05
    # corrector steps: one count per call, the convergence checks in their own region
    dp.step_pc(2.0, corr_tol=1e-9)
    dp.step_mono(2.0, corr_tol=1e-9)
    r = R.regions_read(dp.mesh, reset=True)
    print(f"[regions pc+mono] {r}", flush=True)
    assert r["steps"] == 2 and r["check_ms"] > 0 and r["solve_ms"] > 0
    R.regions_enable(dp.mesh, False)
    dp.step(1e-13)
    assert R.regions_read(dp.mesh)["steps"] == 0
    dp.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_psnr_against_the_oracle_run(torch_cuda, precision):
    from paper_2409_13036_amd import report
    from paper_2409_13036_amd.sim import DeviceProblem
    p = ri.make_problem("tet", 11, 0)
    ref, _ = Model(p).simulate(5, 1e-15)
    dp = DeviceProblem(p)
    states, _ = dp.simulate(5, tol=1e-13, precision=precision, keep=True)
    dp.close()
    for k, field in enumerate(("T", "V")):
        a = [r[k] for r in ref]
        b = [s[k] for s in states]
        s = report.summary(a, b)
        print(f"[psnr {precision} {field}] min {s['min_db']:.1f} dB, controls "
              f"{s['control_db']}", flush=True)
        # well above the 1e-5 noise line, as the paper's accepted solvers are
        assert s["min_db"] > s["control_db"]["1e-05"] + 40

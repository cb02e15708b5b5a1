"""Throughput of coupled RFA time steps on one MI355X: FP64 Jacobi-PCG vs FP32-inner / FP64-refined.

Workload: the 101^3-node hex cube (1,030,301 DOF, 27,270,901 nnz per matrix), coupled
potential + bioheat steps of dt = 1 s from the seeded synthetic problem.  A step is one
pass of the whole hot path: sigma(T) and colour-by-colour assembly of the potential
matrix, Dirichlet lifting, potential PCG, Joule + bioheat right-hand side, bioheat PCG
(the bioheat matrix does not depend on T and is assembled once, before timing).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 101]

Prints one JSON line.  value = coupled steps/s of the mixed-precision path when its
state stays within 1e-8 of the FP64 path's, else of the FP64 path.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TOL = 1e-13


def spmv_bytes(n: int, nnz: int, fp32: bool) -> int:
    """Algorithmic bytes of one CSR SpMV fused with p.Ap: values + column ids + row
    pointers + x read once + y written once."""
    w = 4 if fp32 else 8
    return (w + 4) * nnz + 4 * (n + 1) + 2 * w * n


def layout_bytes(stats, fp32: bool) -> int:
    """Bytes one PCG SpMV (fused with p.Ap) must move on the mesh's own slab layout: every
    stored value slot (padding included), the column data it reads (slab pointers, shared
    offset lists, 16/32-bit per-slot offsets), x read once, y written once, and the
    per-group partial sums."""
    w = 4 if fp32 else 8
    groups = (int(stats.slabs) + 7) // 8
    return (w * int(stats.value_slots) + int(stats.index_bytes) + 2 * w * int(stats.n_nodes)
            + 8 * groups)


def traffic_key(kernel: str, workload: str, nnz: int) -> str:
    """Key of a kernel's byte counters in profiles/traffic.json: the counters depend on the
    matrix the kernel ran on, not only on its name."""
    return f"{kernel} | {workload} | nnz={nnz}"


def kernel_hash() -> str:
    """Hash of the source of the row kernels (the SpMV whose traffic is quoted): the text of
    pcg.hip between its row-kernel markers, so that changes elsewhere in the file do not
    void the recorded counters."""
    with open(os.path.join(ROOT, "paper_2409_13036_amd", "csrc", "pcg.hip")) as f:
        text = f.read()
    a, b = text.find("[row-kernels-begin]"), text.find("[row-kernels-end]")
    if a < 0 or b < a:
        raise RuntimeError("pcg.hip lacks its row-kernel markers")
    return hashlib.sha256(text[a:b].encode()).hexdigest()[:16]


def spmv_kernel_name(mesh, fp32: bool) -> str:
    """rocprofv3's name of the PCG SpMV (fused with p.Ap) that this mesh launches."""
    t = "float" if fp32 else "double"
    st = mesh.stats()
    nt = "_nt" if (st.streamed_values32 if fp32 else st.streamed_values) else ""
    mb = st.launch_bound32 if fp32 else st.launch_bound
    if st.int16_columns and st.int32_column_slabs:
        return f"k_sell_wide{nt}<{t}, 1, {mb}>"
    return f"k_sell{nt}<{t}, 1, {'true' if st.int16_columns else 'false'}, {mb}>"


def copy_probe(mib: int) -> None:
    """A plain device-to-device copy of known size, launched a few times: the reference the
    HBM byte counters are scaled by (it reads and writes mib MiB per launch)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"[bench] copy probe: {mib} MiB read + {mib} MiB written per launch, 3 launches",
          file=sys.stderr, flush=True)
    del a, b


_COPY_GBS = None


def copy_ceiling() -> float:
    """Device copy bandwidth of this GPU (GB/s): a plain copy of 1 GiB (torch's copy kernel),
    read + write bytes over the mean of 10 event-timed launches after 3 untimed ones;
    measured once per process."""
    global _COPY_GBS
    if _COPY_GBS is None:
        import torch
        n = (1 << 30) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        _COPY_GBS = 2 * 4 * n / (ms * 1e6)
        del a, b
    return _COPY_GBS


def measured_traffic(kernel: str, workload: str, nnz: int):
    """HBM bytes per launch of `kernel` on this workload's matrix (nnz entries) from the
    committed rocprofv3 counter summary, if it was taken on the current kernel source (else
    None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    entry = data.get(traffic_key(kernel, workload, nnz))
    if not isinstance(entry, dict) or entry.get("kernels_sha") != kernel_hash():
        return None
    return entry.get("bytes_per_launch")


def cpu_baseline_child(n: int) -> None:
    """Time one coupled step of the CPU oracle from the initial state (run in a child
    process, 1 thread): the whole step, and inside it each PCG solve with its iterations,
    so that the cost per iteration and the cost outside the solves are known."""
    import numpy as np
    import rafem_inputs as ri
    from oracle.rafem import Model

    p = ri.config1(n=n, steps=1)
    t0 = time.perf_counter()
    m = Model(p)
    setup = time.perf_counter() - t0
    _, lift_T = bio = m.bioheat_system()
    T0, V0 = p.initial_T(), p.initial_V()
    t0 = time.perf_counter()
    T1, V1, info = m.step(T0, V0, TOL, bioheat=bio)
    step_s = time.perf_counter() - t0
    # the same step's two solves timed on their own (the oracle's own routines, same inputs)
    sig = m.sigma(T0)
    A_V, b_V = m.potential_system(sig)
    x0 = V0.copy()
    t0 = time.perf_counter()
    V1b, iV = m.solve(A_V, b_V, x0, TOL, "pcg")
    solve_V = time.perf_counter() - t0
    b_T = m.bioheat_rhs(T0, m.joule(sig, V1b), lift_T)
    t0 = time.perf_counter()
    _, iT = m.solve(bio[0], b_T, T0.copy(), TOL, "pcg")
    solve_T = time.perf_counter() - t0
    print(json.dumps({"step_s": step_s, "setup_s": setup, "V_iters": info.V.iters,
                      "T_iters": info.T.iters, "solve_V_s": solve_V, "solve_T_s": solve_T,
                      "iter_V_s": solve_V / max(1, iV.iters), "iter_T_s": solve_T / max(1, iT.iters),
                      "outside_solves_s": max(0.0, step_s - solve_V - solve_T)}), flush=True)


def cpu_baseline(n: int) -> dict:
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                          "--n", str(n)], env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                         text=True, timeout=900)
    if out.returncode != 0:
        raise RuntimeError(f"cpu baseline failed:\n{out.stderr[-2000:]}")
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": 1.0 / r["step_s"], "unit": "coupled steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"one coupled step (potential + bioheat PCG to tol {TOL:g}, "
                       f"{r['V_iters']}+{r['T_iters']} iterations) of the {n}^3 hex workload from "
                       f"its initial state, NumPy/SciPy FP64 oracle, 1 thread; mesh setup "
                       f"({r['setup_s']:.1f} s) excluded"),
            "raw": r, "host_cpus": len(os.sched_getaffinity(0)), "host_cpu_count": os.cpu_count()}


def equal_work_cpu(cpu: dict, v_iters: float, t_iters: float) -> dict:
    """The oracle's step time scaled to the iterations the device's FP64 path needs per step
    (its solves start from the predictor, the oracle's from the previous state): the part
    outside the solves plus the oracle's measured cost per iteration of each solve times
    the device's mean iteration counts.  Replaces value (the raw figure stays in raw)."""
    r = cpu["raw"]
    t = r["outside_solves_s"] + r["iter_V_s"] * v_iters + r["iter_T_s"] * t_iters
    out = dict(cpu)
    out["value"] = 1.0 / t
    out["raw_value"] = cpu["value"]
    out["sample"] = (cpu["sample"] + f"; value scaled to the device FP64 path's mean "
                     f"{v_iters:.1f}+{t_iters:.1f} iterations per step: outside the solves "
                     f"{r['outside_solves_s']:.2f} s + {1e3 * r['iter_V_s']:.1f} ms per "
                     f"potential iteration + {1e3 * r['iter_T_s']:.1f} ms per bioheat "
                     f"iteration; raw_value is the unscaled step")
    return out


def spmv_roofline(mesh, kernel: str, wl_key: str, fp32: bool, warm_us: float,
                  warm_count: int, copies: int = 0) -> dict:
    """Roofline of the PCG SpMV on this mesh's potential matrix.  achieved = the layout's own
    bytes per launch (layout_bytes) / the kernel's mean duration with a cold Infinity Cache:
    rafem_spmv_timing rotates the launches through enough copies of the values (> 1.2 GB in
    all) that none finds its matrix in the 256 MB cache; each launch is timed by events
    stamped at the kernel's own start and end.  Beside it: the same bytes over the mean
    in-solve duration (warm, measured over the PCG iterations of extra steps), the CSR
    count of the same product, and the counter bytes (FETCH_SIZE + WRITE_SIZE) when
    profiles/traffic.json holds them for this kernel, workload and matrix."""
    from paper_2409_13036_amd import _lib as R
    st = mesh.stats()
    prec = "mixed" if fp32 else "fp64"
    nbytes = layout_bytes(st, fp32)
    value_bytes = int(st.value_slots) * (4 if fp32 else 8)
    if copies <= 0:
        copies = max(4, -(-int(1.2e9) // max(1, value_bytes)))
    t_cold = R.spmv_timing(mesh, prec, copies=copies, reps=max(20, 10 * copies))
    t_one = R.spmv_timing(mesh, prec, copies=1, reps=max(20, 10 * copies))
    traffic = measured_traffic(kernel, wl_key, int(st.nnz))
    csr = spmv_bytes(int(st.n_nodes), int(st.nnz), fp32)
    print(f"[bench] SpMV {kernel} on {wl_key}: {nbytes / 1e6:.1f} MB per launch; cold "
          f"({copies} copies) {t_cold:.2f} us, one copy {t_one:.2f} us, in solves "
          f"{warm_us:.2f} us", file=sys.stderr, flush=True)
    gbs = lambda b, us: b / (us * 1e3) if us > 0 else None
    copy_gbs = copy_ceiling()
    return {"bound": "hbm", "achieved": gbs(nbytes, t_cold), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs(nbytes, t_cold) / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": kernel, "workload": wl_key, "bytes_per_launch": nbytes,
            "bytes": {"values": value_bytes, "column_data": int(st.index_bytes),
                      "x_and_y": 2 * (4 if fp32 else 8) * int(st.n_nodes),
                      "partials": 8 * ((int(st.slabs) + 7) // 8)},
            "mean_launch_us": t_cold, "cold_cache_copies": copies,
            "warm": {"mean_launch_us": warm_us, "launches_measured": warm_count,
                     "achieved": gbs(nbytes, warm_us),
                     "frac": (gbs(nbytes, warm_us) or 0.0) / HBM_PEAK_GBS,
                     "one_copy_mean_launch_us": t_one},
            "csr_equivalent": {"bytes_per_launch": csr, "achieved_cold": gbs(csr, t_cold),
                               "achieved_warm": gbs(csr, warm_us)},
            "measured_GBs_cold": gbs(traffic, t_cold) if traffic else None,
            "value_loads": ({"streamed_past_MiB": (int(st.resident_slots32 if fp32 else
                                                       st.resident_slots) * (4 if fp32 else 8)
                                                   / 1048576)}
                            if (st.streamed_values32 if fp32 else st.streamed_values)
                            else "ordinary"),
            "copy_ceiling": {"GBs": copy_gbs, "frac_of_copy": gbs(nbytes, t_cold) / copy_gbs,
                             "how": "plain device copy of 1 GiB on this GPU, read + write "
                                    "bytes over the event-timed mean of 10 launches"},
            "note": ("achieved = bytes_per_launch (the slab layout's values with padding, its "
                     "column data, x once, y once) / mean launch time with a cold Infinity "
                     "Cache; warm = the same bytes over the in-solve launches, whose matrix "
                     "can sit in the 256 MB cache; csr_equivalent = the CSR count of the same "
                     "product; traffic = FETCH_SIZE + WRITE_SIZE bytes per launch")}


def run_path(dp, precision: str, steps: int, warmup: int, profile_steps: int, **kw):
    import torch
    from paper_2409_13036_amd import _lib as R
    dp.reset()
    for _ in range(warmup):
        dp.step(TOL, precision, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, marks = [], [t0]
    for _ in range(steps):
        infos.append(dp.step(TOL, precision, **kw))
        marks.append(time.perf_counter())  # a step ends with a host poll of its last solve
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dp.step_times = [b - a for a, b in zip(marks, marks[1:])]
    T_end, V_end = dp.T.clone(), dp.V.clone()
    # measurement pass: the same kind of steps again, with every PCG SpMV bracketed by events
    R.profile_enable(dp.mesh, True)
    R.profile_read(dp.mesh, precision, reset=True)
    for _ in range(profile_steps):
        dp.step(TOL, precision, **kw)
    torch.cuda.synchronize()
    mean_us, count = R.profile_read(dp.mesh, precision, reset=True)
    R.profile_enable(dp.mesh, False)
    dp.regions = regions_pass(dp, lambda: dp.step(TOL, precision, **kw), 2)
    return elapsed, infos, (T_end, V_end), (mean_us, count)


def step_stats(times) -> dict:
    """Per-step wall times: median, mean and the half-width of the 99.7% interval of the mean
    (3 standard errors), in ms."""
    import statistics
    ms = [1e3 * t for t in times]
    mean = statistics.mean(ms)
    half = 3.0 * statistics.stdev(ms) / len(ms) ** 0.5 if len(ms) > 1 else None
    return {"median_ms": statistics.median(ms), "mean_ms": mean, "ci997_halfwidth_ms": half,
            "steps": len(ms)}


def regions_pass(dp, step, n):
    """Mean assembly / solve / check milliseconds per step over n more steps, timed by the
    library's region events (the breakdown of the paper's traced regions)."""
    from paper_2409_13036_amd import _lib as R
    R.regions_enable(dp.mesh, True)
    R.regions_read(dp.mesh, reset=True)
    for _ in range(n):
        step()
    r = R.regions_read(dp.mesh, reset=True)
    R.regions_enable(dp.mesh, False)
    return r


def adjoint_leg(args) -> dict:
    """Differentiation workload: 101^3 hex, 60 coupled steps, lesion loss, gradients with respect
    to k_e and w_e by the reverse sweep (checkpoints every 10 steps), timed; then central
    finite differences on 32 single parameters drawn from the 1% of elements with the
    largest adjoint gradients and along the two directions k and w (all entries scaled),
    forward solves at tol 1e-14.  Steps are relative to the parameter:
      k singles: 1e-6 (the stated step), 1e-5 and 1e-4.  The reference is the 1e-5 value:
        its round-off noise is a tenth of the stated step's and its truncation error is
        bounded by its spread to the 1e-4 value (truncation grows as h^2);
      w singles: 0.1 and 0.05, Richardson-extrapolated (a 1e-6 step moves the loss below
        the solves' round-off; the response is linear far below the tolerance);
      direction k: 1e-6 (and 1e-5 for its spread); direction w: 1e-3."""
    import numpy as np
    import torch
    import rafem_inputs as ri
    from paper_2409_13036_amd.adjoint import lesion_loss
    from paper_2409_13036_amd.sim import DeviceProblem

    tol = 1e-14
    p = ri.config3(n=args.n, steps=args.adj_steps)
    dp = DeviceProblem(p)
    dev = dp.dev
    k = torch.tensor(p.k_e, dtype=torch.float64, device=dev, requires_grad=True)
    w = torch.tensor(p.perf_e, dtype=torch.float64, device=dev, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = lesion_loss(dp, k, w, p.steps, checkpoint_every=10, tol=tol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gk, gw = k.grad.cpu().numpy(), w.grad.cpu().numpy()
    rows = fd_rows(dp, p, gk, gw, args.fd_params // 2, args.fd_params - args.fd_params // 2,
                   seed=0, tol=tol)
    dp.close()
    ks = [r for r in rows if r["param"].startswith("k")]
    return {"workload": f"C3 adjoint, {args.n}^3 hex, {p.steps} steps, checkpoints every 10",
            "loss": float(L.detach()), "forward_s": t1 - t0, "backward_s": t2 - t1,
            "fd_checks": len(rows),
            "fd_max_rel_err_k": max(r["rel_err"] for r in ks),
            "fd_max_rel_err_k_at_stated_step": max(r["rel_err_h1e-06"] for r in ks),
            "fd_max_noise_k_at_stated_step": max(r["noise_h1e-06"] for r in ks),
            "fd_max_truncation_k_h1e-05": max(r["trunc_h1e-05"] for r in ks),
            "fd_max_rel_err_directional": max(r["rel_err"] for r in rows
                                              if r["param"].startswith("direction")),
            "fd_max_rel_err_w": max(r["rel_err"] for r in rows if r["param"].startswith("w")),
            "fd": rows}


def adjoint_timing_leg(args) -> dict:
    """The differentiation workload's timing alone (101^3 hex, 60 coupled steps, lesion
    loss, reverse sweep with checkpoints every 10 steps, tol 1e-14), for the default run;
    `--adjoint` adds the finite-difference checks."""
    import torch
    import rafem_inputs as ri
    from paper_2409_13036_amd.adjoint import lesion_loss
    from paper_2409_13036_amd.sim import DeviceProblem

    p = ri.config3(n=args.n, steps=args.adj_steps)
    dp = DeviceProblem(p)
    k = torch.tensor(p.k_e, dtype=torch.float64, device=dp.dev, requires_grad=True)
    w = torch.tensor(p.perf_e, dtype=torch.float64, device=dp.dev, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = lesion_loss(dp, k, w, p.steps, checkpoint_every=10, tol=1e-14)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = {"workload": f"C3 adjoint, {args.n}^3 hex, {p.steps} steps, checkpoints every 10",
           "loss": float(L.detach()), "forward_s": t1 - t0, "backward_s": t2 - t1,
           "grad_k_norm": float(torch.linalg.norm(k.grad)),
           "grad_w_norm": float(torch.linalg.norm(w.grad)),
           "fd_checks": "tests/test_gpu_adjoint.py at this size; bench.py --adjoint for 32"}
    dp.close()
    print(f"[bench] adjoint: forward {t1 - t0:.2f} s, backward {t2 - t1:.2f} s",
          file=sys.stderr, flush=True)
    return out


def fd_rows(dp, p, gk, gw, n_k: int, n_w: int, seed: int = 0, tol: float = 1e-14) -> list:
    """Finite-difference checks of the adjoint gradients (gk, gw) of problem p on device
    problem dp: n_k conductivity singles and n_w perfusion singles drawn with
    default_rng(seed) from the 1% of elements with the largest |gradient|, and the two
    directions; steps as in adjoint_leg.  Returns one row per check."""
    import numpy as np
    from paper_2409_13036_amd.adjoint import fd_directional

    rng = np.random.default_rng(seed)
    top_k = np.argsort(-np.abs(gk))[: max(1, p.n_elems // 100)]
    top_w = np.argsort(-np.abs(gw))[: max(1, p.n_elems // 100)]
    picks = [("k", int(e)) for e in rng.choice(top_k, n_k, replace=False)]
    picks += [("w", int(e)) for e in rng.choice(top_w, n_w, replace=False)]

    def fd(dk, dw, h):
        return fd_directional(dp, p.k_e, p.perf_e, dk, dw, h, p.steps, tol)

    rows = []
    for which, e in picks:
        d = np.zeros(p.n_elems)
        d[e] = abs((p.k_e if which == "k" else p.perf_e)[e])
        dk, dw = (d, 0 * d) if which == "k" else (0 * d, d)
        ad = float(gk @ dk + gw @ dw)
        row = {"param": f"{which}[{e}]", "adjoint": ad}
        if which == "k":
            f6, f5, f4 = fd(dk, dw, 1e-6), fd(dk, dw, 1e-5), fd(dk, dw, 1e-4)
            row.update({"h": 1e-5, "fd_h1e-06": f6, "fd_h1e-05": f5, "fd_h1e-04": f4,
                        "noise_h1e-06": abs(f6 - f5) / abs(f5),
                        "trunc_h1e-05": abs(f5 - f4) / abs(f4) / 100.0,
                        "rel_err_h1e-06": abs(ad - f6) / abs(f6), "fd": f5})
        else:
            f1, f2 = fd(dk, dw, 1e-1), fd(dk, dw, 5e-2)
            row.update({"h": 1e-1, "fd_h": f1, "fd_h2": f2, "h_vs_h2": abs(f1 - f2) / abs(f2),
                        "fd": (4.0 * f2 - f1) / 3.0})
        row["rel_err"] = abs(ad - row["fd"]) / abs(row["fd"])
        rows.append(row)
        print(f"[adjoint] {row['param']} adjoint {ad:.10e} fd {row['fd']:.10e} "
              f"rel {row['rel_err']:.2e}"
              + (f" (h=1e-6: rel {row['rel_err_h1e-06']:.2e}, noise {row['noise_h1e-06']:.1e})"
                 if which == "k" else f" (h vs h/2 {row['h_vs_h2']:.1e})"),
              file=sys.stderr, flush=True)
    for name, dk, dw, h in (("direction k", p.k_e.copy(), 0 * p.k_e, 1e-6),
                            ("direction w", 0 * p.perf_e, p.perf_e.copy(), 1e-3)):
        ad = float(gk @ dk + gw @ dw)
        f = fd(dk, dw, h)
        row = {"param": name, "h": h, "adjoint": ad, "fd": f, "rel_err": abs(ad - f) / abs(f)}
        if name == "direction k":
            f5 = fd(dk, dw, 1e-5)
            row["noise_h1e-06"] = abs(f - f5) / abs(f5)
        rows.append(row)
        print(f"[adjoint] {name} adjoint {ad:.10e} fd {f:.10e} rel {row['rel_err']:.2e}",
              file=sys.stderr, flush=True)
    return rows


def _counter_rows(d: str, counter: str):
    """Per-dispatch values of one counter from a rocprofv3 --pmc output folder:
    [(dispatch id, kernel name, value in KiB)]."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    per = {}
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                key = (fn, r["Dispatch_Id"])
                name = r["Kernel_Name"]
                per[key] = (name, per.get(key, (name, 0.0))[1] + float(r["Counter_Value"]))
    return [(k[1], v[0], v[1]) for k, v in per.items()]


def _short_kernel(name: str) -> str:
    import re
    n = name.replace("(anonymous namespace)::", "").replace("rafem::", "").replace("void ", "")
    n = re.sub(r"HIP_vector_type<(\w+), (\d)u>", r"\1\2", n)
    return n.split("(")[0][:48]


def trace_summary(d: str) -> None:
    """Summary of a rocprofv3 --kernel-trace --stats folder: the kernel statistics table,
    the gaps between consecutive dispatches (pairs seen >= 50 times, host syncs > 200 us
    left out) and per-kernel durations without launches under 5 us (iterations enqueued
    past convergence, which exit at once)."""
    import csv
    import glob
    import statistics
    st = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if st:
        with open(st[0]) as f:
            rows = list(csv.DictReader(f))
        print(f"{'kernel':50s} {'calls':>6s} {'avg_us':>9s} {'min_us':>8s} {'total_ms':>9s} "
              f"{'pct':>6s}")
        for r in rows[:24]:
            print(f"{_short_kernel(r['Name']):50s} {int(r['Calls']):6d} "
                  f"{float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:8.2f} "
                  f"{float(r['TotalDurationNs']) / 1e6:9.2f} {float(r['Percentage']):6.2f}")
    tr = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if not tr:
        return
    with open(tr[0]) as f:
        ks = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]),
                     _short_kernel(r["Kernel_Name"])) for r in csv.DictReader(f))
    gaps, per = {}, {}
    for (s0, e0, n0), (s1, e1, n1) in zip(ks, ks[1:]):
        g = (s1 - e0) / 1e3
        if g < 200:
            gaps.setdefault((n0, n1), []).append(g)
    for s0, e0, n0 in ks:
        per.setdefault(n0, []).append((e0 - s0) / 1e3)
    print("\ngaps between consecutive kernels (us), pairs with >= 50 occurrences:")
    for (a, b), v in sorted(gaps.items(), key=lambda kv: -len(kv[1])):
        if len(v) >= 50:
            print(f"  {a[:36]:36s} -> {b[:36]:36s} n={len(v):5d} "
                  f"median={statistics.median(v):6.2f} mean={statistics.mean(v):6.2f}")
    print("\nruns of >= 10 back-to-back launches of one kernel (the autotuner's timing and "
          "the cold-cache rotation of rafem_spmv_timing), mean duration (us):")
    i = 0
    while i < len(ks):
        j = i
        while j + 1 < len(ks) and ks[j + 1][2] == ks[i][2]:
            j += 1
        if j - i + 1 >= 10:
            d = [(e - s) / 1e3 for s, e, _ in ks[i:j + 1]]
            print(f"  {ks[i][2]:48s} run of {len(d):4d} mean={statistics.mean(d):8.2f} "
                  f"median={statistics.median(d):8.2f}")
        i = j + 1
    print("\nper-kernel durations excluding launches under 5 us (early exits):")
    for n0, v in per.items():
        w = [x for x in v if x >= 5.0]
        if len(w) >= 20:
            print(f"  {n0:48s} n={len(w):5d} (of {len(v)}) median={statistics.median(w):8.2f} "
                  f"mean={statistics.mean(w):8.2f}")


def counters_summary(fetch_dir: str, write_dir: str, probe_mib: int, workload: str, nnz: int,
                     out_path: str = "") -> None:
    """HBM bytes per launch of the PCG SpMV kernels from two rocprofv3 --pmc runs of
    `bench.py --copy-probe-mib M ...` on one workload (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch).  Each counter is scaled by what it reads for the probe's plain copy of M MiB
    (the first three copy dispatches of the run: the probe runs before anything else), and a
    kernel's figure is the mean over its full launches (value >= 90% of its largest:
    launches enqueued past convergence exit at once, and in an ensemble a launch skips the
    samples that have converged).  Entries are keyed by (kernel, workload, nnz) and merged
    into profiles/traffic.json (entries of other workloads are kept); prints a summary."""
    import statistics
    path = out_path or os.path.join(ROOT, "profiles", "traffic.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        out = {k: v for k, v in old.items()
               if isinstance(v, dict) and v.get("workload") not in (None, workload)}
    lines = []
    factors = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(d, counter)
        copies = [v for i, n, v in sorted(rows, key=lambda t: int(t[0])) if "copy" in n.lower()]
        if len(copies) < 3:
            raise SystemExit(f"{counter}: the copy probe's three dispatches were not found")
        probe = copies[:3]
        factor = statistics.mean(probe) / (probe_mib * 1024.0)
        factors[counter] = factor
        lines.append(f"{counter}: copy probe {len(probe)} dispatches, mean "
                     f"{statistics.mean(probe):.0f} KiB for {probe_mib * 1024} KiB moved "
                     f"-> factor {factor:.4f}")
        by = {}
        for _, n, v in rows:
            short = _short_kernel(n)
            if short.startswith("k_sell") or short.startswith("k_csr"):
                by.setdefault(short, []).append(v)
        for name, vals in sorted(by.items()):
            busy = [v for v in vals if v >= 0.9 * max(vals)]
            kib = statistics.mean(busy)
            e = out.setdefault(traffic_key(name, workload, nnz),
                               {"kernel": name, "workload": workload, "nnz": nnz,
                                "kernels_sha": kernel_hash(), "probe_mib": probe_mib})
            e[counter.lower() + "_copy_factor"] = factor
            e[counter.lower() + "_bytes"] = kib * 1024.0 / factor
            e[counter.lower() + "_launches"] = len(busy)
            lines.append(f"  {name:34s} {len(busy):5d} of {len(vals):5d} launches, mean "
                         f"{kib:10.0f} KiB -> {kib * 1024.0 / factor / 1e6:8.1f} MB scaled")
    for name, e in out.items():
        if isinstance(e, dict) and "fetch_size_bytes" in e and "write_size_bytes" in e:
            e["bytes_per_launch"] = e["fetch_size_bytes"] + e["write_size_bytes"]
            lines.append(f"{name}: HBM bytes per launch {e['bytes_per_launch'] / 1e6:.1f} MB")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("\n".join(lines))


def batch_leg(args) -> dict:
    """Ensemble workload: 64 hex samples of side n ~ U{41..81} nodes with per-sample lognormal
    k, sigma0 and w, advanced together through one batch handle (graph-captured iteration
    chunks, autotuned SpMV slab shape, device-driven solves: one host poll per solve once
    two alike solves have left their counts) for 30 coupled steps, FP64 and mixed, then the
    same host-driven.  Reports sample-steps/s and, per sample, the relative error of the
    mixed state against the FP64 state after the last step."""
    import numpy as np
    import torch
    import rafem_inputs as ri
    from paper_2409_13036_amd import _lib as R
    from paper_2409_13036_amd.sim import BatchProblem

    probs = ri.config4(samples=args.batch_samples, steps=args.batch_steps)
    t0 = time.perf_counter()
    bp = BatchProblem(probs)
    if args.host_driven:
        bp.mesh.set_device_driven(False)
    bp.extrapolate = not args.no_extrapolate
    bp.extrapolate_order = args.extrapolate_order
    setup = time.perf_counter() - t0
    S = len(probs)
    nnz = sum((3 * p.n - 2) ** 3 for p in probs)
    out = {"workload": f"C4 ensemble, {S} hex samples n~U{{41..81}}, {args.batch_steps} coupled "
                       f"steps, one batch handle",
           "samples": S, "n_nodes_total": int(sum(p.n_nodes for p in probs)), "nnz_total": nnz,
           "handle_rows": int(bp.mesh.n_nodes), "handle_nnz": int(bp.mesh.nnz), "setup_s": setup}
    finals = {}

    def timed(precision):
        bp.reset()
        bp.step(TOL, precision)  # warm-up: bioheat assembly, autotuning, graph capture, counts
        bp.reset()
        st0 = bp.mesh.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            bp.step(TOL, precision)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = bp.mesh.stats()
        dd = {"device_driven": bool(st.device_driven),
              "accepted_solves": int(st.device_driven_solves - st0.device_driven_solves),
              "redone_solves": int(st.device_driven_redone - st0.device_driven_redone)}
        return el, dd

    for precision in ("fp64", "mixed"):
        el, dd = timed(precision)
        finals[precision] = [bp.sample(q) for q in range(S)]
        its = [bp.mesh.sample_info(q) for q in range(S)]
        R.profile_enable(bp.mesh, True)
        R.profile_read(bp.mesh, precision, reset=True)
        bp.step(TOL, precision)
        torch.cuda.synchronize()
        mean_us, count = R.profile_read(bp.mesh, precision, reset=True)
        R.profile_enable(bp.mesh, False)
        out[precision] = {
            "sample_steps_per_s": S * args.batch_steps / el, "elapsed_s": el,
            "V_iters_last_step_min_max": [min(i["V"]["iters"] for i in its),
                                          max(i["V"]["iters"] for i in its)],
            "T_iters_last_step_min_max": [min(i["T"]["iters"] for i in its),
                                          max(i["T"]["iters"] for i in its)],
            "spmv_us_mean": mean_us, "spmv_launches": count, "device_driven": dd}
        print(f"[bench] batch {precision}: {S * args.batch_steps / el:.1f} sample-steps/s "
              f"({el:.2f} s), spmv {mean_us:.1f} us x {count}, {dd}", file=sys.stderr, flush=True)
    # the other way of driving the solves, for comparison (same iterates)
    dd_default = bool(bp.mesh.stats().device_driven)
    bp.mesh.set_device_driven(not dd_default)
    for precision in ("fp64", "mixed"):
        el, dd = timed(precision)
        key = "host_driven" if dd_default else "device_driven"
        out[precision][key] = {"sample_steps_per_s": S * args.batch_steps / el, "elapsed_s": el,
                               **dd}
        print(f"[bench] batch {precision} ({key}): {S * args.batch_steps / el:.1f} "
              f"sample-steps/s, {dd}", file=sys.stderr, flush=True)
    bp.mesh.set_device_driven(dd_default)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    eT = [rel(m[0], f[0]) for m, f in zip(finals["mixed"], finals["fp64"])]
    eV = [rel(m[1], f[1]) for m, f in zip(finals["mixed"], finals["fp64"])]
    out["mixed_rel_err_vs_fp64_max"] = {"T": max(eT), "V": max(eV)}
    mixed_ok = max(eT) <= 1e-8 and max(eV) <= 1e-8
    out["path"] = "mixed" if mixed_ok else "fp64"
    out["sample_steps_per_s"] = out[out["path"]]["sample_steps_per_s"]
    # the full-ensemble product (every sample active): its values (1.8 GB FP32, 3.5 GB FP64)
    # exceed the 256 MB Infinity Cache by themselves, so two rotated copies suffice; the
    # in-solve mean ("warm") also averages launches in which converged samples are skipped
    for precision in ("mixed", "fp64"):
        fp32 = precision == "mixed"
        out[f"roofline_{'fp32' if fp32 else 'fp64'}"] = spmv_roofline(
            bp.mesh, spmv_kernel_name(bp.mesh, fp32), "C4 ensemble", fp32,
            out[precision]["spmv_us_mean"], out[precision]["spmv_launches"], copies=2)
    bp.close()
    return out


def pc_leg(dp, args) -> dict:
    """Predictor-corrector workload on the same mesh: the application's outer loop
    (extrapolated predictor, Picard corrector on sigma(T) until the relative change of T is
    below eps, at most 50 corrector iterations, halving on rejection) from rest over
    t_total seconds with nominal step dt0, FP64 and mixed.  Reports accepted steps/s,
    simulated seconds per wall second, corrector and solver iterations, and the mixed
    final state against the FP64 one."""
    import numpy as np
    import torch
    out = {"workload": f"predictor-corrector run, {args.pc_t:g} s in steps of {args.pc_dt0:g} s, "
                       f"eps {args.pc_eps:g}, at most 50 corrector iterations per step",
           "t_total_s": args.pc_t, "dt0_s": args.pc_dt0, "eps": args.pc_eps}
    finals = {}
    for precision in ("fp64", "mixed"):
        dp.reset()
        dp.step_pc(args.pc_dt0, corr_tol=args.pc_eps, tol=TOL, precision=precision)  # warm-up
        dp.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = dp.simulate_pc(args.pc_t, args.pc_dt0, corr_tol=args.pc_eps, max_iters=50, tol=TOL,
                             precision=precision)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        finals[precision] = (dp.T.clone(), dp.V.clone())
        reg = regions_pass(dp, lambda: dp.step_pc(args.pc_dt0, corr_tol=args.pc_eps, tol=TOL,
                                                  precision=precision), 1)
        its = [r["iters"] for r in rec]
        out[precision] = {
            "accepted_steps": len(rec), "rejected": sum(r["rejected_before"] for r in rec),
            "elapsed_s": el, "accepted_steps_per_s": len(rec) / el,
            "simulated_s_per_s": args.pc_t / el,
            "corrector_iters_mean": float(np.mean(its)), "corrector_iters_max": max(its),
            "corrector_iters_per_s": sum(its) / el,
            "solver_iters_total": int(sum(r["solver_iters"] for r in rec)),
            "regions_ms_one_step": reg}
        print(f"[bench] predictor-corrector {precision}: {len(rec)} steps in {el:.2f} s, "
              f"corrector iterations {its}", file=sys.stderr, flush=True)
    (Tm, Vm), (T64, V64) = finals["mixed"], finals["fp64"]
    out["mixed_rel_err_vs_fp64"] = {
        "T": float(torch.linalg.norm(Tm - T64) / torch.linalg.norm(T64)),
        "V": float(torch.linalg.norm(Vm - V64) / torch.linalg.norm(V64))}
    return out


def arnoldi_bytes(n: int, nnz: int, m: int, fp32: bool = False) -> float:
    """Algorithmic HBM bytes of one Arnoldi step of GMRES(m), averaged over a cycle: the block
    SpMV (per node pair 4 values + an int32 column, row pointers, x and y per node) and the
    three CGS2 passes over the k = j + 1 basis vectors (dots: k + 1 vectors; update with the
    second dots: k + 2; normalisation with M^-1: k + 5 vector-sized streams), k averaged
    over j = 0..m-1.  Values and vectors are FP32 in the mixed Arnoldi process."""
    vb = 4.0 if fp32 else 8.0
    spmv = (4 * vb + 4.0) * nnz + 4.0 * (n + 1) + 4 * vb * n
    k_mean = (m + 1) / 2.0
    return spmv + (3.0 * k_mean + 8.0) * 2 * vb * n


def mono_leg(dp, args) -> dict:
    """Monolithic corrector on the same mesh: GMRES(m) solves of one Newton system (the
    Jacobian at the state after one staggered step, T^n = the initial state) for each m of
    the sweep -- time, iterations, cycles, slowdown against the best m, and stagnating
    cycles (residual reduced by less than 2x over a cycle); then the predictor-corrector run
    of the Picard leg with the Newton corrector at the best m."""
    import numpy as np
    import torch
    from paper_2409_13036_amd import _lib as R
    p = dp.p
    N, nnz = dp.mesh.n_nodes, dp.mesh.nnz
    dp.reset()
    dp.step(TOL)
    T1, V1 = dp.T.clone(), dp.V.clone()
    T0 = torch.as_tensor(p.initial_T(), dtype=torch.float64, device=dp.dev)
    dt_save = dp.phys.dt
    dp.phys.dt = args.pc_dt0
    sweep = []
    hist_len = 20000
    # warm-up (short solves that allocate the workspace for the largest m, both precisions)
    for precision in ("fp64", "mixed"):
        R.mono_solve(dp.mesh, dp.phys, dp.k_e, dp.perf_e, dp.sigma0_e, T0, T1, V1,
                     m=max(args.mono_m), tol=1e-10, max_iters=50, precision=precision,
                     check=False)
    for precision in ("fp64", "mixed"):
        for mm in args.mono_m:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info, hist = R.mono_solve(dp.mesh, dp.phys, dp.k_e, dp.perf_e, dp.sigma0_e, T0, T1,
                                         V1, m=mm, tol=1e-10, precision=precision,
                                         hist_len=hist_len, check=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            h = hist.cpu().numpy()[:min(info["iters"], hist_len)]
            ends = [min(c * mm, len(h)) - 1 for c in range(1, info["cycles"] + 1)]
            starts = [1.0] + [h[e] for e in ends[:-1]]
            stagn = sum(1 for s0, e in zip(starts, ends) if e >= 0 and h[e] > 0.5 * s0)
            per_step = arnoldi_bytes(N, nnz, mm, precision == "mixed")
            row = {"precision": precision, "m": mm, "status": info["status"],
                   "iters": info["iters"], "cycles": info["cycles"], "seconds": el,
                   "relres_true": info["relres_true"],
                   "us_per_arnoldi_step": el / max(1, info["iters"]) * 1e6,
                   "arnoldi_GBs": per_step * info["iters"] / el / 1e9,
                   "stagnating_cycles": stagn}
            sweep.append(row)
            print(f"[bench] GMRES({mm}) {precision}: {info['iters']} iterations, "
                  f"{info['cycles']} cycles, {el:.3f} s, {row['us_per_arnoldi_step']:.0f} us/step, "
                  f"{row['arnoldi_GBs']:.0f} GB/s, stagnating cycles {stagn}",
                  file=sys.stderr, flush=True)
    ok = [r for r in sweep if r["status"] == 0 and r["relres_true"] <= 1e-10]
    best = min(ok, key=lambda r: r["seconds"]) if ok else None
    for r in sweep:
        same = [q for q in ok if q["precision"] == r["precision"]]
        r["slowdown_vs_best_of_precision"] = (r["seconds"] / min(q["seconds"] for q in same)
                                              if same else None)
    dp.phys.dt = dt_save
    out = {"workload": f"monolithic (T, V) Newton-GMRES corrector, {N}-node hex mesh, "
                       f"2N = {2 * N} unknowns, {4 * nnz} nonzeros",
           "unknowns": 2 * N, "nonzeros": 4 * nnz, "gmres_tol": 1e-10, "m_sweep": sweep,
           "best": {"m": best["m"], "precision": best["precision"]} if best else None}
    if best:
        r = best
        out["roofline"] = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                           "achieved": r["arnoldi_GBs"], "frac": r["arnoldi_GBs"] / HBM_PEAK_GBS,
                           "bytes_per_arnoldi_step": arnoldi_bytes(N, nnz, r["m"],
                                                                   r["precision"] == "mixed"),
                           "note": "whole Arnoldi steps of the best (m, precision) (block SpMV "
                                   "+ CGS2), cycle ends and restarts included in the time"}
        gp = r["precision"]
        dp.reset()
        dp.step_mono(args.pc_dt0, corr_tol=args.pc_eps, m=r["m"], gmres_precision=gp)  # warm-up
        dp.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = dp.simulate_pc(args.pc_t, args.pc_dt0, corr_tol=args.pc_eps, max_iters=50,
                             corrector="newton", m=r["m"], gmres_tol=1e-10, gmres_precision=gp)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        its = [x["iters"] for x in rec]
        reg = regions_pass(dp, lambda: dp.step_mono(args.pc_dt0, corr_tol=args.pc_eps, m=r["m"],
                                                    gmres_precision=gp), 1)
        out["predictor_corrector"] = {
            "regions_ms_one_step": reg,
            "t_total_s": args.pc_t, "dt0_s": args.pc_dt0, "eps": args.pc_eps,
            "accepted_steps": len(rec), "rejected": sum(x["rejected_before"] for x in rec),
            "elapsed_s": el, "accepted_steps_per_s": len(rec) / el,
            "newton_iters": its, "gmres_iters_total": int(sum(x["solver_iters"] for x in rec))}
        print(f"[bench] monolithic predictor-corrector: {len(rec)} steps in {el:.2f} s, Newton "
              f"iterations {its}", file=sys.stderr, flush=True)
    return out


def psnr_leg(dp, args) -> dict:
    """PSNR per step (the paper's result-quality metric) of GPU runs against the FP64 run at
    tol 1e-13 from the same initial state: the mixed path, and FP64 at tol 1e-6 (the
    paper's low-tolerance solver setting); min and median over the steps with the 1e-5 and
    1e-12 control lines."""
    from paper_2409_13036_amd import report

    def run(precision, tol):
        dp.reset()
        T, V = [], []
        for _ in range(args.psnr_steps):
            dp.step(tol, precision)
            T.append(dp.T.cpu().numpy())
            V.append(dp.V.cpu().numpy())
        return T, V

    refT, refV = run("fp64", TOL)
    out = {"workload": f"{args.psnr_steps} coupled steps from the initial state; reference: "
                       f"FP64 at tol {TOL:g}"}
    for label, precision, tol in (("mixed", "mixed", TOL), ("fp64_tol_1e-6", "fp64", 1e-6)):
        T, V = run(precision, tol)
        out[label] = {"T": report.summary(refT, T), "V": report.summary(refV, V)}
        print(f"[bench] PSNR {label}: T min {out[label]['T']['min_db']:.1f} dB, V min "
              f"{out[label]['V']['min_db']:.1f} dB (controls {out[label]['T']['control_db']})",
              file=sys.stderr, flush=True)
    return out


def liver_leg(args) -> dict:
    """Unstructured liver-like tet meshes (Delaunay, two needle electrodes): the stand-ins for
    the paper's meshes A and B (about 3.5k and 8.4k nodes) in RCM order, then one of --liver-nodes nodes in the delivered (shuffled) order, in
    RCM order, and in RCM order with degree-sorted windows -- coupled steps/s (FP64 and
    mixed, extrapolated starting points unless --no-extrapolate) and the PCG SpMV's launch
    time and CSR-count bandwidth."""
    import numpy as np
    import torch
    import rafem_inputs as ri
    from paper_2409_13036_amd.sim import DeviceProblem, rcm_reordered

    def bandwidth(conn, order):
        pos = np.argsort(order) if order is not None else np.arange(conn.max() + 1)
        c = pos[conn]
        return int((c.max(axis=1) - c.min(axis=1)).max())

    inner_tol = args.inner_tol if args.inner_tol is not None else 1e-3

    def measure(prob, steps, warmup, label, roofline=False):
        dp = DeviceProblem(prob)
        dp.extrapolate = not args.no_extrapolate
        dp.extrapolate_order = args.extrapolate_order
        st = dp.mesh.stats()
        N, nnz = dp.mesh.n_nodes, dp.mesh.nnz
        row = {"n_nodes": N, "n_elems": dp.mesh.n_elems, "nnz": nnz, "colours": st.n_colours,
               "slabs": int(st.slabs), "int16_columns": int(st.int16_columns),
               "int32_column_slabs": int(st.int32_column_slabs),
               "mixed_inner_tol": inner_tol}
        for precision in ("fp64", "mixed"):
            kw = {"inner_tol": inner_tol} if precision == "mixed" else {}
            el, infos, _, (us, cnt) = run_path(dp, precision, steps, warmup, 1, **kw)
            fp32 = precision == "mixed"
            row[precision] = {
                "steps_per_s": steps / el,
                "V_iters": float(np.mean([i["V"]["iters"] for i in infos])),
                "spmv_us": us, "spmv_GBs": spmv_bytes(N, nnz, fp32) / (us * 1e3) if us else None}
            if roofline:
                row[precision]["roofline"] = spmv_roofline(
                    dp.mesh, spmv_kernel_name(dp.mesh, fp32), f"liver {N} {label}", fp32, us, cnt)
            print(f"[bench] liver {label} {precision}: {steps / el:.2f} steps/s, spmv {us:.1f} us",
                  file=sys.stderr, flush=True)
        dp.close()
        return row

    out = {"workload": "unstructured liver-like tet meshes, bipolar needle electrodes"}
    for name, make in (("mesh_A", ri.liver_mesh_a), ("mesh_B", ri.liver_mesh_b)):
        q, _ = rcm_reordered(make())
        out[name] = measure(q, args.liver_steps, 3, name)
    t0 = time.perf_counter()
    p = ri.make_liver(args.liver_nodes, 0)
    out["large_mesh_generation_s"] = time.perf_counter() - t0
    q, order = rcm_reordered(p)
    qs, order_s = rcm_reordered(p, window=512)
    for label, prob, o in (("shuffled", p, None), ("rcm", q, order),
                           ("rcm_degree_sorted", qs, order_s)):
        row = measure(prob, args.liver_steps, 2, f"{args.liver_nodes} {label}",
                      roofline=label == "rcm")
        row["bandwidth"] = bandwidth(p.conn, o)
        out[f"large_{label}"] = row
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=101)
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="relative tolerance of each FP32 inner solve (default: 1e-4 for the "
                         "worse-conditioned c2 potential system, else the library's 3e-5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-child", action="store_true")
    ap.add_argument("--adjoint", action="store_true",
                    help="run only the differentiation workload (timing + finite-difference check)")
    ap.add_argument("--adj-steps", type=int, default=60)
    ap.add_argument("--no-adjoint-timing", action="store_true",
                    help="leave the differentiation timing out of the default run")
    ap.add_argument("--fd-params", type=int, default=32)
    ap.add_argument("--workload", choices=["c1", "c2"], default="c1",
                    help="c1: 101^3 hex (default); c2: 161^3-node jittered Kuhn tets")
    ap.add_argument("--extrapolate-order", type=int, default=2, choices=(1, 2, 3, 4),
                    help="order of the predictor of the solves' starting points")
    ap.add_argument("--no-extrapolate", action="store_true",
                    help="start every solve from the previous state instead of the linear "
                         "extrapolation of the last two")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the mixed refinement's inner tolerance and restart mode with "
                         "paper_2409_13036_amd.tune (cached on disk) before timing")
    ap.add_argument("--restart-inner", action="store_true",
                    help="mixed precision: plain restarted refinement (a new inner Krylov space "
                         "per refinement) instead of the default reliable updates")
    ap.add_argument("--no-batch", action="store_true", help="skip the ensemble leg")
    ap.add_argument("--no-pc", action="store_true", help="skip the predictor-corrector leg")
    ap.add_argument("--no-mono", action="store_true", help="skip the monolithic GMRES leg")
    ap.add_argument("--no-psnr", action="store_true", help="skip the PSNR leg")
    ap.add_argument("--psnr-steps", type=int, default=20)
    ap.add_argument("--liver", action="store_true",
                    help="run only the unstructured liver-mesh leg (meshes A, B and a large one)")
    ap.add_argument("--liver-nodes", type=int, default=400000)
    ap.add_argument("--liver-steps", type=int, default=10)
    ap.add_argument("--mono-only", action="store_true",
                    help="run only the monolithic GMRES leg (on the c1 mesh)")
    ap.add_argument("--mono-m", type=int, nargs="+", default=[10, 20, 30, 50, 100],
                    help="restart lengths of the GMRES(m) sweep")
    ap.add_argument("--pc-t", type=float, default=10.0, help="predictor-corrector: total time (s)")
    ap.add_argument("--pc-dt0", type=float, default=2.0, help="predictor-corrector: nominal step (s)")
    ap.add_argument("--pc-eps", type=float, default=1e-9,
                    help="predictor-corrector: relative change of T that ends a corrector")
    ap.add_argument("--batch-only", action="store_true", help="run only the ensemble leg")
    ap.add_argument("--host-driven", action="store_true",
                    help="ensemble leg: time the host-driven solves first (host polls inside each "
                         "solve) and the device-driven default second")
    ap.add_argument("--batch-samples", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=30)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first launch a plain copy of this many MiB (byte-counter reference)")
    ap.add_argument("--counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of a "
                         "bench run with --copy-probe-mib into profiles/traffic.json")
    ap.add_argument("--traffic-workload", default="",
                    help="with --counters: the workload key of the profiled run (C1 hex101, "
                         "C2 tet161, C4 ensemble)")
    ap.add_argument("--traffic-nnz", type=int, default=0,
                    help="with --counters: nonzeros of the profiled run's matrix")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="summarise a rocprofv3 --kernel-trace --stats output folder")
    args = ap.parse_args()
    if args.summarize_trace:
        trace_summary(args.summarize_trace)
        return
    if args.counters:
        if not args.traffic_workload or args.traffic_nnz <= 0:
            raise SystemExit("--counters needs --traffic-workload and --traffic-nnz")
        counters_summary(args.counters[0], args.counters[1], args.copy_probe_mib or 1024,
                         args.traffic_workload, args.traffic_nnz)
        return
    if args.cpu_baseline_child:
        cpu_baseline_child(args.n)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the solve is not sharded across GPUs); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    if args.adjoint:
        print(json.dumps(adjoint_leg(args)), flush=True)
        return
    if args.batch_only:
        if args.copy_probe_mib > 0:
            copy_probe(args.copy_probe_mib)
        print(json.dumps(batch_leg(args)), flush=True)
        return
    if args.liver:
        print(json.dumps(liver_leg(args)), flush=True)
        return
    if args.mono_only:
        import rafem_inputs as ri
        from paper_2409_13036_amd.sim import DeviceProblem
        dp = DeviceProblem(ri.config1(n=args.n, steps=1))
        print(json.dumps(mono_leg(dp, args)), flush=True)
        dp.close()
        return

    # CPU oracle first, before this process touches the GPU
    cpu = None if (args.no_cpu_baseline or args.workload != "c1") else cpu_baseline(args.n)
    print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)

    import numpy as np
    import torch
    import rafem_inputs as ri
    from paper_2409_13036_amd import _lib as R
    from paper_2409_13036_amd.sim import DeviceProblem

    if args.copy_probe_mib > 0:
        copy_probe(args.copy_probe_mib)
    if args.workload == "c2":
        n = 161 if args.n == 101 else args.n
        p = ri.config2(n=n, steps=args.steps)
        workload = f"C2 coupled RFA step, {n}^3-node jittered Kuhn-tet mesh"
    else:
        n = args.n
        p = ri.config1(n=n, steps=args.steps)
        workload = f"C1 coupled RFA step, {n}^3-node hex cube"
    dp = DeviceProblem(p)
    dp.extrapolate = not args.no_extrapolate
    dp.extrapolate_order = args.extrapolate_order
    N, nnz = dp.mesh.n_nodes, dp.mesh.nnz
    mesh_stats = dp.mesh.stats()
    tuned = None
    if args.autotune:
        from paper_2409_13036_amd.tune import tune_mixed
        tuned = tune_mixed(dp, tol=TOL)
        args.inner_tol = tuned["inner_tol"]
        args.restart_inner = bool(tuned["restart_inner"])
        print(f"[bench] autotune: {tuned}", file=sys.stderr, flush=True)
    res = {}
    for precision in ("fp64", "mixed"):
        inner_tol = args.inner_tol
        if inner_tol is None:
            inner_tol = 1e-4 if args.workload == "c2" else 0.0
        kw = ({"inner_tol": inner_tol, "restart_inner": int(args.restart_inner)}
              if precision == "mixed" else {})
        el, infos, state, (mean_us, count) = run_path(dp, precision, args.steps, args.warmup,
                                                      args.profile_steps, **kw)
        it_v = float(np.mean([i["V"]["iters"] for i in infos]))
        it_t = float(np.mean([i["T"]["iters"] for i in infos]))
        res[precision] = {"elapsed": el, "state": state, "spmv_us": mean_us, "spmv_count": count,
                          "regions": dp.regions, "step_ms": step_stats(dp.step_times),
                          "V_iters": it_v, "T_iters": it_t,
                          "V_outer": float(np.mean([i["V"]["outer"] for i in infos])),
                          "relres_true_max": max(max(i["V"]["relres_true"], i["T"]["relres_true"])
                                                 for i in infos)}
        print(f"[bench] {precision}: {args.steps / el:.2f} steps/s, V iters {it_v:.1f}, "
              f"T iters {it_t:.1f}, spmv {mean_us:.1f} us x {count}", file=sys.stderr, flush=True)
    T64, V64 = res["fp64"]["state"]
    Tm, Vm = res["mixed"]["state"]
    errT = float(torch.linalg.norm(Tm - T64) / torch.linalg.norm(T64))
    errV = float(torch.linalg.norm(Vm - V64) / torch.linalg.norm(V64))
    mixed_ok = errT <= 1e-8 and errV <= 1e-8
    head = "mixed" if mixed_ok else "fp64"
    r = res[head]
    sps = args.steps / r["elapsed"]
    fp32 = head == "mixed"
    kernel = spmv_kernel_name(dp.mesh, fp32)
    wl_key = f"C2 tet{n}" if args.workload == "c2" else f"C1 hex{n}"
    roof = spmv_roofline(dp.mesh, kernel, wl_key, fp32, r["spmv_us"], r["spmv_count"])
    line = {
        "metric": "coupled time-step solves/s at 1M DOF (101^3 hex), FP64 vs mixed at 1e-8 rel err; SpMV HBM GB/s",
        "value": sps, "unit": "coupled steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 / sps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-inner/f64-refined" if fp32 else "f64", "data": "synthetic",
        "config": {"workload": workload, "n_nodes": N,
                   "nnz": nnz, "dt_s": p.dt, "tol": TOL, "path": head,
                   "slabs": int(mesh_stats.slabs),
                   "shared_offset_slabs": int(mesh_stats.shared_offset_slabs),
                   "predictor_order": (None if args.no_extrapolate
                                       else args.extrapolate_order),
                   "inner_tol": inner_tol if inner_tol else "library default (3e-5)",
                   "refinement": "restarted" if args.restart_inner else "reliable updates",
                   "autotune": tuned},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64": {"steps_per_s": args.steps / res["fp64"]["elapsed"],
                 "V_iters": res["fp64"]["V_iters"], "T_iters": res["fp64"]["T_iters"],
                 "spmv_us": res["fp64"]["spmv_us"],
                 "spmv_GBs": spmv_bytes(N, nnz, False) / (res["fp64"]["spmv_us"] * 1e-6) / 1e9
                 if res["fp64"]["spmv_us"] > 0 else None,
                 "relres_true_max": res["fp64"]["relres_true_max"],
                 "step_ms": res["fp64"]["step_ms"],
                 "regions_ms_per_step": res["fp64"]["regions"]},
        "mixed": {"steps_per_s": args.steps / res["mixed"]["elapsed"],
                  "V_inner_iters": res["mixed"]["V_iters"], "V_outer": res["mixed"]["V_outer"],
                  "T_inner_iters": res["mixed"]["T_iters"], "spmv_us": res["mixed"]["spmv_us"],
                  "spmv_GBs": spmv_bytes(N, nnz, True) / (res["mixed"]["spmv_us"] * 1e-6) / 1e9
                  if res["mixed"]["spmv_us"] > 0 else None,
                  "relres_true_max": res["mixed"]["relres_true_max"],
                  "rel_err_vs_fp64": {"T": errT, "V": errV},
                  "step_ms": res["mixed"]["step_ms"],
                  "regions_ms_per_step": res["mixed"]["regions"]},
    }
    if cpu:
        line["cpu_baseline"] = equal_work_cpu(cpu, res["fp64"]["V_iters"], res["fp64"]["T_iters"])
        line["speedup_vs_cpu_oracle"] = sps / line["cpu_baseline"]["value"]
    if not args.no_pc:
        line["predictor_corrector"] = pc_leg(dp, args)
    if not args.no_psnr:
        line["psnr"] = psnr_leg(dp, args)
    if not args.no_mono:
        line["monolithic"] = mono_leg(dp, args)
    dp.close()
    del dp
    if not args.no_adjoint_timing and args.workload == "c1":
        line["adjoint"] = adjoint_timing_leg(args)
    if not args.no_batch and args.workload == "c1":
        line["batch"] = batch_leg(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

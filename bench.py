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


def kernel_hash() -> str:
    """Hash of the source of the PCG kernels (the SpMV whose traffic is quoted)."""
    with open(os.path.join(ROOT, "paper_2409_13036_amd", "csrc", "pcg.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def spmv_kernel_name(mesh, fp32: bool) -> str:
    """rocprofv3's name of the PCG SpMV (fused with p.Ap) that this mesh launches."""
    t = "float" if fp32 else "double"
    return f"k_sell<{t}, 1, {'true' if mesh.stats().int16_columns else 'false'}>"


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


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    entry = data.get(kernel)
    if not entry or entry.get("kernels_sha") != kernel_hash():
        return None
    return entry.get("bytes_per_launch")


def cpu_baseline_child(n: int) -> None:
    """Time one coupled step of the CPU oracle (run in a child process, 1 thread)."""
    import numpy as np
    import rafem_inputs as ri
    from oracle.rafem import Model

    p = ri.config1(n=n, steps=1)
    t0 = time.perf_counter()
    m = Model(p)
    setup = time.perf_counter() - t0
    bio = m.bioheat_system()
    t0 = time.perf_counter()
    T, V, info = m.step(p.initial_T(), p.initial_V(), TOL, bioheat=bio)
    dt = time.perf_counter() - t0
    print(json.dumps({"step_s": dt, "setup_s": setup, "V_iters": info.V.iters,
                      "T_iters": info.T.iters}), flush=True)


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
            "host_cpus": len(os.sched_getaffinity(0))}


def run_path(dp, precision: str, steps: int, warmup: int, profile_steps: int, **kw):
    import torch
    from paper_2409_13036_amd import _lib as R
    dp.reset()
    for _ in range(warmup):
        dp.step(TOL, precision, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        infos.append(dp.step(TOL, precision, **kw))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    T_end, V_end = dp.T.clone(), dp.V.clone()
    # measurement pass: the same kind of steps again, with every PCG SpMV bracketed by events
    R.profile_enable(dp.mesh, True)
    R.profile_read(dp.mesh, precision, reset=True)
    for _ in range(profile_steps):
        dp.step(TOL, precision, **kw)
    torch.cuda.synchronize()
    mean_us, count = R.profile_read(dp.mesh, precision, reset=True)
    R.profile_enable(dp.mesh, False)
    return elapsed, infos, (T_end, V_end), (mean_us, count)


def adjoint_leg(args) -> dict:
    """Differentiation workload: 101^3 hex, 60 coupled steps, lesion loss, gradients with respect
    to k_e and w_e by the reverse sweep (checkpoints every 10 steps), timed; then central
    finite differences (relative step 1e-6) on 32 single parameters drawn from the 1% of
    elements with the largest adjoint gradients (16 k_e, 16 w_e) and along the two directions
    k and w (all entries scaled), forward solves at tol 1e-14."""
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
    rng = np.random.default_rng(0)
    # single parameters where the sensitivity is large: the 1% largest |dL/dk_e| and |dL/dw_e|
    top_k = np.argsort(-np.abs(gk))[: p.n_elems // 100]
    top_w = np.argsort(-np.abs(gw))[: p.n_elems // 100]
    picks = [("k", int(e)) for e in rng.choice(top_k, args.fd_params // 2, replace=False)]
    picks += [("w", int(e)) for e in rng.choice(top_w, args.fd_params - args.fd_params // 2,
                                                 replace=False)]

    def final_T(kk, ww):
        dp.set_params(torch.as_tensor(kk, device=dev), torch.as_tensor(ww, device=dev))
        dp.reset()
        for _ in range(p.steps):
            dp.step(tol)
        return dp.T.cpu().numpy()

    ids, tgt = p.loss_ids, p.T_target

    def fd_along(dk, dw, h=1e-6):
        Tp = final_T(p.k_e + h * dk, p.perf_e + h * dw)
        Tm = final_T(p.k_e - h * dk, p.perf_e - h * dw)
        a, b = Tp[ids], Tm[ids]
        return float(np.sum((a - b) * (a + b - 2 * tgt))) / (2 * h)

    rows = []
    cases = []
    for which, e in picks:
        d = np.zeros(p.n_elems)
        d[e] = abs((p.k_e if which == "k" else p.perf_e)[e])
        cases.append((f"{which}[{e}]", d if which == "k" else 0 * d, d if which == "w" else 0 * d,
                      1e-6))
    cases.append(("direction k", p.k_e.copy(), 0 * p.k_e, 1e-6))
    # perfusion moves T by ~1e-9 K at a 1e-6 step (FP64 round-off floor): 1e-3 in its direction
    cases.append(("direction w", 0 * p.perf_e, p.perf_e.copy(), 1e-3))
    for name, dk, dw, h in cases:
        fd = fd_along(dk, dw, h)
        ad = float(gk @ dk + gw @ dw)
        rows.append({"param": name, "h": h, "adjoint": ad, "fd": fd,
                     "rel_err": abs(ad - fd) / abs(fd)})
        print(f"[adjoint] {name} adjoint {ad:.10e} fd {fd:.10e} rel {rows[-1]['rel_err']:.2e}",
              file=sys.stderr, flush=True)
    dp.close()
    return {"workload": f"C3 adjoint, {args.n}^3 hex, {p.steps} steps, checkpoints every 10",
            "loss": float(L), "forward_s": t1 - t0, "backward_s": t2 - t1,
            "fd_checks": len(rows),
            "fd_max_rel_err_k": max(r["rel_err"] for r in rows if r["param"].startswith("k")),
            "fd_max_rel_err_directional": max(r["rel_err"] for r in rows
                                              if r["param"].startswith("direction")),
            "fd_max_rel_err_w_single": max(r["rel_err"] for r in rows if r["param"].startswith("w")),
            "fd": rows}


def batch_leg(args) -> dict:
    """Ensemble workload: 64 hex samples of side n ~ U{41..81} nodes with per-sample lognormal
    k, sigma0 and w, advanced together through one batch handle (graph-captured iteration
    chunks, autotuned SpMV slab shape) for 30 coupled steps, FP64 and mixed.  Reports
    sample-steps/s and, per sample, the relative error of the mixed state against the FP64
    state after the last step."""
    import numpy as np
    import torch
    import rafem_inputs as ri
    from paper_2409_13036_amd import _lib as R
    from paper_2409_13036_amd.sim import BatchProblem

    probs = ri.config4(samples=args.batch_samples, steps=args.batch_steps)
    t0 = time.perf_counter()
    bp = BatchProblem(probs)
    setup = time.perf_counter() - t0
    S = len(probs)
    nnz = sum((3 * p.n - 2) ** 3 for p in probs)
    out = {"workload": f"C4 ensemble, {S} hex samples n~U{{41..81}}, {args.batch_steps} coupled "
                       f"steps, one batch handle",
           "samples": S, "n_nodes_total": int(sum(p.n_nodes for p in probs)), "nnz_total": nnz,
           "setup_s": setup}
    finals = {}
    for precision in ("fp64", "mixed"):
        bp.reset()
        bp.step(TOL, precision)  # warm-up: bioheat assembly, autotuning, graph capture
        bp.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            bp.step(TOL, precision)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
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
            "V_iters_last_step": [min(i["V"]["iters"] for i in its),
                                  max(i["V"]["iters"] for i in its)],
            "T_iters_last_step": [min(i["T"]["iters"] for i in its),
                                  max(i["T"]["iters"] for i in its)],
            "spmv_us_mean": mean_us, "spmv_launches": count}
        print(f"[bench] batch {precision}: {S * args.batch_steps / el:.1f} sample-steps/s "
              f"({el:.2f} s), spmv {mean_us:.1f} us x {count}", file=sys.stderr, flush=True)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    eT = [rel(m[0], f[0]) for m, f in zip(finals["mixed"], finals["fp64"])]
    eV = [rel(m[1], f[1]) for m, f in zip(finals["mixed"], finals["fp64"])]
    out["mixed_rel_err_vs_fp64_max"] = {"T": max(eT), "V": max(eV)}
    mixed_ok = max(eT) <= 1e-8 and max(eV) <= 1e-8
    out["path"] = "mixed" if mixed_ok else "fp64"
    out["sample_steps_per_s"] = out[out["path"]]["sample_steps_per_s"]
    bp.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=101)
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="relative tolerance of each FP32 inner solve (0: library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-child", action="store_true")
    ap.add_argument("--adjoint", action="store_true",
                    help="run only the differentiation workload (timing + finite-difference check)")
    ap.add_argument("--adj-steps", type=int, default=60)
    ap.add_argument("--fd-params", type=int, default=32)
    ap.add_argument("--workload", choices=["c1", "c2"], default="c1",
                    help="c1: 101^3 hex (default); c2: 161^3-node jittered Kuhn tets")
    ap.add_argument("--no-batch", action="store_true", help="skip the ensemble leg")
    ap.add_argument("--batch-only", action="store_true", help="run only the ensemble leg")
    ap.add_argument("--batch-samples", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=30)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first launch a plain copy of this many MiB (byte-counter reference)")
    args = ap.parse_args()
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
        print(json.dumps(batch_leg(args)), flush=True)
        return

    # CPU oracle first, before this process touches the GPU
    cpu = None if (args.no_cpu_baseline or args.workload != "c1") else cpu_baseline(args.n)
    print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)

    import numpy as np
    import torch
    import rafem_inputs as ri
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
    N, nnz = dp.mesh.n_nodes, dp.mesh.nnz
    res = {}
    for precision in ("fp64", "mixed"):
        kw = {"inner_tol": args.inner_tol} if precision == "mixed" else {}
        el, infos, state, (mean_us, count) = run_path(dp, precision, args.steps, args.warmup,
                                                      args.profile_steps, **kw)
        it_v = float(np.mean([i["V"]["iters"] for i in infos]))
        it_t = float(np.mean([i["T"]["iters"] for i in infos]))
        res[precision] = {"elapsed": el, "state": state, "spmv_us": mean_us, "spmv_count": count,
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
    per_launch = spmv_bytes(N, nnz, fp32)
    achieved = per_launch / (r["spmv_us"] * 1e-6) / 1e9 if r["spmv_us"] > 0 else 0.0
    line = {
        "metric": "coupled time-step solves/s at 1M DOF (101^3 hex), FP64 vs mixed at 1e-8 rel err; SpMV HBM GB/s",
        "value": sps, "unit": "coupled steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 / sps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-inner/f64-refined" if fp32 else "f64", "data": "synthetic",
        "config": {"workload": workload, "n_nodes": N,
                   "nnz": nnz, "dt_s": p.dt, "tol": TOL, "path": head},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kernel),
                     "kernel": kernel, "bytes_per_launch": per_launch,
                     "mean_launch_us": r["spmv_us"], "launches_measured": r["spmv_count"]},
        "cpu_baseline": cpu,
        "fp64": {"steps_per_s": args.steps / res["fp64"]["elapsed"],
                 "V_iters": res["fp64"]["V_iters"], "T_iters": res["fp64"]["T_iters"],
                 "spmv_us": res["fp64"]["spmv_us"],
                 "spmv_GBs": spmv_bytes(N, nnz, False) / (res["fp64"]["spmv_us"] * 1e-6) / 1e9
                 if res["fp64"]["spmv_us"] > 0 else None,
                 "relres_true_max": res["fp64"]["relres_true_max"]},
        "mixed": {"steps_per_s": args.steps / res["mixed"]["elapsed"],
                  "V_inner_iters": res["mixed"]["V_iters"], "V_outer": res["mixed"]["V_outer"],
                  "T_inner_iters": res["mixed"]["T_iters"], "spmv_us": res["mixed"]["spmv_us"],
                  "spmv_GBs": spmv_bytes(N, nnz, True) / (res["mixed"]["spmv_us"] * 1e-6) / 1e9
                  if res["mixed"]["spmv_us"] > 0 else None,
                  "relres_true_max": res["mixed"]["relres_true_max"],
                  "rel_err_vs_fp64": {"T": errT, "V": errV}},
    }
    if cpu:
        line["speedup_vs_cpu_oracle"] = sps / cpu["value"]
    dp.close()
    del dp
    if not args.no_batch and args.workload == "c1":
        line["batch"] = batch_leg(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

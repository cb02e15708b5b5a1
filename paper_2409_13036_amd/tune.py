"""Autotuning of the mixed-precision refinement for one problem, with an on-disk cache.

The library tunes what it can without changing a result: the slab shape of the SpMV (2 or
4 slabs per wavefront; the partial sums cover fixed groups of slabs whatever the shape),
timed at the first step and cached on disk per layout (``RAFEM_TUNE_CACHE``).  The
parameters that do change the iterates -- the inner tolerance of the FP32 solves (how far
each refinement reduces the residual before x is refined) and whether the inner recurrence
is continued across refinements or restarted -- are a per-problem choice: ``tune_mixed``
times a few coupled steps of each candidate from the same state and keeps the fastest,
caching it by the mesh's layout and the device (``RAFEM_MIXED_TUNE_CACHE``, else
``~/.cache/rafem/mixed_tune.json``).  Every candidate meets the same FP64 stopping test, so
the choice moves only the speed.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional, Sequence, Tuple

CANDIDATES: Tuple[Tuple[float, int], ...] = ((3e-5, 0), (1e-4, 0), (1e-3, 0), (1e-2, 0), (3e-5, 1))


def cache_path() -> str:
    p = os.environ.get("RAFEM_MIXED_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "rafem", "mixed_tune.json")


def layout_key(mesh) -> str:
    import torch
    st = mesh.stats()
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(dev, "gcnArchName", dev.name).replace(" ", "_")
    return (f"{arch}/n{st.n_nodes}/nnz{st.nnz}/slots{st.value_slots}/slabs{st.slabs}"
            f"/shared{st.shared_offset_slabs}/S{st.n_samples}/npe{st.nodes_per_elem}")


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, entry: dict) -> None:
    data = _load(path)
    data[key] = entry
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass


def tune_mixed(dp, *, tol: float = 1e-13, warmup: int = 2, steps: int = 4,
               candidates: Sequence[Tuple[float, int]] = CANDIDATES, use_cache: bool = True,
               path: Optional[str] = None) -> dict:
    """Fastest (inner_tol, restart_inner) of `candidates` for device problem `dp` (a
    DeviceProblem or BatchProblem), timing `steps` mixed coupled steps after `warmup` steps
    from the problem's initial state for each, with the predictor's starting points as dp
    has them.  Returns {"inner_tol", "restart_inner", "cached", "timings"}; dp is left reset."""
    import torch
    path = path or cache_path()
    key = layout_key(dp.mesh)
    if use_cache:
        hit = _load(path).get(key)
        if hit and "inner_tol" in hit and "restart_inner" in hit:
            dp.reset()
            return {"inner_tol": float(hit["inner_tol"]), "restart_inner": int(hit["restart_inner"]),
                    "cached": True, "timings": hit.get("timings", {})}
    timings = {}
    best = None
    for inner_tol, restart in candidates:
        kw = {"inner_tol": inner_tol, "restart_inner": restart}
        dp.reset()
        for _ in range(warmup):
            dp.step(tol, "mixed", **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dp.step(tol, "mixed", **kw)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        timings[f"{inner_tol:g}/{'restart' if restart else 'continue'}"] = ms
        if best is None or ms < best[0]:
            best = (ms, inner_tol, restart)
    dp.reset()
    out = {"inner_tol": best[1], "restart_inner": best[2], "cached": False, "timings": timings}
    if use_cache:
        _store(path, key, {"inner_tol": best[1], "restart_inner": best[2], "timings": timings})
    return out

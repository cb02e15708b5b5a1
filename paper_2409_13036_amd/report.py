"""Result-quality and region reports of the paper's methodology.

PSNR per simulation step (Sec. IV, Eq. 1): with A the reference run and B the run under test,
each a sequence of per-step nodal fields (temperature or potential),

    MSE_i  = (1/n) sum_j (A_ij - B_ij)^2,
    PSNR_i = 20 log10( MAX(A) / sqrt(MSE_i) ),

MAX(A) being the largest value of the field over all steps of the reference.  The paper's
control lines are the PSNR of the reference against itself plus a noise of a given size
(1e-5 and 1e-12) at every node, i.e. 20 log10(MAX(A) / noise).  Identical steps give an
infinite PSNR.
"""
from __future__ import annotations

from typing import Iterable, List

import numpy as np


def psnr(reference: Iterable[np.ndarray], other: Iterable[np.ndarray]) -> np.ndarray:
    """PSNR of every step of ``other`` against the same step of ``reference`` [steps]."""
    ref = [np.asarray(a, dtype=np.float64) for a in reference]
    oth = [np.asarray(b, dtype=np.float64) for b in other]
    if len(ref) != len(oth) or not ref:
        raise ValueError("the two runs must have the same, non-zero number of steps")
    peak = max(float(np.max(a)) for a in ref)
    out = np.empty(len(ref))
    for i, (a, b) in enumerate(zip(ref, oth)):
        if a.shape != b.shape:
            raise ValueError(f"step {i}: shapes {a.shape} and {b.shape} differ")
        mse = float(np.mean((a - b) ** 2))
        out[i] = np.inf if mse == 0.0 else 20.0 * np.log10(peak / np.sqrt(mse))
    return out


def control_psnr(reference: Iterable[np.ndarray], noise: float) -> float:
    """The control line: PSNR of the reference plus ``noise`` at every node."""
    peak = max(float(np.max(np.asarray(a))) for a in reference)
    return 20.0 * np.log10(peak / noise)


def summary(reference: List[np.ndarray], other: List[np.ndarray],
            noises=(1e-5, 1e-12)) -> dict:
    """min / median PSNR over the steps and the control lines."""
    p = psnr(reference, other)
    finite = p[np.isfinite(p)]
    return {"min_db": float(p.min()), "median_db": float(np.median(finite)) if finite.size else
            float("inf"), "steps": int(p.size),
            "control_db": {f"{n:g}": control_psnr(reference, n) for n in noises}}

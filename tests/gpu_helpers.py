"""Shared helpers of the GPU parity tests (inputs to the device, comparisons)."""
import numpy as np

EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps


def to_dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def to_host(t):
    return t.detach().cpu().numpy()


def rel_err(x, ref):
    d = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (d if d > 0 else 1.0))


def spmv_bound(A, x, eps, k=64):
    """Entrywise forward-error bound of a sum of products: k eps sum_j |A_ij x_j|."""
    import scipy.sparse as sp
    absA = sp.csr_matrix((np.abs(A.data), A.indices, A.indptr), shape=A.shape)
    return k * eps * (absA @ np.abs(x))


def assembly_bound(S, vals_abs, eps, k=64):
    """Per-entry bound for an assembled value: k eps times the largest magnitude in its row."""
    rowmax = np.maximum.reduceat(np.abs(vals_abs), S.row_ptr[:-1])
    return k * eps * np.repeat(rowmax, np.diff(S.row_ptr))

"""ctypes binding of librafem.so (argument marshalling only).

Every function here checks dtypes, devices and contiguity, then calls the C ABI
of the same name.  All computation happens in the library's HIP kernels; there
is no Python or CPU fallback: if the shared library is missing or fails to
load, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RAFEM_LIB_VARIANT=asan loads the host-sanitizer build (librafem_asan.so, built by
# `python -m paper_2409_13036_amd.build --sanitize`; its runtime must be preloaded)
_VARIANT = os.environ.get("RAFEM_LIB_VARIANT", "")
LIB_PATH = os.path.join(_HERE, f"librafem_{_VARIANT}.so" if _VARIANT else "librafem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2409_13036_amd.build)")
# torch ships its own HIP runtime; loading it first makes the library bind to that same
# runtime, in which the caller's tensors and streams live (loaded the other way round, the
# library's runtime instance finds no device)
import torch  # noqa: E402,F401
_lib = C.CDLL(LIB_PATH)

OK, E_ARG, E_MESH, E_NOCONV, E_BREAKDOWN, E_HIP, E_NOMEM, E_STATE = range(8)
FP64, MIXED = 0, 1
STATUS_NAMES = {OK: "OK", E_ARG: "E_ARG", E_MESH: "E_MESH", E_NOCONV: "E_NOCONV",
                E_BREAKDOWN: "E_BREAKDOWN", E_HIP: "E_HIP", E_NOMEM: "E_NOMEM", E_STATE: "E_STATE"}

# names every declaration in include/rafem.h maps to
EXPORTS = ("rafem_last_error", "rafem_abi_version", "rafem_csr_structure", "rafem_colour_elements",
           "rafem_mesh_create", "rafem_mesh_destroy", "rafem_mesh_get_stats", "rafem_assemble_csr",
           "rafem_solve", "rafem_solve_adjoint", "rafem_spmv", "rafem_profile_enable",
           "rafem_profile_read", "rafem_step", "rafem_step_vjp", "rafem_lesion_loss",
           "rafem_mesh_create_batch", "rafem_mesh_sample_layout", "rafem_mesh_set_graphs",
           "rafem_sample_info", "rafem_spmv_timing", "rafem_step_pc", "rafem_mono_jacobian",
           "rafem_mono_solve", "rafem_step_mono", "rafem_rcm_order", "rafem_regions_enable",
           "rafem_regions_read", "rafem_degree_sort", "rafem_spmv_step",
           "rafem_solve_noalloc", "rafem_mesh_set_device_driven", "rafem_solve_enqueue")


class RafemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class MeshStats(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_elems", C.c_int64), ("nnz", C.c_int64),
                ("n_dirichlet", C.c_int64), ("nodes_per_elem", C.c_int32), ("n_colours", C.c_int32),
                ("n_samples", C.c_int32), ("slabs_per_block", C.c_int32),
                ("slabs_per_block32", C.c_int32), ("int16_columns", C.c_int32),
                ("slabs", C.c_int64), ("shared_offset_slabs", C.c_int64),
                ("row_assembly", C.c_int32), ("max_row_entries", C.c_int32),
                ("value_slots", C.c_int64), ("index_bytes", C.c_int64),
                ("device_driven", C.c_int32), ("tuned_from_cache", C.c_int32),
                ("device_driven_solves", C.c_int64), ("device_driven_redone", C.c_int64),
                ("int32_column_slabs", C.c_int64), ("streamed_values", C.c_int32),
                ("streamed_values32", C.c_int32), ("resident_slots", C.c_int64),
                ("resident_slots32", C.c_int64), ("launch_bound", C.c_int32),
                ("launch_bound32", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("precision", C.c_int32),
                ("inner_tol", C.c_double), ("max_outer", C.c_int32), ("poll_every", C.c_int32),
                ("restart_inner", C.c_int32), ("pad", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("outer", C.c_int32),
                ("launched", C.c_int32), ("relres", C.c_double), ("relres_true", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CorrectorOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iters", C.c_int32)]


class CorrectorInfo(C.Structure):
    _fields_ = [("accepted", C.c_int32), ("iters", C.c_int32), ("change", C.c_double),
                ("solver_iters", C.c_int32), ("status", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


GMRES_MAX_M = 200


class GmresOpts(C.Structure):
    _fields_ = [("m", C.c_int32), ("max_iters", C.c_int32), ("tol", C.c_double),
                ("precision", C.c_int32), ("pad", C.c_int32)]


class GmresInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("cycles", C.c_int32),
                ("pad", C.c_int32), ("relres", C.c_double), ("relres_true", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class MonoInfo(C.Structure):
    _fields_ = [("accepted", C.c_int32), ("iters", C.c_int32), ("change", C.c_double),
                ("gmres_iters", C.c_int32), ("gmres_cycles", C.c_int32), ("status", C.c_int32),
                ("pad", C.c_int32), ("relres_true_max", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class Regions(C.Structure):
    _fields_ = [("assembly_ms", C.c_double), ("solve_ms", C.c_double), ("check_ms", C.c_double),
                ("steps", C.c_int64)]


class Phys(C.Structure):
    _fields_ = [("rho_c", C.c_double), ("dt", C.c_double), ("T_a", C.c_double),
                ("alpha_sigma", C.c_double), ("T_ref", C.c_double), ("coupled", C.c_int32),
                ("reuse_bioheat", C.c_int32), ("extrapolate", C.c_int32),
                ("extrapolate_order", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("V", SolveInfo), ("T", SolveInfo)]


_p = C.c_void_p
_i64, _i32 = C.c_int64, C.c_int32
_lib.rafem_last_error.restype = C.c_char_p
_lib.rafem_abi_version.restype = C.c_int32
_lib.rafem_csr_structure.argtypes = [_i64, _i64, _i32, _p, C.POINTER(C.c_int64), _p, _p]
_lib.rafem_colour_elements.argtypes = [_i64, _i64, _i32, _p, _p, C.POINTER(C.c_int32)]
_lib.rafem_rcm_order.argtypes = [_i64, _i64, _i32, _p, _p]
_lib.rafem_degree_sort.argtypes = [_i64, _i64, _i32, _p, _i64, _p]
_lib.rafem_mesh_create.argtypes = [_i64, _i64, _i32, _p, _p, _p, _i64, C.POINTER(_p)]
_lib.rafem_mesh_destroy.argtypes = [_p]
_lib.rafem_mesh_get_stats.argtypes = [_p, C.POINTER(MeshStats)]
_lib.rafem_assemble_csr.argtypes = [_p, _p, _p, _p, _p, _p, _p, _p, _p, _p]
_lib.rafem_solve.argtypes = [_p, _p, _p, _p, _p, _p, _p, C.POINTER(SolveOpts), C.POINTER(SolveInfo), _p]
_lib.rafem_solve_enqueue.argtypes = [_p, _p, _p, _p, _p, _p, _p, C.POINTER(SolveOpts), _i32, _i32,
                                     _p, _p]
_lib.rafem_solve_adjoint.argtypes = [_p, _p, _p, _p, _p, _p, _p, C.POINTER(SolveOpts),
                                     C.POINTER(SolveInfo), _p]
_lib.rafem_spmv.argtypes = [_p, _p, _p, _p, _p, _p, _p, _p, _p, _p]
_lib.rafem_spmv_step.argtypes = [_p, _i32, _i32, _p, _p, _p, _p, _p]
_lib.rafem_solve_noalloc.argtypes = [_i64, _i64, _p, _p, _p, _p, _p, _p, C.POINTER(SolveOpts),
                                     C.POINTER(SolveInfo), _p]
_lib.rafem_profile_enable.argtypes = [_p, _i32]
_lib.rafem_profile_read.argtypes = [_p, _i32, C.POINTER(C.c_double), C.POINTER(C.c_int64), _i32]
_lib.rafem_regions_enable.argtypes = [_p, _i32]
_lib.rafem_regions_read.argtypes = [_p, C.POINTER(Regions), _i32]
_lib.rafem_spmv_timing.argtypes = [_p, _i32, _i32, _i32, C.POINTER(C.c_double)]
_lib.rafem_step.argtypes = [_p, C.POINTER(Phys), _p, _p, _p, _p, _p, _p, _p, C.POINTER(SolveOpts),
                            C.POINTER(StepInfo), _p]
_lib.rafem_step_pc.argtypes = [_p, C.POINTER(Phys), _p, _p, _p, _p, _p, _p, C.c_double, _p, _p,
                               C.POINTER(SolveOpts), C.POINTER(CorrectorOpts),
                               C.POINTER(CorrectorInfo), _p]
_lib.rafem_mono_jacobian.argtypes = [_p, C.POINTER(Phys), _p, _p, _p, _p, _p, _p, _p, _p, _p]
_lib.rafem_mono_solve.argtypes = [_p, C.POINTER(Phys), _p, _p, _p, _p, _p, _p,
                                  C.POINTER(GmresOpts), _p, _p, _i32, C.POINTER(GmresInfo), _p]
_lib.rafem_step_mono.argtypes = [_p, C.POINTER(Phys), _p, _p, _p, _p, _p, _p, C.c_double, _p, _p,
                                 C.POINTER(GmresOpts), C.POINTER(CorrectorOpts),
                                 C.POINTER(MonoInfo), _p]
_lib.rafem_step_vjp.argtypes = [_p, C.POINTER(Phys), _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p,
                                C.POINTER(SolveOpts), C.POINTER(StepInfo), _p]
_lib.rafem_lesion_loss.argtypes = [_p, _i64, _p, _p, _p, C.c_double, _p, _p, _p]
_lib.rafem_mesh_create_batch.argtypes = [_i32, _p, _p, _i32, _p, _p, _p, _p, C.POINTER(_p)]
_lib.rafem_mesh_sample_layout.argtypes = [_p, _p, _p, _p]
_lib.rafem_mesh_set_graphs.argtypes = [_p, _i32]
_lib.rafem_mesh_set_device_driven.argtypes = [_p, _i32, C.c_double]
_lib.rafem_sample_info.argtypes = [_p, _i32, C.POINTER(StepInfo)]
for _name in EXPORTS:
    if _name not in ("rafem_last_error", "rafem_abi_version"):
        getattr(_lib, _name).restype = C.c_int32

# the structures above mirror include/rafem.h at this version
ABI_VERSION = 3
if _lib.rafem_abi_version() != ABI_VERSION:
    raise ImportError(f"{_lib._name} has ABI version {_lib.rafem_abi_version()}, the binding "
                      f"expects {ABI_VERSION}: rebuild the library")


def lib():
    return _lib


def last_error() -> str:
    return _lib.rafem_last_error().decode(errors="replace")


def _check(status: int, allow=(OK,)):
    if status not in allow:
        raise RafemError(status, last_error())
    return status


def abi_version() -> int:
    return int(_lib.rafem_abi_version())


# --------------------------------------------------------------------------------------
# host-only analysis
# --------------------------------------------------------------------------------------
def _host_i32(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a


def csr_structure(conn: np.ndarray, n_nodes: int):
    """rafem_csr_structure: CSR pattern of the node graph -> (row_ptr, col_idx) int32 arrays."""
    conn = _host_i32(conn)
    E, npe = conn.shape
    nnz = C.c_int64(0)
    _check(_lib.rafem_csr_structure(n_nodes, E, npe, conn.ctypes.data, C.byref(nnz), None, None))
    rp = np.empty(n_nodes + 1, dtype=np.int32)
    ci = np.empty(nnz.value, dtype=np.int32)
    _check(_lib.rafem_csr_structure(n_nodes, E, npe, conn.ctypes.data, C.byref(nnz),
                                    rp.ctypes.data, ci.ctypes.data))
    return rp, ci


def colour_elements(conn: np.ndarray, n_nodes: int):
    """rafem_colour_elements -> (colour int32 [E], n_colours)."""
    conn = _host_i32(conn)
    E, npe = conn.shape
    col = np.empty(E, dtype=np.int32)
    nc = C.c_int32(0)
    _check(_lib.rafem_colour_elements(n_nodes, E, npe, conn.ctypes.data, col.ctypes.data, C.byref(nc)))
    return col, int(nc.value)


def degree_sort(order: np.ndarray, conn: np.ndarray, n_nodes: int, window: int) -> np.ndarray:
    """rafem_degree_sort -> the order with each window of positions sorted by node degree."""
    conn = _host_i32(conn)
    E, npe = conn.shape
    out = np.ascontiguousarray(np.array(order, dtype=np.int32, copy=True))
    _check(_lib.rafem_degree_sort(n_nodes, E, npe, conn.ctypes.data, int(window), out.ctypes.data))
    return out


def regions_enable(mesh: "Mesh", enable: bool = True):
    """rafem_regions_enable: time the assembly / solve / check regions of every step."""
    _check(_lib.rafem_regions_enable(mesh.handle, 1 if enable else 0))


def regions_read(mesh: "Mesh", reset: bool = True) -> dict:
    """rafem_regions_read -> mean milliseconds per step of each region, and the step count."""
    r = Regions()
    _check(_lib.rafem_regions_read(mesh.handle, C.byref(r), 1 if reset else 0))
    k = max(1, int(r.steps))
    return {"assembly_ms": r.assembly_ms / k, "solve_ms": r.solve_ms / k,
            "check_ms": r.check_ms / k, "steps": int(r.steps)}


def rcm_order(conn: np.ndarray, n_nodes: int) -> np.ndarray:
    """rafem_rcm_order -> order int32 [n_nodes] (order[k] = node placed at position k)."""
    conn = _host_i32(conn)
    E, npe = conn.shape
    order = np.empty(n_nodes, dtype=np.int32)
    _check(_lib.rafem_rcm_order(n_nodes, E, npe, conn.ctypes.data, order.ctypes.data))
    return order


# --------------------------------------------------------------------------------------
# device entry points (torch tensors for device memory and streams)
# --------------------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _dev(t, dtype, n: Optional[int] = None, name: str = "tensor", allow_none: bool = False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device (cuda) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return t


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _precision(precision) -> int:
    return {"fp64": FP64, "mixed": MIXED}.get(precision, precision)


def make_opts(tol=1e-10, maxit=0, precision="fp64", inner_tol=0.0, max_outer=0, poll_every=0,
              restart_inner=0):
    return SolveOpts(tol, maxit, _precision(precision), inner_tol, max_outer, poll_every,
                     int(restart_inner), 0)


class Mesh:
    """rafem_mesh_create / rafem_mesh_destroy: structure, colouring and workspaces on the device."""

    def __init__(self, xyz: np.ndarray, conn: np.ndarray, dir_ids: np.ndarray):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("rafem needs a HIP device")
        torch.cuda.init()
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        conn = _host_i32(conn)
        dir_ids = _host_i32(dir_ids)
        h = C.c_void_p()
        _check(_lib.rafem_mesh_create(int(xyz.shape[0]), conn.shape[0], conn.shape[1], xyz.ctypes.data,
                                      conn.ctypes.data, dir_ids.ctypes.data if dir_ids.size else None,
                                      int(dir_ids.size), C.byref(h)))
        self._adopt(h)

    @classmethod
    def batch(cls, meshes):
        """rafem_mesh_create_batch from a list of (xyz, conn, dir_ids) of one element type."""
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("rafem needs a HIP device")
        torch.cuda.init()
        S = len(meshes)
        keep = []
        nn = np.empty(S, dtype=np.int64)
        ne = np.empty(S, dtype=np.int64)
        nd = np.empty(S, dtype=np.int64)
        xp = (C.c_void_p * S)()
        cp = (C.c_void_p * S)()
        dp = (C.c_void_p * S)()
        npe = None
        for q, (xyz, conn, dirs) in enumerate(meshes):
            xyz = np.ascontiguousarray(xyz, dtype=np.float64)
            conn = _host_i32(conn)
            dirs = _host_i32(dirs)
            npe = conn.shape[1] if npe is None else npe
            keep += [xyz, conn, dirs]
            nn[q], ne[q], nd[q] = xyz.shape[0], conn.shape[0], dirs.size
            xp[q], cp[q] = xyz.ctypes.data, conn.ctypes.data
            dp[q] = dirs.ctypes.data if dirs.size else None
        h = C.c_void_p()
        _check(_lib.rafem_mesh_create_batch(S, nn.ctypes.data, ne.ctypes.data, int(npe), xp, cp, dp,
                                            nd.ctypes.data, C.byref(h)))
        self = cls.__new__(cls)
        self._adopt(h)
        return self

    def _adopt(self, h):
        self.handle = h
        st = self.stats()
        self.n_nodes = int(st.n_nodes)
        self.n_elems = int(st.n_elems)
        self.npe = int(st.nodes_per_elem)
        self.n_dir = int(st.n_dirichlet)
        self.nnz = int(st.nnz)
        self.n_colours = int(st.n_colours)
        self.n_samples = int(st.n_samples)
        S = self.n_samples
        self.node_off = np.empty(S + 1, dtype=np.int64)
        self.elem_off = np.empty(S + 1, dtype=np.int64)
        self.dir_off = np.empty(S + 1, dtype=np.int64)
        _check(_lib.rafem_mesh_sample_layout(self.handle, self.node_off.ctypes.data,
                                             self.elem_off.ctypes.data, self.dir_off.ctypes.data))

    def stats(self) -> MeshStats:
        st = MeshStats()
        _check(_lib.rafem_mesh_get_stats(self.handle, C.byref(st)))
        return st

    def set_device_driven(self, enable: bool, budget_scale: float = 0.0):
        """rafem_mesh_set_device_driven: whole solves enqueued at once, one poll per solve."""
        _check(_lib.rafem_mesh_set_device_driven(self.handle, 1 if enable else 0,
                                                 float(budget_scale)))

    def set_graphs(self, enable: bool):
        _check(_lib.rafem_mesh_set_graphs(self.handle, 1 if enable else 0))

    def sample_info(self, q: int):
        info = StepInfo()
        _check(_lib.rafem_sample_info(self.handle, int(q), C.byref(info)))
        return {"V": info.V.as_dict(), "T": info.T.as_dict()}

    def close(self):
        if getattr(self, "handle", None):
            _lib.rafem_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def profile_enable(mesh: Mesh, enable: bool = True):
    """rafem_profile_enable: bracket every PCG SpMV launch with HIP events."""
    _check(_lib.rafem_profile_enable(mesh.handle, 1 if enable else 0))


def profile_read(mesh: Mesh, precision: str = "fp64", reset: bool = True):
    """rafem_profile_read -> (mean SpMV kernel duration in us, number of launches measured)."""
    mean = C.c_double(0.0)
    cnt = C.c_int64(0)
    prec = {"fp64": FP64, "mixed": MIXED}.get(precision, precision)
    _check(_lib.rafem_profile_read(mesh.handle, prec, C.byref(mean), C.byref(cnt), 1 if reset else 0))
    return float(mean.value), int(cnt.value)


def spmv_timing(mesh: Mesh, precision: str = "fp64", copies: int = 1, reps: int = 20) -> float:
    """rafem_spmv_timing -> mean duration (us) of the PCG SpMV on the mesh's potential matrix,
    rotating through `copies` copies of its values (enough copies defeat the Infinity Cache)."""
    mean = C.c_double(0.0)
    prec = {"fp64": FP64, "mixed": MIXED}.get(precision, precision)
    _check(_lib.rafem_spmv_timing(mesh.handle, prec, int(copies), int(reps), C.byref(mean)))
    return float(mean.value)


def assemble_csr(mesh: Mesh, stiff_coef=None, mass_coef=None, dir_vals=None, *, want_structure=True,
                 want_f32=False, stream=None):
    """rafem_assemble_csr -> dict(row_ptr, col_idx, vals, vals32, rhs_lift) of device tensors."""
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device())
    stiff_coef = _dev(stiff_coef, torch.float64, mesh.n_elems, "stiff_coef", allow_none=True)
    mass_coef = _dev(mass_coef, torch.float64, mesh.n_elems, "mass_coef", allow_none=True)
    dir_vals = _dev(dir_vals, torch.float64, mesh.n_dir, "dir_vals", allow_none=True)
    out = {"vals": torch.empty(mesh.nnz, dtype=torch.float64, device=dev)}
    if want_structure:
        out["row_ptr"] = torch.empty(mesh.n_nodes + 1, dtype=torch.int32, device=dev)
        out["col_idx"] = torch.empty(mesh.nnz, dtype=torch.int32, device=dev)
    if want_f32:
        out["vals32"] = torch.empty(mesh.nnz, dtype=torch.float32, device=dev)
    if dir_vals is not None:
        out["rhs_lift"] = torch.empty(mesh.n_nodes, dtype=torch.float64, device=dev)
    _check(_lib.rafem_assemble_csr(mesh.handle, _ptr(mass_coef), _ptr(stiff_coef), _ptr(dir_vals),
                                   _ptr(out.get("row_ptr")), _ptr(out.get("col_idx")), _ptr(out["vals"]),
                                   _ptr(out.get("vals32")), _ptr(out.get("rhs_lift")), _stream(stream)))
    return out


def solve(mesh: Mesh, row_ptr, col_idx, vals, b, x, *, vals32=None, tol=1e-10, precision="fp64",
          maxit=0, inner_tol=0.0, max_outer=0, poll_every=0, restart_inner=0, stream=None, check=True):
    """rafem_solve: Jacobi-PCG (FP64 or mixed) on A x = b, x in/out.  Returns the info dict."""
    torch = _torch()
    n = mesh.n_nodes
    row_ptr = _dev(row_ptr, torch.int32, n + 1, "row_ptr")
    col_idx = _dev(col_idx, torch.int32, None, "col_idx")
    vals = _dev(vals, torch.float64, col_idx.numel(), "vals")
    vals32 = _dev(vals32, torch.float32, col_idx.numel(), "vals32", allow_none=True)
    b = _dev(b, torch.float64, n, "b")
    x = _dev(x, torch.float64, n, "x")
    opts = make_opts(tol, maxit, precision, inner_tol, max_outer, poll_every, restart_inner)
    info = SolveInfo()
    st = _lib.rafem_solve(mesh.handle, _ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(vals32), _ptr(b),
                          _ptr(x), C.byref(opts), C.byref(info), _stream(stream))
    if check:
        _check(st)
    return info.as_dict()


class DeviceInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("outer", C.c_int32),
                ("pad", C.c_int32), ("relres_true", C.c_double)]


def device_info_buffer(device=None):
    """A device buffer for rafem_solve_enqueue's report (uint8 tensor of its size)."""
    torch = _torch()
    return torch.zeros(C.sizeof(DeviceInfo), dtype=torch.uint8,
                       device=device if device is not None else "cuda")


def read_device_info(buf) -> dict:
    """The report in a device_info_buffer, read back (a stream-ordered copy)."""
    raw = bytes(buf.cpu().numpy().tobytes())
    d = DeviceInfo.from_buffer_copy(raw)
    return {"status": d.status, "iters": d.iters, "outer": d.outer, "relres_true": d.relres_true}


def solve_enqueue(mesh: Mesh, row_ptr, col_idx, vals, b, x, info_buf, *, iterations: int,
                  refinements: int = 1, vals32=None, tol=1e-10, precision="fp64", maxit=0,
                  inner_tol=0.0, restart_inner=0, stream=None, check=True):
    """rafem_solve_enqueue: the whole solve enqueued with fixed budgets and its report
    written to info_buf (device_info_buffer); no host synchronisation.  Returns the call's
    status (argument errors only)."""
    torch = _torch()
    n = mesh.n_nodes
    row_ptr = _dev(row_ptr, torch.int32, n + 1, "row_ptr")
    col_idx = _dev(col_idx, torch.int32, None, "col_idx")
    vals = _dev(vals, torch.float64, col_idx.numel(), "vals")
    vals32 = _dev(vals32, torch.float32, col_idx.numel(), "vals32", allow_none=True)
    b = _dev(b, torch.float64, n, "b")
    x = _dev(x, torch.float64, n, "x")
    if not (info_buf.is_cuda and info_buf.dtype == torch.uint8
            and info_buf.numel() >= C.sizeof(DeviceInfo) and info_buf.is_contiguous()):
        raise ValueError("info_buf must be a contiguous device uint8 tensor from device_info_buffer")
    opts = make_opts(tol, maxit, precision, inner_tol, 0, 0, restart_inner)
    st = _lib.rafem_solve_enqueue(mesh.handle, _ptr(row_ptr), _ptr(col_idx), _ptr(vals),
                                  _ptr(vals32), _ptr(b), _ptr(x), C.byref(opts), int(iterations),
                                  int(refinements), _ptr(info_buf), _stream(stream))
    if check:
        _check(st)
    return st


def solve_noalloc(row_ptr, col_idx, vals, b, x, *, vals32=None, tol=1e-10, precision="fp64",
                  maxit=0, inner_tol=0.0, max_outer=0, poll_every=0, restart_inner=0, stream=None, check=True):
    """rafem_solve_noalloc: rafem_solve without a handle, in the library's static device
    workspace (no device allocation).  Returns the info dict."""
    torch = _torch()
    n = int(b.numel())
    row_ptr = _dev(row_ptr, torch.int32, n + 1, "row_ptr")
    col_idx = _dev(col_idx, torch.int32, None, "col_idx")
    vals = _dev(vals, torch.float64, col_idx.numel(), "vals")
    vals32 = _dev(vals32, torch.float32, col_idx.numel(), "vals32", allow_none=True)
    b = _dev(b, torch.float64, n, "b")
    x = _dev(x, torch.float64, n, "x")
    opts = make_opts(tol, maxit, precision, inner_tol, max_outer, poll_every, restart_inner)
    info = SolveInfo()
    st = _lib.rafem_solve_noalloc(n, int(col_idx.numel()), _ptr(row_ptr), _ptr(col_idx), _ptr(vals),
                                  _ptr(vals32), _ptr(b), _ptr(x), C.byref(opts), C.byref(info),
                                  _stream(stream))
    if check:
        _check(st)
    return info.as_dict()


def solve_adjoint(mesh: Mesh, row_ptr, col_idx, vals, g, lam, *, vals32=None, tol=1e-10,
                  precision="fp64", maxit=0, inner_tol=0.0, max_outer=0, poll_every=0, restart_inner=0, stream=None,
                  check=True):
    """rafem_solve_adjoint: A^T lambda = g (g zeroed on Dirichlet rows), lambda in/out."""
    torch = _torch()
    n = mesh.n_nodes
    row_ptr = _dev(row_ptr, torch.int32, n + 1, "row_ptr")
    col_idx = _dev(col_idx, torch.int32, None, "col_idx")
    vals = _dev(vals, torch.float64, col_idx.numel(), "vals")
    vals32 = _dev(vals32, torch.float32, col_idx.numel(), "vals32", allow_none=True)
    g = _dev(g, torch.float64, n, "g")
    lam = _dev(lam, torch.float64, n, "lambda")
    opts = make_opts(tol, maxit, precision, inner_tol, max_outer, poll_every, restart_inner)
    info = SolveInfo()
    st = _lib.rafem_solve_adjoint(mesh.handle, _ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(vals32),
                                  _ptr(g), _ptr(lam), C.byref(opts), C.byref(info), _stream(stream))
    if check:
        _check(st)
    return info.as_dict()


def spmv(mesh: Mesh, row_ptr, col_idx, vals, x, y, *, stream=None):
    """rafem_spmv: y = A x (FP64 if vals is float64, else the FP32 kernel)."""
    torch = _torch()
    n = mesh.n_nodes
    row_ptr = _dev(row_ptr, torch.int32, n + 1, "row_ptr")
    col_idx = _dev(col_idx, torch.int32, None, "col_idx")
    if vals.dtype == torch.float64:
        vals = _dev(vals, torch.float64, col_idx.numel(), "vals")
        x, y = _dev(x, torch.float64, n, "x"), _dev(y, torch.float64, n, "y")
        _check(_lib.rafem_spmv(mesh.handle, _ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(x), _ptr(y),
                               None, None, None, _stream(stream)))
    else:
        vals = _dev(vals, torch.float32, col_idx.numel(), "vals32")
        x, y = _dev(x, torch.float32, n, "x32"), _dev(y, torch.float32, n, "y32")
        _check(_lib.rafem_spmv(mesh.handle, _ptr(row_ptr), _ptr(col_idx), None, None, None, _ptr(vals),
                               _ptr(x), _ptr(y), _stream(stream)))


def spmv_step(mesh: Mesh, x, y, *, matrix="potential", b=None, dots=True, stream=None):
    """rafem_spmv_step: y = A x (or y = b - A x when b is given) with the PCG kernels on the
    mesh's slab layout.  x, y float64 (FP64 kernel) or float32 (FP32 kernel).  Returns the
    per-sample x.(A x) (or (||b - A x||^2, ||b||^2) pairs) as a NumPy array when dots."""
    torch = _torch()
    n, S = mesh.n_nodes, mesh.n_samples
    which = {"potential": 0, "bioheat": 1}[matrix]
    dt = torch.float64 if x.dtype == torch.float64 else torch.float32
    x, y = _dev(x, dt, n, "x"), _dev(y, dt, n, "y")
    b = _dev(b, torch.float64, n, "b", allow_none=True)
    out = np.zeros(2 * S if b is not None else S) if dots else None
    prec = FP64 if dt == torch.float64 else MIXED
    _check(_lib.rafem_spmv_step(mesh.handle, which, prec, _ptr(x), _ptr(y), _ptr(b),
                                out.ctypes.data if dots else None, _stream(stream)))
    return out


def step(mesh: Mesh, phys: Phys, k_e, perf_e, sigma0_e, dir_V, dir_T, T, V, *, tol=1e-12,
         precision="fp64", maxit=0, inner_tol=0.0, max_outer=0, poll_every=0, restart_inner=0, stream=None, check=True):
    """rafem_step: one coupled step, T and V updated in place.  Returns {"V": info, "T": info}."""
    torch = _torch()
    E, n = mesh.n_elems, mesh.n_nodes
    k_e = _dev(k_e, torch.float64, E, "k_e")
    perf_e = _dev(perf_e, torch.float64, E, "perf_e")
    sigma0_e = _dev(sigma0_e, torch.float64, E, "sigma0_e", allow_none=not phys.coupled)
    dir_V = _dev(dir_V, torch.float64, mesh.n_dir, "dir_V", allow_none=not phys.coupled)
    dir_T = _dev(dir_T, torch.float64, mesh.n_dir, "dir_T")
    T = _dev(T, torch.float64, n, "T")
    V = _dev(V, torch.float64, n, "V", allow_none=not phys.coupled)
    opts = make_opts(tol, maxit, precision, inner_tol, max_outer, poll_every, restart_inner)
    info = StepInfo()
    st = _lib.rafem_step(mesh.handle, C.byref(phys), _ptr(k_e), _ptr(perf_e), _ptr(sigma0_e),
                         _ptr(dir_V), _ptr(dir_T), _ptr(T), _ptr(V), C.byref(opts), C.byref(info),
                         _stream(stream))
    if check:
        _check(st)
    return {"status": st, "V": info.V.as_dict(), "T": info.T.as_dict()}


def step_pc(mesh: Mesh, phys: Phys, k_e, perf_e, sigma0_e, dir_V, dir_T, T_prev, dt_prev, T, V, *,
            corr_tol=1e-10, max_iters=50, tol=1e-12, precision="fp64", maxit=0, inner_tol=0.0,
            max_outer=0, poll_every=0, restart_inner=0, stream=None, check=True):
    """rafem_step_pc: one predictor-corrector step of size phys.dt; T and V are advanced in
    place when the step is accepted.  Returns the corrector info as a dict."""
    torch = _torch()
    E, n = mesh.n_elems, mesh.n_nodes
    k_e = _dev(k_e, torch.float64, E, "k_e")
    perf_e = _dev(perf_e, torch.float64, E, "perf_e")
    sigma0_e = _dev(sigma0_e, torch.float64, E, "sigma0_e", allow_none=not phys.coupled)
    dir_V = _dev(dir_V, torch.float64, mesh.n_dir, "dir_V", allow_none=not phys.coupled)
    dir_T = _dev(dir_T, torch.float64, mesh.n_dir, "dir_T")
    T_prev = _dev(T_prev, torch.float64, n, "T_prev", allow_none=True)
    T = _dev(T, torch.float64, n, "T")
    V = _dev(V, torch.float64, n, "V", allow_none=not phys.coupled)
    opts = make_opts(tol, maxit, precision, inner_tol, max_outer, poll_every, restart_inner)
    copts = CorrectorOpts(float(corr_tol), int(max_iters))
    info = CorrectorInfo()
    st = _lib.rafem_step_pc(mesh.handle, C.byref(phys), _ptr(k_e), _ptr(perf_e), _ptr(sigma0_e),
                            _ptr(dir_V), _ptr(dir_T), _ptr(T_prev),
                            float(dt_prev) if dt_prev else 0.0, _ptr(T), _ptr(V), C.byref(opts),
                            C.byref(copts), C.byref(info), _stream(stream))
    if check:
        _check(st)
    return info.as_dict()


def _mono_fields(mesh: Mesh, k_e, perf_e, sigma0_e):
    torch = _torch()
    E = mesh.n_elems
    return (_dev(k_e, torch.float64, E, "k_e"), _dev(perf_e, torch.float64, E, "perf_e"),
            _dev(sigma0_e, torch.float64, E, "sigma0_e"))


def mono_jacobian(mesh: Mesh, phys: Phys, k_e, perf_e, sigma0_e, T_n, T, V, *, stream=None):
    """rafem_mono_jacobian: the monolithic Jacobian at (T, V) as four planes (TT, TV, VT, VV)
    in the mesh's CSR order, and the residual R interleaved by node.  Returns (planes
    [4, nnz], R [2 n]) on the device."""
    torch = _torch()
    n = mesh.n_nodes
    k_e, perf_e, sigma0_e = _mono_fields(mesh, k_e, perf_e, sigma0_e)
    T_n = _dev(T_n, torch.float64, n, "T_n")
    T = _dev(T, torch.float64, n, "T")
    V = _dev(V, torch.float64, n, "V")
    planes = torch.empty((4, mesh.nnz), dtype=torch.float64, device=T.device)
    R = torch.empty(2 * n, dtype=torch.float64, device=T.device)
    _check(_lib.rafem_mono_jacobian(mesh.handle, C.byref(phys), _ptr(k_e), _ptr(perf_e),
                                    _ptr(sigma0_e), _ptr(T_n), _ptr(T), _ptr(V), _ptr(planes),
                                    _ptr(R), _stream(stream)))
    return planes, R


def mono_solve(mesh: Mesh, phys: Phys, k_e, perf_e, sigma0_e, T_n, T, V, *, m=30, max_iters=0,
               tol=1e-10, precision="fp64", hist_len=0, stream=None, check=True):
    """rafem_mono_solve: assemble J, R at (T, V) and solve J delta = -R by GMRES(m)
    (precision "mixed": FP32 Arnoldi process inside FP64 restarts).  Returns (delta [2 n]
    interleaved, info dict, residual history [hist_len] or None)."""
    torch = _torch()
    n = mesh.n_nodes
    k_e, perf_e, sigma0_e = _mono_fields(mesh, k_e, perf_e, sigma0_e)
    T_n = _dev(T_n, torch.float64, n, "T_n")
    T = _dev(T, torch.float64, n, "T")
    V = _dev(V, torch.float64, n, "V")
    delta = torch.empty(2 * n, dtype=torch.float64, device=T.device)
    hist = torch.zeros(hist_len, dtype=torch.float64, device=T.device) if hist_len else None
    opts = GmresOpts(int(m), int(max_iters), float(tol), _precision(precision), 0)
    info = GmresInfo()
    st = _lib.rafem_mono_solve(mesh.handle, C.byref(phys), _ptr(k_e), _ptr(perf_e),
                               _ptr(sigma0_e), _ptr(T_n), _ptr(T), _ptr(V), C.byref(opts),
                               _ptr(delta), _ptr(hist), int(hist_len), C.byref(info),
                               _stream(stream))
    if check:
        _check(st)
    return delta, info.as_dict(), hist


def step_mono(mesh: Mesh, phys: Phys, k_e, perf_e, sigma0_e, dir_V, dir_T, T_prev, dt_prev, T, V,
              *, corr_tol=1e-10, max_iters=50, m=30, gmres_max_iters=0, gmres_tol=1e-10,
              gmres_precision="fp64", stream=None, check=True):
    """rafem_step_mono: one predictor-corrector step of size phys.dt with the monolithic
    Newton-GMRES corrector; T and V advance in place when accepted.  Returns the info dict."""
    torch = _torch()
    n = mesh.n_nodes
    k_e, perf_e, sigma0_e = _mono_fields(mesh, k_e, perf_e, sigma0_e)
    dir_V = _dev(dir_V, torch.float64, mesh.n_dir, "dir_V")
    dir_T = _dev(dir_T, torch.float64, mesh.n_dir, "dir_T")
    T_prev = _dev(T_prev, torch.float64, n, "T_prev", allow_none=True)
    T = _dev(T, torch.float64, n, "T")
    V = _dev(V, torch.float64, n, "V")
    opts = GmresOpts(int(m), int(gmres_max_iters), float(gmres_tol), _precision(gmres_precision), 0)
    copts = CorrectorOpts(float(corr_tol), int(max_iters))
    info = MonoInfo()
    st = _lib.rafem_step_mono(mesh.handle, C.byref(phys), _ptr(k_e), _ptr(perf_e), _ptr(sigma0_e),
                              _ptr(dir_V), _ptr(dir_T), _ptr(T_prev),
                              float(dt_prev) if dt_prev else 0.0, _ptr(T), _ptr(V), C.byref(opts),
                              C.byref(copts), C.byref(info), _stream(stream))
    if check:
        _check(st)
    return info.as_dict()


def step_vjp(mesh: Mesh, phys: Phys, k_e, perf_e, sigma0_e, dir_V, dir_T, T_prev, V, T, lam, grad_k,
             grad_perf, *, tol=1e-12, precision="fp64", maxit=0, inner_tol=0.0, max_outer=0,
             poll_every=0, restart_inner=0, stream=None, check=True):
    """rafem_step_vjp: reverse of one step.  lam in: dL/dT^n, out: dL/dT^{n-1}; grads accumulate."""
    torch = _torch()
    E, n = mesh.n_elems, mesh.n_nodes
    k_e = _dev(k_e, torch.float64, E, "k_e")
    perf_e = _dev(perf_e, torch.float64, E, "perf_e")
    sigma0_e = _dev(sigma0_e, torch.float64, E, "sigma0_e", allow_none=not phys.coupled)
    dir_V = _dev(dir_V, torch.float64, mesh.n_dir, "dir_V", allow_none=not phys.coupled)
    dir_T = _dev(dir_T, torch.float64, mesh.n_dir, "dir_T")
    T_prev = _dev(T_prev, torch.float64, n, "T_prev", allow_none=not phys.coupled)
    V = _dev(V, torch.float64, n, "V", allow_none=not phys.coupled)
    T = _dev(T, torch.float64, n, "T")
    lam = _dev(lam, torch.float64, n, "lambda")
    grad_k = _dev(grad_k, torch.float64, E, "grad_k")
    grad_perf = _dev(grad_perf, torch.float64, E, "grad_perf")
    opts = make_opts(tol, maxit, precision, inner_tol, max_outer, poll_every, restart_inner)
    info = StepInfo()
    st = _lib.rafem_step_vjp(mesh.handle, C.byref(phys), _ptr(k_e), _ptr(perf_e), _ptr(sigma0_e),
                             _ptr(dir_V), _ptr(dir_T), _ptr(T_prev), _ptr(V), _ptr(T), _ptr(lam),
                             _ptr(grad_k), _ptr(grad_perf), C.byref(opts), C.byref(info),
                             _stream(stream))
    if check:
        _check(st)
    return {"status": st, "V": info.V.as_dict(), "T": info.T.as_dict()}


def lesion_loss(mesh: Mesh, ids, target, T, *, scale=1.0, grad=None, stream=None):
    """rafem_lesion_loss -> loss as a 1-element device tensor; grad (if given) = dL/dT."""
    torch = _torch()
    ids = _dev(ids, torch.int32, None, "ids")
    target = _dev(target, torch.float64, ids.numel(), "target")
    T = _dev(T, torch.float64, mesh.n_nodes, "T")
    grad = _dev(grad, torch.float64, mesh.n_nodes, "grad", allow_none=True)
    out = torch.empty(1, dtype=torch.float64, device=T.device)
    _check(_lib.rafem_lesion_loss(mesh.handle, ids.numel(), _ptr(ids), _ptr(target), _ptr(T),
                                  float(scale), _ptr(out), _ptr(grad), _stream(stream)))
    return out

"""ctypes binding of ``libhodbf.so`` (argument marshalling only; all compute runs in the library)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhodbf.so")

HODBF_OK = 0
STATUS = {0: "OK", -1: "E_ARG", -2: "E_NOMEM", -3: "E_HIP", -4: "E_NUMERIC", -5: "E_NOCONV",
          -6: "E_STATE"}
C64, C128 = 0, 1
P_NONE, P_FP32, P_BF16, P_BOTH, P_FP16 = 0, 1, 2, 3, 4

EXPORTED = ["hodbf_build", "hodbf_apply", "hodbf_precond_apply", "vie_solve", "hodbf_plane_wave",
            "hodbf_apply_tree", "hodbf_solve_workspace",
            "hodbf_stats", "hodbf_export", "hodbf_free", "hodbf_last_error", "hodbf_plan_probe",
            "hodbf_set_allocator"]

# allocator hook types: alloc(bytes, stream, ctx) -> device pointer; release(ptr, ctx)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class BuildParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("h", C.c_double), ("k0", C.c_double), ("eps_r", C.POINTER(C.c_double)),
                ("tol_con", C.c_double), ("tol_fact", C.c_double), ("leaf_size", C.c_int32),
                ("precond_prec", C.c_int32), ("precond_min_level", C.c_int32),
                ("precond_dense_levels", C.c_int32), ("seed", C.c_uint64), ("hbm_budget", C.c_size_t), ("stream", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("use_precond", C.c_int32), ("fp32_only", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.POINTER(C.c_int32)), ("converged", C.POINTER(C.c_int32)),
                ("relres", C.POINTER(C.c_double))]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("levels", C.c_int32), ("leaves", C.c_int32),
                ("max_rank", C.c_int32), ("precond_max_rank", C.c_int32),
                ("entries_fwd", C.c_int64), ("entries_pre", C.c_int64),
                ("bytes_fwd", C.c_int64), ("bytes_pre", C.c_int64), ("bytes_total", C.c_int64),
                ("fwd_stages", C.c_int32), ("pre_stages", C.c_int32),
                ("build_seconds", C.c_double), ("precond_seconds", C.c_double),
                ("id_count", C.c_int64), ("io_rows_fwd", C.c_int64), ("io_rows_pre", C.c_int64),
                ("precond_reconstructions", C.c_int64), ("precond_sketch_cols", C.c_int64)]


class HodbfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load the HIP library; fails loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # torch is the process's device-memory and stream provider: load its HIP runtime
    # first so that the library binds to the same one
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2111_01730_amd._build.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.hodbf_build.argtypes = [C.POINTER(BuildParams), C.POINTER(vp)]
    L.hodbf_apply.argtypes = [vp, i32, i32, vp, i64, vp, i64, vp]
    L.hodbf_precond_apply.argtypes = [vp, i32, i32, vp, i64, vp, i64, vp]
    L.hodbf_apply_noalloc.argtypes = [vp, i32, i32, vp, i64, vp, i64, vp]
    L.vie_solve.argtypes = [vp, i32, vp, i64, vp, i64, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
    L.hodbf_plane_wave.argtypes = [vp, i32, C.POINTER(C.c_double), vp, i64, vp]
    L.hodbf_solve_workspace.argtypes = [vp, i32, C.POINTER(SolveOpts), C.POINTER(C.c_size_t)]
    L.hodbf_stats.argtypes = [vp, C.POINTER(Stats)]
    L.hodbf_export.argtypes = [vp, i32, vp, C.POINTER(C.c_size_t)]
    L.hodbf_plan_probe.argtypes = [C.POINTER(BuildParams), i32, vp, C.POINTER(C.c_size_t)]
    L.hodbf_precond_probe.argtypes = [C.POINTER(BuildParams), i32, vp, C.POINTER(C.c_size_t)]
    L.hodbf_apply_tree.argtypes = [vp, i32, i32, vp, vp, vp]
    L.hodbf_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
    L.hodbf_free.argtypes = [vp]
    L.hodbf_free.restype = None
    L.hodbf_last_error.restype = C.c_char_p
    for name in ["hodbf_build", "hodbf_apply", "hodbf_apply_noalloc", "hodbf_precond_apply", "vie_solve", "hodbf_apply_tree",
                 "hodbf_plane_wave", "hodbf_solve_workspace", "hodbf_stats", "hodbf_export", "hodbf_plan_probe",
                 "hodbf_precond_probe", "hodbf_set_allocator"]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(code: int):
    if code != HODBF_OK:
        raise HodbfError(code, lib().hodbf_last_error().decode(errors="replace"))
    return code


def make_params(grid, tol_con, tol_fact=0.0, leaf_size=64, precond_prec=P_NONE,
                precond_min_level=0, seed=1, hbm_budget=0, stream=None, precond_dense_levels=0):
    eps = np.ascontiguousarray(np.asarray(grid.eps, dtype=np.complex128)).view(np.float64)
    p = BuildParams(nx=grid.nx, ny=grid.ny, nz=grid.nz, h=grid.h, k0=grid.k0,
                    eps_r=eps.ctypes.data_as(C.POINTER(C.c_double)), tol_con=tol_con,
                    tol_fact=tol_fact, leaf_size=leaf_size, precond_prec=precond_prec,
                    precond_min_level=precond_min_level,
                    precond_dense_levels=precond_dense_levels, seed=seed, hbm_budget=hbm_budget,
                    stream=stream)
    p._keep = eps  # keep the host array alive with the struct
    return p


def probe(params: BuildParams, which: int, dtype, entry="hodbf_plan_probe"):
    """Host-only export (no GPU needed): the forward plan (hodbf_plan_probe) or the
    host run of the preconditioner construction (hodbf_precond_probe)."""
    fn = getattr(lib(), entry)
    n = C.c_size_t(0)
    check(fn(C.byref(params), which, None, C.byref(n)))
    out = np.empty(n.value // np.dtype(dtype).itemsize, dtype=dtype)
    check(fn(C.byref(params), which, out.ctypes.data_as(C.c_void_p), C.byref(n)))
    return out

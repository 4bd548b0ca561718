"""Python face of the hodbf library: torch tensors for device memory and streams only.

Every method marshals arguments to one C-ABI call of ``libhodbf.so``; no arithmetic of
the method happens here.  Vectors are torch tensors of shape (N,) or (N, R) on the GPU,
complex64 or complex128, in the user's voxel order (i = ix + nx*(iy + ny*iz)).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import C64, C128, P_BF16, P_BOTH, P_FP16, P_FP32, P_NONE, check, lib


_hook_refs: list = []  # the installed ctypes callbacks must outlive their use


def use_torch_allocator(enable: bool = True) -> None:
    """Route the library's device memory (operator arenas and per-call workspace) through
    torch's caching allocator, so torch's pool owns and accounts for the bytes; False
    restores hipMalloc.  Change it only while no library call is running."""
    if not enable:
        check(lib().hodbf_set_allocator(_lib.ALLOC_FN(0), _lib.FREE_FN(0), None))
        _hook_refs.clear()
        return

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:  # reported to the caller of the library as E_NOMEM
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    a, f = _lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free)
    check(lib().hodbf_set_allocator(a, f, None))
    _hook_refs[:] = [a, f]


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _as_cols(x: torch.Tensor, n: int):
    """View (N,) or (N, R) as a column-major block: returns (tensor of shape (R, N), R)."""
    if x.dim() == 1:
        x = x.unsqueeze(1)
    if x.shape[0] != n:
        raise ValueError(f"expected {n} rows, got {tuple(x.shape)}")
    if not x.is_cuda:
        raise ValueError("vectors must live on the GPU")
    if x.dtype not in (torch.complex64, torch.complex128):
        raise ValueError("vectors must be complex64 or complex128")
    return x.t().contiguous(), x.shape[1]


class Operator:
    """A compressed VIE system matrix (and optional preconditioner) resident on the GPU."""

    def __init__(self, grid, tol_con=1e-4, tol_fact=0.0, leaf_size=64, precond=P_NONE,
                 precond_min_level=0, seed=1, hbm_budget=0, precond_dense_levels=0):
        self.grid = grid
        self.n = grid.n
        p = _lib.make_params(grid, tol_con, tol_fact, leaf_size, precond, precond_min_level,
                             seed, hbm_budget, _stream(), precond_dense_levels)
        h = C.c_void_p()
        check(lib().hodbf_build(C.byref(p), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().hodbf_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call_apply(self, fn, x, out_dtype=None):
        xc, R = _as_cols(x, self.n)
        dt = C128 if xc.dtype == torch.complex128 else C64
        y = torch.empty_like(xc)
        check(fn(self._h, R, dt, C.c_void_p(xc.data_ptr()), self.n, C.c_void_p(y.data_ptr()),
                 self.n, _stream()))
        y = y.t()
        return y[:, 0] if x.dim() == 1 else y

    def apply(self, x: torch.Tensor) -> torch.Tensor:
        """y = Z_con x."""
        return self._call_apply(lib().hodbf_apply, x)

    def precond_apply(self, x: torch.Tensor) -> torch.Tensor:
        """y = P x with P ~ Z^{-1}."""
        return self._call_apply(lib().hodbf_precond_apply, x)

    def apply_tree(self, x: torch.Tensor, which: int = 0) -> torch.Tensor:
        """Products on internal-layout vectors: x of shape (N, R) complex64 in tree order
        (row t = user index perm[t]), contiguous, so element (t, q) sits at t*R + q.
        which: 0 Z_con, 1 P (default copy), 2 P FP32 copy, 3 P BF16 copy, 4 P FP16 copy,
        5 Z_con and 6 P FP32 copy with split-BF16 arithmetic."""
        if x.dtype != torch.complex64 or not x.is_contiguous() or x.dim() != 2:
            raise ValueError("x must be a contiguous (N, R) complex64 tensor")
        y = torch.empty_like(x)
        check(lib().hodbf_apply_tree(self._h, which, x.shape[1], C.c_void_p(x.data_ptr()),
                                     C.c_void_p(y.data_ptr()), _stream()))
        return y

    def plane_wave(self, dirs) -> torch.Tensor:
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        R = d.shape[0]
        b = torch.empty((R, self.n), dtype=torch.complex128, device="cuda")
        check(lib().hodbf_plane_wave(self._h, R, d.ctypes.data_as(C.POINTER(C.c_double)),
                                     C.c_void_p(b.data_ptr()), self.n, _stream()))
        return b.t()

    @staticmethod
    def _solve_opts(tol, restart, max_iter, use_precond, fp32_only=False):
        up = {"fp32": 8 + P_FP32, "bf16": 8 + P_BF16, "fp16": 8 + P_FP16,
              "fp32_split": 16 + P_FP32}.get(use_precond, use_precond)
        return _lib.SolveOpts(tol=tol, restart=restart, max_iter=max_iter, use_precond=int(up),
                              fp32_only=int(bool(fp32_only)))

    def solve_workspace(self, nrhs: int, restart=20, use_precond=1) -> int:
        """Device bytes the library allocates for one solve of nrhs columns (b, x and
        this binding's transposed copies not included)."""
        n = C.c_size_t(0)
        opts = self._solve_opts(1e-4, restart, 1, use_precond)
        check(lib().hodbf_solve_workspace(self._h, int(nrhs), C.byref(opts), C.byref(n)))
        return n.value

    def solve(self, b: torch.Tensor, tol=1e-4, restart=20, max_iter=3000, use_precond=1,
              fp32_only=False):
        """x ~ Z^{-1} b by right-preconditioned FGMRES; returns (x, info dict).

        use_precond: 0 none, 1 the operator's default copy, 'fp32', 'bf16' or 'fp16', or
        'fp32_split' (the FP32 copy with split-BF16 arithmetic).  fp32_only: every
        product with Z in FP32 (no FP64 products for the last few columns).
        """
        if b.dtype != torch.complex128:
            raise ValueError("b must be complex128")
        bc, R = _as_cols(b, self.n)
        x = torch.empty_like(bc)
        opts = self._solve_opts(tol, restart, max_iter, use_precond, fp32_only)
        iters = np.zeros(R, dtype=np.int32)
        conv = np.zeros(R, dtype=np.int32)
        rel = np.zeros(R, dtype=np.float64)
        info = _lib.SolveInfo(iters.ctypes.data_as(C.POINTER(C.c_int32)),
                              conv.ctypes.data_as(C.POINTER(C.c_int32)),
                              rel.ctypes.data_as(C.POINTER(C.c_double)))
        code = lib().vie_solve(self._h, R, C.c_void_p(bc.data_ptr()), self.n,
                               C.c_void_p(x.data_ptr()), self.n, C.byref(opts), C.byref(info),
                               _stream())
        if code not in (_lib.HODBF_OK, -5):
            check(code)
        x = x.t()
        out = dict(iters=iters, converged=conv.astype(bool), relres=rel, status=_lib.STATUS[code])
        return (x[:, 0] if b.dim() == 1 else x), out

    def stats(self) -> dict:
        s = _lib.Stats()
        check(lib().hodbf_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in s._fields_}

    def export(self, which: int, dtype):
        n = C.c_size_t(0)
        check(lib().hodbf_export(self._h, which, None, C.byref(n)))
        out = np.empty(n.value // np.dtype(dtype).itemsize, dtype=dtype)
        check(lib().hodbf_export(self._h, which, out.ctypes.data_as(C.c_void_p), C.byref(n)))
        return out

    def perm(self) -> np.ndarray:
        return self.export(0, np.int32)

    def forward_blocks(self):
        """(table as int64 (k, 12), values complex64) of the forward operator."""
        return self.export(1, np.int64).reshape(-1, 12), self.export(2, np.complex64)

    def precond_blocks(self, copy="fp32"):
        vals = self.export({"fp32": 4, "bf16": 5, "fp16": 6}[copy], np.complex64)
        return self.export(3, np.int64).reshape(-1, 12), vals


__all__ = ["Operator", "P_NONE", "P_FP32", "P_BF16", "P_BOTH", "P_FP16"]

"""hodbf_apply_noalloc through the C ABI: the same result as hodbf_apply bit for bit, on
two calls in a row (the second with a smaller input, on scratch the first call left
dirty), without one allocation (an allocator hook that counts calls sees none, while
hodbf_apply does use it), and a clear E_ARG when the sizes exceed the static scratch."""
import ctypes as C

import numpy as np
import pytest

from synth.workloads import small_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _call(fn, op, x, dtype):
    from paper_2111_01730_amd import _lib
    R, n = x.shape
    y = torch.full_like(x, complex(np.nan, np.nan))
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = fn(op._h, R, dtype, _ptr(x), n, _ptr(y), n, st)
    return code, y


def test_noalloc_apply_equals_apply_without_allocating():
    from paper_2111_01730_amd import _lib
    from paper_2111_01730_amd.hodbf import Operator
    L = _lib.lib()
    counts = {"alloc": 0}

    def _alloc(nbytes, stream, ctx):
        counts["alloc"] += 1
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    cases = [(small_case(81, sides=(12, 10, 9), h=0.1, eps_range=(2.0, 8.0), loss=0.5, nrhs=8), 8),
             (small_case(82, sides=(8, 8, 8), h=0.1, eps_range=(2.0, 4.0), loss=0.1, nrhs=3), 3)]
    ops = [Operator(c["grid"], tol_con=1e-4) for c, _ in cases]
    hooks = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))
    _lib.check(L.hodbf_set_allocator(hooks[0], hooks[1], None))
    try:
        for (c, R), op in zip(cases, ops):
            for dtype, tdt in ((_lib.C128, torch.complex128), (_lib.C64, torch.complex64)):
                x = torch.as_tensor(np.ascontiguousarray(c["x"][:, :R].T)).to("cuda", tdt)
                counts["alloc"] = 0
                code, y_na = _call(L.hodbf_apply_noalloc, op, x, dtype)
                torch.cuda.synchronize()
                assert code == _lib.HODBF_OK, _lib.lib().hodbf_last_error()
                assert counts["alloc"] == 0
                code, y_ref = _call(L.hodbf_apply, op, x, dtype)
                torch.cuda.synchronize()
                assert code == _lib.HODBF_OK
                assert counts["alloc"] > 0  # the allocating entry point does use the hook
                assert torch.equal(y_na, y_ref)
                print(f"[noalloc N={op.n} R={R} dtype {dtype}: equal to hodbf_apply]", flush=True)
        # sizes beyond the 64 MiB scratch are refused with a message, nothing launched
        big = (64 << 20) // (2 * 8 * ops[0].n) + 1
        x = torch.zeros((big, ops[0].n), dtype=torch.complex64, device="cuda")
        code, _ = _call(L.hodbf_apply_noalloc, ops[0], x, _lib.C64)
        assert code == -1  # HODBF_E_ARG
        assert b"scratch" in L.hodbf_last_error()
    finally:
        _lib.check(L.hodbf_set_allocator(_lib.ALLOC_FN(0), _lib.FREE_FN(0), None))
    for op in ops:
        op.close()

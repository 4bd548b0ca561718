"""The rounding bounds of tests/bounds.py, pinned on the CPU with no library code: a
numpy emulation of the stage-by-stage arithmetic of a HOD-BF apply (every stage's output
stored in FP32; products either FP32 or the split-BF16 form hi hi + hi lo + lo hi) on a
small oracle operator stays inside both the element-wise and the norm-wise bound, and the
same emulation with the hi_a lo_x cross term dropped (a planted arithmetic mistake)
breaks the norm-wise bound on inputs whose BF16 remainders are coherent (every x_k =
m_k (1 + 2^-9) with m_k a BF16 value, so lo(x_k) = 2^-9 m_k exactly and the dropped
terms add up to 2^-9 of the result instead of averaging out)."""
import numpy as np
import pytest

from oracle.butterfly import build_hodbf
from synth.workloads import small_case
from tests import bounds


_bf16 = bounds.bf16


def _split(a):
    a = np.asarray(a, dtype=np.complex64)
    out = []
    for part in (a.real, a.imag):
        hi = _bf16(part)
        lo = _bf16(part - hi)
        out.append((hi.astype(np.float64), lo.astype(np.float64)))
    (rh, rl), (ih, il) = out
    return rh + 1j * ih, rl + 1j * il


def _mm(mode):
    def fp32(A, X):
        return (A.astype(np.complex64).astype(np.complex128) @ X)

    def split(A, X, drop=False):
        ah, al = _split(A)
        xh, xl = _split(X)
        y = ah @ xh + ah @ xl
        return y if drop else y + al @ xh

    return {"fp32": fp32, "split": split, "drop": lambda A, X: split(A, X, True)}[mode]


def _round32(t):
    return t.astype(np.complex64).astype(np.complex128)


def _emulate(h, xt, mode):
    """Stage by stage like the kernels: V^0, W^1..W^L into FP32 workspace, then every
    leaf's dense block plus outer factors summed into its output rows (FP32 store)."""
    mm = _mm(mode)
    tr = h.tree
    LH = tr.depth
    y = np.zeros_like(xt)
    acc = {}
    for i, (lo, hi) in enumerate(tr.ranges[LH]):
        acc[i] = mm(h.D[i], xt[lo:hi])
    for (l, i), bf in h.bf.items():
        t = {}
        for b, (lo, hi) in enumerate(bf.col_ranges):
            t[(0, b)] = _round32(mm(bf.V0[b], xt[lo:hi]))
        for lv in range(1, bf.L + 1):
            t = {(a, b): _round32(mm(bf.W[lv][a][b], np.vstack([t[(a // 2, 2 * b)],
                                                                t[(a // 2, 2 * b + 1)]])))
                 for a in range(1 << lv) for b in range(1 << (bf.L - lv))}
        o_leaf0 = i << (LH - l)
        for a in range(1 << bf.L):
            acc[o_leaf0 + a] = acc[o_leaf0 + a] + mm(bf.B[a], t[(a, 0)])
    for i, (lo, hi) in enumerate(tr.ranges[LH]):
        y[lo:hi] = _round32(acc[i])
    return y


@pytest.fixture(scope="module")
def model():
    c = small_case(71, sides=(8, 8, 8), h=0.125, eps_range=(2.0, 10.0), loss=0.5, nrhs=8)
    h = build_hodbf(c["grid"], 1e-4)
    xt = _round32(c["x"])
    ref = h.apply_tree(xt)
    absref = bounds.absolute_hodbf(h).apply_tree(np.abs(xt))
    # stage dimensions straight from the oracle's factors (the device table's layout)
    dims = [max(v.shape[1] for bf in h.bf.values() for v in bf.V0)]
    for lv in range(1, h.tree.depth):
        ws = [w.shape[1] for bf in h.bf.values() if bf.L >= lv for row in bf.W[lv] for w in row]
        if ws:
            dims.append(max(ws))
    leaf = [d.shape[1] for d in h.D]
    for (l, i), bf in h.bf.items():
        for a in range(1 << bf.L):
            leaf[(i << bf.L) + a] += bf.B[a].shape[1]
    dims.append(max(leaf))
    return h, xt, ref, absref, dims


_coherent = bounds.coherent


@pytest.mark.parametrize("mode,split", [("fp32", False), ("split", True)])
@pytest.mark.parametrize("coherent", [False, True])
def test_emulated_arithmetic_is_inside_both_bounds(model, mode, split, coherent):
    h, xt, ref, absref, dims = model
    if coherent:
        xt = _coherent(xt)
        ref = h.apply_tree(xt)
        absref = bounds.absolute_hodbf(h).apply_tree(np.abs(xt))
    y = _emulate(h, xt, mode)
    ratio, col_ref, col_abs = bounds.check(y, ref, absref, dims, split)
    tol = bounds.normwise_tolerance(dims, split)
    assert ratio <= 1.0, ratio
    assert col_ref <= tol and col_abs <= tol, (col_ref, col_abs, tol)
    assert col_ref > 0  # the emulation does round


def test_dropped_cross_term_breaks_the_normwise_bound(model):
    h, xt, _, _, dims = model
    xt = _coherent(xt)
    ref = h.apply_tree(xt)
    absref = bounds.absolute_hodbf(h).apply_tree(np.abs(xt))
    y = _emulate(h, xt, "drop")
    _, col_ref, _ = bounds.check(y, ref, absref, dims, True)
    tol = bounds.normwise_tolerance(dims, True)
    assert col_ref > 2 * tol, (col_ref, tol)


def test_stage_dims_of_a_device_style_table_match_the_factors(model):
    """forward_stage_dims reads the same dimensions from a table laid out like the
    library's export (kind, hod level, node, ca, cb, butterfly level, a, b, m, n, off, lda)."""
    h, _, _, _, dims = model
    rows = []
    LH = h.tree.depth
    for i, d in enumerate(h.D):
        rows.append([0, LH, i, 0, 0, 0, 0, 0, d.shape[0], d.shape[1], 0, d.shape[0]])
    for (l, i), bf in h.bf.items():
        for b, v in enumerate(bf.V0):
            rows.append([1, l, i, 0, 0, 0, 0, b, v.shape[0], v.shape[1], 0, v.shape[0]])
        for lv in range(1, bf.L + 1):
            for a, row in enumerate(bf.W[lv]):
                for b, w in enumerate(row):
                    rows.append([2, l, i, 0, 0, lv, a, b, w.shape[0], w.shape[1], 0, w.shape[0]])
        for a, bb in enumerate(bf.B):
            rows.append([3, l, i, 0, 0, bf.L, a, 0, bb.shape[0], bb.shape[1], 0, bb.shape[0]])
    assert bounds.forward_stage_dims(np.array(rows, dtype=np.int64), LH) == dims

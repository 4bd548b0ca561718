"""Rounding-error bounds for GPU products re-applied by the oracle (test-side only).

A product computed as a chain of stages t_s = F_s t_{s-1} (x = t_0), each stage an
inner product of length n_s formed with rounding unit u per operation, satisfies to
first order, element by element,

    |y_hat - y| <= sum_s g_s * (|F_S| ... |F_1| |x|),     g_s = (2 n_s + 2) u

(the complex product is a real inner product of length 2 n_s; one more rounding stores
the stage output; errors of earlier stages pass through the later |F|).  With the
split-BF16 arithmetic every product is within 2^-15 (1 + 2^-7) |a| |x| of the exact one
(the per-product bound pinned on the CPU by tests/test_split_bf16_bound.py), so
g_s = 2^-15 (1 + 2^-7) + (2 n_s + 2) 2^-24.  The "abs chain" |F_S| ... |F_1| |x| is the
same oracle apply run on the absolute values of the exported factors and of x.

Besides this worst-case, element-wise bound, whose accumulation term grows like n_s u, a
norm-wise bound follows the usual probabilistic model (rounding errors of independent
operations add in quadrature): per stage 2^-15 (1 + 2^-7) for the split products plus
(2 sqrt(2 n_s) + 2) u for the FP32 accumulation, summed over the dependent stages and
doubled, relative to the column norm of the exact result (forward products, which do
not cancel much) or of the abs chain (the multiplicative preconditioner, which does).
"""
import copy

import numpy as np

from oracle.precond import DenseBlock

U32 = 2.0 ** -24
SPLIT = 2.0 ** -15 * (1 + 2.0 ** -7)


def bf16(v):
    """float32 -> the nearest bfloat16 value (ties to even), returned as float32."""
    u = np.asarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    return (((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)).astype(
        np.uint32).view(np.float32)


def coherent(x):
    """Inputs whose BF16 remainders are coherent: each real and imaginary part is a BF16
    value times (1 + 2^-9), exact in FP32, so its split is hi = that BF16 value and
    lo = 2^-9 hi.  A split product that dropped the hi_a lo_x term would then be off by
    2^-9 of the result, not by terms that average out."""
    hr, hi_ = bf16(x.real.astype(np.float32)), bf16(x.imag.astype(np.float32))
    f = np.float32(1 + 2.0 ** -9)
    return (hr * f).astype(np.float64) + 1j * (hi_ * f).astype(np.float64)


def _abs_bf(b):
    c = copy.copy(b)
    c.V0 = [np.abs(v) for v in b.V0]
    c.W = [None] + [[[np.abs(w) for w in row] for row in lev] for lev in b.W[1:]]
    c.B = [np.abs(v) for v in b.B]
    return c


def absolute_hodbf(h):
    """The same HODBF with every stored factor replaced by its absolute value."""
    c = copy.copy(h)
    c.D = [np.abs(d) for d in h.D]
    c.bf = {k: _abs_bf(b) for k, b in h.bf.items()}
    return c


def absolute_precond(p):
    """The same multiplicative form with |D^-1| and |X_tau| blocks (z += |X| z)."""
    c = copy.copy(p)
    c.Dinv = [np.abs(d) for d in p.Dinv]
    X = {}
    for key, blocks in p.X.items():
        X[key] = [[DenseBlock(np.abs(b.M)) if isinstance(b, DenseBlock) else _abs_bf(b)
                   for b in row] for row in blocks]
    c.X = X
    return c


def forward_stage_dims(table, depth):
    """Largest inner dimension of each dependent stage of the forward apply: V^0 (leaf
    columns), W^1 .. W^{L_H - 1} (r1 + r2), and the final per-leaf sum of the dense leaf
    block and every outer factor B^L covering the leaf."""
    t = np.asarray(table)
    dims = []
    v0 = t[t[:, 0] == 1]
    dims.append(int(v0[:, 9].max()) if len(v0) else 0)
    w = t[t[:, 0] == 2]
    for lev in range(1, depth):
        sel = w[w[:, 5] == lev]
        if len(sel):
            dims.append(int(sel[:, 9].max()))
    leaf_n = {}
    for row in t:
        kind, l, i = int(row[0]), int(row[1]), int(row[2])
        if kind == 0:
            leaf_n[i] = leaf_n.get(i, 0) + int(row[9])
        elif kind == 3:
            L = depth - l
            g = (i << L) + int(row[6])
            leaf_n[g] = leaf_n.get(g, 0) + int(row[9])
    dims.append(max(leaf_n.values()))
    return dims


def precond_stage_dims(table, depth):
    """Inner dimensions of the preconditioner's dependent stages: the dense first stage,
    then for each tree level (leaves towards the root) its X_tau butterflies' V^0, W and
    outer-factor stages, the last adding into z (one more term)."""
    t = np.asarray(table)
    dense = t[t[:, 0] == 0]
    dims = [int(dense[:, 9].max())]
    lb = int(dense[0, 1])
    for l in range(lb - 1, -1, -1):
        lv = t[(t[:, 1] == l) & (t[:, 0] != 0)]
        if not len(lv):
            continue
        L = depth - l - 1
        v0 = lv[lv[:, 0] == 1]
        dims.append(int(v0[:, 9].max()) if len(v0) else 0)
        for s in range(1, L + 1):
            sel = lv[(lv[:, 0] == 2) & (lv[:, 5] == s)]
            dims.append(int(sel[:, 9].max()) if len(sel) else 0)
        b = lv[lv[:, 0] == 3]
        # per output leaf: the outer blocks of the (up to) two butterflies covering it
        per = {}
        for row in b:
            key = (int(row[2]), int(row[3]), int(row[6]))
            per[key] = per.get(key, 0) + int(row[9])
        dims.append((max(per.values()) if per else 0) + 1)
    return dims


def worst_case_gamma(dims, split=False):
    """Sum over stages of the per-stage element-wise bound g_s (see the module text)."""
    return float(sum((SPLIT if split else 0.0) + (2 * n + 2) * U32 for n in dims))


def normwise_tolerance(dims, split=False, safety=2.0):
    """Norm-wise bound of the module text (probabilistic accumulation term)."""
    return float(safety * sum((SPLIT if split else 0.0) + (2 * np.sqrt(2 * n) + 2) * U32
                              for n in dims))


def check(y, ref, absref, dims, split=False):
    """(worst ratio of |y - ref| to its element-wise bound, worst column error relative to
    the exact column norm, worst column error relative to the abs-chain column norm)."""
    absref = np.real(absref)
    g = worst_case_gamma(dims, split)
    err = np.abs(y - ref)
    tiny = np.finfo(np.float64).tiny
    ratio = float(np.max(err / np.maximum(g * absref, tiny)))
    en = np.linalg.norm(err, axis=0)
    return (ratio, float(np.max(en / np.linalg.norm(ref, axis=0))),
            float(np.max(en / np.linalg.norm(absref, axis=0))))

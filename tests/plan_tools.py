"""Turn the library's exported factors into oracle butterflies (test-side glue only).

The oracle applies them with its own FP64 code, so a product-vs-oracle comparison
checks the library's arithmetic (exported factors) or host construction (probe).
"""
import numpy as np

from oracle import vie
from oracle.butterfly import HODBF, Butterfly
from oracle.precond import DenseBlock, Precond
from oracle.tree import Tree


def tree_from_perm(perm, n, depth):
    """Rebuild node ranges of a complete tree whose leaves split as the library does."""
    ranges = [[(0, n)]]
    for _ in range(depth):
        nxt = []
        for lo, hi in ranges[-1]:
            n1 = (hi - lo + 1) // 2
            nxt += [(lo, lo + n1), (lo + n1, hi)]
        ranges.append(nxt)
    return Tree(np.asarray(perm, dtype=np.int64), ranges)


def _mat(vals, off, m, n, lda=None):
    lda = m if not lda else lda
    cols = [np.asarray(vals[off + k * lda: off + k * lda + m], dtype=np.complex128) for k in range(n)]
    return np.stack(cols, axis=1) if n else np.zeros((m, 0), dtype=np.complex128)


def butterflies_from_table(tree, table, vals, skel=None, grid=None, precond=False):
    """Group table rows into oracle Butterfly objects keyed like the library's blocks."""
    LH = tree.depth
    groups = {}
    for row in table:
        kind, l, i, ca, cb, lev, a, b, m, n, off, lda = (int(v) for v in row)
        if kind == 0:
            continue
        groups.setdefault((l, i, ca, cb), []).append((kind, lev, a, b, m, n, off, lda))
    out = {}
    perm = tree.perm
    for (l, i, ca, cb), rows in groups.items():
        if precond:
            lev_bf, oi, si = l + 1, 2 * i + ca, 2 * i + cb
        else:
            lev_bf, oi, si = l, i, i ^ 1
        L = LH - lev_bf
        rr = [tree.node(LH, (oi << L) + a) for a in range(1 << L)]
        cr = [tree.node(LH, (si << L) + b) for b in range(1 << L)]
        V0 = [None] * (1 << L)
        W = [None] + [[[None] * (1 << (L - lv)) for _ in range(1 << lv)] for lv in range(1, L + 1)]
        B = [None] * (1 << L)
        # zero-rank factors are absent from device tables: default to empty matrices
        for kind, lev, a, b, m, n, off, lda in rows:
            if kind == 1:
                V0[b] = _mat(vals, off, m, n, lda)
            elif kind == 2:
                W[lev][a][b] = _mat(vals, off, m, n, lda)
            elif kind == 3:
                if skel is not None:
                    cols = skel[off:off + n]
                    lo, hi = rr[a]
                    B[a] = vie.entries(grid, perm[np.arange(lo, hi)], perm[cols])
                else:
                    B[a] = _mat(vals, off, m, n, lda)
        out[(l, i, ca, cb)] = (L, rr, cr, V0, W, B)
    return out


def fill_missing(L, rr, cr, V0, W, B):
    """Zero-rank blocks are not stored; rebuild consistent empty shapes."""
    for b in range(1 << L):
        if V0[b] is None:
            V0[b] = np.zeros((0, cr[b][1] - cr[b][0]), dtype=complex)
    ranks = [v.shape[0] for v in V0]
    for lv in range(1, L + 1):
        nb = 1 << (L - lv)
        new = []
        for a in range(1 << lv):
            for b in range(nb):
                cin = ranks[(a // 2) * 2 * nb + 2 * b] + ranks[(a // 2) * 2 * nb + 2 * b + 1]
                if W[lv][a][b] is None:
                    W[lv][a][b] = np.zeros((0, cin), dtype=complex)
                new.append(W[lv][a][b].shape[0])
        ranks = new
    for a in range(1 << L):
        if B[a] is None:
            B[a] = np.zeros((rr[a][1] - rr[a][0], ranks[a]), dtype=complex)
    return Butterfly(L, rr, cr, V0, W, B)


def hodbf_from_export(grid, perm, table, vals, skel=None):
    n = grid.n
    depth = int(round(np.log2(max(1, sum(1 for r in table if r[0] == 0))))) if skel is None else None
    if depth is None:
        # probe tables carry no dense rows: recover the depth from the largest hod level
        lv = [int(r[1]) for r in table]
        depth = max(lv) if lv else 0
    tree = tree_from_perm(perm, n, depth)
    LH = tree.depth
    if skel is None:
        D = [None] * (1 << LH)
        for row in table:
            if int(row[0]) == 0:
                D[int(row[2])] = _mat(vals, int(row[10]), int(row[8]), int(row[9]), int(row[11]))
    else:
        D = [vie.entries(grid, tree.perm[lo:hi], tree.perm[lo:hi]) for lo, hi in tree.ranges[LH]]
    groups = butterflies_from_table(tree, table, vals, skel, grid)
    bf = {}
    for (l, i, _, _), parts in groups.items():
        bf[(l, i)] = fill_missing(*parts)
    for l in range(1, LH + 1):  # blocks whose every factor has rank 0
        for i in range(1 << l):
            if (l, i) not in bf:
                L = LH - l
                rr = [tree.node(LH, (i << L) + a) for a in range(1 << L)]
                cr = [tree.node(LH, ((i ^ 1) << L) + b) for b in range(1 << L)]
                bf[(l, i)] = fill_missing(L, rr, cr, [None] * (1 << L),
                                          [None] + [[[None] * (1 << (L - v)) for _ in range(1 << v)]
                                                    for v in range(1, L + 1)], [None] * (1 << L))
    return HODBF(tree, D, bf)


class DenseBottomPrecond(Precond):
    """The multiplicative form started from the exported dense inverses of the level-lb
    nodes' diagonal blocks (the library's precond_dense_levels = L_H - lb), then the X_tau
    of the levels above, applied in FP64 like the oracle's own form."""

    def __init__(self, tree, lb, Dinv, X):
        super().__init__(tree, Dinv, X)
        self.lb = lb

    def apply_tree(self, xt):
        tr = self.tree
        z = np.empty_like(xt, dtype=np.complex128)
        for i, (lo, hi) in enumerate(tr.ranges[self.lb]):
            z[lo:hi] = self.Dinv[i] @ xt[lo:hi]
        for l in range(self.lb - 1, -1, -1):
            for i in range(1 << l):
                blocks = self.X[(l, i)]
                c = [tr.node(l + 1, 2 * i), tr.node(l + 1, 2 * i + 1)]
                zc = [z[lo:hi].copy() for (lo, hi) in c]
                for a in range(2):
                    lo, hi = c[a]
                    z[lo:hi] += blocks[a][0].apply(zc[0]) + blocks[a][1].apply(zc[1])
        return z


def precond_from_export(grid, perm, table, vals, depth):
    tree = tree_from_perm(perm, grid.n, depth)
    LH = tree.depth
    dense = [row for row in table if int(row[0]) == 0]
    lb = int(dense[0][1])  # level of the dense inverses (L_H: the leaves)
    Dinv = [None] * (1 << lb)
    for row in dense:
        assert int(row[1]) == lb
        Dinv[int(row[2])] = _mat(vals, int(row[10]), int(row[8]), int(row[9]), int(row[11]))
    groups = butterflies_from_table(tree, table, vals, precond=True)
    X = {}
    levels = sorted({k[0] for k in groups})
    for l in range(LH):
        for i in range(1 << l):
            blocks = []
            for ca in range(2):
                row = []
                for cb in range(2):
                    key = (l, i, ca, cb)
                    if key in groups:
                        row.append(fill_missing(*groups[key]))
                    else:
                        a_lo, a_hi = tree.node(l + 1, 2 * i + ca)
                        b_lo, b_hi = tree.node(l + 1, 2 * i + cb)
                        row.append(DenseBlock(np.zeros((a_hi - a_lo, b_hi - b_lo), dtype=complex)))
                blocks.append(row)
            X[(l, i)] = blocks
    del levels
    return Precond(tree, Dinv, X) if lb == LH else DenseBottomPrecond(tree, lb, Dinv, X)

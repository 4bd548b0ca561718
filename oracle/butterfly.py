"""Oracle: nested-ID butterflies and the HOD-BF operator (Section III-A). Test infrastructure only.

HOD-BF partition: D_tau = Z(tau, tau) is kept dense at every leaf tau of T_H; every
pair of siblings (tau1, tau2) at level l >= 1 gives two off-diagonal blocks
B_tau1 = Z(tau1, tau2) and B_tau2 = Z(tau2, tau1), each compressed as a butterfly
of L = L_H - l levels with row tree T_o (rooted at o) and column tree T_s.

Butterfly of B = Z(o, s), eqs. (ID), (nested_basis), (butterfly_mat):

* level 0: for every leaf nu of T_s, Z(o, nu) ~ Z(o, nubar) V_{o,nu};
* level l = 1..L: for tau at level l of T_o and nu at level L-l of T_s with children
  nu1, nu2, the transfer matrix W_{tau,nu} comes from the ID
  Z(tau, nubar) W_{tau,nu} ~ [Z(tau, nubar_1), Z(tau, nubar_2)], where nubar_i are the
  skeletons found for (p_tau, nu_i) one level up;
* B^L = diag(Z(tau, sbar_tau)) over the leaves tau of T_o.

Then Z(o, s) ~ B^L W^L ... W^1 V^0 and the product is applied right to left.  This
oracle uses every row of tau in each ID (no row sampling), the most accurate form of
eq. (ID).
"""
from __future__ import annotations

import numpy as np

from . import vie
from .idec import interp_decomp
from .tree import Tree, build_tree


class Butterfly:
    """Factors of one butterfly; rows/cols are tree-order position ranges.

    V0[b]       : r x |nu_b|           for leaf b of T_s
    W[l][a][b]  : r x (r1 + r2)        for tau index a at level l of T_o (l = 1..L),
                                        nu index b at level L - l of T_s
    B[a]        : |tau_a| x r          for leaf a of T_o
    row_ranges[a], col_ranges[b]: the leaf ranges of T_o and T_s.
    """

    def __init__(self, L, row_ranges, col_ranges, V0, W, B, skel=None):
        self.L = L
        self.row_ranges = row_ranges
        self.col_ranges = col_ranges
        self.V0 = V0
        self.W = W
        self.B = B
        self.skel = skel

    @property
    def shape(self):
        return (self.row_ranges[-1][1] - self.row_ranges[0][0],
                self.col_ranges[-1][1] - self.col_ranges[0][0])

    def ranks(self):
        out = [m.shape[0] for m in self.V0]
        for lev in self.W[1:]:
            for row in lev:
                out.extend(m.shape[0] for m in row)
        return out

    def stored_entries(self) -> int:
        n = sum(m.size for m in self.V0) + sum(m.size for m in self.B)
        for lev in self.W[1:]:
            for row in lev:
                n += sum(m.size for m in row)
        return n

    def apply(self, x: np.ndarray) -> np.ndarray:
        """y = B^L W^L ... W^1 V^0 x for x of shape (|s|, R) in local column order."""
        c0 = self.col_ranges[0][0]
        r0 = self.row_ranges[0][0]
        t = {}
        for b, (lo, hi) in enumerate(self.col_ranges):
            t[(0, b)] = self.V0[b] @ x[lo - c0:hi - c0]
        for l in range(1, self.L + 1):
            nt = {}
            for a in range(1 << l):
                for b in range(1 << (self.L - l)):
                    u = np.vstack([t[(a // 2, 2 * b)], t[(a // 2, 2 * b + 1)]])
                    nt[(a, b)] = self.W[l][a][b] @ u
            t = nt
        y = np.zeros((self.shape[0], x.shape[1]), dtype=np.complex128)
        for a, (lo, hi) in enumerate(self.row_ranges):
            y[lo - r0:hi - r0] = self.B[a] @ t[(a, 0)]
        return y

    def factor_matrices(self):
        """The factors of eq. (butterfly_mat) as explicit (block-sparse) dense matrices.

        Intermediate vectors at level l are ordered tau-major, nu-minor.  Returns
        [V^0, W^1, ..., W^L, B^L]; their right-to-left product is the block.
        """
        m, n = self.shape
        c0 = self.col_ranges[0][0]
        r0 = self.row_ranges[0][0]
        # offsets of every (a, b) segment per level
        offs = []
        sizes0 = [v.shape[0] for v in self.V0]
        offs.append(np.concatenate([[0], np.cumsum(sizes0)]))
        lev_sizes = [sizes0]
        for l in range(1, self.L + 1):
            sz = [self.W[l][a][b].shape[0] for a in range(1 << l) for b in range(1 << (self.L - l))]
            lev_sizes.append(sz)
            offs.append(np.concatenate([[0], np.cumsum(sz)]))
        mats = []
        V = np.zeros((offs[0][-1], n), dtype=np.complex128)
        for b, (lo, hi) in enumerate(self.col_ranges):
            V[offs[0][b]:offs[0][b + 1], lo - c0:hi - c0] = self.V0[b]
        mats.append(V)
        for l in range(1, self.L + 1):
            nb_prev = 1 << (self.L - l + 1)
            nb = 1 << (self.L - l)
            Wm = np.zeros((offs[l][-1], offs[l - 1][-1]), dtype=np.complex128)
            for a in range(1 << l):
                for b in range(nb):
                    row = a * nb + b
                    p = a // 2
                    c1 = p * nb_prev + 2 * b
                    cols = np.r_[offs[l - 1][c1]:offs[l - 1][c1 + 1], offs[l - 1][c1 + 1]:offs[l - 1][c1 + 2]]
                    Wm[offs[l][row]:offs[l][row + 1], cols] = self.W[l][a][b]
            mats.append(Wm)
        Bm = np.zeros((m, offs[self.L][-1]), dtype=np.complex128)
        for a, (lo, hi) in enumerate(self.row_ranges):
            Bm[lo - r0:hi - r0, offs[self.L][a]:offs[self.L][a + 1]] = self.B[a]
        mats.append(Bm)
        return mats


def build_butterfly(entry, tree: Tree, level: int, oi: int, si: int, L: int, chi: float) -> Butterfly:
    """Compress entry(rows, cols) on o = node(level, oi), s = node(level, si) with L levels.

    ``entry`` maps two arrays of tree positions to the dense sub-block.
    """
    leaf_level = level + L
    row_ranges = [tree.node(leaf_level, oi * (1 << L) + a) for a in range(1 << L)]
    col_ranges = [tree.node(leaf_level, si * (1 << L) + b) for b in range(1 << L)]
    o_lo, o_hi = tree.node(level, oi)
    rows_o = np.arange(o_lo, o_hi)
    skel = {}
    V0 = []
    for b, (lo, hi) in enumerate(col_ranges):
        nu = np.arange(lo, hi)
        J, V = interp_decomp(entry(rows_o, nu), chi)
        skel[(0, b)] = nu[J]
        V0.append(V)
    W = [None]
    for l in range(1, L + 1):
        nskel = {}
        lev = []
        for a in range(1 << l):
            t_lo, t_hi = tree.node(level + l, oi * (1 << l) + a)
            rows = np.arange(t_lo, t_hi)
            row_w = []
            for b in range(1 << (L - l)):
                cols = np.concatenate([skel[(a // 2, 2 * b)], skel[(a // 2, 2 * b + 1)]])
                J, V = interp_decomp(entry(rows, cols), chi)
                nskel[(a, b)] = cols[J]
                row_w.append(V)
            lev.append(row_w)
        W.append(lev)
        skel = nskel
    B = []
    for a, (lo, hi) in enumerate(row_ranges):
        B.append(entry(np.arange(lo, hi), skel[(a, 0)]))
    return Butterfly(L, row_ranges, col_ranges, V0, W, B, skel)


class HODBF:
    """Dense leaves D[i] plus butterflies bf[(l, i)] for the block (node i, node i^1) at level l."""

    def __init__(self, tree: Tree, D, bf):
        self.tree = tree
        self.D = D
        self.bf = bf

    @property
    def n(self):
        return len(self.tree.perm)

    def apply_tree(self, xt: np.ndarray) -> np.ndarray:
        """y = Z_con x with x, y in tree order, shape (N, R)."""
        tr = self.tree
        LH = tr.depth
        y = np.zeros_like(xt, dtype=np.complex128)
        for i, (lo, hi) in enumerate(tr.ranges[LH]):
            y[lo:hi] += self.D[i] @ xt[lo:hi]
        for (l, i), bf in self.bf.items():
            o_lo, o_hi = tr.node(l, i)
            s_lo, s_hi = tr.node(l, i ^ 1)
            y[o_lo:o_hi] += bf.apply(xt[s_lo:s_hi])
        return y

    def apply(self, x: np.ndarray) -> np.ndarray:
        """y = Z_con x in user order; x has shape (N,) or (N, R)."""
        x2 = x.reshape(self.n, -1)
        perm = self.tree.perm
        yt = self.apply_tree(x2[perm])
        y = np.empty_like(yt)
        y[perm] = yt
        return y.reshape(x.shape)

    def stored_entries(self) -> int:
        return sum(d.size for d in self.D) + sum(b.stored_entries() for b in self.bf.values())

    def max_rank(self) -> int:
        return max([0] + [max(b.ranks() or [0]) for b in self.bf.values()])


def build_hodbf(grid, chi: float, leaf_size: int = 64, tree: Tree | None = None) -> HODBF:
    """HOD-BF compression of the voxel system matrix with full-row IDs at tolerance chi."""
    tree = tree if tree is not None else build_tree(grid, leaf_size)
    perm = tree.perm

    def entry(r, c):
        return vie.entries(grid, perm[r], perm[c])

    LH = tree.depth
    D = [entry(np.arange(lo, hi), np.arange(lo, hi)) for (lo, hi) in tree.ranges[LH]]
    bf = {}
    for l in range(1, LH + 1):
        for i in range(1 << l):
            bf[(l, i)] = build_butterfly(entry, tree, l, i, i ^ 1, LH - l, chi)
    return HODBF(tree, D, bf)

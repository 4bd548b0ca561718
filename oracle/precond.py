"""Oracle: the HOD-BF approximate inverse in multiplicative form (Section III-B). Test infrastructure only.

Algorithm 1 writes, for a non-leaf tau with children tau1, tau2,
    D_tau = [D_tau1, B_tau1; B_tau2, D_tau2] = diag(D_tau1, D_tau2) A_tau,
    A_tau = [I, D_tau1^{-1} B_tau1; D_tau2^{-1} B_tau2, I],
    D_tau^{-1} = A_tau^{-1} diag(D_tau1^{-1}, D_tau2^{-1}),
and Algorithm 2 returns A_tau^{-1} - I =: X_tau as a butterfly.  Unrolled from the
leaves to the root this gives
    Z^{-1} = (I + X_root) diag over level 1 of (I + X_tau) ... diag over leaves of D_tau^{-1}.

The paper reaches X_tau with randomized butterfly reconstruction (BF_random_matvec)
and the butterfly Sherman-Morrison-Woodbury recursion (BF_SMW).  This oracle computes
the same object by its plain definition instead, which is feasible on small grids:
X_tau = D_tau^{-1} diag(D_tau1, D_tau2) - I from exact dense inverses of the
diagonal blocks of Z, then compresses each of its four child blocks X_tau(tau_i, tau_j)
as a butterfly with L_H - l - 1 levels (row tree T_tau_i, column tree T_tau_j) by
full-row nested IDs at chi_fact.  Leaves keep D_tau^{-1} dense.

Parity: with dense (uncompressed) X_tau the product equals Z^{-1} to rounding (pinned
by a test).  The compressed factors are tolerance-dependent and not unique, so only
products of this preconditioner are pinned (P Z ~ I to O(chi_fact), P -> Z^{-1} as
chi_fact -> 0); the factors themselves are "parity unpinned".
"""
from __future__ import annotations

import numpy as np

from . import vie
from .butterfly import build_butterfly
from .tree import Tree, build_tree


class DenseBlock:
    def __init__(self, M):
        self.M = M

    def apply(self, x):
        return self.M @ x

    def stored_entries(self):
        return self.M.size


class Precond:
    """Dinv[i]: dense inverse of leaf i; X[(l, i)][a][b]: block (child a, child b) of X_tau."""

    def __init__(self, tree: Tree, Dinv, X):
        self.tree = tree
        self.Dinv = Dinv
        self.X = X

    @property
    def n(self):
        return len(self.tree.perm)

    def apply_tree(self, xt: np.ndarray) -> np.ndarray:
        tr = self.tree
        LH = tr.depth
        z = np.empty_like(xt, dtype=np.complex128)
        for i, (lo, hi) in enumerate(tr.ranges[LH]):
            z[lo:hi] = self.Dinv[i] @ xt[lo:hi]
        for l in range(LH - 1, -1, -1):
            for i in range(1 << l):
                blocks = self.X[(l, i)]
                c = [tr.node(l + 1, 2 * i), tr.node(l + 1, 2 * i + 1)]
                zc = [z[lo:hi].copy() for (lo, hi) in c]
                for a in range(2):
                    lo, hi = c[a]
                    z[lo:hi] += blocks[a][0].apply(zc[0]) + blocks[a][1].apply(zc[1])
        return z

    def apply(self, x: np.ndarray) -> np.ndarray:
        x2 = x.reshape(self.n, -1)
        perm = self.tree.perm
        zt = self.apply_tree(x2[perm])
        z = np.empty_like(zt)
        z[perm] = zt
        return z.reshape(x.shape)

    def stored_entries(self) -> int:
        n = sum(d.size for d in self.Dinv)
        for blocks in self.X.values():
            n += sum(b.stored_entries() for row in blocks for b in row)
        return n


def build_precond(grid, chi_fact: float, leaf_size: int = 64, tree: Tree | None = None,
                  compress: bool = True) -> Precond:
    """Multiplicative-form inverse; compress=False keeps every X_tau block dense."""
    tree = tree if tree is not None else build_tree(grid, leaf_size)
    perm = tree.perm
    Zt = vie.entries(grid, perm, perm)  # dense, tree order
    LH = tree.depth
    Dinv = [np.linalg.inv(Zt[lo:hi, lo:hi]) for (lo, hi) in tree.ranges[LH]]
    X = {}
    for l in range(LH - 1, -1, -1):
        for i in range(1 << l):
            lo, hi = tree.node(l, i)
            inv_tau = np.linalg.inv(Zt[lo:hi, lo:hi])
            diag = np.zeros_like(inv_tau)
            kids = [tree.node(l + 1, 2 * i), tree.node(l + 1, 2 * i + 1)]
            for (clo, chi_) in kids:
                diag[clo - lo:chi_ - lo, clo - lo:chi_ - lo] = Zt[clo:chi_, clo:chi_]
            Xt = inv_tau @ diag - np.eye(hi - lo)

            def entry(r, c, Xt=Xt, lo=lo):
                return Xt[np.ix_(r - lo, c - lo)]

            blocks = []
            for a in range(2):
                row = []
                for b in range(2):
                    if compress:
                        row.append(build_butterfly(entry, tree, l + 1, 2 * i + a, 2 * i + b,
                                                   LH - l - 1, chi_fact))
                    else:
                        (alo, ahi), (blo, bhi) = kids[a], kids[b]
                        row.append(DenseBlock(Xt[alo - lo:ahi - lo, blo - lo:bhi - lo]))
                blocks.append(row)
            X[(l, i)] = blocks
    return Precond(tree, Dinv, X)

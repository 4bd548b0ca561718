"""Oracle: the cluster tree T_H by recursive KD bisection (Section III-A). Test infrastructure only.

Reading of the paper's "tree clustering (such as KD) ... approximately equal numbers
of unknowns ... until the subscatterer contains a prescribed number of unknowns":

* a node is split along the axis of largest extent of its voxel centres, ties going
  to x before y before z;
* the ceil(n/2) members with the smallest coordinate along that axis (ties broken by
  position in the parent) form the first child, the rest the second; both children
  keep the parent's relative order (a stable partition);
* every node is split to the same depth L_H, the smallest L with
  ceil(N / 2^L) <= leaf_size, so T_H is a complete binary tree (a node with fewer
  than 2 members cannot split; such grids are rejected).

Tree order lists the leaves left to right; every node is then a contiguous range.
"""
from __future__ import annotations

import numpy as np

from .vie import voxel_index


def depth_for(n: int, leaf_size: int) -> int:
    """Smallest L with ceil(n / 2^L) <= leaf_size."""
    L = 0
    while -(-n // (1 << L)) > leaf_size:
        L += 1
    return L


class Tree:
    """perm[tree position] = user index; ranges[l][i] = (lo, hi) of node i at level l."""

    def __init__(self, perm: np.ndarray, ranges: list):
        self.perm = perm
        self.ranges = ranges
        self.depth = len(ranges) - 1

    def node(self, level: int, i: int):
        return self.ranges[level][i]

    def size(self, level: int, i: int) -> int:
        lo, hi = self.ranges[level][i]
        return hi - lo


def build_tree(grid, leaf_size: int = 64) -> Tree:
    n = grid.n
    if n <= 0:
        raise ValueError("empty grid")
    L = depth_for(n, leaf_size)
    if L > 0 and n < (1 << L):
        raise ValueError("grid too small to split to a complete tree")
    coords = voxel_index(grid, np.arange(n)).astype(np.float64)
    levels = [[np.arange(n)]]
    for _ in range(L):
        nxt = []
        for members in levels[-1]:
            c = coords[members]
            ext = c.max(axis=0) - c.min(axis=0)
            axis = int(np.argmax(ext))  # argmax returns the first maximum: x < y < z
            order = np.argsort(c[:, axis], kind="stable")
            n1 = -(-len(members) // 2)
            first = np.zeros(len(members), dtype=bool)
            first[order[:n1]] = True  # stable partition: both halves keep parent order
            nxt.append(members[first])
            nxt.append(members[~first])
        levels.append(nxt)
    perm = np.concatenate(levels[-1])
    # each level's nodes, concatenated left to right, is a permutation of perm's order
    ranges = []
    for lev in levels:
        lo = 0
        rr = []
        for members in lev:
            rr.append((lo, lo + len(members)))
            lo += len(members)
        ranges.append(rr)
    # sanity: the node at level l covers exactly its leaves' members
    for l, lev in enumerate(levels):
        for i, members in enumerate(lev):
            lo, hi = ranges[l][i]
            assert np.array_equal(np.sort(perm[lo:hi]), np.sort(members))
    return Tree(perm, ranges)


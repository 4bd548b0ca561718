"""Pins for the oracle's KD cluster tree and interpolative decomposition (Section III-A)."""
import os

import numpy as np
import pytest

from oracle.idec import interp_decomp
from oracle.tree import build_tree, depth_for
from synth.workloads import make_grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def morton_position(ix, iy, iz, bits):
    """Closed form for 2^b cubes, leaf 4x4x4: leaf = interleave(bx, by, bz) with x the
    most significant bit at every level, then x-fastest order inside the brick."""
    bx, by, bz = ix >> 2, iy >> 2, iz >> 2
    leaf = 0
    for j in range(bits - 3, -1, -1):
        leaf = (leaf << 3) | (((bx >> j) & 1) << 2) | (((by >> j) & 1) << 1) | ((bz >> j) & 1)
    return leaf * 64 + (ix & 3) + 4 * (iy & 3) + 16 * (iz & 3)


@pytest.mark.parametrize("side", [8, 16])
def test_kd_tree_equals_morton_closed_form(side):
    g = make_grid(side, side, side, 1.0 / side, 2.0)
    tr = build_tree(g, 64)
    bits = side.bit_length() - 1
    n = g.n
    idx = np.arange(n)
    ix, iy, iz = idx % side, (idx // side) % side, idx // (side * side)
    pos = morton_position(ix, iy, iz, bits)
    expect = np.empty(n, dtype=np.int64)
    expect[pos] = idx
    assert np.array_equal(tr.perm, expect)
    assert tr.depth == 3 * (bits - 2)


def test_kd_golden_leaf_order_8cube():
    rows = np.loadtxt(os.path.join(GOLDEN, "kd_8cube_leaf_order.txt"), dtype=int)
    g = make_grid(8, 8, 8, 0.125, 2.0)
    tr = build_tree(g, 64)
    for leaf, (lo, hi) in enumerate(tr.ranges[tr.depth]):
        first = tr.perm[lo]
        ix, iy, iz = first % 8, (first // 8) % 8, first // 64
        assert (ix // 4, iy // 4, iz // 4) == tuple(rows[leaf])


def test_ragged_tree_structure():
    g = make_grid(12, 10, 9, 0.1, 2.0)
    tr = build_tree(g, 64)
    assert tr.depth == depth_for(g.n, 64) == 5
    assert sorted(tr.perm) == list(range(g.n))
    for l in range(tr.depth + 1):
        sizes = [hi - lo for lo, hi in tr.ranges[l]]
        assert len(sizes) == 1 << l and max(sizes) - min(sizes) <= 1
        if l < tr.depth:
            for i, (lo, hi) in enumerate(tr.ranges[l]):
                assert tr.ranges[l + 1][2 * i] == (lo, tr.ranges[l + 1][2 * i][1])
                assert tr.ranges[l + 1][2 * i + 1][1] == hi
    assert max(hi - lo for lo, hi in tr.ranges[tr.depth]) <= 64
    # children of the root are separated by a plane along the longest (x) axis
    lo, hi = tr.ranges[1][0]
    xs_first = tr.perm[lo:hi] % 12
    xs_second = tr.perm[hi:] % 12
    assert xs_first.max() <= xs_second.min()


def test_single_leaf_tree():
    g = make_grid(4, 4, 4, 0.1, 2.0)
    tr = build_tree(g, 64)
    assert tr.depth == 0 and list(tr.perm) == list(range(64))


def _rand(rng, m, n):
    return rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))


def test_id_invariants_and_error_bound():
    rng = np.random.default_rng(1)
    # numerically low-rank matrix with geometrically decaying spectrum
    U, _ = np.linalg.qr(_rand(rng, 80, 40))
    W, _ = np.linalg.qr(_rand(rng, 60, 40))
    s = 10.0 ** (-np.arange(40) / 4.0)
    M = (U * s) @ W.conj().T
    for chi in [1e-2, 1e-4, 1e-8]:
        J, V = interp_decomp(M, chi)
        r = len(J)
        assert np.allclose(V[:, J], np.eye(r), atol=1e-12)  # V(:, J) = I
        err = np.linalg.norm(M - M[:, J] @ V) / np.linalg.norm(M)
        assert err <= chi * (1 + 1e-10)
        # no ID of rank r can beat the truncated SVD, so r >= the chi-rank of the spectrum
        tails = np.sqrt(np.cumsum((s**2)[::-1]))[::-1] / np.linalg.norm(s)
        svd_rank = int(np.argmax(np.append(tails, 0.0) <= chi))
        assert r >= svd_rank


def test_id_exact_rank_and_zero():
    rng = np.random.default_rng(2)
    for r in [1, 5, 13]:
        M = _rand(rng, 40, r) @ _rand(rng, r, 30)
        J, V = interp_decomp(M, 1e-10)
        assert len(J) == r
        assert np.linalg.norm(M - M[:, J] @ V) <= 1e-10 * np.linalg.norm(M)
    J, V = interp_decomp(np.zeros((10, 7), dtype=complex), 1e-4)
    assert len(J) == 0 and V.shape == (0, 7)
    # a wide matrix: rank is capped by the row count
    M = _rand(rng, 6, 20)
    J, V = interp_decomp(M, 1e-12)
    assert len(J) == 6

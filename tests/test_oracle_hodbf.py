"""Pins for the oracle's nested-ID butterflies and HOD-BF operator (Section III-A)."""
import numpy as np
import pytest

from oracle import butterfly, vie
from oracle.idec import interp_decomp
from oracle.tree import build_tree
from synth.workloads import make_grid, small_case


@pytest.fixture(scope="module")
def ragged():
    c = small_case(11, sides=(12, 10, 9), h=0.1, eps_range=(2.0, 10.0), loss=1.0)
    g = c["grid"]
    return c, g, vie.dense(g)


@pytest.fixture(scope="module")
def ragged_op(ragged):
    c, g, Z = ragged
    return butterfly.build_hodbf(g, 1e-4)


def test_hodbf_product_within_ten_chi(ragged, ragged_op):
    c, g, Z = ragged
    x = c["x"]
    y = Z @ x
    err = np.linalg.norm(ragged_op.apply(x) - y, axis=0) / np.linalg.norm(y, axis=0)
    assert np.all(err <= 1e-3), err


def test_hodbf_tighter_tolerance_tightens_error(ragged):
    c, g, Z = ragged
    x = c["x"][:, :1]
    op = butterfly.build_hodbf(g, 1e-7)
    y = Z @ x
    assert np.linalg.norm(op.apply(x) - y) <= 1e-6 * np.linalg.norm(y)


def test_butterfly_factor_chain_equals_apply(ragged, ragged_op):
    # eq. (butterfly_mat): the literal product of block-sparse factors equals the apply
    tr = ragged_op.tree
    for key in [(1, 0), (2, 3), (tr.depth - 1, 1), (tr.depth, 6)]:
        bf = ragged_op.bf[key]
        mats = bf.factor_matrices()
        assert len(mats) == bf.L + 2
        prod = mats[0]
        for m in mats[1:]:
            prod = m @ prod
        eye = np.eye(bf.shape[1], dtype=complex)
        assert np.allclose(prod, bf.apply(eye), atol=1e-12)
        # 2^L blocks per factor
        assert len(bf.V0) == len(bf.B) == 1 << bf.L
        for l in range(1, bf.L + 1):
            assert sum(len(r) for r in bf.W[l]) == 1 << bf.L


def test_leaf_level_block_is_plain_id(ragged, ragged_op):
    c, g, Z = ragged
    tr = ragged_op.tree
    LH = tr.depth
    bf = ragged_op.bf[(LH, 4)]
    assert bf.L == 0
    (olo, ohi), (slo, shi) = tr.node(LH, 4), tr.node(LH, 5)
    perm = tr.perm
    M = Z[np.ix_(perm[olo:ohi], perm[slo:shi])]
    J, V = interp_decomp(M, 1e-4)
    assert np.allclose(bf.B[0] @ bf.V0[0], M[:, J] @ V, atol=1e-13)


def test_single_leaf_grid_is_dense():
    c = small_case(5, sides=(4, 4, 3))
    g = c["grid"]
    op = butterfly.build_hodbf(g, 1e-4)
    assert op.tree.depth == 0 and not op.bf
    assert np.allclose(op.apply(c["x"]), vie.dense(g) @ c["x"], atol=1e-14)


def test_free_space_gives_identity():
    g = make_grid(8, 8, 8, 0.125, 1.0)
    op = butterfly.build_hodbf(g, 1e-4)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((g.n, 2)) + 0j
    assert np.array_equal(op.apply(x), x)
    assert op.max_rank() == 0


def test_planted_transfer_mistake_is_caught(ragged, ragged_op):
    # swapping the two child segments feeding one transfer matrix must break the product
    import copy
    c, g, Z = ragged
    op = copy.deepcopy(ragged_op)
    bf = op.bf[(1, 0)]
    W = bf.W[2][1][0]
    cols = W.shape[1]
    bf.W[2][1][0] = np.roll(W, cols // 2, axis=1)
    x = c["x"][:, :1]
    y = Z @ x
    assert np.linalg.norm(op.apply(x) - y) > 1e-3 * np.linalg.norm(y)


def test_c1_operator_error_and_memory():
    from synth import config
    cfg = config("c1_plain_16")
    g = cfg["grid"]
    tr = build_tree(g, 64)
    op = butterfly.build_hodbf(g, cfg["tol"], tree=tr)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(g.n) + 1j * rng.standard_normal(g.n)
    y = vie.fft_matvec(g, x)
    assert np.linalg.norm(op.apply(x) - y) <= 10 * cfg["tol"] * np.linalg.norm(y)
    # compression: fewer stored entries than the dense N^2
    assert op.stored_entries() < 0.3 * g.n * g.n

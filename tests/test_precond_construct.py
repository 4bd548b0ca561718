"""The library's preconditioner construction (Algorithm 1 with the butterfly
Sherman-Morrison-Woodbury recursion of Algorithm 2, every new butterfly reconstructed
from products with structured random vectors), run on the host through
hodbf_precond_probe (complex FP64, no GPU) and checked against the oracle:

* chi -> 0 (compression and factorization at 1e-10): P is Z^{-1} up to the FP32 storage
  of its factors, and equals the oracle's multiplicative inverse (Algorithm 1 computed
  densely) to the same level;
* at chi_fact = 1e-2 and 1e-4 on a ragged grid: ||P Z x - x|| is of the size of the
  oracle's own (the same tolerance gives the same quality), and P differs from the
  oracle's P by O(chi_fact);
* run through the device path's packed programs (forward and transposed, leaves above
  the tree's for the recursion's coarser butterflies) by a host interpreter of their
  descriptors, the same results;
* the number of reconstructions is what the recursion of Algorithm 2 predicts (one for
  line 7 of Algorithm 1 per level, then per BF_SMW call: A22^{-1}, the Schur update
  and A11^{-1} recursively, and the final product);
* started from the dense inverses of larger nodes (precond_dense_levels), those blocks
  are the inverses of the diagonal blocks of the dense operator, only the levels above
  them are reconstructed, and the preconditioner is no worse."""
import numpy as np
import pytest

from oracle import precond as oprecond
from oracle import vie
from synth.workloads import small_case

_lib = pytest.importorskip("paper_2111_01730_amd._lib")


def _probe(g, chi_con, chi_fact, seed=1, programs=False, dense=0):
    """programs: run every product through the device path's packed grouped-GEMM
    programs (forward and transposed), interpreted on the host.  dense: the recursion
    starts from the dense inverses of the nodes that many levels above the leaves."""
    from tests.plan_tools import precond_from_export
    p = _lib.make_params(g, chi_con, chi_fact, precond_prec=1, seed=seed,
                         precond_dense_levels=dense)
    o = 16 if programs else 0
    perm = _lib.probe(p, 0 + o, np.int32, "hodbf_precond_probe")
    tab = _lib.probe(p, 3 + o, np.int64, "hodbf_precond_probe").reshape(-1, 12)
    vals = _lib.probe(p, 4 + o, np.complex128, "hodbf_precond_probe")
    stats = _lib.probe(p, 7 + o, np.int64, "hodbf_precond_probe")
    from oracle.tree import depth_for
    lb = int(tab[tab[:, 0] == 0][0, 1])  # level of the dense inverses
    return precond_from_export(g, perm, tab, vals, depth_for(g.n, 64)), stats, lb


def _rel(a, b):
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


@pytest.mark.parametrize("programs", [False, True])
def test_tight_tolerances_give_the_inverse(programs):
    c = small_case(61, sides=(8, 8, 8), h=0.1, eps_range=(2.0, 6.0), loss=0.3, nrhs=4)
    g = c["grid"]
    P, stats, _ = _probe(g, 1e-10, 1e-10, programs=programs)
    Z = vie.dense(g)
    x = c["x"]
    assert np.all(_rel(P.apply(Z @ x), x) <= 1e-6)  # FP32 storage of the factors
    po = oprecond.build_precond(g, 1e-10)
    assert np.all(_rel(P.apply(x), po.apply(x)) <= 1e-6)


@pytest.fixture(scope="module")
def ragged():
    c = small_case(61, sides=(10, 9, 8), h=0.1, eps_range=(2.0, 8.0), loss=0.5, nrhs=6)
    return c, vie.dense(c["grid"])


@pytest.mark.parametrize("chi_fact,programs", [(1e-2, False), (1e-4, False), (1e-2, True)])
def test_quality_matches_the_oracle(ragged, chi_fact, programs):
    c, Z = ragged
    g = c["grid"]
    P, _, _ = _probe(g, 1e-6, chi_fact, programs=programs)
    x = c["x"]
    po = oprecond.build_precond(g, chi_fact)
    mine = _rel(P.apply(Z @ x), x).max()
    theirs = _rel(po.apply(Z @ x), x).max()
    assert mine <= 3 * theirs, (mine, theirs)
    # both approximate Z^{-1} to O(chi_fact) times the amplification of this grid
    assert np.all(_rel(P.apply(x), po.apply(x)) <= 30 * chi_fact)


def _predicted_reconstructions(depth, top=None):
    def smw(lc, has22):
        return inv(lc, has22) + inv(lc, True) + 1

    def inv(lc, present):
        if not present:
            return 0
        if lc - 2 < 0:
            return 1
        return 1 + smw(lc - 2, True)

    return sum(1 + smw(depth - l - 1, False) for l in range(depth if top is None else top))


@pytest.mark.parametrize("sides", [(8, 8, 8), (10, 9, 8), (16, 16, 8)])
def test_reconstruction_count_follows_algorithm_2(sides):
    c = small_case(7, sides=sides, h=0.1, eps_range=(2.0, 4.0), loss=0.1, nrhs=1)
    _, stats, depth = _probe(c["grid"], 1e-4, 1e-2)
    assert int(stats[0]) == _predicted_reconstructions(depth)
    assert _predicted_reconstructions(3) == 12 and _predicted_reconstructions(4) == 18


def test_dense_bottom_levels(ragged):
    c, Z = ragged
    g = c["grid"]
    P0, _, depth = _probe(g, 1e-6, 1e-2)
    P, stats, lb = _probe(g, 1e-6, 1e-2, dense=2)
    assert lb == depth - 2
    # the recursion's leaves: inverses of Z(tau, tau) in tree order (FP32 storage)
    Zt = Z[np.ix_(P.tree.perm, P.tree.perm)]
    for i, (lo, hi) in enumerate(P.tree.ranges[lb]):
        inv = np.linalg.inv(Zt[lo:hi, lo:hi])
        assert np.linalg.norm(P.Dinv[i] - inv) <= 1e-6 * np.linalg.norm(inv)
    # only the levels above them are built by Algorithm 1
    assert int(stats[0]) == _predicted_reconstructions(depth, top=lb)
    x = c["x"]
    assert _rel(P.apply(Z @ x), x).max() <= _rel(P0.apply(Z @ x), x).max()
    # d = L_H: the root's dense inverse, Z^{-1} to FP32 storage
    Pr, stats_r, lr = _probe(g, 1e-6, 1e-2, dense=depth)
    assert lr == 0 and int(stats_r[0]) == 0
    assert np.all(_rel(Pr.apply(Z @ x), x) <= 1e-5)

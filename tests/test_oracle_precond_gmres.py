"""Pins for the oracle's multiplicative inverse (Algorithm 1 form) and its FGMRES / LU solvers."""
import numpy as np
import pytest

from oracle import butterfly, gmres, precond, vie
from synth.workloads import make_grid, small_case


@pytest.fixture(scope="module")
def case():
    c = small_case(21, sides=(10, 9, 8), h=0.1, eps_range=(2.0, 8.0), loss=0.5)
    g = c["grid"]
    return c, g, vie.dense(g)


def test_uncompressed_multiplicative_form_is_exact_inverse(case):
    c, g, Z = case
    p = precond.build_precond(g, 0.1, compress=False)
    x = c["x"]
    assert np.linalg.norm(p.apply(Z @ x) - x) <= 1e-11 * np.linalg.norm(x)
    assert np.linalg.norm(Z @ p.apply(x) - x) <= 1e-11 * np.linalg.norm(x)


def test_tight_fact_tolerance_approaches_inverse(case):
    c, g, Z = case
    p = precond.build_precond(g, 1e-9)
    x = c["x"]
    assert np.linalg.norm(p.apply(Z @ x) - x) <= 1e-6 * np.linalg.norm(x)


def test_loose_fact_tolerance_still_preconditions(case):
    c, g, Z = case
    p = precond.build_precond(g, 1e-2)
    x = c["x"]
    assert np.linalg.norm(p.apply(Z @ x) - x) <= 0.3 * np.linalg.norm(x)
    b = vie.plane_wave(g, c["dirs"])[:, 0]
    A = lambda v: Z @ v
    _, it_p, conv_p, _ = gmres.fgmres(A, b, p.apply, tol=1e-6)
    _, it_n, conv_n, _ = gmres.fgmres(A, b, None, tol=1e-6, max_iter=400)
    assert conv_p and it_p <= 12
    assert it_n > 3 * it_p


def test_fgmres_matches_lu_and_history_monotone(case):
    c, g, Z = case
    b = vie.plane_wave(g, c["dirs"])[:, 1]
    xs = gmres.lu_solve(Z, b)
    x, it, conv, hist = gmres.fgmres(lambda v: Z @ v, b, None, tol=1e-10, restart=400, max_iter=1000)
    assert conv
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
    assert np.linalg.norm(Z @ xs - b) <= 1e-12 * np.linalg.norm(b)
    # full (unrestarted) GMRES residual is non-increasing
    assert all(b2 <= b1 * (1 + 1e-12) for b1, b2 in zip(hist, hist[1:]))


def test_fgmres_exact_preconditioner_one_step(case):
    c, g, Z = case
    b = vie.plane_wave(g, c["dirs"])[:, 2]
    Zi = np.linalg.inv(Z)
    x, it, conv, _ = gmres.fgmres(lambda v: Z @ v, b, lambda v: Zi @ v, tol=1e-10)
    assert conv and it == 1


def test_fgmres_identity_operator():
    g = make_grid(4, 4, 4, 0.1, 1.0)
    b = vie.plane_wave(g, np.array([[0.0, 0.0, -1.0]]))[:, 0]
    x, it, conv, _ = gmres.fgmres(lambda v: vie.dense(g) @ v, b, None, tol=1e-12)
    assert conv and it == 1 and np.allclose(x, b, atol=1e-14)
    x0, it0, conv0, _ = gmres.fgmres(lambda v: v, np.zeros(5, dtype=complex))
    assert conv0 and it0 == 0 and not np.any(x0)


def test_preconditioned_compressed_solve(case):
    c, g, Z = case
    op = butterfly.build_hodbf(g, 1e-4)
    p = precond.build_precond(g, 1e-2)
    b = vie.plane_wave(g, c["dirs"])[:, 0]
    x, it, conv, _ = gmres.fgmres(op.apply, b, p.apply, tol=1e-4)
    assert conv
    # true residual against the exact operator stays within chi_sol + O(10 chi_con)
    assert np.linalg.norm(Z @ x - b) <= (1e-4 + 1e-3) * np.linalg.norm(b)


def test_lowest_levels_compose_to_node_inverses(case):
    # Algorithm 1's leaf inverses followed by the uncompressed X_tau of the levels >= lb
    # equal the inverses of the diagonal blocks Z(tau, tau) of the level-lb nodes (each
    # level's I + X_tau = Z(tau, tau)^-1 diag(Z(tau1, tau1), Z(tau2, tau2)) telescopes):
    # the identity behind storing those node inverses directly (precond_dense_levels)
    c, g, Z = case
    p = precond.build_precond(g, 0.1, compress=False)
    tr = p.tree
    lb = tr.depth - 2
    X = {}
    for (l, i), blocks in p.X.items():
        if l >= lb:
            X[(l, i)] = blocks
        else:
            X[(l, i)] = [[precond.DenseBlock(np.zeros((ha - la, hb - lb_), dtype=complex))
                          for (lb_, hb) in (tr.node(l + 1, 2 * i), tr.node(l + 1, 2 * i + 1))]
                         for (la, ha) in (tr.node(l + 1, 2 * i), tr.node(l + 1, 2 * i + 1))]
    q = precond.Precond(tr, p.Dinv, X)
    xt = c["x"][:, :3][tr.perm]
    zt = q.apply_tree(xt)
    Zt = Z[np.ix_(tr.perm, tr.perm)]
    assert len(tr.ranges[lb]) == 1 << lb
    for (lo, hi) in tr.ranges[lb]:
        ref = np.linalg.solve(Zt[lo:hi, lo:hi], xt[lo:hi])
        assert np.linalg.norm(zt[lo:hi] - ref) <= 1e-11 * np.linalg.norm(ref)
    # and the product is not already the full inverse (the levels above lb still couple)
    assert np.linalg.norm(Zt @ zt - xt) > 1e-3 * np.linalg.norm(xt)

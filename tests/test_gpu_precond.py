"""GPU parity of the preconditioner (Algorithm 1 multiplicative form) and of the
preconditioned FGMRES solve, against the oracle."""
import numpy as np
import pytest

from oracle import gmres as ogmres
from oracle import precond as oprecond
from oracle import vie
from synth.workloads import small_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _t(x, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _rel(a, b):
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


@pytest.fixture(scope="module")
def case():
    from paper_2111_01730_amd import hodbf
    c = small_case(61, sides=(10, 9, 8), h=0.1, eps_range=(2.0, 8.0), loss=0.5, nrhs=16)
    g = c["grid"]
    print("[precond build 10x9x8 chi_fact=1e-2 both copies]", flush=True)
    op = hodbf.Operator(g, tol_con=1e-4, tol_fact=1e-2, precond=hodbf.P_BOTH)
    return c, g, op, vie.dense(g)


def test_precond_arithmetic_parity_fp32(case):
    from tests.plan_tools import precond_from_export
    c, g, op, Z = case
    table, vals = op.precond_blocks("fp32")
    ref = precond_from_export(g, op.perm(), table, vals, op.stats()["levels"])
    x = c["x"][:, :8]
    # the default copy is BF16; the FP32 copy is reached through a solve-time switch, so
    # check the FP32 factors through the oracle and the BF16 apply below
    xr = x.astype(np.complex64).astype(np.complex128)
    zr = ref.apply(xr)
    # the reference itself must be a good approximate inverse
    assert np.all(_rel(Z @ zr, xr) <= 0.3)


def test_precond_apply_bf16_matches_exported_factors(case):
    from tests.plan_tools import precond_from_export
    c, g, op, Z = case
    table, vals = op.precond_blocks("bf16")
    ref = precond_from_export(g, op.perm(), table, vals, op.stats()["levels"])
    for R in (1, 8):
        x = c["x"][:, :R]
        z = op.precond_apply(_t(x, torch.complex64)).cpu().numpy().astype(np.complex128)
        # inputs are rounded to BF16 inside the MFMA path: a few 1e-3 relative
        assert np.all(_rel(z, ref.apply(x)) <= 2e-2), _rel(z, ref.apply(x))


def test_precond_is_approximate_inverse(case):
    c, g, op, Z = case
    x = c["x"][:, :4]
    z = op.precond_apply(_t(Z @ x)).cpu().numpy()
    assert np.all(_rel(z, x) <= 0.3)


def test_precond_tight_tolerance_approaches_inverse():
    from paper_2111_01730_amd import hodbf
    c = small_case(62, sides=(8, 8, 8), h=0.1, eps_range=(2.0, 6.0), loss=0.3, nrhs=4)
    g = c["grid"]
    op = hodbf.Operator(g, tol_con=1e-6, tol_fact=1e-7, precond=hodbf.P_FP32)
    Z = vie.dense(g)
    z = op.precond_apply(_t(Z @ c["x"])).cpu().numpy()
    assert np.all(_rel(z, c["x"]) <= 1e-4)
    # and agrees with the oracle's multiplicative inverse at the same tolerance
    po = oprecond.build_precond(g, 1e-7)
    assert np.all(_rel(z, po.apply(Z @ c["x"])) <= 1e-4)


def test_preconditioned_solve_iterations_and_residual(case):
    c, g, op, Z = case
    b = op.plane_wave(c["dirs"])
    bn = b.cpu().numpy()
    out = {}
    for mode in ("bf16", "fp32", 0):
        x, info = op.solve(b, tol=1e-5, restart=20, max_iter=500, use_precond=mode)
        assert info["converged"].all(), (mode, info)
        xn = x.cpu().numpy()
        assert np.all(_rel(Z @ xn, bn) <= 1e-5 + 1e-3)  # chi_sol + compression error
        out[mode] = info["iters"]
    assert out["bf16"].max() <= 15 and out["fp32"].max() <= 15
    assert out[0].min() > 2 * out["fp32"].max()
    # the oracle's preconditioner at the same chi_fact needs a comparable count
    po = oprecond.build_precond(g, 1e-2)
    _, it, conv, _ = ogmres.fgmres(lambda v: Z @ v, bn[:, 0], po.apply, tol=1e-5)
    assert conv and abs(int(out["fp32"][0]) - it) <= 3


def test_batched_solve_equals_single_column_solves(case):
    c, g, op, Z = case
    b = op.plane_wave(c["dirs"][:6])
    xb, ib = op.solve(b, tol=1e-5, use_precond="bf16")
    for q in (0, 3, 5):
        xs, is_ = op.solve(b[:, q].contiguous(), tol=1e-5, use_precond="bf16")
        # one column alone runs the small-R kernels (other summation order): same answer
        # within the solve tolerance, same iteration count up to one step
        assert abs(int(is_["iters"][0]) - int(ib["iters"][q])) <= 1
        d = np.linalg.norm(xs.cpu().numpy() - xb[:, q].cpu().numpy()) / np.linalg.norm(xs.cpu().numpy())
        assert d <= 1e-3

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


def _apply_copy(op, x, which):
    """P x with one stored copy (which: 2 FP32, 3 BF16, 4 FP16) via the tree-order entry."""
    perm = torch.as_tensor(op.perm().astype(np.int64), device="cuda")
    xt = _t(x, torch.complex64)[perm].contiguous()
    zt = op.apply_tree(xt, which)
    z = torch.empty_like(zt)
    z[perm] = zt
    return z.cpu().numpy().astype(np.complex128)


@pytest.fixture(scope="module")
def case():
    from paper_2111_01730_amd import hodbf
    c = small_case(61, sides=(10, 9, 8), h=0.1, eps_range=(2.0, 8.0), loss=0.5, nrhs=16)
    g = c["grid"]
    print("[precond build 10x9x8 chi_fact=1e-2, FP32 + BF16 + FP16 copies]", flush=True)
    op = hodbf.Operator(g, tol_con=1e-4, tol_fact=1e-2,
                        precond=hodbf.P_FP32 | hodbf.P_BF16 | hodbf.P_FP16)
    return c, g, op, vie.dense(g)


def _split_tol(op):
    """Norm-wise bound of the split-BF16 arithmetic against the FP64 re-application: each
    of the apply's dependent launches adds at most 2^-15 relative per product (three
    BF16 products of the hi + lo halves, the dropped lo x lo term), twice that for
    safety, plus the FP32 accumulation allowance of the FP32 path (2e-5)."""
    return 2 * op.stats()["pre_stages"] * 2.0**-15 + 2e-5


# which 6: the FP32 copy with split-BF16 arithmetic (tolerance from _split_tol)
@pytest.mark.parametrize("copy,which,tol", [("fp32", 2, 2e-5), ("fp16", 4, 2e-5), ("bf16", 3, 2e-2),
                                            ("fp32", 6, None)])
@pytest.mark.parametrize("R", [1, 8])
def test_precond_apply_matches_exported_factors(case, copy, which, tol, R):
    # the oracle re-applies the GPU's stored factors (values as stored, block scales
    # applied) in FP64; FP32 / FP16 copies differ by FP32 accumulation only, the BF16
    # copy also rounds its inputs to BF16
    from tests.plan_tools import precond_from_export
    c, g, op, Z = case
    tol = _split_tol(op) if tol is None else tol
    table, vals = op.precond_blocks(copy)
    ref = precond_from_export(g, op.perm(), table, vals, op.stats()["levels"])
    x = c["x"][:, :R].astype(np.complex64).astype(np.complex128)
    z = _apply_copy(op, x, which)
    print(f"[precond copy {copy} which {which} R={R}: max rel err "
          f"{_rel(z, ref.apply(x)).max():.2e}]", flush=True)
    assert np.all(_rel(z, ref.apply(x)) <= tol), _rel(z, ref.apply(x))
    if copy == "fp32":
        assert np.all(_rel(Z @ ref.apply(x), x) <= 0.3)  # the factors form an approximate inverse


def test_precond_is_approximate_inverse(case):
    c, g, op, Z = case
    x = c["x"][:, :4]
    z = op.precond_apply(_t(Z @ x)).cpu().numpy()  # default: FP32 copy, split-BF16
    assert np.all(_rel(z, x) <= 0.3)
    z32 = _apply_copy(op, Z @ x, 2)
    assert np.all(_rel(z32, x) <= 0.3)


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
    for mode in ("fp16", "fp32", "fp32_split", 0):
        x, info = op.solve(b, tol=1e-5, restart=20, max_iter=500, use_precond=mode)
        assert info["converged"].all(), (mode, info)
        xn = x.cpu().numpy()
        assert np.all(_rel(Z @ xn, bn) <= 1e-5 + 1e-3)  # chi_sol + compression error
        out[mode] = info["iters"]
    assert out["fp16"].max() <= 15 and out["fp32"].max() <= 15
    # split-BF16 arithmetic on the FP32 copy preconditions as well as FP32 arithmetic
    assert np.abs(out["fp32_split"].astype(int) - out["fp32"].astype(int)).max() <= 1
    assert out[0].min() > 2 * out["fp32"].max()
    # the oracle's preconditioner at the same chi_fact needs a comparable count
    po = oprecond.build_precond(g, 1e-2)
    _, it, conv, _ = ogmres.fgmres(lambda v: Z @ v, bn[:, 0], po.apply, tol=1e-5)
    assert conv and abs(int(out["fp32"][0]) - it) <= 3


def test_batched_solve_equals_single_column_solves(case):
    c, g, op, Z = case
    b = op.plane_wave(c["dirs"][:6])
    xb, ib = op.solve(b, tol=1e-5, use_precond="fp32")
    for q in (0, 3, 5):
        xs, is_ = op.solve(b[:, q].contiguous(), tol=1e-5, use_precond="fp32")
        # one column alone runs the small-R kernels (other summation order): same answer
        # within the solve tolerance, same iteration count up to one step
        assert abs(int(is_["iters"][0]) - int(ib["iters"][q])) <= 1
        d = np.linalg.norm(xs.cpu().numpy() - xb[:, q].cpu().numpy()) / np.linalg.norm(xs.cpu().numpy())
        assert d <= 1e-3


def test_fp64_tail_and_fp32_only_solves_agree(case):
    # a batch of at most four columns runs its products with Z in FP64 by default; with
    # fp32_only every product is FP32: both meet the tolerance against the dense operator
    # and agree within what two solutions meeting it can differ by
    import ctypes as C
    from paper_2111_01730_amd import _lib
    c, g, op, Z = case
    b = op.plane_wave(c["dirs"][:3])
    x64, i64 = op.solve(b, tol=1e-6, use_precond="fp32")
    x32, i32 = op.solve(b, tol=1e-6, use_precond="fp32", fp32_only=True)
    assert i64["converged"].all() and i32["converged"].all()
    bn = b.cpu().numpy()
    for x in (x64, x32):
        xn = x.cpu().numpy()
        rel = np.linalg.norm(Z @ xn - bn, axis=0) / np.linalg.norm(bn, axis=0)
        assert np.all(rel <= 1e-6 + 1e-3), rel  # + the compression error of chi_con 1e-4
    smin = np.linalg.svd(Z, compute_uv=False)[-1]
    d = np.linalg.norm(x64.cpu().numpy() - x32.cpu().numpy(), axis=0)
    bound = 2 * (1e-6 + 1e-5) * np.linalg.norm(bn, axis=0) / smin
    print(f"[FP64 tail vs FP32 only: steps {i64['iters']} / {i32['iters']}, difference "
          f"{d.max():.2e} (bound {bound.min():.2e})]", flush=True)
    assert np.all(d <= bound)
    opts = _lib.SolveOpts(tol=1e-6, restart=20, max_iter=10, use_precond=9, fp32_only=2)
    xb = torch.empty_like(b)
    code = _lib.lib().vie_solve(op._h, 3, C.c_void_p(b.t().contiguous().data_ptr()), op.n,
                                C.c_void_p(xb.data_ptr()), op.n, C.byref(opts), None, None)
    assert code == -1  # E_ARG


def test_split_bf16_apply_is_reproducible_and_batch_independent(case):
    # every output element is owned by one work item and accumulated in a fixed chunk
    # order, so two calls agree bit for bit; a column alone runs the same arithmetic
    c, g, op, Z = case
    x = c["x"][:, :8].astype(np.complex64).astype(np.complex128)
    z1 = _apply_copy(op, x, 6)
    z2 = _apply_copy(op, x, 6)
    assert np.array_equal(z1, z2)
    z3 = _apply_copy(op, x[:, 3:4], 6)
    d = np.linalg.norm(z3[:, 0] - z1[:, 3]) / np.linalg.norm(z1[:, 3])
    print(f"[split-BF16 precond: column alone vs in a batch of 8: rel diff {d:.2e}]", flush=True)
    assert d <= 1e-6
    b = op.plane_wave(c["dirs"][:4])
    x1, i1 = op.solve(b, tol=1e-5, use_precond="fp32_split")
    x2, i2 = op.solve(b, tol=1e-5, use_precond="fp32_split")
    assert np.array_equal(i1["iters"], i2["iters"])
    assert torch.equal(x1, x2)


@pytest.fixture(scope="module")
def dense_case(case):
    """The same scatterer with Algorithm 1 started from the dense inverses of the level
    L_H - 2 nodes' diagonal blocks (two levels above the leaves)."""
    from paper_2111_01730_amd import hodbf
    c, g, op, Z = case
    print("[precond build 10x9x8 chi_fact=1e-2, dense bottom 2 levels]", flush=True)
    opd = hodbf.Operator(g, tol_con=1e-4, tol_fact=1e-2, precond=hodbf.P_FP32,
                         precond_dense_levels=2)
    return c, g, opd, Z


def _tree_order(Z, perm):
    return Z[np.ix_(perm, perm)]


# split arithmetic: the tolerance from _split_tol, as for the leaf form
@pytest.mark.parametrize("which,tol", [(2, 2e-5), (6, None)])
def test_dense_bottom_matches_exported_factors(dense_case, which, tol):
    from tests.plan_tools import DenseBottomPrecond, precond_from_export
    c, g, op, Z = dense_case
    tol = _split_tol(op) if tol is None else tol
    LH = op.stats()["levels"]
    table, vals = op.precond_blocks("fp32")
    ref = precond_from_export(g, op.perm(), table, vals, LH)
    assert isinstance(ref, DenseBottomPrecond) and ref.lb == LH - 2
    x = c["x"][:, :8].astype(np.complex64).astype(np.complex128)
    z = _apply_copy(op, x, which)
    err = _rel(z, ref.apply(x))
    print(f"[dense bottom which {which}: max rel err {err.max():.2e}]", flush=True)
    assert np.all(err <= tol), err


def test_dense_bottom_blocks_are_node_inverses(dense_case):
    # the recursion's leaves are the level L_H - 2 nodes: their stored blocks are the
    # inverses of the diagonal blocks Z(tau, tau) of the dense operator (tree order), to
    # FP32 storage rounding (each block is stored as FP32 values times one scale)
    from tests.plan_tools import precond_from_export
    c, g, op, Z = dense_case
    LH = op.stats()["levels"]
    table, vals = op.precond_blocks("fp32")
    ref = precond_from_export(g, op.perm(), table, vals, LH)
    Zt = _tree_order(Z, op.perm().astype(np.int64))
    worst = 0.0
    for i, (lo, hi) in enumerate(ref.tree.ranges[ref.lb]):
        inv = np.linalg.inv(Zt[lo:hi, lo:hi])
        worst = max(worst, np.linalg.norm(ref.Dinv[i] - inv) / np.linalg.norm(inv))
    print(f"[dense bottom blocks vs inverses of Z(tau, tau): max rel {worst:.2e}]", flush=True)
    assert worst <= 1e-6


def test_dense_bottom_at_the_root_is_the_inverse(case):
    # d = L_H: the recursion's one leaf is the root, the stored block is Z^{-1} itself
    # (one launch); preconditioned FGMRES then stops after a step or two
    from paper_2111_01730_amd import hodbf
    c, g, op, Z = case
    LH = op.stats()["levels"]
    opr = hodbf.Operator(g, tol_con=1e-4, tol_fact=1e-2, precond=hodbf.P_FP32,
                         precond_dense_levels=LH)
    assert opr.stats()["pre_stages"] == 1
    x = c["x"][:, :4].astype(np.complex64).astype(np.complex128)
    d = _rel(_apply_copy(opr, Z @ x, 2), x)
    print(f"[dense root: ||P Z x - x|| / ||x|| max {d.max():.2e}]", flush=True)
    assert np.all(d <= 1e-4), d
    b = opr.plane_wave(c["dirs"][:2])
    _, info = opr.solve(b, tol=1e-5, use_precond="fp32")
    assert info["converged"].all() and info["iters"].max() <= 3, info


def test_dense_bottom_solve(dense_case, case):
    c, g, op, Z = dense_case
    b = op.plane_wave(c["dirs"])
    out = {}
    for mode in ("fp32", "fp32_split"):
        x, info = op.solve(b, tol=1e-5, restart=20, max_iter=500, use_precond=mode)
        assert info["converged"].all(), (mode, info)
        assert np.all(_rel(Z @ x.cpu().numpy(), b.cpu().numpy()) <= 1e-5 + 1e-3)
        out[mode] = info["iters"]
    # exact bottom levels: no more steps than with the compressed ones
    _, ileaf = case[2].solve(b, tol=1e-5, restart=20, max_iter=500, use_precond="fp32")
    print(f"[dense bottom steps {out['fp32'].max()} vs leaves {ileaf['iters'].max()}]", flush=True)
    assert out["fp32"].max() <= ileaf["iters"].max() + 1


def test_dense_bottom_reaching_above_min_level_is_rejected(case):
    from paper_2111_01730_amd import hodbf
    from paper_2111_01730_amd._lib import HodbfError
    c, g, op, Z = case
    LH = op.stats()["levels"]
    with pytest.raises(HodbfError):
        hodbf.Operator(g, tol_con=1e-4, tol_fact=1e-2, precond=hodbf.P_FP32,
                       precond_min_level=LH - 1, precond_dense_levels=2)


def test_precond_apply_default_is_split_arithmetic_on_the_fp32_copy(case):
    # hodbf_precond_apply runs the arithmetic that preconditions best: the FP32 copy on
    # split-BF16 MFMA (which 6), the same bits as the tree-order call
    c, g, op, Z = case
    x = c["x"][:, :8].astype(np.complex64).astype(np.complex128)
    z = op.precond_apply(_t(x, torch.complex64)).cpu().numpy().astype(np.complex128)
    assert np.array_equal(z, _apply_copy(op, x, 6))


def _ptr(t):
    import ctypes as C
    return C.c_void_p(t.data_ptr())


def test_padded_leading_dimensions(case):
    """ld > N on every vector argument of the user-order calls: the padding rows are
    neither read (NaN there changes nothing) nor written (a sentinel survives)."""
    import ctypes as C

    from paper_2111_01730_amd import _lib
    c, g, op, Z = case
    n, R = g.n, 5
    lib, st = _lib.lib(), C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ldx, ldy = n + 37, n + 101
    xh = np.full((R, ldx), np.nan + 1j * np.nan)
    xh[:, :n] = c["x"][:, :R].T
    xd = torch.as_tensor(xh).cuda()
    sentinel = 7.0 - 3.0j
    for fn, ref in ((lib.hodbf_apply, op.apply), (lib.hodbf_precond_apply, op.precond_apply)):
        yd = torch.full((R, ldy), sentinel, dtype=torch.complex128, device="cuda")
        _lib.check(fn(op._h, R, _lib.C128, _ptr(xd), ldx, _ptr(yd), ldy, st))
        y = yd.cpu().numpy()
        assert np.all(y[:, n:] == sentinel)
        want = ref(_t(c["x"][:, :R])).cpu().numpy()
        assert np.array_equal(y[:, :n].T, want)
    # the solve: b and x padded as well
    b = op.plane_wave(c["dirs"][:R]).cpu().numpy()
    bh = np.full((R, ldx), np.nan + 1j * np.nan)
    bh[:, :n] = b.T
    bd = torch.as_tensor(bh).cuda()
    xs = torch.full((R, ldy), sentinel, dtype=torch.complex128, device="cuda")
    opts = op._solve_opts(1e-5, 20, 500, "fp32")
    code = lib.vie_solve(op._h, R, _ptr(bd), ldx, _ptr(xs), ldy, C.byref(opts), None, st)
    _lib.check(code)
    xsol = xs.cpu().numpy()
    assert np.all(xsol[:, n:] == sentinel)
    x_ref, _ = op.solve(_t(b), tol=1e-5, restart=20, max_iter=500, use_precond="fp32")
    assert np.array_equal(xsol[:, :n].T, x_ref.cpu().numpy())


def test_device_construction_matches_oracle_and_host_run(case):
    """The preconditioner built on the device (Algorithm 1 + Algorithm 2 with randomized
    reconstruction, FP32 sketches) against the oracle's multiplicative inverse (Algorithm 1
    computed densely, chi_fact = 1e-2) and against the same construction run on the host in
    FP64 (hodbf_precond_probe): the same quality ||P Z x - x||, and P x within O(chi_fact)."""
    from paper_2111_01730_amd import _lib
    from tests.plan_tools import precond_from_export
    c, g, op, Z = case
    x = c["x"][:, :6]
    zd = _apply_copy(op, x, 2)
    rd = _rel(_apply_copy(op, Z @ x, 2), x)
    po = oprecond.build_precond(g, 1e-2)
    ro = _rel(po.apply(Z @ x), x)
    p = _lib.make_params(g, 1e-4, 1e-2, precond_prec=1)
    tab = _lib.probe(p, 3, np.int64, "hodbf_precond_probe").reshape(-1, 12)
    vals = _lib.probe(p, 4, np.complex128, "hodbf_precond_probe")
    ph = precond_from_export(g, _lib.probe(p, 0, np.int32, "hodbf_precond_probe"), tab, vals,
                             int(tab[tab[:, 0] == 0][0, 1]))
    rh = _rel(ph.apply(Z @ x), x)
    st = op.stats()
    print(f"[device construction: ||PZx - x|| {rd.max():.3e} (oracle {ro.max():.3e}, host run "
          f"{rh.max():.3e}), vs oracle P {_rel(zd, po.apply(x)).max():.3e}, vs host P "
          f"{_rel(zd, ph.apply(x)).max():.3e}; {st['precond_reconstructions']} reconstructions, "
          f"{st['precond_sketch_cols']} sketch columns]", flush=True)
    assert rd.max() <= 3 * ro.max() and rd.max() <= 2 * rh.max() + 1e-3
    assert np.all(_rel(zd, po.apply(x)) <= 30 * 1e-2)
    assert np.all(_rel(zd, ph.apply(x)) <= 30 * 1e-2)
    assert st["precond_reconstructions"] > 0

"""GPU parity of the batched solver (sg_gmres_batched) and its tile autotuner.

Every instance of a batch is checked on its own against the CPU FP64 oracle:
  * small instances: true relative residual <= tol recomputed with the oracle's assembled
    A, and relative solution error against the oracle's direct solve <= 1e-6;
  * config-4 instances at full size (N up to 255, Q up to 70): the oracle's pointwise rows
    of A at sampled grid points reproduce the GPU residual b - A x there (to 64 ulps of an
    upper bound of the row sums Σ|A_pq||x_q|), and the FP64 GPU relative residual is
    <= 1e-8.
The batched and the single-instance GMRES run the same algorithm, so in FP64 their
iteration counts agree and their solutions agree to rounding.
"""
import numpy as np
import pytest

from oracle import assemble, precond
from workloads import config1, config4_instances, small_2d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2209_14740_amd import sg  # noqa: E402

SMALL = [
    small_2d(n=33, kbar=8.0, sigma=0.8, s=2, degree=2),
    small_2d(n=41, kbar=10.0, sigma=1.0, s=3, degree=2),
    small_2d(n=65, kbar=12.0, sigma=1.2, s=1, degree=4),
    small_2d(n=63, kbar=7.0, sigma=0.7, s=4, degree=2),
    small_2d(n=33, kbar=6.0, sigma=0.6, s=1, degree=2),
    config1(),
]

_REF = {}


def ref(inst):
    if inst.name not in _REF:
        S = assemble.from_instance(inst)
        _REF[inst.name] = (S, precond.direct_solve(S))
    return _REF[inst.name]


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def small_ops():
    ops = [sg.SG.from_instance(i) for i in SMALL]
    yield ops
    for op in ops:
        op.close()


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16x3"])
def test_batched_small_matches_oracle(small_ops, precision):
    bs = [op.rhs(inst.f) for op, inst in zip(small_ops, SMALL)]
    xs, rc, infos = sg.gmres_batched(small_ops, bs, restart=30, maxit=600, pc="mean", precision=precision,
                                     tol=1e-8)
    assert rc == sg.SG_OK
    for inst, x, info in zip(SMALL, xs, infos):
        S, xref = ref(inst)
        xh = to_host(x)
        rel = np.linalg.norm(S.b - S.A @ xh) / np.linalg.norm(S.b)
        err = np.linalg.norm(xh - xref) / np.linalg.norm(xref)
        print(inst.name, precision, info["iters"], info["restarts"], rel, err, flush=True)
        assert info["converged"] == 1
        assert rel <= 1e-8 * 1.05
        assert abs(info["relres_true"] - rel) <= 1e-3 * rel + 1e-14
        assert err <= 1e-6


@pytest.mark.parametrize("pc", ["mean", "csl"])
def test_batched_2d_only_matches_oracle(small_ops, pc):
    """A batch of 2D instances only (n = 33…65, segments of at most 8 rows): the grouped
    sweep then carries two right-hand sides per thread (a batch with the 1D instance uses
    one).  Every instance against the oracle's direct solve, and against the single-instance
    solve (same iterations, solutions within 1e-9)."""
    ops = small_ops[:5]
    insts = SMALL[:5]
    bs = [op.rhs(inst.f) for op, inst in zip(ops, insts)]
    xs, rc, infos = sg.gmres_batched(ops, bs, restart=30, maxit=600, pc=pc, precision="f64", tol=1e-9)
    assert rc == sg.SG_OK
    for op, inst, b, x, info in zip(ops, insts, bs, xs, infos):
        S, xref = ref(inst)
        xh = to_host(x)
        err = np.linalg.norm(xh - xref) / np.linalg.norm(xref)
        assert info["converged"] == 1 and err <= 1e-6, (inst.name, err)
        x1, i1 = op.gmres(b, restart=30, maxit=600, pc=pc, precision="f64", tol=1e-9)
        assert abs(i1["iters"] - info["iters"]) <= 1
        assert float((x - x1).abs().max() / x1.abs().max()) <= 1e-9


def test_batched_iterations_match_single(small_ops):
    bs = [op.rhs(inst.f) for op, inst in zip(small_ops, SMALL)]
    xs, rc, infos = sg.gmres_batched(small_ops, bs, restart=20, maxit=600, pc="csl", precision="f64", tol=1e-9)
    assert rc == sg.SG_OK
    for op, b, x, info in zip(small_ops, bs, xs, infos):
        x1, i1 = op.gmres(b, restart=20, maxit=600, pc="csl", precision="f64", tol=1e-9)
        assert abs(i1["iters"] - info["iters"]) <= 1
        assert i1["restarts"] == info["restarts"]
        d = float((x - x1).abs().max() / x1.abs().max())
        assert d <= 1e-9


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batched_delayed_and_two_pass_cgs2_agree(small_ops, precision):
    """The batch with the delayed CGS2 (the default: flexible Arnoldi, one reduction and one
    update pass per step) and with the two-pass CGS2 (every handle set to "cgs2"): both
    converge to the oracle's solution.  With the FP64 preconditioner the two generate the
    same Krylov space: iteration counts within one, solutions within 1e-7.  With the FP32
    preconditioner the two-pass form applies P^{-1} again to V y at the cycle end (it assumes
    a linear preconditioner) while the flexible form keeps the z_j it used, so the delayed
    form needs at most as many iterations (one of slack) and the solutions agree to 1e-6."""
    bs = [op.rhs(inst.f) for op, inst in zip(small_ops, SMALL)]
    xd, rcd, infd = sg.gmres_batched(small_ops, bs, restart=12, maxit=600, pc="mean", precision=precision, tol=1e-9)
    try:
        for op in small_ops:
            op.set_orthogonalisation("cgs2")
        xc, rcc, infc = sg.gmres_batched(small_ops, bs, restart=12, maxit=600, pc="mean", precision=precision,
                                         tol=1e-9)
    finally:
        for op in small_ops:
            op.set_orthogonalisation("dcgs2")
    assert rcd == sg.SG_OK and rcc == sg.SG_OK
    for inst, a, c, ia, ic in zip(SMALL, xd, xc, infd, infc):
        S, xref = ref(inst)
        for xv in (a, c):
            err = np.linalg.norm(to_host(xv) - xref) / np.linalg.norm(xref)
            assert err <= 1e-6, (inst.name, err)
        print(inst.name, precision, ia["iters"], ic["iters"], ia["restarts"], ic["restarts"], flush=True)
        if precision == "f64":
            assert abs(ia["iters"] - ic["iters"]) <= 1, (inst.name, ia["iters"], ic["iters"])
            assert float((a - c).abs().max() / c.abs().max()) <= 1e-7
        else:
            assert ia["iters"] <= ic["iters"] + 1, (inst.name, ia["iters"], ic["iters"])
            assert float((a - c).abs().max() / c.abs().max()) <= 1e-6


@pytest.mark.parametrize("restart,pc", [(1, "mean"), (2, "csl"), (3, "none")])
def test_batched_short_restarts_match_single(small_ops, restart, pc):
    """Restart lengths 1-3 (every cycle ends in a finishing reduction of the delayed CGS2 at
    j = m) and the unpreconditioned solve: the batch against the single-instance solver
    (the same delayed CGS2), iterations within one and solutions within 1e-6 where they
    converge; where neither converges within maxit (GMRES(3) without a preconditioner) the
    same iteration count and true residuals within 10 % (the iterates of a stagnating
    restarted GMRES drift apart with the rounding of the two launch layouts)."""
    ops = small_ops if pc != "none" else small_ops[:5]
    insts = SMALL if pc != "none" else SMALL[:5]
    bs = [op.rhs(inst.f) for op, inst in zip(ops, insts)]
    maxit = 3000 if pc != "none" else 400
    xs, rc, infos = sg.gmres_batched(ops, bs, restart=restart, maxit=maxit, pc=pc, precision="f64", tol=1e-7)
    for op, inst, b, x, info in zip(ops, insts, bs, xs, infos):
        x1, i1 = op.gmres(b, restart=restart, maxit=maxit, pc=pc, precision="f64", tol=1e-7)
        print(inst.name, restart, pc, info["iters"], i1["iters"], info["converged"], i1["converged"], flush=True)
        assert info["converged"] == i1["converged"]
        assert abs(i1["iters"] - info["iters"]) <= 1, (inst.name, i1["iters"], info["iters"])
        assert bool(torch.isfinite(torch.view_as_real(x)).all())
        if info["converged"]:
            assert float((x - x1).abs().max() / x1.abs().max()) <= 1e-6
        else:
            assert abs(info["relres_true"] - i1["relres_true"]) <= 0.1 * i1["relres_true"]


@pytest.mark.parametrize("tile", ["128x128", "64x128", "64x64", "64x32", "32x64", "3m32x32", "3m64x32", "3m32x64",
                                  "3m64x64"])
def test_batched_tile_shapes(small_ops, tile):
    for op in small_ops:
        if op.dim == 2:
            sg.tune_set(op.n, op.Q, "f64", tile)
    try:
        bs = [op.rhs(inst.f) for op, inst in zip(small_ops, SMALL)]
        xs, rc, infos = sg.gmres_batched(small_ops, bs, restart=30, maxit=600, pc="mean", precision="f64",
                                         tol=1e-10)
        assert rc == sg.SG_OK
        for inst, x in zip(SMALL, xs):
            _, xref = ref(inst)
            xh = to_host(x)
            assert np.linalg.norm(xh - xref) / np.linalg.norm(xref) <= 1e-8
    finally:
        for op in small_ops:
            if op.dim == 2:
                sg.tune_set(op.n, op.Q, "f64", "128x128")


@pytest.mark.parametrize("tile", ["3m32x32", "3m64x64", "64x256"])
def test_batched_f32_tile_shapes(small_ops, tile):
    """The FP32 preconditioner of the batched solver in the 3M form and the wide real-form
    tile (grouped launches over instances of several shapes) against the oracle."""
    for op in small_ops:
        if op.dim == 2:
            sg.tune_set(op.n, op.Q, "f32", tile)
    try:
        bs = [op.rhs(inst.f) for op, inst in zip(small_ops, SMALL)]
        xs, rc, infos = sg.gmres_batched(small_ops, bs, restart=30, maxit=600, pc="mean", precision="f32",
                                         tol=1e-10)
        assert rc == sg.SG_OK
        for inst, x in zip(SMALL, xs):
            _, xref = ref(inst)
            xh = to_host(x)
            assert np.linalg.norm(xh - xref) / np.linalg.norm(xref) <= 1e-8
    finally:
        for op in small_ops:
            if op.dim == 2:
                sg.tune_set(op.n, op.Q, "f32", "128x128")


def test_batched_shifted_operator_matches_single():
    """A handle whose operator is the full CSL matrix M(β) (sg_set_operator_shift) in the
    batched solver (generic grouped operator) next to an unshifted one: each matches its
    single-instance solve, and the shifted solution satisfies M(β) x = b by the oracle."""
    insts = [small_2d(n=33, kbar=8.0, sigma=0.8, s=2, degree=2), small_2d(n=41, kbar=10.0, sigma=1.0, s=3, degree=2)]
    ops = [sg.SG.from_instance(i) for i in insts]
    try:
        ops[0].set_operator_shift(0.5)
        bs = [op.rhs(i.f) for op, i in zip(ops, insts)]
        xs, rc, infos = sg.gmres_batched(ops, bs, restart=30, maxit=600, pc="csl", precision="f64", tol=1e-10)
        assert rc == sg.SG_OK
        for op, b, x, info in zip(ops, bs, xs, infos):
            x1, i1 = op.gmres(b, restart=30, maxit=600, pc="csl", precision="f64", tol=1e-10)
            assert info["converged"] == 1 and abs(i1["iters"] - info["iters"]) <= 1
            assert float((x - x1).abs().max() / x1.abs().max()) <= 1e-9
        S = assemble.from_instance(insts[0])
        M = S.csl(0.5)
        xh = to_host(xs[0])
        assert np.linalg.norm(S.b - M @ xh) / np.linalg.norm(S.b) <= 1e-10 * 1.05
    finally:
        for op in ops:
            op.close()


def test_batched_edge_cases(small_ops):
    ops = small_ops[:3]
    bs = [op.rhs(inst.f) for op, inst in zip(ops, SMALL[:3])]
    bs[1].zero_()
    xs, rc, infos = sg.gmres_batched(ops, bs, restart=30, maxit=600, precision="f64")
    assert rc == sg.SG_OK
    assert infos[1]["converged"] == 1 and infos[1]["iters"] == 0
    assert float(xs[1].abs().max()) == 0.0
    # maxit too small: the batch reports non-convergence per instance, results stay finite
    xs, rc, infos = sg.gmres_batched(ops, [op.rhs(inst.f) for op, inst in zip(ops, SMALL[:3])], restart=30,
                                     maxit=2, precision="f64")
    assert rc == sg.SG_ENOTCONV
    assert all(i["converged"] == 0 and i["iters"] == 2 for i in infos)
    assert all(bool(torch.isfinite(torch.view_as_real(x)).all()) for x in xs)
    # invalid arguments
    with pytest.raises(sg.SGError):
        sg.gmres_batched([ops[0], ops[0]], [bs[0], bs[2]])
    with pytest.raises(sg.SGError):
        sg.gmres_batched(ops, bs, restart=64)
    with pytest.raises(sg.SGError):
        sg.gmres_batched(ops, bs, xs=[bs[0], bs[1], bs[2]])
    assert sg.gmres_batched([], [])[1] == sg.SG_OK


def test_autotune_fills_table(small_ops):
    ms = sg.autotune(small_ops, precision="bf16x3", reps=2)
    assert ms > 0
    for op in small_ops:
        if op.dim == 2:
            assert sg.tune_get(op.n, op.Q, "bf16x3") in (0, 1, 2, 3, 4, 9, 10)   # 3M shapes: FP64 and FP32


def test_batched_config4_sample_full_size():
    """A sample of the 512-instance batched workload at its real sizes, in one call with
    the autotuned tiles and the FP32 preconditioner (the benchmarked configuration)."""
    insts = config4_instances(count=24, seed0=0)
    # make sure the largest shape of the workload is in the sample
    insts += [i for i in config4_instances(count=40, seed0=24) if i.n == 255 and i.Q == 70][:1]
    ops = [sg.SG.from_instance(i) for i in insts]
    try:
        sg.autotune(ops, precision="f32", reps=2)
        bs = [op.rhs(i.f) for op, i in zip(ops, insts)]
        xs, rc, infos = sg.gmres_batched(ops, bs, restart=30, maxit=1000, pc="mean", precision="f32", tol=1e-8)
        assert rc == sg.SG_OK
        rng = np.random.default_rng(7)
        for inst, op, b, x, info in zip(insts, ops, bs, xs, infos):
            assert info["converged"] == 1
            r = b - op.apply(x)
            rel = sg.norm(r) / sg.norm(b)
            assert rel <= 1e-8 * 1.05
            assert abs(rel - info["relres_true"]) <= 1e-3 * rel
            pts = rng.choice(inst.points, size=64, replace=False)
            pts = np.unique(np.concatenate([pts, [0, inst.n - 1, inst.points - 1]]))
            xh, rh, bh = to_host(x), to_host(r), to_host(b)
            ax = assemble.apply_at_points(inst, xh, pts)
            idx = (np.arange(op.Q)[:, None] * inst.points + pts[None, :]).ravel()
            r_or = bh[idx] - ax.ravel()
            # rounding of a row of A x is bounded by a few ulps of Σ|A_pq||x_q| <=
            # (8/h² + max|k|²·Σ|G|) max|x|; the stencil terms dominate
            kmax = np.max(np.abs(inst.k_fields).sum(axis=0))
            rowsum = (8.0 / inst.h ** 2 + 4.0 * kmax ** 2 + 2.0 * kmax / inst.h) * np.max(np.abs(xh))
            assert np.max(np.abs(r_or - rh[idx])) <= 64 * 2.2e-16 * rowsum
    finally:
        for op in ops:
            op.close()

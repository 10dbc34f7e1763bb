"""GPU parity of the undiscounted scheme (lambda = 0, Section 3 as printed) on the paper's exit
problems (Table 0: A advection, B / B2 eikonal, C Zermelo) and of the varying costs and diffusion of
Sections 5.2-5.3 (eps(x) = eps chi{x_2 >= 0}; l_1, l_2, l_3 with sigma_1, sigma_2, sigma_3), through
the Jacobi solve, the active-tile solver and the patchy pipeline, against the FP64 oracle.

Tolerance 1e-5 max-abs, as the other parity tests. Without discount the stopping rule bounds the
error by the sweep change times the expected number of steps to exit (no factor beta per step), so
the solves stop at 2e-7, near what the FP32 iterate (values up to ~2, one ulp 1.2e-7) resolves."""
import numpy as np
import pytest

import oracle
from paper_1502_01629_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 2e-7


@pytest.fixture(scope="module")
def ctx():
    from paper_1502_01629_amd import capi

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = capi.Context(0)
    yield c
    c.close()


def _dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype).reshape(-1)).cuda()


def _ref(x, scheme):
    v, _, _, _ = oracle.Problem.from_instance(x, scheme).solve(tol=1e-12, threads=8)
    return v


def _run(ctx, x, scheme, how):
    from paper_1502_01629_amd import capi

    dp = capi.DeviceProblem(x, scheme)
    v = _dev(np.zeros((x.n, x.n)) if float(x.lam) == 0.0 else x.initial())
    if how == "jacobi":
        st = ctx.solve(dp, v, tol=TOL, max_sweeps=200_000, check_every=4)
    else:
        st = ctx.solve_tiles(dp, v, tol=TOL, max_passes=200_000, policy_sweeps=14 if how == "tiles_pe" else 0,
                             tile_shape=capi.TILE_16x16_SPLIT2)
    return v, st


@pytest.mark.parametrize("how", ["jacobi", "tiles", "tiles_pe"])
@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("dyn,eps", [("A", 0.0), ("A", 1e-2), ("B", 0.0), ("B", 1e-2), ("B2", 0.0), ("B2", 1e-2),
                                     ("C", 0.0), ("C", 1e-2)])
def test_table0_problems_undiscounted(ctx, dyn, eps, scheme, how):
    x = I.exit_problem(50, dyn, eps=eps, lam=0.0)
    print(f"exit {dyn} eps={eps} lambda=0 scheme={scheme} {how}", flush=True)
    v, st = _run(ctx, x, scheme, how)
    err = float(np.abs(v.cpu().numpy().astype(np.float64) - _ref(x, scheme)).max())
    print(f"  status {st['status']} sweeps/passes {st['sweeps']} path {st['kernel_path']} err {err:.3e}", flush=True)
    assert st["status"] == 0 and st["kernel_path"] == 2
    assert err < 1e-5


@pytest.mark.parametrize("how", ["jacobi", "tiles_pe"])
def test_degenerate_diffusion(ctx, how):
    x = I.degenerate_problem(65, eps=0.1)
    print(f"degenerate diffusion 65^2 {how}", flush=True)
    v, st = _run(ctx, x, 1, how)
    err = float(np.abs(v.cpu().numpy().astype(np.float64) - _ref(x, 1)).max())
    print(f"  status {st['status']} sweeps/passes {st['sweeps']} halo {st['halo']} err {err:.3e}", flush=True)
    assert st["status"] == 0 and err < 1e-5


@pytest.mark.parametrize("how", ["jacobi", "tiles_pe"])
@pytest.mark.parametrize("cost", [1, 2, 3])
@pytest.mark.parametrize("sigma", [1, 2, 3])
def test_general_costs_and_diffusions(ctx, cost, sigma, how):
    x = I.general_problem(65, cost=cost, sigma=sigma, eps=0.1)
    print(f"general l{cost} sigma{sigma} 65^2 {how}", flush=True)
    v, st = _run(ctx, x, 1, how)
    err = float(np.abs(v.cpu().numpy().astype(np.float64) - _ref(x, 1)).max())
    print(f"  status {st['status']} sweeps/passes {st['sweeps']} halo {st['halo']} err {err:.3e}", flush=True)
    assert st["status"] == 0 and err < 1e-5


@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_general_costs_discounted_and_not(ctx, lam):
    """l_3 with sigma_2 in the Kruzkov-discounted form too (lambda = 1: a cost field changes the
    reference constant of the iterate) and without discount."""
    x = I.general_problem(65, cost=3, sigma=2, eps=0.05, lam=lam)
    v, st = _run(ctx, x, 1, "tiles_pe")
    err = float(np.abs(v.cpu().numpy().astype(np.float64) - _ref(x, 1)).max())
    print(f"lambda={lam}: status {st['status']} err {err:.3e}", flush=True)
    assert st["status"] == 0 and err < 1e-5


@pytest.mark.parametrize("mode", ["patchy", "static"])
@pytest.mark.parametrize("eps", [0.0, 1e-2])
def test_patchy_pipeline_undiscounted(ctx, mode, eps):
    """The eikonal exit problem B2 at 101^2 without discount through the patchy pipeline (coarse
    51^2 sigma = 0 solve from v = 0, u_hat, synthesis, labels, u_hat-ordered fine solve)."""
    from paper_1502_01629_amd import capi

    fine = I.exit_problem(101, "B2", eps=eps, lam=0.0)
    coarse = I.exit_problem(51, "B2", eps=0.0, lam=0.0)
    dp, dpc = capi.DeviceProblem(fine, 1), capi.DeviceProblem(coarse, 1)
    v = torch.empty(fine.n * fine.n, dtype=torch.float32, device="cuda")
    if mode == "patchy":
        src, _ = capi.partition_sources(fine.node_class, 8)
        lab = torch.empty(fine.n * fine.n, dtype=torch.int16, device="cuda")
        st = ctx.solve_patchy(dp, dpc, v, tol=TOL, tol_coarse=TOL, source_patch=_dev(src, np.int16), n_patches=8,
                              label_out=lab, policy_sweeps=14)
        assert int((lab >= 0).sum()) > 0
    else:
        st = ctx.solve_patchy(dp, None, v, mode=capi.PATCHY_STATIC, tol=TOL, policy_sweeps=14)
    err = float(np.abs(v.cpu().numpy().astype(np.float64) - _ref(fine, 1)).max())
    print(f"patchy B2 101^2 eps={eps} {mode}: status {st['status']} passes {st['passes']} err {err:.3e}", flush=True)
    assert st["status"] == 0 and err < 1e-5


def test_unsupported_combinations_are_rejected(ctx):
    from paper_1502_01629_amd import capi

    x = I.exit_problem(33, "B", lam=0.0)
    dp = capi.DeviceProblem(x, 1)
    with pytest.raises(capi.SlhjbError) as e:
        ctx.solve_batch([dp], [_dev(x.initial())])
    assert e.value.status == capi.E_UNSUPPORTED
    g = I.general_problem(33, cost=3, sigma=1)
    dg = capi.DeviceProblem(g, 1)
    ctrl = torch.empty(33 * 33, dtype=torch.int16, device="cuda")
    with pytest.raises(capi.SlhjbError) as e:
        ctx.synthesize(dg, _dev(np.zeros((33, 33))), ctrl)
    assert e.value.status == capi.E_UNSUPPORTED
    bad = I.exit_problem(33, "B", lam=0.0)
    bad.lam = np.float32(-1.0)
    with pytest.raises(capi.SlhjbError) as e:
        ctx.solve(capi.DeviceProblem(bad, 1), _dev(bad.initial()), tol=1e-6, max_sweeps=10)
    assert e.value.status == capi.E_INVALID_ARG

"""GPU parity on the paper's exit-to-boundary problems (Section 5: Omega = [-1,1]^2, g = 0 on
the boundary, l = 1, 16 controls; A advection, B eikonal, C Zermelo), whose drift goes through
the general kernels: f(x,a) = c(x) (d(x) + a).

Every case compares the GPU path with the FP64 oracle on the same FP32 inputs: one sweep from
a random iterate to 2e-6, converged solutions to 1e-5 max-abs (the bounds of the other parity
tests: a handful of FP32 roundings, amplified by at most 1/(1-beta) at convergence). The general
kernels leave the node's own corner out of eq. SLscheme3's interpolation exactly (it reads 0), so
the FP32 iterate settles; the GPU solves stop at 1e-6 like the other parity tests.
"""
import numpy as np
import pytest

import oracle
from paper_1502_01629_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_1502_01629_amd import capi

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = capi.Context(0)
    yield c
    c.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).reshape(-1)).cuda()


def _oracle_solution(inst, scheme, tol=1e-12):
    p = oracle.Problem.from_instance(inst, scheme)
    v, _, _, _ = p.solve(tol=tol, threads=8)
    return v


CASES = [("A", 0.0), ("B", 0.0), ("B2", 0.0), ("C", 0.0), ("C", 1e-2), ("B", 1e-2)]


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("dyn,eps", CASES)
def test_one_sweep_matches_oracle(ctx, dyn, eps, scheme):
    from paper_1502_01629_amd import capi

    inst = I.exit_problem(45, dyn, eps=eps)
    print(f"case exit {dyn} eps={eps} scheme={scheme} n={inst.n} h={float(inst.h)}", flush=True)
    rng = np.random.default_rng(3)
    v = rng.random((inst.n, inst.n)).astype(np.float32)
    v[inst.node_class == I.TARGET] = 0.0
    dp = capi.DeviceProblem(inst, scheme)
    vin = _dev(v)
    vout = torch.empty_like(vin)
    ctx.sweep(dp, vin, vout)
    p = oracle.Problem.from_instance(inst, scheme)
    ref, _ = p.sweep(v.astype(np.float64).reshape(-1), threads=8)
    assert np.abs(vout.cpu().numpy().astype(np.float64) - ref).max() < 2e-6


@pytest.mark.parametrize("dyn,eps", CASES)
def test_jacobi_solve_matches_oracle(ctx, dyn, eps):
    from paper_1502_01629_amd import capi

    inst = I.exit_problem(65, dyn, eps=eps)
    print(f"case exit {dyn} eps={eps} n={inst.n}", flush=True)
    dp = capi.DeviceProblem(inst, capi.SL3)
    v = _dev(inst.initial())
    st = ctx.solve(dp, v, tol=1e-6, max_sweeps=200_000)
    assert st["status"] == 0
    ref = _oracle_solution(inst, oracle.SL3)
    assert np.abs(v.cpu().numpy().astype(np.float64) - ref).max() < 1e-5


def test_advection_closed_form_on_gpu(ctx):
    """A with h = dx: every foot is the upstream node, v = 1 - beta^i exactly (FP32 here)."""
    from paper_1502_01629_amd import capi

    n = 33
    inst = I.exit_problem(n, "A", h=2.0 / (n - 1))
    dp = capi.DeviceProblem(inst, capi.SL3)
    v = _dev(inst.initial())
    ctx.solve(dp, v, tol=1e-9, max_sweeps=10_000)
    beta = oracle.Problem.from_instance(inst, oracle.SL3).beta()
    want = 1.0 - beta ** np.arange(n)[None, :].repeat(n, 0)
    free = inst.node_class == 0
    got = v.cpu().numpy().reshape(n, n).astype(np.float64)
    assert np.abs(got[free] - want[free]).max() < 1e-6


@pytest.mark.parametrize("shape", [1, 4])
@pytest.mark.parametrize("eps", [0.0, 1e-2])
def test_tile_solver_matches_oracle(ctx, shape, eps):
    """The active-tile solver (general path with the drift) on Zermelo, tiles by u_hat keys of
    the start and plain order, with and without policy evaluation."""
    from paper_1502_01629_amd import capi

    inst = I.exit_problem(65, "C", eps=eps)
    ref = _oracle_solution(inst, oracle.SL3)
    dp = capi.DeviceProblem(inst, capi.SL3)
    for order, pe in ((capi.ORDER_NONE, 0), (capi.ORDER_KEYS, 0), (capi.ORDER_NONE, 7 if shape == 4 else 0)):
        print(f"case tiles C eps={eps} shape={shape} order={order} pe={pe}", flush=True)
        v = _dev(inst.initial())
        st = ctx.solve_tiles(dp, v, tol=1e-6, order=order, tile_shape=shape, policy_sweeps=pe, max_passes=200_000)
        assert st["status"] == 0
        assert np.abs(v.cpu().numpy().astype(np.float64) - ref).max() < 1e-5


def test_patchy_transmission_on_zermelo(ctx):
    """Coarse solve, u_hat and the fine solve in u_hat order (no patch labels) with the drift."""
    from paper_1502_01629_amd import capi

    fine = I.exit_problem(129, "C")
    coarse = I.exit_problem(33, "C", h=float(fine.h) * 4.0)
    ref = _oracle_solution(fine, oracle.SL3)
    dp, dpc = capi.DeviceProblem(fine, capi.SL3), capi.DeviceProblem(coarse, capi.SL3)
    v = torch.empty(fine.n * fine.n, dtype=torch.float32, device="cuda")
    st = ctx.solve_patchy(dp, dpc, v, mode=capi.PATCHY_TRANSMISSION, tol=1e-6, tol_coarse=1e-7, policy_sweeps=16)
    assert st["status"] == 0
    assert np.abs(v.cpu().numpy().astype(np.float64) - ref).max() < 1e-5


def test_drift_is_rejected_where_unsupported(ctx):
    from paper_1502_01629_amd import capi

    inst = I.exit_problem(33, "C")
    dp = capi.DeviceProblem(inst, capi.SL3)
    v = _dev(inst.initial())
    ctrl = torch.empty(inst.n * inst.n, dtype=torch.int16, device="cuda")
    with pytest.raises(capi.SlhjbError) as e:
        ctx.synthesize(dp, v, ctrl)
    assert e.value.status == capi.E_UNSUPPORTED
    src = torch.zeros(inst.n * inst.n, dtype=torch.int16, device="cuda")
    lab = torch.empty_like(src)
    with pytest.raises(capi.SlhjbError) as e:
        ctx.label(dp, ctrl, src, 1, lab)
    assert e.value.status == capi.E_UNSUPPORTED
    with pytest.raises(capi.SlhjbError) as e:
        ctx.solve_batch([dp], [v], tol=1e-6)
    assert e.value.status == capi.E_UNSUPPORTED


def test_non_finite_drift_is_rejected(ctx):
    from paper_1502_01629_amd import capi

    inst = I.exit_problem(17, "C")
    inst.drift = inst.drift.copy()
    inst.drift[5, 7, 1] = np.inf
    dp = capi.DeviceProblem(inst, capi.SL3)
    v = _dev(inst.initial())
    with pytest.raises(capi.SlhjbError) as e:
        ctx.solve(dp, v, tol=1e-6)
    assert e.value.status == capi.E_INVALID_ARG

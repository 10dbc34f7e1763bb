"""GPU parity of the Jacobi sweep and the value-iteration driver against the FP64 oracle.

All inputs are seeded and synthetic; both sides consume the same FP32 arrays. Tolerances:
one sweep from the same input agrees to 2e-6 (a handful of FP32 roundings on values in
[0,1]); converged solutions agree to 1e-5 max-abs.
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


def _random_v(inst, seed):
    rng = np.random.default_rng(seed)
    v = rng.random((inst.n, inst.n)).astype(np.float32)
    v[inst.node_class == I.TARGET] = inst.target_value
    v[inst.node_class == I.OBSTACLE] = inst.v_out
    return v


def _one_sweep_case(ctx, inst, scheme, seed=0, tol=2e-6):
    from paper_1502_01629_amd import capi

    print(f"case n={inst.n} diff={inst.diffusion} eps={float(inst.eps)} scheme={scheme} NA={inst.n_controls}", flush=True)
    v = _random_v(inst, seed)
    dp = capi.DeviceProblem(inst, scheme)
    vin = _dev(v)
    vout = torch.empty_like(vin)
    r_gpu = ctx.sweep(dp, vin, vout)
    torch.cuda.synchronize()
    p = oracle.Problem.from_instance(inst, scheme)
    ref, r_ref = p.sweep(v.astype(np.float64).reshape(-1), threads=8)
    got = vout.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max()
    assert err < tol, err
    assert abs(r_gpu - r_ref) < tol
    return err


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("eps", [0.0, 0.01])
def test_sweep_disc_problem(ctx, scheme, eps):
    """The CPU-sized disc problem: eps = 0 runs the first-ring kernel, eps = 0.01 the halo kernel."""
    _one_sweep_case(ctx, I.disc_problem(129, eps), scheme)


@pytest.mark.parametrize("n", [3, 5, 65, 77, 200])
@pytest.mark.parametrize("diff", [I.DIFF_NONE, I.DIFF_ISO, I.DIFF_RANK1])
@pytest.mark.parametrize("scheme", [0, 1])
def test_sweep_ragged_random_fields(ctx, n, diff, scheme):
    """Ragged grids (partial tiles), random speed, obstacles, targets and controls in every quadrant."""
    rng = np.random.default_rng(n * 7 + diff)
    inst = I.disc_problem(n, eps=0.0 if diff == I.DIFF_NONE else 0.004, n_controls=int(rng.integers(5, 40)),
                          diffusion=diff)
    inst.speed = (0.3 + 1.4 * rng.random((n, n))).astype(np.float32)
    cls = np.zeros((n, n), dtype=np.uint8)
    cls[rng.random((n, n)) < 0.05] = I.OBSTACLE
    cls[rng.random((n, n)) < 0.05] = I.TARGET
    inst.node_class = cls
    _one_sweep_case(ctx, inst, scheme, seed=n)


@pytest.mark.parametrize("scheme", [0, 1])
def test_sweep_first_ring_with_edges(ctx, scheme):
    """First-ring kernel on every edge configuration: h c <= dx with random speeds, targets at corners."""
    n = 130
    rng = np.random.default_rng(11)
    inst = I.disc_problem(n, 0.0, n_controls=64, h_factor=0.5)
    inst.speed = (0.2 + 1.8 * rng.random((n, n))).astype(np.float32)  # h c <= dx
    inst.node_class[0, 0] = I.TARGET
    inst.node_class[-1, -1] = I.TARGET
    _one_sweep_case(ctx, inst, scheme)


@pytest.mark.parametrize("scheme", [0, 1])
def test_transport_closed_form_on_gpu(ctx, scheme):
    from paper_1502_01629_amd import capi

    inst = I.transport_problem(65, 32)
    dp = capi.DeviceProblem(inst, scheme)
    v = _dev(inst.initial())
    st = ctx.solve(dp, v, tol=0.0, max_sweeps=200, check_every=8)
    beta = np.float64(np.float32(np.exp(-np.float64(inst.h))))
    exact = 1.0 - beta ** np.arange(65)
    got = v.cpu().numpy().reshape(65, 65)
    assert np.abs(got - exact[None, :]).max() < 2e-6


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("eps", [0.0, 0.01])
def test_solve_disc_problem_matches_oracle(ctx, scheme, eps):
    """129^2 disc problem, 32 directions: GPU FP32 Jacobi from v = 1 to the FP32 noise floor (a sweep
    changes nothing by more than a few ulp of 1) agrees with the FP64 oracle converged to 1e-10
    within 1e-5."""
    from paper_1502_01629_amd import capi

    inst = I.disc_problem(129, eps)
    print(f"solve n=129 eps={eps} scheme={scheme}", flush=True)
    dp = capi.DeviceProblem(inst, scheme)
    v = _dev(inst.initial())
    st = ctx.solve(dp, v, tol=5e-7, max_sweeps=20000, check_every=4)
    print("gpu", st, flush=True)
    assert st["status"] == 0 or st["residual"] < 2e-6
    p = oracle.Problem.from_instance(inst, scheme)
    ref, sweeps, r, _ = p.solve(tol=1e-10, threads=8)
    got = v.cpu().numpy().reshape(-1).astype(np.float64)
    err = np.abs(got - ref).max()
    print("max abs err", err, "gpu sweeps", st["sweeps"], "oracle sweeps", sweeps, flush=True)
    assert err < 1e-5


def test_solve_reports_not_converged(ctx):
    from paper_1502_01629_amd import capi

    inst = I.disc_problem(65, 0.0)
    dp = capi.DeviceProblem(inst, 1)
    v = _dev(inst.initial())
    st = ctx.solve(dp, v, tol=1e-12, max_sweeps=5, check_every=2)
    assert st["status"] == capi.NOT_CONVERGED and st["sweeps"] == 5


def test_invalid_arguments_launch_nothing(ctx):
    from paper_1502_01629_amd import capi

    inst = I.disc_problem(33, 0.0)
    dp = capi.DeviceProblem(inst, 1)
    v = _dev(inst.initial())
    before = v.clone()
    dp.struct.h = -1.0
    with pytest.raises(capi.SlhjbError) as e:
        ctx.solve(dp, v)
    assert e.value.status == capi.E_INVALID_ARG
    dp.struct.h = float(inst.h)
    dp.speed[3] = -1.0
    with pytest.raises(capi.SlhjbError) as e:
        ctx.solve(dp, v)
    assert e.value.status == capi.E_INVALID_ARG
    assert torch.equal(v, before)

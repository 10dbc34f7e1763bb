"""slhjb_solve_noalloc, the Jacobi solve that allocates nothing (its scratch is a static device array
of the library): the same results and statistics as slhjb_solve, bit for bit, on two calls in a
row, the second on a smaller grid (the static scratch keeps the first call's contents), and a clear
rejection of a grid above its maximum."""
import numpy as np
import pytest

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


def test_noalloc_equals_solve_on_two_calls(ctx):
    from paper_1502_01629_amd import capi

    big = I.scattered_problem(1, n=257, n_coarse=65, eps=8e-3)[0]  # general kernels, halo 3
    small = I.disc_problem(129, 0.0)                                 # first-ring kernels
    for inst in (big, small):
        print(f"noalloc n={inst.n} eps={float(inst.eps)}", flush=True)
        dp = capi.DeviceProblem(inst, capi.SL3)
        v_ref = _dev(inst.initial())
        s_ref = ctx.solve(dp, v_ref, tol=5e-7, max_sweeps=100_000, check_every=8)
        v = _dev(inst.initial())
        s = ctx.solve_noalloc(dp, v, tol=5e-7, max_sweeps=100_000, check_every=8)
        print("  solve", s_ref["sweeps"], s_ref["residual"], "noalloc", s["sweeps"], s["residual"], flush=True)
        assert s_ref["status"] == 0 and s["status"] == 0
        assert torch.equal(v, v_ref)
        for k in ("sweeps", "converged_sweep", "node_updates", "residual", "kernel_path", "halo"):
            assert s[k] == s_ref[k], k


def test_noalloc_rejects_grids_above_its_maximum(ctx):
    from paper_1502_01629_amd import capi

    inst = I.disc_problem(1027, 0.0)
    dp = capi.DeviceProblem(inst, capi.SL3)
    v = _dev(inst.initial())
    before = v.clone()
    with pytest.raises(capi.SlhjbError) as e:
        ctx.solve_noalloc(dp, v, tol=1e-6, max_sweeps=10)
    assert e.value.status == capi.E_INVALID_ARG and "at most 1025^2" in str(e.value)
    assert torch.equal(v, before)

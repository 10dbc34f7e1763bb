"""Batched solve of independent instances: every instance bit-for-bit equal to its own
single-instance Jacobi solve (same arithmetic, check cadence and stopping rule), whatever the
tile shape, with instances of different sizes, diffusions and control sets in the same launches."""
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


def _mixed(seed):
    """Sizes with ragged tiles, first-ring and general paths, ISO and RANK1 diffusion."""
    out = I.batch_problems(seed, count=6, sizes=(65, 100, 129))
    out.append(I.disc_problem(129, 0.0))                    # sigma = 0, first-ring path
    out.append(I.disc_problem(97, 0.01))                     # ISO, general path
    fine, _ = I.scattered_problem(seed, n=161, n_coarse=41)  # obstacles, variable speed, sigma = 0
    out.append(fine)
    out.append(I.rank1_walk_problem(33))                     # RANK1
    return out


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("shapes", ["default", "mixed"])
def test_batch_bit_exact_vs_single_instance(ctx, scheme, shapes):
    from paper_1502_01629_amd import capi

    insts = _mixed(scheme)
    probs = [capi.DeviceProblem(x, scheme) for x in insts]
    starts = [x.initial() for x in insts]
    tile_shapes = None if shapes == "default" else [k % 4 for k in range(len(insts))]
    vs = [_dev(s0) for s0 in starts]
    print(f"batch of {len(insts)} scheme={scheme} shapes={shapes}", flush=True)
    stats, tot = ctx.solve_batch(probs, vs, tol=1e-6, max_sweeps=20000, check_every=8, tile_shapes=tile_shapes)
    print(tot, flush=True)
    assert tot["status"] == 0 and tot["converged"] == len(insts)
    for k, (p, s0) in enumerate(zip(probs, starts)):
        v1 = _dev(s0)
        st1 = ctx.solve(p, v1, tol=1e-6, max_sweeps=20000, check_every=8)
        assert torch.equal(vs[k], v1), f"instance {k} differs from its single-instance solve"
        assert stats[k]["sweeps"] == st1["sweeps"] and stats[k]["converged_sweep"] == st1["converged_sweep"]
        assert stats[k]["residual"] == st1["residual"] and stats[k]["node_updates"] == st1["node_updates"]


def test_batch_max_sweeps_and_partial_last_batch(ctx):
    """A sweep budget that is not a multiple of check_every: the last batch is shorter, and every
    instance stops where the single-instance call stops."""
    from paper_1502_01629_amd import capi

    insts = _mixed(3)[:5]
    probs = [capi.DeviceProblem(x, 1) for x in insts]
    vs = [_dev(x.initial()) for x in insts]
    stats, tot = ctx.solve_batch(probs, vs, tol=1e-9, max_sweeps=45, check_every=16)
    assert tot["status"] == 1 and tot["sweeps"] == 45
    for k, p in enumerate(probs):
        v1 = _dev(insts[k].initial())
        st1 = ctx.solve(p, v1, tol=1e-9, max_sweeps=45, check_every=16)
        assert st1["status"] == 1 and stats[k]["status"] == 1
        assert torch.equal(vs[k], v1) and stats[k]["sweeps"] == 45


def test_batch_matches_oracle(ctx):
    from paper_1502_01629_amd import capi

    insts = [I.disc_problem(129, 0.01), I.disc_problem(129, 0.0)] + I.batch_problems(5, count=2, sizes=(65,))
    probs = [capi.DeviceProblem(x, 1) for x in insts]
    vs = [_dev(x.initial()) for x in insts]
    # FP32 iterates near w = 1 stagnate at a few ulp (6e-8): 1e-6 is the tolerance of the method
    stats, tot = ctx.solve_batch(probs, vs, tol=1e-6, max_sweeps=50000, check_every=4)
    assert tot["converged"] == len(insts)
    for k, x in enumerate(insts):
        ref, _, _, _ = oracle.Problem.from_instance(x, 1).solve(tol=1e-10, threads=8)
        err = np.abs(vs[k].cpu().numpy().astype(np.float64) - ref).max()
        print(k, "max abs err vs oracle", err, flush=True)
        assert err < 1e-5


def test_batch_rejects_bad_arguments(ctx):
    from paper_1502_01629_amd import capi

    a, b = I.disc_problem(33, 0.0), I.disc_problem(33, 0.0)
    pa, pb = capi.DeviceProblem(a, 0), capi.DeviceProblem(b, 1)
    va, vb = _dev(a.initial()), _dev(b.initial())
    with pytest.raises(capi.SlhjbError):
        ctx.solve_batch([pa, pb], [va, vb])  # schemes differ
    with pytest.raises(capi.SlhjbError):
        ctx.solve_batch([pb], [vb], tile_shapes=[7])

"""GPU parity of the solver paths the benchmark times, at their default settings, against the FP64
oracle's exact fixed points (stored by tests/golden/make_parity_references.py, which calls only the
oracle: Howard's policy iteration, certified by max |T(v) - v| <= 1e-14).

* rank-1 diffusion sigma = sqrt(2 eps) a on a 257^2 bump-speed problem with eps = 2 dx (noise feet
  two cells out: interpolation halo 4), through the active-tile solver from the cold start and from
  u_hat of a coarse sigma = 0 solve (tiles by increasing u_hat), 14 policy-evaluation iterations per
  full one, and through plain Jacobi sweeps;
* the scattered-targets geometry (obstacles, c = 1 + 0.5 sin sin, 64 controls, h = dx / 1.5) on
  257^2 with isotropic diffusion at eps = 8e-3 and 8e-2, the benchmark's 1e-3 and 1e-2 scaled to
  the same noise reach in cells (halos 3 and 5), through the whole patchy pipeline (coarse solve,
  u_hat, synthesis, 64 patch labels, u_hat-ordered fine solve) and the static decomposition.

Tolerance: 1e-5 max-abs over every node (the bound of the other parity tests). The solves stop at a
full-sweep change of 5e-7 (below that the FP32 iterate of the rank-1 case changes by a few ulp per
sweep and never settles); the a-posteriori bound of the contraction (factor beta / (1 - beta) <= 192
on these grids) allows 1e-4 at worst, the errors measured are about 1e-6.
"""
import os

import numpy as np
import pytest

from paper_1502_01629_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL_STOP = 5e-7
POLICY_SWEEPS_DIFFUSION = 14


@pytest.fixture(scope="module")
def ctx():
    from paper_1502_01629_amd import capi

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = capi.Context(0)
    yield c
    c.close()


def _ref(name):
    g = np.load(os.path.join(GOLDEN, f"{name}_fixed_point.npz"))
    assert g["bellman_residual"] <= 1e-13
    return g["v"]


def _dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype).reshape(-1)).cuda()


def _err(v, ref):
    return float(np.abs(v.cpu().numpy().astype(np.float64) - ref).max())


@pytest.mark.parametrize("start", ["cold", "uhat", "jacobi"])
def test_rank1_bumps_257(ctx, start):
    from paper_1502_01629_amd import capi

    x = I.bumps_problem(0, n=257, eps=2.0 * 2.0 / 256)
    print(f"rank-1 bumps 257^2 eps={float(x.eps)} start={start}", flush=True)
    ref = _ref("bumps257_rank1")
    dp = capi.DeviceProblem(x, capi.SL3)
    if start == "jacobi":
        v = _dev(x.initial())
        st = ctx.solve(dp, v, tol=TOL_STOP, max_sweeps=200_000)
    elif start == "cold":
        v = _dev(x.initial())
        st = ctx.solve_tiles(dp, v, tol=TOL_STOP, order=capi.ORDER_NONE, max_passes=200_000,
                             policy_sweeps=POLICY_SWEEPS_DIFFUSION)
    else:
        # u_hat of a sigma = 0 coarse solve (ratio 16, as the benchmark's 257^2 -> 4097^2)
        xc = I.bumps_problem(0, n=17, eps=0.0)
        xc.diffusion = I.DIFF_NONE
        dpc = capi.DeviceProblem(xc, capi.SL3)
        vc = _dev(xc.initial())
        ctx.solve_tiles(dpc, vc, tol=1e-7, tile_shape=capi.TILE_8x8_SPLIT4, max_passes=20000)
        v = torch.empty(x.n * x.n, dtype=torch.float32, device="cuda")
        ctx.upsample(vc, xc.n, v, x.n)
        st = ctx.solve_tiles(dp, v, tol=TOL_STOP, order=capi.ORDER_KEYS, max_passes=200_000,
                             policy_sweeps=POLICY_SWEEPS_DIFFUSION)
    err = _err(v, ref)
    print(f"  status {st['status']} halo {st['halo']} passes/sweeps {st['sweeps']} max|gpu - oracle| {err:.3e}",
          flush=True)
    assert st["status"] == 0 and st["halo"] == 4
    assert err < 1e-5


@pytest.mark.parametrize("mode", ["patchy", "static"])
@pytest.mark.parametrize("eps,halo", [(8e-3, 3), (8e-2, 5)])
def test_scattered_257_diffusion(ctx, eps, halo, mode):
    from paper_1502_01629_amd import capi

    fine, coarse = I.scattered_problem(1, n=257, n_coarse=65, eps=eps)
    print(f"scattered 257^2 eps={eps} mode={mode}", flush=True)
    ref = _ref({8e-3: "scattered257_eps8e-3", 8e-2: "scattered257_eps8e-2"}[eps])
    dp, dpc = capi.DeviceProblem(fine, capi.SL3), capi.DeviceProblem(coarse, capi.SL3)
    v = torch.empty(fine.n * fine.n, dtype=torch.float32, device="cuda")
    if mode == "patchy":
        src, _ = capi.partition_sources(fine.node_class, 64)
        lab = torch.empty(fine.n * fine.n, dtype=torch.int16, device="cuda")
        st = ctx.solve_patchy(dp, dpc, v, mode=capi.PATCHY_TRANSMISSION, tol=TOL_STOP, tol_coarse=1e-7,
                              source_patch=_dev(src, np.int16), n_patches=64, label_out=lab,
                              policy_sweeps=POLICY_SWEEPS_DIFFUSION)
        assert int((lab >= 0).sum()) > 0
    else:
        st = ctx.solve_patchy(dp, None, v, mode=capi.PATCHY_STATIC, tol=TOL_STOP,
                              policy_sweeps=POLICY_SWEEPS_DIFFUSION)
    err = _err(v, ref)
    print(f"  status {st['status']} passes {st['passes']} max|gpu - oracle| {err:.3e}", flush=True)
    assert st["status"] == 0
    j = ctx.solve(dp, v.clone(), tol=1.0, max_sweeps=1)
    assert j["halo"] == halo
    assert err < 1e-5

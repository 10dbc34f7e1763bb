"""GPU parity of the active-tile solver (transmission and independent patches, static and u_hat
order) against the FP64 oracle's fixed points."""
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


def _dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype).reshape(-1)).cuda()


def _uhat(fine, coarse):
    vc, _, _, _ = oracle.Problem.from_instance(coarse, oracle.SL3).solve(tol=1e-10, threads=8)
    return oracle.upsample_bilinear(vc, fine.n).astype(np.float32)


@pytest.mark.parametrize("shape", [1, 2, 3, 4])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("eps", [0.0, 0.01])
@pytest.mark.parametrize("scheme", [0, 1])
def test_tiles_transmission_matches_global_fixed_point(ctx, order, eps, scheme, shape):
    from paper_1502_01629_amd import capi

    inst = I.disc_problem(129, eps)
    print(f"tiles disc eps={eps} order={order} scheme={scheme}", flush=True)
    dp = capi.DeviceProblem(inst, scheme)
    if order == 1:
        # start from u_hat of a coarse (65^2, sigma = 0) solve, as the paper's computation step does
        coarse = I.disc_problem(65, 0.0)
        v = _dev(_uhat(inst, coarse))
    else:
        v = _dev(inst.initial())
    st = ctx.solve_tiles(dp, v, tol=5e-7, order=order, max_passes=20000, tile_shape=shape)
    print(st, flush=True)
    assert st["status"] == 0 and st["residual"] <= 5e-7
    ref, _, _, _ = oracle.Problem.from_instance(inst, scheme).solve(tol=1e-10, threads=8)
    err = np.abs(v.cpu().numpy().astype(np.float64) - ref).max()
    print("max abs err", err, flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("order", [0, 1])
def test_tiles_scattered_obstacles(ctx, order, shape):
    """Point targets, obstacles and variable speed on 257^2 (ragged tiles), cold and u_hat starts."""
    from paper_1502_01629_amd import capi

    fine, coarse = I.scattered_problem(1, n=257, n_coarse=65)
    dp = capi.DeviceProblem(fine, 1)
    v = _dev(_uhat(fine, coarse) if order == 1 else fine.initial())
    st = ctx.solve_tiles(dp, v, tol=5e-7, order=order, max_passes=20000, tile_shape=shape)
    print(st, flush=True)
    assert st["status"] == 0
    ref, sweeps, _, _ = oracle.Problem.from_instance(fine, 1).solve(tol=1e-10, threads=8)
    err = np.abs(v.cpu().numpy().astype(np.float64) - ref).max()
    print("max abs err", err, "oracle Jacobi sweeps", sweeps, "tile updates per node",
          st["node_updates"] / (fine.node_class == 0).sum(), flush=True)
    assert err < 1e-5


def _independent_fixed_point(p, label):
    w = p.initial()
    for _ in range(100000):
        w, r = p.sweep_independent(label, w, threads=8)
        if r < 1e-12:
            break
    return w


@pytest.mark.parametrize("shape", [1, 2, 3])
@pytest.mark.parametrize("layout", ["sectors", "stripes"])
def test_tiles_independent_patches_match_oracle(ctx, layout, shape):
    """State constraints at patch interfaces: the fixed point of the per-patch problems. Sectors around
    the target are invariant under the optimal (radial) dynamics, so the constraint costs nothing
    (the property the patchy decomposition is built for, Section 2); stripes cut the characteristics
    and change the solution near the interfaces."""
    from paper_1502_01629_amd import capi

    n = 129
    inst = I.disc_problem(n, 0.0)
    X1, X2 = I.node_coords(n)
    if layout == "sectors":
        label = np.minimum((4 * (np.arctan2(X2, X1) + np.pi) / (2 * np.pi)).astype(np.int16), 3)
    else:
        label = ((np.arange(n)[None, :] // 24) % 3 + np.zeros((n, 1), dtype=np.int64)).astype(np.int16)
    dp = capi.DeviceProblem(inst, 1)
    v = _dev(inst.initial())
    st = ctx.solve_tiles(dp, v, tol=5e-7, mode=capi.MODE_INDEPENDENT, label=_dev(label, np.int16), max_passes=20000,
                         tile_shape=shape)
    assert st["status"] == 0
    p = oracle.Problem.from_instance(inst, 1)
    w = _independent_fixed_point(p, label)
    got = v.cpu().numpy().astype(np.float64)
    err = np.abs(got - w).max()
    glob, _, _, _ = p.solve(tol=1e-10, threads=8)
    dec = np.abs(w - glob).max()
    print(layout, "independent err", err, "decomposition error", dec, flush=True)
    assert err < 1e-5
    if layout == "sectors":
        assert dec < 1e-9
    else:
        assert dec > 1e-2


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
def test_persistent_and_host_driven_agree_bit_for_bit(ctx, order, shape):
    """Both drivers read the previous pass's iterate in every visit (the host-driven passes write
    each tile to the other of two arrays, the cooperative kernel stages and commits after all
    visits), so the result does not depend on which workgroup visits which tile, nor on the
    driver."""
    from paper_1502_01629_amd import capi

    fine, coarse = I.scattered_problem(2, n=257, n_coarse=65)
    dp = capi.DeviceProblem(fine, 1)
    start = _uhat(fine, coarse) if order == 1 else fine.initial()
    out = []
    for persistent in (0, 1):
        v = _dev(start)
        st = ctx.solve_tiles(dp, v, tol=5e-7, order=order, tile_shape=shape, persistent=persistent,
                             max_passes=20000)
        print("persistent", persistent, st, flush=True)
        assert st["status"] == 0
        out.append((v.cpu().numpy(), st["sweeps"], st["node_updates"]))
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("eps,shape,pe", [(0.0, 4, 16), (0.008, 4, 8), (0.0, 1, 0)])
@pytest.mark.parametrize("max_passes", [5, 37])
def test_stopped_solve_matches_the_cooperative_driver(ctx, order, eps, shape, pe, max_passes):
    """A solve stopped at max_passes before it converged. The batched driver (one instance) and the
    cooperative driver both stop after exactly max_passes passes that did work; the first writes
    tiles to the other of two arrays and gathers the ones left there at the end, the second
    stages and commits after every pass. Their iterates must agree bit for bit, so the gather of
    an unfinished solve is checked too."""
    from paper_1502_01629_amd import capi

    fine, coarse = I.scattered_problem(2, n=257, n_coarse=65, eps=eps)
    dp = capi.DeviceProblem(fine, 1)
    start = _uhat(fine, coarse) if order == 1 else fine.initial()
    print(f"stopped solve order={order} eps={eps} shape={shape} pe={pe} max_passes={max_passes}", flush=True)
    v_b = _dev(start)
    stats, tot = ctx.solve_tiles_batch([dp], [v_b], tol=1e-9, max_passes=max_passes, order=order,
                                       tile_shape=shape, policy_sweeps=pe)
    v_c = _dev(start)
    st = ctx.solve_tiles(dp, v_c, tol=1e-9, max_passes=max_passes, order=order, tile_shape=shape,
                         policy_sweeps=pe, persistent=1)
    # (the 16 x 16 one-node-per-lane tiles in plain order reach an exact FP32 fixed point within 37
    # passes: then both drivers must have stopped at the same converged pass)
    assert (tot["converged"] == 1) == (st["status"] == 0)
    assert stats[0]["sweeps"] == st["sweeps"]
    assert st["status"] == 0 or st["sweeps"] == max_passes
    assert stats[0]["node_updates"] == st["node_updates"]
    assert torch.equal(v_b, v_c)
    assert not torch.equal(v_b, _dev(start))  # the passes did change the iterate


@pytest.mark.parametrize("shape", [2, 4])
@pytest.mark.parametrize("pe", [2, 8])
@pytest.mark.parametrize("eps,scheme", [(0.0, 1), (0.0, 0), (0.01, 1)])
def test_policy_evaluation_iterations_reach_the_same_fixed_point(ctx, shape, pe, eps, scheme):
    """Modified policy iteration inside the visits: cheap iterations with each node's maximising
    control between full ones; the fixed point, and so the oracle's solution, is unchanged."""
    from paper_1502_01629_amd import capi

    inst = I.disc_problem(129, eps)
    dp = capi.DeviceProblem(inst, scheme)
    v = _dev(inst.initial())
    st = ctx.solve_tiles(dp, v, tol=5e-7, order=0, max_passes=20000, tile_shape=shape, policy_sweeps=pe,
                         max_inner=16 if eps > 0 else 0)
    print(st, flush=True)
    assert st["status"] == 0 and st["residual"] <= 5e-7
    assert st["policy_updates"] > 0
    ref, _, _, _ = oracle.Problem.from_instance(inst, scheme).solve(tol=1e-10, threads=8)
    err = np.abs(v.cpu().numpy().astype(np.float64) - ref).max()
    print("max abs err", err, flush=True)
    assert err < 1e-5


def test_policy_evaluation_on_scattered_obstacles_uhat_order(ctx):
    from paper_1502_01629_amd import capi

    fine, coarse = I.scattered_problem(1, n=257, n_coarse=65)
    dp = capi.DeviceProblem(fine, 1)
    v = _dev(_uhat(fine, coarse))
    st = ctx.solve_tiles(dp, v, tol=5e-7, order=1, max_passes=20000, policy_sweeps=4)
    assert st["status"] == 0 and st["policy_updates"] > 0
    ref, _, _, _ = oracle.Problem.from_instance(fine, 1).solve(tol=1e-10, threads=8)
    assert np.abs(v.cpu().numpy().astype(np.float64) - ref).max() < 1e-5


def test_cached_pass_graphs_replay_and_rekey(ctx):
    """The context keeps instantiated pass graphs keyed by every launch argument. A repeated solve
    (cache hit) must give the same bits and statistics as the first; a solve that differs in one
    argument (the tolerance) must not replay the old graph: it meets its own tolerance and equals,
    bit for bit, the same solve on a fresh context (which has to capture it)."""
    from paper_1502_01629_amd import capi

    inst = I.scattered_problem(3, n=257, n_controls=32, n_coarse=65)[0]
    dp = capi.DeviceProblem(inst, capi.SL3)
    v0 = _dev(inst.initial())
    outs = []
    for tol in (1e-5, 1e-5, 1e-6):
        v = v0.clone()
        st = ctx.solve_tiles(dp, v, tol=tol, order=capi.ORDER_KEYS, policy_sweeps=16, max_passes=100_000)
        assert st["status"] == 0 and st["residual"] <= tol
        outs.append((v.cpu().numpy(), st))
    assert np.array_equal(outs[0][0], outs[1][0])
    for k in ("sweeps", "node_updates", "policy_updates", "residual"):
        assert outs[0][1][k] == outs[1][1][k], k
    fresh = capi.Context(0)
    try:
        v = v0.clone()
        st = fresh.solve_tiles(dp, v, tol=1e-6, order=capi.ORDER_KEYS, policy_sweeps=16, max_passes=100_000)
        assert np.array_equal(v.cpu().numpy(), outs[2][0])
        assert st["sweeps"] == outs[2][1]["sweeps"]
    finally:
        fresh.close()

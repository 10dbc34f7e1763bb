"""The learned warm start on the GPU: network forward pass and gradients against the FP64
reference (bfloat16 rounding emulated at the same points), Adam against its definition, the
projection to a start of the SL iteration, and what a trained network gains over u_hat."""
import numpy as np
import pytest

from oracle import cnn
from paper_1502_01629_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DIL = (1, 2, 4, 8, 16, 1)


@pytest.fixture(scope="module")
def ctx():
    from paper_1502_01629_amd import capi

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = capi.Context(0)
    yield c
    c.close()


def _frame(seed, n=65):
    """A problem and synthetic u_hat / v* fields on it (host float32 and device copies)."""
    from paper_1502_01629_amd import capi

    fine, _ = I.warmstart_problems(seed, count=1, n=n, n_coarse=17)[0]
    rng = np.random.default_rng(seed)
    X1, X2 = I.node_coords(n)
    uhat = (0.5 + 0.3 * np.sin(3 * X1) * np.cos(2 * X2)).astype(np.float32)
    vstar = (uhat + 0.05 * rng.standard_normal((n, n))).astype(np.float32)
    dp = capi.DeviceProblem(fine, capi.SL3)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).cuda()
    return fine, dp, uhat, vstar, dev(uhat), dev(vstar)


def _random_params(net, seed):
    from paper_1502_01629_amd import warmstart

    p = warmstart.init_params(net, seed)
    rng = np.random.default_rng(seed + 100)
    lay, _ = cnn.layout(net.layers, net.channels)
    for name, o, shape in lay:
        if name.startswith("b"):
            p[o:o + shape[0]] = rng.normal(0.0, 0.05, size=shape).astype(np.float32)
        if name == "hw":
            p[o:o + shape[0]] = rng.normal(0.0, 0.2, size=shape).astype(np.float32)
    return p


def _ref_inputs(fine, uhat, vstar, crops, margin=sum(DIL)):
    feats, uh, vs, mask = [], [], [], []
    f = cnn.features(uhat.astype(np.float64), fine.speed.astype(np.float64), fine.node_class, float(fine.eps))
    for (x0, y0, c) in crops:
        sl = (slice(y0, y0 + c), slice(x0, x0 + c))
        feats.append(f[sl])
        uh.append(uhat[sl].astype(np.float64))
        vs.append(vstar[sl].astype(np.float64))
        mask.append(cnn.crop_mask(fine.node_class, x0, y0, c, fine.n, margin))
    return np.stack(feats), np.stack(uh), np.stack(vs), np.stack(mask)


@pytest.mark.parametrize("crop", [40, 65])
def test_forward_matches_reference(ctx, crop):
    from paper_1502_01629_amd import capi

    fine, dp, uhat, vstar, duh, dvs = _frame(1)
    net = capi.Net(ctx, 6, 32, DIL)
    p = _random_params(net, 3)
    net.set_params(p)
    crops = [(0, 0, crop), (65 - crop, 65 - crop, crop)]
    out = torch.empty(len(crops) * crop * crop, dtype=torch.float32, device="cuda")
    net.forward([(duh, None, dp, x0, y0) for (x0, y0, _) in crops], crop, out)
    feats, _, _, _ = _ref_inputs(fine, uhat, vstar, crops)
    _, ref = cnn.forward(p.astype(np.float64), 6, 32, DIL, feats, emulate=True)
    got = out.cpu().numpy().reshape(ref.shape)
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    print(f"crop {crop}: delta scale {scale:.3e}, max err {err.max():.3e}, mean err {err.mean():.3e}", flush=True)
    # bfloat16 activations: where the FP32 and FP64 sums land on opposite sides of a rounding
    # boundary an activation flips by one bfloat16 ulp (2^-8 relative, 2^-7 at magnitude ~1); a
    # flip reaches every pixel of its 65-pixel receptive field through weights of ~0.2, and a few
    # can meet at one pixel: the maximum is bounded by 1% of the scale, the mean by 1e-3 of it; a
    # systematic difference would move the median, which these rare flips leave near zero
    print(f"  median err {np.median(err):.3e}", flush=True)
    assert err.max() <= 1e-2 * scale
    assert err.mean() <= 1e-3 * scale
    assert np.median(err) <= 2e-4 * scale
    net.close()


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_features_are_exact(ctx, k):
    """A one-layer network whose centre tap copies feature k into channels k and k + 8 with signs
    + and -, and a head (+1, -1): delta = relu(f) - relu(-f) = f exactly (every product is by 1)."""
    from paper_1502_01629_amd import capi

    fine, dp, uhat, vstar, duh, dvs = _frame(6)
    net = capi.Net(ctx, 1, 32, (1,))
    lay, total = cnn.layout(1, 32)
    p = np.zeros(total, dtype=np.float32)
    W = p[:9 * 32 * cnn.CIN0].reshape(9, 32, cnn.CIN0)
    W[4, k, k] = 1.0
    W[4, k + 8, k] = -1.0
    hw = dict((name, o) for name, o, _ in lay)["hw"]
    p[hw + k] = 1.0
    p[hw + k + 8] = -1.0
    net.set_params(p)
    out = torch.empty(65 * 65, dtype=torch.float32, device="cuda")
    net.forward([(duh, None, dp, 0, 0)], 65, out)
    f = cnn.features(uhat.astype(np.float64), fine.speed.astype(np.float64), fine.node_class, float(fine.eps))
    assert np.array_equal(out.cpu().numpy().reshape(65, 65).astype(np.float64), f[..., k])
    net.close()


def test_gradients_match_reference(ctx):
    from paper_1502_01629_amd import capi

    fine, dp, uhat, vstar, duh, dvs = _frame(2)
    net = capi.Net(ctx, 6, 32, DIL)
    p = _random_params(net, 5)
    net.set_params(p)
    # crops that touch two sides of the frame keep a masked region beyond the receptive-field margin
    crops = [(0, 0, 48), (17, 17, 48), (0, 17, 48), (17, 0, 48)]
    loss = net.loss_grad([(duh, dvs, dp, x0, y0) for (x0, y0, _) in crops], 48)
    g = net.get_grads().astype(np.float64)
    feats, uh, vs, mask = _ref_inputs(fine, uhat, vstar, crops)
    rloss, rg = cnn.loss_and_grads(p.astype(np.float64), 6, 32, DIL, feats, uh, vs, mask, emulate=True)
    print("loss", loss, rloss, flush=True)
    assert abs(loss - rloss) <= 1e-3 * rloss
    lay, _ = cnn.layout(6, 32)
    for name, o, shape in lay:
        k = int(np.prod(shape))
        a, b = g[o:o + k], rg[o:o + k]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        scale = np.abs(b).max()
        d = np.abs(a - b) / max(scale, 1e-30)
        print(f"{name}: |g| {np.linalg.norm(b):.3e} rel err {rel:.2e}; per element / block max: max {d.max():.2e} "
              f"p99 {np.quantile(d, 0.99):.2e} median {np.median(d):.2e}", flush=True)
        # Element by element, relative to the block's largest gradient: both sides round the same
        # activations and back-propagated errors to bfloat16 (relative step 2^-8), so the only
        # difference is FP32 against FP64 accumulation order, which moves a rounding of the
        # reference by one bfloat16 ulp where a sum lands near a rounding boundary. Measured: at
        # most 4.5e-4 of the block scale; the bound is 2^-9 (half a bfloat16 ulp) of it.
        assert d.max() <= 2.0 ** -9, name
        assert rel <= 2e-3, name
    net.close()


def test_adam_steps_match_reference(ctx):
    from paper_1502_01629_amd import capi

    fine, dp, uhat, vstar, duh, dvs = _frame(3)
    net = capi.Net(ctx, 2, 32, (1, 2))
    p = _random_params(net, 7)
    net.set_params(p)
    m = np.zeros(p.size)
    v = np.zeros(p.size)
    ref = p.astype(np.float64)
    for step in (1, 2):
        net.loss_grad([(duh, dvs, dp, 25, 25 * (step - 1))], 40)
        g = net.get_grads().astype(np.float64)
        net.adam_step(1e-3)
        ref, m, v = cnn.adam(ref, g, m, v, step, 1e-3)
        got = net.get_params().astype(np.float64)
        # FP32 state on the device: a few ulp of the parameters, relative to the step size 1e-3
        assert np.abs(got - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
        ref = got
    net.close()


def test_warm_start_projection(ctx):
    """A network with only its head bias set: delta is that constant, and the start is the clamped
    u_hat + delta on FREE nodes and the boundary data elsewhere."""
    from paper_1502_01629_amd import capi

    fine, dp, uhat, vstar, duh, dvs = _frame(4)
    net = capi.Net(ctx, 2, 32, (1, 1))
    p = np.zeros(net.param_count, dtype=np.float32)
    p[-1] = 0.25
    net.set_params(p)
    g = torch.empty_like(duh)
    net.warm_start(dp, duh, g)
    want = np.where(fine.node_class == I.FREE, np.clip(uhat + np.float32(0.25), 0.0, 1.0),
                    np.where(fine.node_class == I.TARGET, fine.target_value, fine.v_out)).astype(np.float32)
    assert np.array_equal(g.cpu().numpy().reshape(want.shape), want)
    net.close()


def test_trained_network_gains_over_uhat(ctx):
    """Train on the method's own solves (257^2, coarse 65^2, the batch law), then on held-out
    problems compare the start error and the plain Jacobi sweeps from u_hat and from the network."""
    from paper_1502_01629_amd import capi, warmstart

    pairs = I.warmstart_problems(21, count=20, n=257, n_coarse=65)
    frames = warmstart.make_frames(ctx, pairs)
    train, test = frames[:16], frames[16:]
    net = capi.Net(ctx, 6, 32, DIL)
    net.set_params(warmstart.init_params(net, 0))
    losses = warmstart.train(net, train, steps=600, batch=8, crop=128, lr=2e-3)
    print("loss first/last", np.mean(losses[:20]), np.mean(losses[-20:]), flush=True)
    rows = warmstart.evaluate(ctx, net, test)
    for r in rows:
        print({k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}, flush=True)
    e_u = np.mean([r["err_mean_uhat"] for r in rows])
    e_n = np.mean([r["err_mean_network"] for r in rows])
    s_u = np.mean([r["jacobi_sweeps_uhat"] for r in rows])
    s_n = np.mean([r["jacobi_sweeps_network"] for r in rows])
    print(f"held-out mean |start - v*|: u_hat {e_u:.3e}, network {e_n:.3e}; Jacobi sweeps {s_u:.0f} -> {s_n:.0f}",
          flush=True)
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:20])
    assert e_n < e_u
    net.close()

"""The 4-level U-Net warm start on the GPU (slhjb_net with arch = 1): forward pass and gradients
against the FP64 reference oracle/unet.py (bfloat16 rounding emulated at the same points), the
skip wiring exactly, the whole-frame start with padding, and Adam."""
import numpy as np
import pytest

from oracle import cnn, unet
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


def _frame(seed, n=129):
    from paper_1502_01629_amd import capi

    fine, _ = I.warmstart_problems(seed, count=1, n=n, n_coarse=17)[0]
    rng = np.random.default_rng(seed)
    X1, X2 = I.node_coords(n)
    uhat = (0.5 + 0.3 * np.sin(3 * X1) * np.cos(2 * X2)).astype(np.float32)
    vstar = (uhat + 0.05 * rng.standard_normal((n, n))).astype(np.float32)
    dp = capi.DeviceProblem(fine, capi.SL3)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).cuda()
    return fine, dp, uhat, vstar, dev(uhat), dev(vstar)


def _params(seed):
    """He-normal weights (a random sign pattern over every channel), biases of 0.05 scale."""
    rng = np.random.default_rng(seed)
    lay, total = unet.layout()
    p = np.zeros(total, dtype=np.float32)
    for name, o, shape in lay:
        k = int(np.prod(shape))
        if name.startswith("W"):
            p[o:o + k] = rng.normal(0.0, np.sqrt(2.0 / (9 * shape[2])), size=k)
        elif name == "hw":
            p[o:o + k] = rng.normal(0.0, 0.2, size=k)
        else:
            p[o:o + k] = rng.normal(0.0, 0.05, size=k)
    W0 = p[:9 * 32 * 16].reshape(9, 32, 16)
    W0[:, :, 5:] = 0.0
    return p


def _ref_inputs(fine, uhat, vstar, crops, margin=unet.MARGIN):
    f = cnn.features(uhat.astype(np.float64), fine.speed.astype(np.float64), fine.node_class, float(fine.eps))
    feats, uh, vs, mask = [], [], [], []
    for (x0, y0, c) in crops:
        sl = (slice(y0, y0 + c), slice(x0, x0 + c))
        feats.append(f[sl])
        uh.append(uhat[sl].astype(np.float64))
        vs.append(vstar[sl].astype(np.float64))
        mask.append(cnn.crop_mask(fine.node_class, x0, y0, c, fine.n, margin))
    return np.stack(feats), np.stack(uh), np.stack(vs), np.stack(mask)


@pytest.fixture
def net(ctx):
    from paper_1502_01629_amd import capi

    n = capi.Net(ctx, arch=capi.NET_UNET)
    yield n
    n.close()


@pytest.mark.parametrize("crop", [64, 128])
def test_unet_forward_matches_reference(ctx, net, crop):
    fine, dp, uhat, vstar, duh, dvs = _frame(1)
    p = _params(3)
    net.set_params(p)
    crops = [(0, 0, crop), (129 - crop, 129 - crop, crop)]
    out = torch.empty(len(crops) * crop * crop, dtype=torch.float32, device="cuda")
    net.forward([(duh, None, dp, x0, y0) for (x0, y0, _) in crops], crop, out)
    feats, _, _, _ = _ref_inputs(fine, uhat, vstar, crops)
    _, ref = unet.forward(p.astype(np.float64), feats, emulate=True)
    got = out.cpu().numpy().reshape(ref.shape)
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    print(f"crop {crop}: scale {scale:.3e} max {err.max():.3e} mean {err.mean():.3e} median {np.median(err):.3e}",
          flush=True)
    # 14 layers of bfloat16 activations: where an FP32 sum and the FP64 one round an activation to
    # neighbouring bfloat16 values (one ulp, 2^-8 relative) the difference travels on through the
    # following layers and the three scales. Evaluating the same reference with FP32 accumulation
    # (numpy float32 matmuls) differs from the FP64 one by mean 0.8-1.2e-3, median 0.4-1.0e-3 and
    # max 0.75% of the scale on these crops; the bounds are about 3x that.
    assert err.max() <= 2e-2 * scale
    assert err.mean() <= 3e-3 * scale
    assert np.median(err) <= 3e-3 * scale


def test_unet_gradients_match_reference(ctx, net):
    fine, dp, uhat, vstar, duh, dvs = _frame(2)
    p = _params(5)
    net.set_params(p)
    crops = [(0, 0, 128), (1, 1, 128), (0, 1, 128), (1, 0, 128)]
    loss = net.loss_grad([(duh, dvs, dp, x0, y0) for (x0, y0, _) in crops], 128)
    g = net.get_grads().astype(np.float64)
    feats, uh, vs, mask = _ref_inputs(fine, uhat, vstar, crops)
    rloss, rg = unet.loss_and_grads(p.astype(np.float64), feats, uh, vs, mask, emulate=True)
    print("loss", loss, rloss, flush=True)
    assert abs(loss - rloss) <= 1e-3 * rloss
    lay, _ = unet.layout()
    bad = []
    for name, o, shape in lay:
        k = int(np.prod(shape))
        a, b = g[o:o + k], rg[o:o + k]
        scale = np.abs(b).max()
        d = np.abs(a - b) / max(scale, 1e-30)
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print(f"{name}: scale {scale:.3e} rel {rel:.2e} max {d.max():.2e} p99 {np.quantile(d, 0.99):.2e}", flush=True)
        # the FP32-accumulation evaluation of the reference differs from the FP64 one by at most
        # 4.4e-3 (relative L2 per block) and 4.8e-3 (largest element / block scale): about 4x that
        if not (rel <= 2e-2 and d.max() <= 2e-2):
            bad.append(name)
    assert not bad, bad


@pytest.mark.parametrize("k", [0, 4])
def test_unet_feature_through_skip_is_exact(ctx, net, k):
    fine, dp, uhat, vstar, duh, dvs = _frame(6)
    lay, total = unet.layout()
    off = {name: o for name, o, _ in lay}
    p = np.zeros(total, dtype=np.float32)

    def W(l):
        ci, co, _ = unet.LAYERS[l]
        return p[off[f"W{l}"]:off[f"W{l}"] + 9 * co * ci].reshape(9, co, ci)

    W(0)[4, k, k], W(0)[4, k + 8, k] = 1.0, -1.0
    for c in (k, k + 8):
        W(1)[4, c, c] = 1.0
        W(12)[4, c, 64 + c] = 1.0
        W(13)[4, c, c] = 1.0
    p[off["hw"] + k], p[off["hw"] + k + 8] = 1.0, -1.0
    net.set_params(p)
    out = torch.empty(128 * 128, dtype=torch.float32, device="cuda")
    net.forward([(duh, None, dp, 1, 0)], 128, out)
    f = cnn.features(uhat.astype(np.float64), fine.speed.astype(np.float64), fine.node_class, float(fine.eps))
    assert np.array_equal(out.cpu().numpy().reshape(128, 128).astype(np.float64), f[0:128, 1:129, k])


def test_unet_warm_start_pads_the_frame(ctx, net):
    """n = 129 is padded to 136: a network with only its head bias set gives clamp(u_hat + 0.25) on
    FREE nodes and the boundary data elsewhere, over the whole frame."""
    fine, dp, uhat, vstar, duh, dvs = _frame(4)
    p = np.zeros(net.param_count, dtype=np.float32)
    p[-1] = 0.25
    net.set_params(p)
    g = torch.empty_like(duh)
    net.warm_start(dp, duh, g)
    want = np.where(fine.node_class == I.FREE, np.clip(uhat + np.float32(0.25), 0.0, 1.0),
                    np.where(fine.node_class == I.TARGET, fine.target_value, fine.v_out)).astype(np.float32)
    assert np.array_equal(g.cpu().numpy().reshape(want.shape), want)


def test_unet_adam_step(ctx, net):
    fine, dp, uhat, vstar, duh, dvs = _frame(3)
    p = _params(7)
    net.set_params(p)
    net.loss_grad([(duh, dvs, dp, 0, 0)], 64)
    g = net.get_grads().astype(np.float64)
    net.adam_step(1e-3)
    ref, _, _ = cnn.adam(p.astype(np.float64), g, np.zeros(p.size), np.zeros(p.size), 1, 1e-3)
    assert np.abs(net.get_params() - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())


def test_trained_unet_start(ctx, net):
    """Train on the method's own solves (257^2, coarse 65^2, the batch law, bicubic u_hat as input),
    then on held-out problems: the loss falls, the network's start is closer to v* than both
    upsamplings on average, and every start's stopping point of the u_hat-ordered active-tile solve
    is within 1e-4 of the refined v* (the same fixed point whatever the start)."""
    from paper_1502_01629_amd import warmstart

    pairs = I.warmstart_problems(22, count=36, n=257, n_coarse=65)
    frames = warmstart.make_frames(ctx, pairs, bicubic=True)
    train, test = frames[:32], frames[32:]
    net.set_params(warmstart.init_params(net, 0))
    losses = warmstart.train(net, train, steps=500, batch=8, crop=128, lr=1e-3)
    print("loss first/last", np.mean(losses[:20]), np.mean(losses[-20:]), flush=True)
    rows = warmstart.evaluate(ctx, net, test)
    for r in rows:
        print({k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}, flush=True)
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:20])
    e = {m: np.mean([r[f"err_mean_{m}"] for r in rows]) for m in ("uhat", "uhat_bicubic", "network")}
    print("held-out mean |start - v*|", e, flush=True)
    assert e["network"] < min(e["uhat"], e["uhat_bicubic"])
    for r in rows:
        for m in ("uhat", "uhat_bicubic", "network"):
            assert r[f"tiles_err_{m}"] <= 1e-4, (m, r)

"""Pins of the FP64 reference U-Net (CPU only): pooling and upsampling against their adjoints,
every gradient block against central finite differences, and the wiring of the skip connection
(a feature carried through level 0's skip to the head exactly)."""
import numpy as np
import pytest

from oracle import cnn, unet


def test_pool_and_up_are_adjoint_to_their_backward_maps():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 8, 8, 3))
    y = rng.normal(size=(2, 4, 4, 3))
    assert np.isclose((unet.pool(x) * y).sum(), (x * 0.25 * unet.up(y)).sum(), rtol=1e-13)
    assert np.isclose((unet.up(y) * x).sum(), (y * unet.up_adjoint(x)).sum(), rtol=1e-13)
    assert np.array_equal(unet.up(y)[:, 2 * 1 + 1, 2 * 3], y[:, 1, 3])


def _tiny(seed, S=16, B=2):
    rng = np.random.default_rng(seed)
    _, total = unet.layout()
    params = rng.normal(0.0, 0.08, size=total)
    feats = np.zeros((B, S, S, cnn.CIN0))
    feats[..., :5] = rng.uniform(0.0, 1.0, size=(B, S, S, 5))
    uhat = feats[..., 0].copy()
    vstar = uhat + rng.normal(0.0, 0.05, size=uhat.shape)
    mask = (rng.random(uhat.shape) < 0.8).astype(np.float64)
    return params, feats, uhat, vstar, mask


def test_gradients_match_finite_differences():
    params, feats, uhat, vstar, mask = _tiny(1)
    loss, g = unet.loss_and_grads(params, feats, uhat, vstar, mask, emulate=False)
    lay, total = unet.layout()
    rng = np.random.default_rng(2)
    idx = []
    for name, o, shape in lay:
        if name == "W0":  # only the 5 used input channels carry a gradient
            co, ci = shape[1], shape[2]
            cand = [o + (t * co + c) * ci + k for t in range(9) for c in range(co) for k in range(5)]
        else:
            cand = list(range(o, o + int(np.prod(shape))))
        idx += list(rng.choice(cand, size=min(4, len(cand)), replace=False))
    h = 1e-6
    for i in idx:
        e = np.zeros(total)
        e[i] = h
        lp, _ = unet.loss_and_grads(params + e, feats, uhat, vstar, mask, emulate=False)
        lm, _ = unet.loss_and_grads(params - e, feats, uhat, vstar, mask, emulate=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 2e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


@pytest.mark.parametrize("k", [0, 4])
def test_feature_through_the_level0_skip_is_exact(k):
    """Layer 0 copies feature k to channels k and k + 8 (signs + and -), layer 1 is the identity on
    them; every deeper weight is 0, so the concatenation before layer 12 holds them in its skip part
    (channels 64 + c); layers 12 and 13 copy them on, and the head (+1, -1) gives
    relu(f) - relu(-f) = f exactly."""
    lay, total = unet.layout()
    off = {name: o for name, o, _ in lay}
    p = np.zeros(total)

    def W(l):
        ci, co, _ = unet.LAYERS[l]
        return p[off[f"W{l}"]:off[f"W{l}"] + 9 * co * ci].reshape(9, co, ci)

    W(0)[4, k, k], W(0)[4, k + 8, k] = 1.0, -1.0
    for c in (k, k + 8):
        W(1)[4, c, c] = 1.0
        W(12)[4, c, 64 + c] = 1.0
        W(13)[4, c, c] = 1.0
    p[off["hw"] + k], p[off["hw"] + k + 8] = 1.0, -1.0
    rng = np.random.default_rng(k)
    feats = np.zeros((1, 16, 24, cnn.CIN0))
    feats[..., :5] = rng.uniform(-1.0, 1.0, size=(1, 16, 24, 5))
    _, delta = unet.forward(p, feats, emulate=False)
    assert np.array_equal(delta, feats[..., k])

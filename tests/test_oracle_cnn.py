"""Pins of the FP64 reference network (CPU only): the dilated convolution against its loop
definition, and every gradient of the chain rule against central finite differences."""
import numpy as np
import pytest

from oracle import cnn


def _loop_conv(x, w, dil):
    B, H, W, C = x.shape
    Co = w.shape[1]
    y = np.zeros((B, H, W, Co))
    for b in range(B):
        for i in range(H):
            for j in range(W):
                for t in range(9):
                    ii, jj = i + (t // 3 - 1) * dil, j + (t % 3 - 1) * dil
                    if 0 <= ii < H and 0 <= jj < W:
                        y[b, i, j] += w[t] @ x[b, ii, jj]
    return y


@pytest.mark.parametrize("dil", [1, 2, 5])
def test_conv3x3_matches_its_loop_definition(dil):
    rng = np.random.default_rng(dil)
    x = rng.normal(size=(2, 7, 9, 5))
    w = rng.normal(size=(9, 3, 5))
    assert np.allclose(cnn.conv3x3(x, w, dil), _loop_conv(x, w, dil), rtol=0, atol=1e-12)


def _tiny(seed, layers=3, channels=32, dil=(1, 2, 1), H=9, W=11):
    rng = np.random.default_rng(seed)
    _, total = cnn.layout(layers, channels)
    params = rng.normal(0.0, 0.15, size=total)
    feats = np.zeros((2, H, W, cnn.CIN0))
    feats[..., :5] = rng.uniform(0.0, 1.0, size=(2, H, W, 5))
    uhat = feats[..., 0].copy()
    vstar = uhat + rng.normal(0.0, 0.05, size=uhat.shape)
    mask = (rng.random(uhat.shape) < 0.8).astype(np.float64)
    return params, feats, uhat, vstar, mask, layers, channels, dil


def test_gradients_match_finite_differences():
    params, feats, uhat, vstar, mask, L, C, dil = _tiny(0)
    loss, g = cnn.loss_and_grads(params, L, C, dil, feats, uhat, vstar, mask, emulate=False)
    lay, total = cnn.layout(L, C)
    rng = np.random.default_rng(1)
    # every block of the layout: weights of each layer (used input channels), biases, head
    idx = []
    for name, o, shape in lay:
        size = int(np.prod(shape))
        if name == "W0":
            cand = [o + (t * C + co) * cnn.CIN0 + ci for t in range(9) for co in range(C) for ci in range(5)]
        else:
            cand = list(range(o, o + size))
        idx += list(rng.choice(cand, size=min(6, len(cand)), replace=False))
    h = 1e-6
    for i in idx:
        e = np.zeros(total)
        e[i] = h
        lp, _ = cnn.loss_and_grads(params + e, L, C, dil, feats, uhat, vstar, mask, emulate=False)
        lm, _ = cnn.loss_and_grads(params - e, L, C, dil, feats, uhat, vstar, mask, emulate=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_unused_input_channels_have_zero_gradient():
    params, feats, uhat, vstar, mask, L, C, dil = _tiny(2)
    _, g = cnn.loss_and_grads(params, L, C, dil, feats, uhat, vstar, mask, emulate=False)
    W0 = g[:9 * C * cnn.CIN0].reshape(9, C, cnn.CIN0)
    assert np.all(W0[:, :, 5:] == 0.0)


def test_bf16_rounding_is_round_to_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -3.140625, 0.0], dtype=np.float32)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1); 1 + 3 * 2^-8 rounds up to 1 + 2^-6
    assert list(cnn.bf16(x)) == [1.0, 1.0, 1.0 + 2 ** -6, 1.0, -3.140625, 0.0]


def test_adam_first_step_is_sign_times_lr():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = cnn.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # the first bias-corrected step is -lr g / (|g| + eps): the sign, up to eps / |g|
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=2e-5)


def test_adam_second_and_third_steps_match_the_recursion_by_hand():
    """Gradients 1, -1, 2 with beta1 = 0.9, beta2 = 0.999, worked out by hand:
    step 2: m = 0.9 * 0.1 - 0.1 = -0.01, v = 0.999 * 0.001 + 0.001 = 0.001999,
            m_hat = -0.01 / (1 - 0.9^2) = -1/19, v_hat = 0.001999 / (1 - 0.999^2) = 1;
    step 3: m = -0.009 + 0.2 = 0.191, v = 0.999 * 0.001999 + 0.004 = 0.005997001,
            m_hat = 0.191 / (1 - 0.9^3) = 0.191 / 0.271, v_hat = 0.005997001 / 0.002997001.
    A wrong bias-correction power or moment recursion changes steps 2 and 3."""
    lr, e = 0.01, 1e-8
    p, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    p, m, v = cnn.adam(p, np.array([1.0]), m, v, 1, lr=lr)
    p1 = -lr * 1.0 / (1.0 + e)
    assert np.isclose(p[0], p1, rtol=1e-12, atol=0)
    p, m, v = cnn.adam(p, np.array([-1.0]), m, v, 2, lr=lr)
    assert np.isclose(m[0], -0.01, rtol=1e-12) and np.isclose(v[0], 0.001999, rtol=1e-12)
    p2 = p1 + lr * (1.0 / 19.0) / (1.0 + e)
    assert np.isclose(p[0], p2, rtol=1e-12, atol=0)
    p, m, v = cnn.adam(p, np.array([2.0]), m, v, 3, lr=lr)
    assert np.isclose(m[0], 0.191, rtol=1e-12) and np.isclose(v[0], 0.005997001, rtol=1e-12)
    p3 = p2 - lr * (0.191 / 0.271) / (np.sqrt(0.005997001 / 0.002997001) + e)
    assert np.isclose(p[0], p3, rtol=1e-12, atol=0)


def test_crop_mask_keeps_the_margin_from_inner_edges_only():
    cls = np.zeros((20, 20), dtype=np.uint8)
    m = cnn.crop_mask(cls, 0, 6, 10, 20, 3)  # left edge is the box side, the others are inside
    want = np.zeros((10, 10))
    want[3:7, 0:7] = 1.0
    assert np.array_equal(m, want)


def test_boundary_feature_is_one_on_the_box_sides():
    f = cnn.features(np.zeros((9, 9)), np.ones((9, 9)), np.zeros((9, 9), dtype=np.uint8), 1e-3, emulate=False)
    assert np.all(f[0, :, 4] == 1.0) and np.all(f[:, -1, 4] == 1.0)
    assert f[4, 4, 4] == np.float32(1.0) / np.float32(2.0)

"""FP64 reference of the 4-level U-Net of the learned warm start (plain NumPy).

TEST INFRASTRUCTURE ONLY: the GPU network kernels are checked against it; nothing on the product
path imports it. It shares no code with the GPU package (it reuses the dilated network's
reference pieces in oracle/cnn.py: bfloat16 rounding, the shifted-image 3 x 3 convolution, the
features and the crop mask).

The network (the definition of the library's slhjb_net with arch = 1):
  features  f = cnn.features(...) (16 channels, 5 used; channel 0 is the u_hat the caller passes)
  conv l    relu(b_l + 3 x 3 convolution with W_l[t][co][ci]), zero padding, layers
            0: 16->32  1: 32->32            (level 0, full resolution)
            2: 32->64  3: 64->64            (level 1)
            4: 64->128 5: 128->128          (level 2)
            6: 128->128 7: 128->128         (level 3, the bottom)
            8: 256->128 9: 128->128         (level 2: [up(out7), out5])
            10: 192->64 11: 64->64          (level 1: [up(out9), out3])
            12: 96->32 13: 32->32           (level 0: [up(out11), out1])
  down      pool(x)[y][x] = ((x[2y][2x] + x[2y][2x+1]) + (x[2y+1][2x] + x[2y+1][2x+1])) / 4
  up        up(x)[y][x] = x[y // 2][x // 2], concatenated before the level's skip
  head      delta = hb + out13 . hw;  loss as in cnn.loss_and_grads, the mask keeping MARGIN pixels
            (the receptive-field radius, 46) from crop edges inside the frame
Parameters, flat FP32: per layer W_l[9][cout][cin] then b_l[cout]; then hw[32], hb[1].

With emulate=True the reference rounds to bfloat16 where the GPU stores bfloat16: features, conv
weights, every activation (conv outputs, pooled tensors), and in the backward pass every stored
gradient (conv input gradients, the 2 x 2 sums of the upsampling's gradient, the encoder outputs'
combined skip and pooling gradients).
"""
from __future__ import annotations

import numpy as np

from . import cnn

LAYERS = [(16, 32, 0), (32, 32, 0), (32, 64, 1), (64, 64, 1), (64, 128, 2), (128, 128, 2), (128, 128, 3),
          (128, 128, 3), (256, 128, 2), (128, 128, 2), (192, 64, 1), (64, 64, 1), (96, 32, 0), (32, 32, 0)]
MARGIN = 48
HEAD = 32


def layout():
    out, off = [], 0
    for l, (ci, co, _) in enumerate(LAYERS):
        out.append((f"W{l}", off, (9, co, ci)))
        off += 9 * co * ci
        out.append((f"b{l}", off, (co,)))
        off += co
    out.append(("hw", off, (HEAD,)))
    off += HEAD
    out.append(("hb", off, (1,)))
    off += 1
    return out, off


def unpack(params: np.ndarray) -> dict:
    lay, total = layout()
    assert params.size == total
    return {name: np.asarray(params[o:o + int(np.prod(shape))], dtype=np.float64).reshape(shape)
            for name, o, shape in lay}


def pool(x):
    return ((x[:, 0::2, 0::2] + x[:, 0::2, 1::2]) + (x[:, 1::2, 0::2] + x[:, 1::2, 1::2])) * 0.25


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_adjoint(g):
    """The adjoint of up: the sum over each 2 x 2 block."""
    return (g[:, 0::2, 0::2] + g[:, 0::2, 1::2]) + (g[:, 1::2, 0::2] + g[:, 1::2, 1::2])


def _below(lv):
    """Index of the last convolution of the level below decoder level lv (7, 9, 11) and the skip (5, 3, 1)."""
    return 2 * (2 - lv) + 7, 2 * lv + 1


def forward(params, feats, emulate=True):
    """feats [B, S, S, 16] (S a multiple of 8) -> (state, delta [B, S, S])."""
    P = unpack(params)
    rd = cnn.bf16 if emulate else (lambda a: a)

    def conv(l, x):
        w = cnn.bf16(P[f"W{l}"]) if emulate else P[f"W{l}"]
        return rd(np.maximum(cnn.conv3x3(x, w, 1) + P[f"b{l}"], 0.0))

    out = [None] * len(LAYERS)
    out[0] = conv(0, feats)
    out[1] = conv(1, out[0])
    pools = []
    for lv in range(3):
        pools.append(rd(pool(out[2 * lv + 1])))
        out[2 * lv + 2] = conv(2 * lv + 2, pools[lv])
        out[2 * lv + 3] = conv(2 * lv + 3, out[2 * lv + 2])
    cats = [None] * 3
    for lv in (2, 1, 0):
        below, skip = _below(lv)
        cats[lv] = np.concatenate([up(out[below]), out[skip]], axis=-1)
        out[below + 1] = conv(below + 1, cats[lv])
        out[below + 2] = conv(below + 2, out[below + 1])
    delta = out[13] @ P["hw"] + P["hb"][0]
    return dict(out=out, pools=pools, cats=cats, feats=feats), delta


def loss_and_grads(params, feats, uhat, vstar, mask, emulate=True):
    """Loss over the masked pixels and the gradient of every parameter, by the chain rule."""
    P = unpack(params)
    rd = cnn.bf16 if emulate else (lambda a: a)
    st, delta = forward(params, feats, emulate)
    out, pools, cats = st["out"], st["pools"], st["cats"]
    n = float(mask.sum())
    e = (uhat + delta - vstar) * mask
    loss = float((e * e).sum() / n)
    g = 2.0 * e
    grads = {"hw": np.einsum("bhw,bhwc->c", g, out[13]), "hb": np.array([g.sum()])}
    G = [None] * len(LAYERS)
    G[13] = rd(g[..., None] * P["hw"] * (out[13] > 0))

    def back(l, x, gated, need_dx=True):
        dy = G[l]
        w = cnn.bf16(P[f"W{l}"]) if emulate else P[f"W{l}"]
        dW = np.zeros_like(P[f"W{l}"])
        for t, (oy, ox) in enumerate(cnn.offsets(1)):
            dW[t] = np.einsum("bhwo,bhwi->oi", dy, cnn.shift(x, oy, ox))
        grads[f"W{l}"] = dW
        grads[f"b{l}"] = dy.sum(axis=(0, 1, 2))
        if not need_dx:
            return None
        dx = np.zeros(x.shape)
        for t, (oy, ox) in enumerate(cnn.offsets(1)):
            dx += cnn.shift(dy, -oy, -ox) @ w[t]
        if gated:
            dx = dx * (x > 0)
        return rd(dx)

    gcat = [None] * 3
    for lv in (0, 1, 2):
        below, skip = _below(lv)
        G[below + 1] = back(below + 2, out[below + 1], True)
        gcat[lv] = back(below + 1, cats[lv], True)
        G[below] = rd(up_adjoint(gcat[lv][..., :out[below].shape[-1]]))
    G[6] = back(7, out[6], True)
    gpool = [None, None, back(6, pools[2], False)]
    for lv in (2, 1, 0):
        b = 2 * lv + 1
        cu = out[_below(lv)[0]].shape[-1]
        G[b] = rd((out[b] > 0) * (gcat[lv][..., cu:] + 0.25 * up(gpool[lv])))
        G[b - 1] = back(b, out[b - 1], True)
        if lv > 0:
            gpool[lv - 1] = back(b - 1, pools[lv - 1], False)
        else:
            back(0, feats, False, need_dx=False)
    lay, total = layout()
    flat = np.zeros(total)
    for name, o, shape in lay:
        flat[o:o + int(np.prod(shape))] = grads[name].reshape(-1) / n
    return loss, flat

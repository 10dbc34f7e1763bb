"""FP64 reference of the learned warm-start network (plain NumPy).

TEST INFRASTRUCTURE ONLY: the GPU network kernels are checked against it; nothing on the product
path imports it. It shares no code with the GPU package.

The network (the definition of the library's slhjb_net):
  features  x0[p] = [u_hat, c, target mask, log10(eps) + 3, 1 / (1 + d / 4), 0 x 11]  (16 channels)
            d = distance in cells from p to the nearest side of the box
  layer l   x_{l+1}[p][co] = relu(b_l[co] + sum_t sum_ci x_l[p + d_l off_t][ci] W_l[t][co][ci])
            off_t = (t // 3 - 1, t % 3 - 1) in (dy, dx), zero outside the image
  head      delta[p] = hb + sum_c x_L[p][c] hw[c]
  loss      L = mean over the masked p of (u_hat + delta - v*)^2: FREE nodes at least R = sum of
            the dilations away from every crop edge inside the frame (crop_mask)
Parameters, flat FP32: per layer W_l[9][C][cin_l] then b_l[C]; then hw[C], hb.

With emulate=True the reference rounds to bfloat16 where the GPU stores bfloat16 (features, conv
weights, activations, the back-propagated gradients of the conv layers), so that the comparison
measures accumulation order only; with emulate=False it is the exact FP64 function, the one the
finite-difference pins check.
"""
from __future__ import annotations

import numpy as np

CIN0 = 16


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layout(layers: int, channels: int):
    """Offsets and shapes of the flat parameter vector."""
    out, off = [], 0
    for l in range(layers):
        cin = CIN0 if l == 0 else channels
        out.append((f"W{l}", off, (9, channels, cin)))
        off += 9 * channels * cin
        out.append((f"b{l}", off, (channels,)))
        off += channels
    out.append(("hw", off, (channels,)))
    off += channels
    out.append(("hb", off, (1,)))
    off += 1
    return out, off


def unpack(params: np.ndarray, layers: int, channels: int) -> dict:
    lay, total = layout(layers, channels)
    assert params.size == total
    return {name: np.asarray(params[o:o + int(np.prod(shape))], dtype=np.float64).reshape(shape)
            for name, o, shape in lay}


def features(uhat, speed, cls, eps, emulate=True):
    """[H, W, 16] input features of a whole frame (cls: 1 = TARGET)."""
    H, W = uhat.shape
    f = np.zeros((H, W, CIN0))
    f[..., 0] = uhat
    f[..., 1] = speed
    f[..., 2] = (cls == 1).astype(np.float64)
    f[..., 3] = np.log10(np.float64(np.float32(eps))) + 3.0
    j, i = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    d = np.minimum(np.minimum(i, j), np.minimum(W - 1 - i, H - 1 - j)).astype(np.float32)
    # in float32, as the device computes it (IEEE division: the same value)
    f[..., 4] = np.float32(1.0) / (np.float32(1.0) + np.float32(0.25) * d)
    if emulate:
        f[..., :5] = bf16(f[..., :5].astype(np.float32))
    return f


def crop_mask(cls, x0, y0, S, n, margin):
    """Loss mask of the S x S crop at (x0, y0) of an n x n frame: FREE nodes (cls 0) at least margin
    cells from every crop edge that lies inside the frame."""
    m = (cls[y0:y0 + S, x0:x0 + S] == 0).copy()
    if x0 > 0:
        m[:, :margin] = False
    if y0 > 0:
        m[:margin, :] = False
    if x0 + S < n:
        m[:, S - margin:] = False
    if y0 + S < n:
        m[S - margin:, :] = False
    return m.astype(np.float64)


def shift(x: np.ndarray, oy: int, ox: int) -> np.ndarray:
    """s[b, y, x] = x[b, y + oy, x + ox], zero outside the image."""
    B, H, W, C = x.shape
    s = np.zeros_like(x)
    ys, ye = max(0, -oy), min(H, H - oy)
    xs, xe = max(0, -ox), min(W, W - ox)
    if ys < ye and xs < xe:
        s[:, ys:ye, xs:xe] = x[:, ys + oy:ye + oy, xs + ox:xe + ox]
    return s


def offsets(dil: int):
    return [((t // 3 - 1) * dil, (t % 3 - 1) * dil) for t in range(9)]


def conv3x3(x: np.ndarray, w: np.ndarray, dil: int) -> np.ndarray:
    """y[p][co] = sum_t sum_ci x[p + off_t][ci] w[t][co][ci] (no bias)."""
    y = np.zeros(x.shape[:3] + (w.shape[1],))
    for t, (oy, ox) in enumerate(offsets(dil)):
        y += shift(x, oy, ox) @ w[t].T
    return y


def forward(params, layers, channels, dilations, feats, emulate=True):
    """feats [B, H, W, 16] -> (activations x_1..x_L, delta [B, H, W])."""
    P = unpack(params, layers, channels)
    acts = []
    x = feats
    for l in range(layers):
        w = bf16(P[f"W{l}"]) if emulate else P[f"W{l}"]
        y = conv3x3(x, w, dilations[l]) + P[f"b{l}"]
        x = np.maximum(y, 0.0)
        if emulate:
            x = bf16(x)
        acts.append(x)
    delta = x @ P["hw"] + P["hb"][0]
    return acts, delta


def loss_and_grads(params, layers, channels, dilations, feats, uhat, vstar, mask, emulate=True):
    """Loss over the FREE pixels (mask) and the gradient of every parameter, by the chain rule."""
    P = unpack(params, layers, channels)
    acts, delta = forward(params, layers, channels, dilations, feats, emulate)
    n = float(mask.sum())
    e = (uhat + delta - vstar) * mask
    loss = float((e * e).sum() / n)
    g = 2.0 * e  # d(sum e^2)/d delta; everything is divided by n at the end
    grads = {}
    xL = acts[-1]
    grads["hw"] = np.einsum("bhw,bhwc->c", g, xL)
    grads["hb"] = np.array([g.sum()])
    dy = g[..., None] * P["hw"][None, None, None, :] * (xL > 0)
    if emulate:
        dy = bf16(dy)
    for l in range(layers - 1, -1, -1):
        x = feats if l == 0 else acts[l - 1]
        w = bf16(P[f"W{l}"]) if emulate else P[f"W{l}"]
        dW = np.zeros_like(P[f"W{l}"])
        for t, (oy, ox) in enumerate(offsets(dilations[l])):
            dW[t] = np.einsum("bhwo,bhwi->oi", dy, shift(x, oy, ox))
        grads[f"W{l}"] = dW
        grads[f"b{l}"] = dy.sum(axis=(0, 1, 2))
        if l > 0:
            dx = np.zeros(x.shape)
            for t, (oy, ox) in enumerate(offsets(dilations[l])):
                dx += shift(dy, -oy, -ox) @ w[t]
            dy = dx * (x > 0)
            if emulate:
                dy = bf16(dy)
    lay, total = layout(layers, channels)
    flat = np.zeros(total)
    for name, o, shape in lay:
        flat[o:o + int(np.prod(shape))] = grads[name].reshape(-1) / n
    return loss, flat


def adam(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (Kingma & Ba, Algorithm 1)."""
    m = b1 * m + (1.0 - b1) * grads
    v = b2 * v + (1.0 - b2) * grads * grads
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v

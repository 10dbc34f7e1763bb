"""Learned warm start: training data from the method's own solves, training with the library's
network kernels (slhjb_net_*), and the comparison of starts.

A frame is one fine problem with u_hat (the bilinear upsampling of its coarse sigma = 0 solve,
Section 4.3), the network's input u_hat (the same bilinear one for the dilated CNN, the bicubic
upsampling for the U-Net) and v* (its converged fine solution). The network learns
delta = v* - u_hat_in from [u_hat_in, c, target mask, log10(eps), distance to the box] on random
crops; the start of the fine iteration is then clamp(u_hat_in + delta, 0, 1). The iteration
converges to the same fixed point from any start, so the comparison measures work only: the
error of the start, and the sweeps and time to the tolerance.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import capi


# (c_in, c_out) of the U-Net's 14 convolutions in parameter order (slhjb_net_config, arch 1)
UNET_LAYERS = [(16, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128), (128, 128), (128, 128), (256, 128),
               (128, 128), (192, 64), (64, 64), (96, 32), (32, 32)]


def init_params(net: "capi.Net", seed: int = 0) -> np.ndarray:
    """He-normal 3 x 3 weights over the used input channels, zero biases, a small head."""
    rng = np.random.default_rng(seed)
    C = net.channels
    parts = []
    if net.arch == capi.NET_UNET:
        for l, (cin, cout) in enumerate(UNET_LAYERS):
            used = 5 if l == 0 else cin
            w = rng.normal(0.0, math.sqrt(2.0 / (9 * used)), size=(9, cout, cin))
            if l == 0:
                w[:, :, 5:] = 0.0
            parts += [w.reshape(-1), np.zeros(cout)]
        parts += [rng.normal(0.0, 1e-2, size=32), np.zeros(1)]
        p = np.concatenate(parts).astype(np.float32)
        assert p.size == net.param_count
        return p
    for l in range(net.layers):
        cin = 16 if l == 0 else C
        used = 5 if l == 0 else C
        w = rng.normal(0.0, math.sqrt(2.0 / (9 * used)), size=(9, C, cin))
        if l == 0:
            w[:, :, 5:] = 0.0
        parts += [w.reshape(-1), np.zeros(C)]
    parts += [rng.normal(0.0, 1e-2, size=C), np.zeros(1)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == net.param_count
    return p


@dataclass
class Frame:
    dp: "capi.DeviceProblem"
    vhat: object   # device float[n*n]: bilinear u_hat (the paper's start)
    vstar: object  # device float[n*n]
    n: int
    eps: float
    seconds_coarse: float
    seconds_fine: float
    feat: object = None  # device float[n*n]: the network's u_hat (bicubic for the U-Net), else vhat


def make_frames(ctx: "capi.Context", pairs, tol: float = 1e-6, bicubic: bool = False) -> list[Frame]:
    """Solve each (fine, coarse) pair with the library: coarse sigma = 0 active-tile solve, u_hat,
    then the fine solve from u_hat in u_hat order to tol. With bicubic the frame also holds the
    bicubic u_hat, the U-Net's input."""
    import torch

    frames = []
    for fine, coarse in pairs:
        dpc = capi.DeviceProblem(coarse, capi.SL3)
        vc = torch.from_numpy(coarse.initial().reshape(-1)).cuda()
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.solve_tiles(dpc, vc, tol=tol, order=capi.ORDER_NONE, tile_shape=capi.TILE_8x8_SPLIT4, max_passes=50000)
        vhat = torch.empty(fine.n * fine.n, dtype=torch.float32, device="cuda")
        ctx.upsample(vc, coarse.n, vhat, fine.n)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t
        dp = capi.DeviceProblem(fine, capi.SL3)
        vstar = vhat.clone()
        t = time.perf_counter()
        st = ctx.solve_tiles(dp, vstar, tol=tol, order=capi.ORDER_KEYS, max_passes=1_000_000)
        torch.cuda.synchronize()
        if st["status"] != 0:
            raise RuntimeError(f"fine solve did not converge: {st}")
        tf = time.perf_counter() - t
        feat = vhat
        if bicubic:
            feat = torch.empty_like(vhat)
            ctx.upsample_bicubic(vc, coarse.n, feat, fine.n)
        frames.append(Frame(dp, vhat, vstar, fine.n, float(fine.eps), tc, tf, feat))
    return frames


def train(net: "capi.Net", frames, steps: int, batch: int = 8, crop: int = 256, lr: float = 2e-3,
          seed: int = 0, lr_final: float = 0.05) -> list[float]:
    """Adam on random crops; cosine decay of the learning rate to lr * lr_final. Each crop coordinate
    is snapped to a side of the box half of the time: the boundary layer (diffusion feet leaving the
    box read v_out) is where u_hat, a sigma = 0 solution, is furthest from v*, and a uniform origin
    would almost never show it."""
    rng = np.random.default_rng(seed)
    losses = []
    c = min(crop, min(f.n for f in frames))
    if net.arch == capi.NET_UNET:
        c -= c % 8

    def origin(n):
        if rng.random() < 0.5:
            return 0 if rng.random() < 0.5 else n - c
        return int(rng.integers(0, n - c + 1))

    for s in range(steps):
        items = []
        for _ in range(batch):
            f = frames[int(rng.integers(len(frames)))]
            items.append((f.feat, f.vstar, f.dp, origin(f.n), origin(f.n)))
        losses.append(net.loss_grad(items, c))
        rate = lr * (lr_final + (1.0 - lr_final) * 0.5 * (1.0 + math.cos(math.pi * s / max(1, steps - 1))))
        net.adam_step(rate)
    return losses


def evaluate(ctx: "capi.Context", net: "capi.Net", frames, tol: float = 1e-6, tol_ref: float = 2e-7,
             max_ref_sweeps: int = 20000) -> list[dict]:
    """For every frame: error of u_hat, of the bicubic u_hat (when the frame has one) and of the
    network's start against v*, and from each start the plain Jacobi solve and the u_hat-ordered
    active-tile solve: sweeps, time, node updates, and the error at the stopping point against v*.
    v* is first refined by Jacobi sweeps to the residual tol_ref (at most max_ref_sweeps), so that
    it is closer to the fixed point than any of the stopping points it is compared with."""
    import torch

    out = []
    for f in frames:
        free = torch.from_numpy((f.dp.inst.node_class.reshape(-1) == 0)).cuda()
        ref = ctx.solve(f.dp, f.vstar, tol=tol_ref, max_sweeps=max_ref_sweeps)
        g = torch.empty_like(f.vhat)
        torch.cuda.synchronize()
        t = time.perf_counter()
        net.warm_start(f.dp, f.feat, g)
        torch.cuda.synchronize()
        t_net = time.perf_counter() - t
        row = {"n": f.n, "eps": f.eps, "t_network_s": t_net, "ref_residual": ref["residual"],
               "ref_sweeps": ref["sweeps"]}
        starts = [("uhat", f.vhat)]
        if f.feat is not f.vhat:
            starts.append(("uhat_bicubic", f.feat))
        starts.append(("network", g))
        for name, start in starts:
            e = (start - f.vstar).abs()[free]
            row[f"err_max_{name}"] = float(e.max())
            row[f"err_mean_{name}"] = float(e.mean())
            v = start.clone()
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = ctx.solve(f.dp, v, tol=tol, max_sweeps=1_000_000)
            torch.cuda.synchronize()
            row[f"jacobi_sweeps_{name}"] = st["sweeps"]
            row[f"jacobi_s_{name}"] = time.perf_counter() - t
            row[f"jacobi_err_{name}"] = float((v - f.vstar).abs()[free].max())
            v = start.clone()
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = ctx.solve_tiles(f.dp, v, tol=tol, order=capi.ORDER_KEYS, max_passes=1_000_000)
            torch.cuda.synchronize()
            row[f"tiles_s_{name}"] = time.perf_counter() - t
            row[f"tiles_updates_per_node_{name}"] = st["node_updates"] / max(1, int(free.sum()))
            row[f"tiles_err_{name}"] = float((v - f.vstar).abs()[free].max())
        out.append(row)
    return out


def main(argv=None):
    """Timing of the U-Net's training step and whole-frame inference on the method's own solves:
    python -m paper_1502_01629_amd.warmstart [--problems P --steps K ...]"""
    import argparse

    import torch

    from . import instances

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--n", type=int, default=1025)
    ap.add_argument("--coarse", type=int, default=129)
    ap.add_argument("--problems", type=int, default=16)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--crop", type=int, default=256)
    a = ap.parse_args(argv)
    ctx = capi.Context(0)
    frames = make_frames(ctx, instances.warmstart_problems(0, count=a.problems, n=a.n, n_coarse=a.coarse),
                         bicubic=True)
    net = capi.Net(ctx, arch=capi.NET_UNET)
    net.set_params(init_params(net, 0))
    train(net, frames, steps=10, batch=a.batch, crop=a.crop, lr=1e-3)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    losses = train(net, frames, steps=a.steps, batch=a.batch, crop=a.crop, lr=1e-3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    g = torch.empty_like(frames[0].vhat)
    net.warm_start(frames[0].dp, frames[0].feat, g)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(10):
        net.warm_start(frames[0].dp, frames[0].feat, g)
    torch.cuda.synchronize()
    ti = (time.perf_counter() - t) / 10
    print(f"U-Net training: {a.steps} steps of {a.batch} x {a.crop}^2 in {dt:.3f} s = {1e3 * dt / a.steps:.3f} ms/step "
          f"(loss {np.mean(losses[:10]):.3e} -> {np.mean(losses[-10:]):.3e}); inference {a.n}^2: {1e3 * ti:.3f} ms",
          flush=True)
    net.close()
    ctx.close()


if __name__ == "__main__":
    main()

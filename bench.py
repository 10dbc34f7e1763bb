#!/usr/bin/env python3
"""Benchmark: time-to-residual-1e-6 and SL node-updates/s of the 2049^2 2-D HJB solve on one MI355X.

Workload (one "step"): the scattered-targets problem on [-1,1]^2 with a 2049 x 2049 grid,
c(x) = 1 + 0.5 sin(2 pi x1) sin(2 pi x2), 64 controls, three point targets, square obstacles on
10% of the box, Kruzkov discount lambda = 1, h = dx/1.5, sigma = 0, scheme SL3 (eq. SLscheme3).
A step is one complete Jacobi value iteration from the cold start v = 1 until the sup-norm change
of a sweep is <= 1e-6, inputs already resident in HBM.

Prints one JSON line (rank 0). `value` is FREE-node Bellman updates per second over the timed
steps; `ms_per_step` is the time-to-residual.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def cpu_baseline(inst, scheme: int, budget_s: float = 12.0) -> dict:
    """The FP64 oracle, as it stands, timed on this host's cores on a bounded sample: whole Jacobi
    sweeps of the same problem from the same cold start until ~budget_s of CPU time."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
    p = oracle.Problem.from_instance(inst, scheme)
    v = p.initial()
    free = int((inst.node_class == 0).sum())
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        v, _ = p.sweep(v, threads=threads)
        sweeps += 1
        if time.perf_counter() - t0 >= budget_s or sweeps >= 50:
            break
    dt = time.perf_counter() - t0
    return {"value": free * sweeps / dt, "unit": "node-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{sweeps} FP64 Jacobi sweeps of the same {inst.n}^2 problem from v=1 ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--eps", type=float, default=0.0)
    ap.add_argument("--scheme", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n", type=int, default=2049)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch

        a = torch.ones(args.copy_calibration * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see DESIGN.md, "
              "'How the path would shard'). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1502_01629_amd import capi
    from paper_1502_01629_amd import instances as I
    from paper_1502_01629_amd import roofline as RL

    fine, _coarse = I.scattered_problem(args.seed, n=args.n, eps=args.eps)
    ctx = capi.Context(0)
    dp = capi.DeviceProblem(fine, args.scheme)
    v0 = torch.from_numpy(fine.initial().reshape(-1)).cuda()
    v = torch.empty_like(v0)
    free = int((fine.node_class == 0).sum())

    def step():
        v.copy_(v0)
        return ctx.solve(dp, v, tol=args.tol, max_sweeps=2_000_000)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    updates = sum(s["node_updates"] for s in stats)
    sweep_s = sum(s["sweep_seconds"] for s in stats)
    launches = sum(s["sweep_launches"] for s in stats)
    avg_launch = sweep_s / launches
    flops = RL.sweep_flops_per_node_update(fine.diffusion, args.scheme, fine.n_controls) * free
    achieved = flops / avg_launch / 1e12
    kernel = ("sweep_ring1<SL3>" if args.scheme == 1 else "sweep_ring1<SL2>") if stats[0]["kernel_path"] == 1 else \
        f"sweep_general<diff={fine.diffusion},{'SL3' if args.scheme == 1 else 'SL2'}>"
    out = {
        "metric": "time-to-residual-1e-6 & SL node-updates/s at 2049^2 2D HJB (cold start)",
        "value": updates / dt,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded instance generator)",
        "config": {
            "workload": f"scattered targets {fine.n}^2, c=1+0.5sin(2pi x1)sin(2pi x2), 64 controls, 3 point targets, "
                        f"10% square obstacles, eps={args.eps}, h=dx/1.5, SL{2 + args.scheme}, Jacobi from v=1 to "
                        f"residual {args.tol:g}",
            "n": fine.n, "eps": args.eps, "n_controls": fine.n_controls, "seed": args.seed, "tol": args.tol,
            "free_nodes": free,
        },
        "time_to_residual_s": float(np.median([s["seconds"] for s in stats])),
        "sweeps_to_residual": int(np.median([s["converged_sweep"] for s in stats])),
        "sweeps_run": int(stats[0]["sweeps"]),
        "roofline": {
            "kernel": kernel,
            "bound": "alu",
            "achieved": achieved,
            "peak": RL.FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / RL.FP32_VECTOR_PEAK_TFLOPS,
            "traffic": None,
            "avg_launch_us": avg_launch * 1e6,
            "flops_per_node_update": RL.sweep_flops_per_node_update(fine.diffusion, args.scheme, fine.n_controls),
            "hbm_frac_algorithmic": RL.SWEEP_BYTES_PER_NODE_UPDATE * free / avg_launch / 1e9 / RL.HBM_PEAK_GBS,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(fine, args.scheme)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

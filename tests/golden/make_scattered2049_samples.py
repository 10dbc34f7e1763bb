#!/usr/bin/env python3
"""Write the FP64 oracle's converged values of the 2049^2 scattered-targets problem at sampled nodes.

The workload is the one the benchmark times (seed 0, eps = 0, 64 controls, three point targets,
square obstacles on 10% of the box, h = dx / 1.5, scheme SL3 of Section 3). The oracle's Jacobi
value iteration runs from v = 1 until the sup-norm change of a sweep is <= TOL; by the
contraction of the scheme its distance to the fixed point is then at most beta / (1 - beta) TOL.
The values at SAMPLES FREE nodes drawn with a fixed seed are stored with the residual and the
sweep count. Only the oracle and the seeded input generator are used.

Usage: python tests/golden/make_scattered2049_samples.py [--threads T] [--checkpoint PATH]
(about 2000 sweeps of 4.2M nodes: tens of minutes on 8 cores; a checkpoint file lets a run resume).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1502_01629_amd import instances as I  # noqa: E402

OUT = os.path.join(HERE, "scattered2049_eps0_samples.npz")
TOL = 1e-11
SAMPLES = 65536
SAMPLE_SEED = 20240611


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--checkpoint", default=None, help="npz file holding the iterate between chunks")
    ap.add_argument("--chunk", type=int, default=50, help="sweeps between progress lines / checkpoints")
    args = ap.parse_args()

    fine, _ = I.scattered_problem(0, n=2049, eps=0.0)
    p = oracle.Problem.from_instance(fine, oracle.SL3)
    v, sweeps = p.initial(), 0
    if args.checkpoint and os.path.exists(args.checkpoint):
        ck = np.load(args.checkpoint)
        v, sweeps = ck["v"].copy(), int(ck["sweeps"])
        print(f"resumed at sweep {sweeps}", flush=True)
    t0 = time.time()
    while True:
        v, s, r, _ = p.solve(v0=v, tol=TOL, max_sweeps=args.chunk, threads=args.threads)
        sweeps += s
        print(f"sweep {sweeps}: residual {r:.3e} ({time.time() - t0:.0f} s)", flush=True)
        if args.checkpoint:
            np.savez(args.checkpoint + ".tmp.npz", v=v, sweeps=sweeps)
            os.replace(args.checkpoint + ".tmp.npz", args.checkpoint)
        if r <= TOL:
            break
    free = np.flatnonzero(p.node_class == oracle.FREE)
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = np.sort(rng.choice(free, size=SAMPLES, replace=False)).astype(np.int64)
    np.savez_compressed(OUT, node=idx, value=v[idx], residual=np.float64(r), sweeps=np.int64(sweeps),
                        beta=np.float64(p.beta()), tol=np.float64(TOL))
    print(f"wrote {OUT}: {SAMPLES} nodes, {sweeps} sweeps, residual {r:.3e}, "
          f"bound {p.beta() / (1 - p.beta()) * r:.2e}")


if __name__ == "__main__":
    main()

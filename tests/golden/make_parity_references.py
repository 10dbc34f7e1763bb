#!/usr/bin/env python3
"""Write the FP64 oracle's exact fixed points of the 257^2 parity cases that mirror the benchmark's
arms (the GPU tests compare with them; computing them inside a test would take minutes).

Cases (seeded inputs from the instance generator):
  bumps257_rank1      rank-1 diffusion sigma = sqrt(2 eps) a, 16 Gaussian speed bumps, disc target,
                      64 controls, h = dx, eps = 2 dx (noise feet 2 cells out: interpolation halo 4);
  scattered257_eps8e-3, scattered257_eps8e-2
                      three point targets, square obstacles, c = 1 + 0.5 sin sin, 64 controls,
                      h = dx / 1.5, isotropic diffusion with eps = 8x the benchmark's 1e-3 and 1e-2
                      (the same noise reach in cells as on the 2049^2 grid: halos 3 and 5).
Each fixed point comes from Howard's policy iteration with exact sparse solves (oracle.policy),
and is certified by one oracle Jacobi sweep of eq. SLscheme3: the stored `bellman_residual` is
max |T(v) - v|, so the distance to the fixed point is at most beta / (1 - beta) times it.
Only the oracle and the seeded input generator are used.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import policy as PI  # noqa: E402
from paper_1502_01629_amd import instances as I  # noqa: E402


def cases():
    return {
        "bumps257_rank1": I.bumps_problem(0, n=257, eps=2.0 * 2.0 / 256),
        "scattered257_eps8e-3": I.scattered_problem(1, n=257, n_coarse=65, eps=8e-3)[0],
        "scattered257_eps8e-2": I.scattered_problem(1, n=257, n_coarse=65, eps=8e-2)[0],
    }


def path(name: str) -> str:
    return os.path.join(HERE, f"{name}_fixed_point.npz")


def main():
    threads = os.cpu_count() or 1
    for name, inst in cases().items():
        t = time.time()
        p = oracle.Problem.from_instance(inst, oracle.SL3)
        v, _, its = PI.sparse_policy_iteration(p, threads=threads)
        _, r = p.sweep(v, threads=threads)
        np.savez_compressed(path(name), v=v, bellman_residual=np.float64(r), howard_iterations=np.int64(its),
                            beta=np.float64(p.beta()), n=np.int64(inst.n), eps=np.float64(inst.eps))
        print(f"{name}: {its} policy iterations, max|T(v) - v| = {r:.2e}, {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main()

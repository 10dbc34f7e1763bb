#!/usr/bin/env python3
"""Benchmark: time-to-residual-1e-6 of the 2049^2 2-D HJB solve on one MI355X, warm vs cold start.

Workload: the scattered-targets problem on [-1,1]^2, 2049 x 2049 nodes, c(x) = 1 + 0.5 sin(2 pi x1)
sin(2 pi x2), 64 controls, three point targets, square obstacles on 10% of the box, Kruzkov
discount lambda = 1, h = dx/1.5, sigma = 0, scheme SL3 (eq. SLscheme3); coarse grid 129^2, 64 patches.

One step = the patchy method of Section 4.3 end to end with inputs resident in HBM: coarse solve
(sigma = 0) -> u_hat -> synthesis of the control -> integer patch labels (64 patches) -> the fine
solve from u_hat with tiles taken by increasing u_hat (each tile visit alternating full Bellman
iterations with policy-evaluation iterations, modified policy iteration), until one full Jacobi
sweep changes no node by more than 1e-6. `value` is the mean wall time of a step (lower is better).

Beside the timed steps, each comparison arm runs once (progress on stderr):
  c2     the plain cold-start global Jacobi value iteration (the SL sweep kernel at full rate), the
         same from u_hat, and the static decomposition (active tiles, fixed order, cold start);
  c2eps  the same 2049^2 workload with isotropic diffusion eps = 1e-3 and 1e-2: patchy pipeline
         against the cold global Jacobi iteration;
  batch  256 independent instances (65^2..1025^2, eps > 0): the batched Jacobi solve and the batched
         active-tile solve, each against the same instances solved one by one (bit-exact
         agreement counted);
  bumps  4097^2 with rank-1 diffusion: full sweeps against active tiles (cold, and u_hat-ordered);
  learned  the U-Net warm start trained on the method's own 1025^2 solves against the cold start,
         the bilinear and the bicubic u_hat on held-out problems (time to the tolerance and error
         at the stopping point);
  indep  the independent (state-constraint) patch solves at eps = 0, 1e-3, 1e-2 against the
         transmission solve: the decomposition error, near the patch interfaces and away from them;
  hdx    the same step with h = dx (feet up to 1.5 cells: the general kernels);
  balance  balanced patches on the step's workload: the patch sizes of the rounds of
         slhjb_balance_sources from the equal angular sectors;
  exit   the paper's exit-to-boundary experiments (Table 0, the eps sweeps of Tables 1-2).
The full record of every arm goes to a JSON file (--arms-out); stdout ends with one JSON line of
at most a few KB: the headline, the roofline, the CPU baseline, the accuracy against the oracle's
stored values and a summary of each arm.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# modified policy iteration inside the tile visits of the active-tile solves (0 = off): policy
# iterations after each full one, for sigma = 0 (the main step) and with diffusion (the arms, where
# a visit is one full iteration and these)
POLICY_SWEEPS = 16
POLICY_SWEEPS_DIFFUSION = 14


# the files that define the dominant kernel (the tile visit) and everything it inlines
KERNEL_SOURCES = ("tiles.hip", "sweep_device.h", "select_device.h", "internal.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1502_01629_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None when the
    kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(inst, scheme: int, jacobi_sweeps: int, budget_s: float = 12.0) -> dict:
    """The FP64 oracle, as it stands, on this host's cores: whole Jacobi sweeps of the same problem from
    the same cold start for ~budget_s, scaled to the sweeps the global Jacobi needs to reach 1e-6."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
    p = oracle.Problem.from_instance(inst, scheme)
    v = p.initial()
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        v, _ = p.sweep(v, threads=threads)
        sweeps += 1
        if time.perf_counter() - t0 >= budget_s or sweeps >= 50:
            break
    dt = time.perf_counter() - t0
    per_sweep = dt / sweeps
    free = int((inst.node_class == 0).sum())
    return {"value": per_sweep * jacobi_sweeps, "unit": "s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{sweeps} FP64 Jacobi sweeps of the same {inst.n}^2 problem from v=1 in {dt:.1f} s "
                      f"({free * sweeps / dt:.3g} node-updates/s), scaled to the {jacobi_sweeps} sweeps the "
                      f"global Jacobi iteration needs to reach residual 1e-6"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


GOLDEN_2049 = os.path.join(ROOT, "tests", "golden", "scattered2049_eps0_samples.npz")


def oracle_samples_error(v, fine, seed: int, eps: float) -> dict | None:
    """max |v - v_oracle| at the nodes where the committed oracle solution of the same 2049^2
    problem (seed 0, eps 0) stores its converged FP64 values (written by
    tests/golden/make_scattered2049_samples.py, which calls only the oracle)."""
    if fine.n != 2049 or seed != 0 or eps != 0.0 or not os.path.exists(GOLDEN_2049):
        return None
    g = np.load(GOLDEN_2049)
    idx = g["node"]
    got = v.cpu().numpy()[idx].astype(np.float64)
    d = np.abs(got - g["value"])
    return {"nodes": int(idx.size), "max_abs": float(d.max()), "mean_abs": float(d.mean()),
            "oracle_residual": float(g["residual"]), "oracle_sweeps": int(g["sweeps"])}


def log(msg: str) -> None:
    """Progress of the long arms, on stderr (stdout carries the one JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def arm_batch(ctx, seed: int, tol: float) -> dict:
    """256 independent instances (grid sizes 65..1025, 1-4 disc targets, 8 speed bumps, eps
    log-uniform in [1e-4, 1e-2], 32-64 controls, isotropic diffusion, h = dx): one batched solve
    (tile shapes from the autotuner) against the same instances solved one after the other with
    the single-instance Jacobi solve; the two must agree bit for bit."""
    import torch

    from paper_1502_01629_amd import autotune, capi
    from paper_1502_01629_amd import instances as I

    xs = I.batch_problems(seed, count=256)
    probs = [capi.DeviceProblem(x, capi.SL3) for x in xs]
    starts = [torch.from_numpy(x.initial().reshape(-1)).cuda() for x in xs]
    t = time.perf_counter()
    shapes = autotune.tune(ctx, xs, cache=os.path.join(ROOT, "_build", "batch_tiles.json"))
    t_tune = time.perf_counter() - t
    log(f"batch: autotuned {len(set(autotune.bucket_key(x) for x in xs))} buckets in {t_tune:.1f} s")
    vb = [s0.clone() for s0 in starts]
    torch.cuda.synchronize()
    t = time.perf_counter()
    stats, tot = ctx.solve_batch(probs, vb, tol=tol, max_sweeps=1_000_000, check_every=16, tile_shapes=shapes)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    log(f"batch: batched solve {t_batch:.2f} s, {tot['sweeps']} sweeps")
    t = time.perf_counter()
    equal = 0
    upd = 0
    for k, p in enumerate(probs):
        v1 = starts[k].clone()
        st1 = ctx.solve(p, v1, tol=tol, max_sweeps=1_000_000, check_every=16)
        upd += st1["node_updates"]
        equal += int(bool(torch.equal(v1, vb[k])) and st1["sweeps"] == stats[k]["sweeps"])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    log(f"batch: sequential single-instance solves {t_seq:.2f} s")
    # the active-tile solver on the same instances: batched against one after the other
    vt = [s0.clone() for s0 in starts]
    torch.cuda.synchronize()
    t = time.perf_counter()
    tstats, ttot = ctx.solve_tiles_batch(probs, vt, tol=tol, policy_sweeps=POLICY_SWEEPS_DIFFUSION)
    torch.cuda.synchronize()
    t_tb = time.perf_counter() - t
    log(f"batch: batched active-tile solve {t_tb:.2f} s, {ttot['converged']} converged")
    t = time.perf_counter()
    equal_t = 0
    upd_t = 0
    for k, p in enumerate(probs):
        v1 = starts[k].clone()
        st1 = ctx.solve_tiles(p, v1, tol=tol, policy_sweeps=POLICY_SWEEPS_DIFFUSION)
        upd_t += st1["node_updates"]
        equal_t += int(bool(torch.equal(v1, vt[k])) and st1["sweeps"] == tstats[k]["sweeps"])
    torch.cuda.synchronize()
    t_tseq = time.perf_counter() - t
    log(f"batch: sequential single-instance active-tile solves {t_tseq:.2f} s")
    diff = max(float((vt[k] - vb[k]).abs().max()) for k in range(len(xs)))
    sizes = sorted({x.n for x in xs})
    return {
        "instances": len(xs), "nodes": int(sum(x.n * x.n for x in xs)),
        "grid_sizes": {str(n): sum(1 for x in xs if x.n == n) for n in sizes},
        "time_s_batched": t_batch, "device_s_batched": tot["seconds"], "time_s_sequential": t_seq,
        "speedup": t_seq / t_batch, "node_updates": tot["node_updates"],
        "node_updates_per_s_batched": tot["node_updates"] / t_batch, "node_updates_per_s_sequential": upd / t_seq,
        "sweeps_max": tot["sweeps"], "graph_replays": tot["replays"], "converged": tot["converged"],
        "bit_exact_vs_single": f"{equal}/{len(xs)}", "autotune_s": t_tune,
        "active_tiles": {"time_s_batched": t_tb, "device_s_batched": ttot["seconds"],
                         "time_s_sequential": t_tseq, "speedup": t_tseq / t_tb,
                         "speedup_vs_sequential_jacobi": t_seq / t_tb, "node_updates": ttot["node_updates"],
                         "passes_total": ttot["sweeps"], "graph_replays": ttot["replays"],
                         "converged": ttot["converged"], "bit_exact_vs_single": f"{equal_t}/{len(xs)}",
                         "max_abs_diff_vs_batched_jacobi": diff},
        "tile_shapes": {capi.BATCH_TILE_SHAPES[k][0] * 1000 + capi.BATCH_TILE_SHAPES[k][1]: shapes.count(k)
                        for k in set(shapes)},
    }


def arm_bumps(ctx, seed: int, tol: float, n: int) -> dict:
    """Degenerate (rank-1) diffusion on 4097^2: full Jacobi sweeps against the active-tile work list
    with per-tile convergence flags, both from the cold start, plus the active tiles ordered by the
    u_hat of a coarse sigma = 0 solve."""
    import torch

    from paper_1502_01629_amd import capi
    from paper_1502_01629_amd import instances as I

    x = I.bumps_problem(seed, n=n)
    free = int((x.node_class == 0).sum())
    dp = capi.DeviceProblem(x, capi.SL3)
    v0 = torch.from_numpy(x.initial().reshape(-1)).cuda()
    out = {"n": n, "eps": float(x.eps), "free_nodes": free, "diffusion": "rank-1 sqrt(2 eps) a"}
    vf = v0.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    sf = ctx.solve(dp, vf, tol=tol, max_sweeps=200_000)
    torch.cuda.synchronize()
    out["full_sweeps"] = {"time_s": time.perf_counter() - t, "sweeps": sf["sweeps"],
                          "node_updates_per_free_node": sf["node_updates"] / free,
                          "sweep_kernel_us": 1e6 * sf["sweep_seconds"] / sf["sweep_launches"], "halo": sf["halo"]}
    log(f"bumps: full sweeps {out['full_sweeps']['time_s']:.2f} s")
    vt = v0.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = ctx.solve_tiles(dp, vt, tol=tol, order=capi.ORDER_NONE, max_passes=200_000, policy_sweeps=POLICY_SWEEPS_DIFFUSION)
    torch.cuda.synchronize()
    out["active_tiles_cold"] = {"time_s": time.perf_counter() - t, "passes": st["sweeps"],
                                "node_updates_per_free_node": st["node_updates"] / free,
                                "policy_updates_per_free_node": st["policy_updates"] / free,
                                "max_abs_diff_vs_full": float((vt - vf).abs().max())}
    log(f"bumps: active tiles {out['active_tiles_cold']['time_s']:.2f} s")
    # u_hat from a coarse sigma = 0 solve, tiles by increasing u_hat
    xc = I.bumps_problem(seed, n=257, eps=0.0)
    xc.diffusion = I.DIFF_NONE
    dpc = capi.DeviceProblem(xc, capi.SL3)
    vc = torch.from_numpy(xc.initial().reshape(-1)).cuda()
    vk = torch.empty_like(v0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sc = ctx.solve_tiles(dpc, vc, tol=tol, order=capi.ORDER_NONE, tile_shape=capi.TILE_8x8_SPLIT4, max_passes=20000)
    ctx.upsample(vc, xc.n, vk, n)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t
    sk = ctx.solve_tiles(dp, vk, tol=tol, order=capi.ORDER_KEYS, max_passes=200_000, policy_sweeps=POLICY_SWEEPS_DIFFUSION)
    torch.cuda.synchronize()
    out["active_tiles_uhat"] = {"time_s": time.perf_counter() - t, "coarse_and_upsample_s": t_pre,
                                "coarse_passes": sc["sweeps"], "passes": sk["sweeps"],
                                "node_updates_per_free_node": sk["node_updates"] / free,
                                "policy_updates_per_free_node": sk["policy_updates"] / free,
                                "max_abs_diff_vs_full": float((vk - vf).abs().max())}
    log(f"bumps: active tiles from u_hat {out['active_tiles_uhat']['time_s']:.2f} s")
    out["speedup_active_tiles_cold"] = out["full_sweeps"]["time_s"] / out["active_tiles_cold"]["time_s"]
    out["speedup_active_tiles_uhat"] = out["full_sweeps"]["time_s"] / out["active_tiles_uhat"]["time_s"]
    return out


# Table 0 of the paper (Section 5.1): Gauss-Seidel iterations of eq. SLscheme2 / eq. SLscheme3
# on a 50 x 50 grid, as printed; context for the GPU's Jacobi counts, not a target.
PAPER_TABLE0 = {("A", 0.0): (176, 2), ("A", 1e-2): (458, 102), ("B", 0.0): (145, 26), ("B", 1e-2): (353, 98),
                ("B2", 0.0): (276, 33), ("B2", 1e-2): (305, 78), ("C", 0.0): (716, 116), ("C", 1e-2): (961, 325)}


def arm_exit(ctx, tol: float) -> dict:
    """The paper's exit-to-boundary experiments (Section 5) in the paper's own undiscounted form
    (lambda = 0: beta = 1, rho = h l): g = 0 on the boundary, l = 1, 16 controls,
    h = dx / (1 + Upsilon) / f_min. (1) Table 0: Jacobi sweeps of SL2 and SL3 for the
    advection (A), eikonal (B, B2) and Zermelo (C) dynamics at eps = 0 and 1e-2 on 50 x 50 nodes.
    (2) Tables 1 and 2: the patchy solve (coarse 51^2 sigma = 0 solve, u_hat, tiles by increasing
    u_hat) against the static decomposition (cold, fixed order) over eps, on 101^2 and 201^2
    nodes (dx = 0.02, 0.01), for the eikonal-diffusion (threshold eps < dx/4) and Zermelo
    (eps < dx/120) problems: work per node and time across the upwind diffusion ball threshold."""
    import torch

    from paper_1502_01629_amd import capi
    from paper_1502_01629_amd import instances as I

    out = {"table0": [], "threshold": {}}
    for (dyn, eps), (p2, p3) in PAPER_TABLE0.items():
        x = I.exit_problem(50, dyn, eps=eps, lam=0.0)
        row = {"equation": dyn, "eps": eps, "lambda": 0.0, "paper_gauss_seidel_sl2_sl3": [p2, p3]}
        for name, scheme in (("sl2", capi.SL2), ("sl3", capi.SL3)):
            dp = capi.DeviceProblem(x, scheme)
            # the undiscounted cold start: v = 0 (boundary data 0), from which the iterates climb
            v = torch.from_numpy(x.initial(free_value=0.0).reshape(-1)).cuda()
            st = ctx.solve(dp, v, tol=tol, max_sweeps=1_000_000, check_every=1)
            row[f"jacobi_sweeps_{name}"] = st["converged_sweep"] if st["status"] == 0 else None
        out["table0"].append(row)
    log("exit: Table 0 done")
    eps_sets = {"B": [1e-9, 1e-8, 1e-7, 1e-6, 1e-5, 1e-4, 6.25e-4, 1.25e-3, 2.5e-3, 5e-3, 1e-2],
                "C": [1e-9, 1e-8, 1e-7, 1e-6, 1e-5, 2.083e-5, 4.16e-5, 8.3e-5, 1.6e-4, 1e-3, 5e-3]}
    for dyn, eps_list in eps_sets.items():
        per_grid = {}
        for n in (101, 201):
            dx = 2.0 / (n - 1)
            rows = []
            for eps in eps_list:
                fine = I.exit_problem(n, dyn, eps=eps, lam=0.0)
                coarse = I.exit_problem(51, dyn, eps=0.0, lam=0.0)
                free = int((fine.node_class == 0).sum())
                dp, dpc = capi.DeviceProblem(fine, capi.SL3), capi.DeviceProblem(coarse, capi.SL3)
                row = {"eps": eps}
                for name, mode, cp in (("patchy", capi.PATCHY_TRANSMISSION, dpc), ("static", capi.PATCHY_STATIC, None)):
                    v = torch.empty(n * n, dtype=torch.float32, device="cuda")
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    st = ctx.solve_patchy(dp, cp, v, mode=mode, tol=tol, tol_coarse=tol, max_passes=100_000,
                                          policy_sweeps=POLICY_SWEEPS_DIFFUSION if eps > 0 else POLICY_SWEEPS)
                    torch.cuda.synchronize()
                    row[name] = {"time_s": time.perf_counter() - t, "passes": st["passes"],
                                 "node_updates_per_free_node": st["node_updates"] / free,
                                 "policy_updates_per_free_node": st["policy_updates"] / free,
                                 "converged": st["status"] == 0}
                rows.append(row)
            f_min, f_max = fine.meta["f_min"], fine.meta["f_max"]
            per_grid[str(n)] = {"dx": dx, "h": float(I.exit_problem(n, dyn).h),
                                "eps_threshold": dx * f_min / (2.0 * (1.0 + f_max / f_min)), "rows": rows}
        out["threshold"]["eikonal-diffusion" if dyn == "B" else "zermelo"] = per_grid
        log(f"exit: threshold sweep {dyn} done (" + ", ".join(
            f"n={n}: {g['rows'][0]['patchy']['node_updates_per_free_node']:.1f} -> "
            f"{g['rows'][-1]['patchy']['node_updates_per_free_node']:.1f} upd/node" for n, g in per_grid.items()) + ")")
    return out


def arm_c2_eps(ctx, seed: int, tol: float, patches: int, eps_list=(1e-3, 1e-2)) -> dict:
    """The same 2049^2 workload with isotropic diffusion: the patchy pipeline (coarse sigma = 0
    solve, u_hat, synthesis, labels, u_hat-ordered active tiles) against the cold global Jacobi
    iteration."""
    import torch

    from paper_1502_01629_amd import capi
    from paper_1502_01629_amd import instances as I

    out = {}
    for eps in eps_list:
        fine, coarse = I.scattered_problem(seed, eps=eps)
        free = int((fine.node_class == 0).sum())
        dp = capi.DeviceProblem(fine, capi.SL3)
        dpc = capi.DeviceProblem(coarse, capi.SL3)
        src_host, _ = capi.partition_sources(fine.node_class, patches)
        src = torch.from_numpy(src_host.reshape(-1)).cuda()
        v = torch.empty(fine.n * fine.n, dtype=torch.float32, device="cuda")
        lab = torch.empty(fine.n * fine.n, dtype=torch.int16, device="cuda")
        times = []
        for _ in range(2):  # warm-up, then timed
            torch.cuda.synchronize()
            t = time.perf_counter()
            sp = ctx.solve_patchy(dp, dpc, v, mode=capi.PATCHY_TRANSMISSION, tol=tol, tol_coarse=1e-7,
                                  source_patch=src, n_patches=patches, label_out=lab, policy_sweeps=POLICY_SWEEPS_DIFFUSION)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        vj = torch.from_numpy(fine.initial().reshape(-1)).cuda()
        torch.cuda.synchronize()
        t = time.perf_counter()
        sj = ctx.solve(dp, vj, tol=tol, max_sweeps=200_000)
        torch.cuda.synchronize()
        tj = time.perf_counter() - t
        out[f"eps={eps:g}"] = {
            "patchy_time_s": times[-1], "patchy_stages_s": {k: sp[k] for k in ("t_coarse", "t_synthesize", "t_label",
                                                                                "t_solve")},
            "patchy_passes": sp["passes"], "patchy_node_updates_per_free_node": sp["node_updates"] / free,
            "patchy_policy_updates_per_free_node": sp["policy_updates"] / free,
            "global_jacobi_cold_s": tj, "global_jacobi_sweeps": sj["sweeps"], "halo": sj["halo"],
            "sweep_kernel_us": 1e6 * sj["sweep_seconds"] / sj["sweep_launches"],
            "speedup": tj / times[-1], "max_abs_diff": float((v - vj).abs().max()),
        }
        log(f"c2 eps={eps:g}: patchy {times[-1]:.3f} s, global Jacobi {tj:.3f} s")
    return out


def interface_band(lab, radius: int):
    """Nodes within `radius` cells (Chebyshev) of a node of another patch; label -1 (no patch:
    obstacles, unreached nodes) is ignored on both sides."""
    import torch

    n = int(round(lab.numel() ** 0.5))
    L = lab.view(1, 1, n, n).float()
    big = float(1 << 20)
    hi = torch.nn.functional.max_pool2d(L, 2 * radius + 1, stride=1, padding=radius)
    lo = -torch.nn.functional.max_pool2d(-torch.where(L < 0, torch.full_like(L, big), L), 2 * radius + 1, stride=1,
                                         padding=radius)
    return ((hi != lo) & (lo < big)).view(-1)


def arm_indep(ctx, seed: int, tol: float, patches: int, eps_list=(0.0, 1e-3, 1e-2)) -> dict:
    """Decomposition error of the independent patch solves (state constraints at the patch
    interfaces, Section 2) on the 2049^2 workload: max |v_indep - v_transmission| over all FREE
    nodes, inside the band of `halo` cells around the interfaces (where the paper expects the
    error of a first-order patchy decomposition to sit) and away from it."""
    import torch

    from paper_1502_01629_amd import capi
    from paper_1502_01629_amd import instances as I

    out = {}
    for eps in eps_list:
        fine, coarse = I.scattered_problem(seed, eps=eps)
        dp, dpc = capi.DeviceProblem(fine, capi.SL3), capi.DeviceProblem(coarse, capi.SL3)
        src_host, _ = capi.partition_sources(fine.node_class, patches)
        src = torch.from_numpy(src_host.reshape(-1)).cuda()
        N = fine.n * fine.n
        vg = torch.empty(N, dtype=torch.float32, device="cuda")
        vi = torch.empty_like(vg)
        lab = torch.empty(N, dtype=torch.int16, device="cuda")
        ps = POLICY_SWEEPS_DIFFUSION if eps > 0 else POLICY_SWEEPS
        res = {}
        for name, mode, v in (("transmission", capi.PATCHY_TRANSMISSION, vg), ("independent", capi.PATCHY_INDEPENDENT, vi)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = ctx.solve_patchy(dp, dpc, v, mode=mode, tol=tol, tol_coarse=1e-7, source_patch=src,
                                  n_patches=patches, label_out=lab, policy_sweeps=ps)
            torch.cuda.synchronize()
            res[name] = {"time_s": time.perf_counter() - t, "passes": st["passes"], "converged": st["status"] == 0}
        # a node reads the corners of the cells its feet fall in: up to floor(reach) + 1 cells away
        reach = capi.lib().slhjb_foot_reach(capi.DeviceProblem.host_struct(fine), float(fine.speed.max()))
        halo = int(np.floor(reach + 1e-6)) + 1
        free = torch.from_numpy(np.ascontiguousarray(fine.node_class).reshape(-1) == 0).cuda()
        band = interface_band(lab, halo) & free
        inner = free & ~band
        d = (vi - vg).abs()
        out[f"eps={eps:g}"] = {
            "halo": halo, "time_s_transmission": res["transmission"]["time_s"],
            "time_s_independent": res["independent"]["time_s"],
            "passes_independent": res["independent"]["passes"], "converged": res["independent"]["converged"],
            "decomposition_error_max": float(d[free].max()), "decomposition_error_mean": float(d[free].mean()),
            "band_max": float(d[band].max()) if bool(band.any()) else 0.0,
            "band_mean": float(d[band].mean()) if bool(band.any()) else 0.0,
            "interior_max": float(d[inner].max()), "interior_mean": float(d[inner].mean()),
            "band_fraction": float(band.sum()) / float(free.sum()),
        }
        log(f"indep eps={eps:g}: decomposition error max {out[f'eps={eps:g}']['decomposition_error_max']:.3g} "
            f"(band {out[f'eps={eps:g}']['band_max']:.3g}, interior {out[f'eps={eps:g}']['interior_max']:.3g})")
    return out


def arm_hdx(ctx, seed: int, tol: float, patches: int) -> dict:
    """The headline workload with h = dx instead of dx / 1.5: drift feet up
    to 1.5 cells away, so the fine solve takes the general kernels; patchy step against the cold
    global Jacobi iteration. The integer labeler takes first-ring feet only, so this step runs
    without labels (the transmission-mode solve does not read them)."""
    import torch

    from paper_1502_01629_amd import capi
    from paper_1502_01629_amd import instances as I

    fine, coarse = I.scattered_problem(seed, eps=0.0, h_factor=1.0)
    dp, dpc = capi.DeviceProblem(fine, capi.SL3), capi.DeviceProblem(coarse, capi.SL3)
    N = fine.n * fine.n
    free = int((fine.node_class == 0).sum())
    v = torch.empty(N, dtype=torch.float32, device="cuda")
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        sp = ctx.solve_patchy(dp, dpc, v, tol=tol, tol_coarse=1e-7, policy_sweeps=POLICY_SWEEPS)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    vj = torch.from_numpy(fine.initial().reshape(-1)).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    sj = ctx.solve(dp, vj, tol=tol, max_sweeps=200_000)
    torch.cuda.synchronize()
    tj = time.perf_counter() - t
    out = {"h": float(fine.h), "dx": fine.dx, "patchy_time_s": float(np.median(times[1:])), "patchy_passes": sp["passes"],
           "patchy_node_updates_per_free_node": sp["node_updates"] / free, "halo": sj["halo"],
           "kernel_path": "general" if sj["kernel_path"] == 0 else "first-ring",
           "global_jacobi_cold_s": tj, "global_jacobi_sweeps": sj["sweeps"],
           "sweep_kernel_us": 1e6 * sj["sweep_seconds"] / sj["sweep_launches"],
           "speedup": tj / float(np.median(times[1:])), "max_abs_diff": float((v - vj).abs().max())}
    log(f"hdx: patchy {out['patchy_time_s'] * 1e3:.1f} ms, global Jacobi {tj:.3f} s")
    return out


def arm_balance(ctx, seed: int, patches: int, rounds: int = 4) -> dict:
    """Balanced patches on the step's workload (2049^2 scattered targets, eps = 0): the coarse solve,
    u_hat and the synthesized control as in the step, then slhjb_balance_sources from the equal
    angular sectors; the patch sizes of every round and the time."""
    import torch

    from paper_1502_01629_amd import capi
    from paper_1502_01629_amd import instances as I

    fine, coarse = I.scattered_problem(seed)
    dp, dpc = capi.DeviceProblem(fine, capi.SL3), capi.DeviceProblem(coarse, capi.SL3)
    vc = torch.from_numpy(coarse.initial().reshape(-1)).cuda()
    ctx.solve_tiles(dpc, vc, tol=1e-7, order=capi.ORDER_NONE, tile_shape=capi.TILE_8x8_SPLIT4, max_passes=50000,
                    policy_sweeps=POLICY_SWEEPS)
    vhat = torch.empty(fine.n * fine.n, dtype=torch.float32, device="cuda")
    ctx.upsample(vc, coarse.n, vhat, fine.n)
    ctrl = torch.empty(fine.n * fine.n, dtype=torch.int16, device="cuda")
    ctx.synthesize(dp, vhat, ctrl)
    src_host, _ = capi.partition_sources(fine.node_class, patches)
    src = torch.from_numpy(src_host.reshape(-1)).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    sizes, best = ctx.balance_sources(dp, ctrl, src, patches, rounds, v_hat=vhat)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ratio = lambda s: float(np.max(s) / np.mean(s))
    log(f"balance: largest/mean patch {[round(ratio(s), 3) for s in sizes]}, kept round {best}, {dt:.2f} s")
    return {"n": fine.n, "patches": patches, "rounds": rounds, "time_s": dt, "kept_round": best,
            "largest_over_mean": [ratio(s) for s in sizes],
            "smallest_over_mean": [float(np.min(s) / np.mean(s)) for s in sizes],
            "sizes_start": [int(v) for v in sizes[0]], "sizes_kept": [int(v) for v in sizes[best]]}


def arm_learned(ctx, seed: int, tol: float, n: int = 1025, n_coarse: int = 129, train_count: int = 192,
                test_count: int = 8, steps: int = 2000) -> dict:
    """Learned warm start: the 4-level U-Net (BF16 matrix-core kernels of the library) trained on
    the method's own solves of the batch law at n^2 (coarse n_coarse^2, bicubic u_hat as input),
    then on held-out problems the cold start (v = 1), the bilinear u_hat, the bicubic u_hat and the
    network's start, each solved to tol by Jacobi and by the u_hat-ordered active-tile solver."""
    import torch

    from paper_1502_01629_amd import capi, warmstart
    from paper_1502_01629_amd import instances as I

    pairs = I.warmstart_problems(seed, count=train_count + test_count, n=n, n_coarse=n_coarse)
    t = time.perf_counter()
    frames = []
    for k in range(0, len(pairs), 32):
        frames += warmstart.make_frames(ctx, pairs[k:k + 32], tol=tol, bicubic=True)
        log(f"learned: {len(frames)} of {len(pairs)} solves, {time.perf_counter() - t:.1f} s")
    t_data = time.perf_counter() - t
    train, test = frames[:train_count], frames[train_count:]
    net = capi.Net(ctx, arch=capi.NET_UNET)
    net.set_params(warmstart.init_params(net, seed))
    torch.cuda.synchronize()
    t = time.perf_counter()
    losses = warmstart.train(net, train, steps=steps, batch=8, crop=256, lr=1e-3, seed=seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t
    log(f"learned: {steps} training steps in {t_train:.1f} s, loss {np.mean(losses[:20]):.2e} -> "
        f"{np.mean(losses[-20:]):.2e}")
    rows = warmstart.evaluate(ctx, net, test, tol=tol)
    for f, r in zip(test, rows):
        free = torch.from_numpy((f.dp.inst.node_class.reshape(-1) == 0)).cuda()
        v = torch.from_numpy(f.dp.inst.initial().reshape(-1)).cuda()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = ctx.solve(f.dp, v, tol=tol, max_sweeps=1_000_000)
        torch.cuda.synchronize()
        r["jacobi_sweeps_cold"] = st["sweeps"]
        r["jacobi_s_cold"] = time.perf_counter() - t
        r["jacobi_err_cold"] = float((v - f.vstar).abs()[free].max())
    net.close()
    names = ("uhat", "uhat_bicubic", "network")
    mean = lambda k: float(np.mean([r[k] for r in rows]))
    per = lambda key, extra=(): {m: mean(f"{key}_{m}") for m in tuple(extra) + names}
    out = {
        "n": n, "coarse": n_coarse, "network": "unet4", "train_problems": train_count,
        "test_problems": test_count, "data_generation_s": t_data, "training_steps": steps,
        "training_s": t_train, "loss_first": float(np.mean(losses[:20])),
        "loss_last": float(np.mean(losses[-20:])), "inference_s": mean("t_network_s"),
        "start_error_mean": per("err_mean"), "start_error_max": per("err_max"),
        "jacobi_sweeps": per("jacobi_sweeps", ("cold",)), "jacobi_time_s": per("jacobi_s", ("cold",)),
        "jacobi_stop_error_max": per("jacobi_err", ("cold",)),
        "active_tiles_time_s": per("tiles_s"), "active_tiles_updates_per_node": per("tiles_updates_per_node"),
        "active_tiles_stop_error_max": per("tiles_err"),
        "reference_residual_max": max(r["ref_residual"] for r in rows),
    }
    for r in rows:
        log(f"learned test n={r['n']} eps={r['eps']:.2e}: start err max uhat {r['err_max_uhat']:.3e} "
            f"bicubic {r['err_max_uhat_bicubic']:.3e} net {r['err_max_network']:.3e}; tiles s "
            f"{r['tiles_s_uhat']:.3f}/{r['tiles_s_uhat_bicubic']:.3f}/{r['tiles_s_network']:.3f}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--eps", type=float, default=0.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n", type=int, default=2049)
    ap.add_argument("--patches", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-arms", action="store_true", help="skip the comparison arms")
    ap.add_argument("--arms", default="c2,c2eps,indep,hdx,batch,bumps,balance,learned,exit",
                    help="comparison arms: c2 (global Jacobi, static decomposition), c2eps (the same workload "
                         "with eps = 1e-3 and 1e-2), indep (decomposition error of the independent patch solves), "
                         "hdx (the step with h = dx), batch (256 instances), bumps (4097^2 rank-1 diffusion), "
                         "balance (balanced patches on the step's workload), "
                         "learned (U-Net warm start at 1025^2), exit (the paper's exit-to-boundary experiments: "
                         "Table 0 on the GPU and the eps-threshold sweeps of Tables 1 and 2)")
    ap.add_argument("--arms-out", default=os.path.join(ROOT, "_build", "bench_arms.json"),
                    help="file that receives the full record (every arm); the stdout line holds a summary")
    ap.add_argument("--bumps-n", type=int, default=4097)
    ap.add_argument("--learned-train", type=int, default=192, help="training solves of the learned arm")
    ap.add_argument("--learned-steps", type=int, default=2000, help="training steps of the learned arm")
    ap.add_argument("--policy-sweeps", type=int, default=POLICY_SWEEPS,
                    help="policy-evaluation iterations after each full iteration of a tile visit")
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
        print("bench.py measures one GPU only: there is no multi-GPU path (the library runs on one device). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1502_01629_amd import capi
    from paper_1502_01629_amd import instances as I
    from paper_1502_01629_amd import roofline as RL

    scheme = capi.SL3
    fine, coarse = I.scattered_problem(args.seed, n=args.n, eps=args.eps)
    free = int((fine.node_class == 0).sum())
    ctx = capi.Context(0)
    dp = capi.DeviceProblem(fine, scheme)
    dpc = capi.DeviceProblem(coarse, scheme)
    t_part = time.perf_counter()
    src_host, n_targets = capi.partition_sources(fine.node_class, args.patches)
    t_part = time.perf_counter() - t_part
    src = torch.from_numpy(src_host.reshape(-1)).cuda()
    v = torch.empty(fine.n * fine.n, dtype=torch.float32, device="cuda")
    lab = torch.empty(fine.n * fine.n, dtype=torch.int16, device="cuda")

    def step(kernel_time: int = 0):
        return ctx.solve_patchy(dp, dpc, v, mode=capi.PATCHY_TRANSMISSION, tol=args.tol, tol_coarse=1e-7,
                                source_patch=src, n_patches=args.patches, label_out=lab,
                                collect_kernel_time=kernel_time, policy_sweeps=args.policy_sweeps)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert all(s["status"] == 0 for s in stats), stats
    v_pdd = v.clone()
    # The timed steps run the passes as graph replays; events inside a graph cannot be timed, so
    # the kernel's own durations come from the same number of steps with the passes launched one
    # by one and HIP events around every visit launch, on its stream, right after.
    kstats = [step(1) for _ in range(args.steps)]
    assert all(s["status"] == 0 for s in kstats), kstats
    # The same step without the patch labels: the transmission-mode solve does not read them, so
    # this is the cost of the labeler running beside it (reported, not the value)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nl = [ctx.solve_patchy(dp, dpc, v, mode=capi.PATCHY_TRANSMISSION, tol=args.tol, tol_coarse=1e-7,
                           policy_sweeps=args.policy_sweeps) for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt_nolabels = time.perf_counter() - t0
    assert all(s["status"] == 0 for s in nl), nl

    med = lambda k: float(np.median([s[k] for s in stats]))
    visit_s = sum(s["t_visit"] for s in kstats)
    visit_launches = sum(s["passes"] for s in kstats)
    fine_updates = sum(s["node_updates"] for s in kstats)
    policy_updates = sum(s["policy_updates"] for s in kstats)
    check_sweeps = sum(s["check_sweeps"] for s in kstats)
    check_visit_s = sum(s["t_check_visit"] for s in kstats)
    flop_per_update = RL.sweep_flops_per_node_update(fine.diffusion, scheme, fine.n_controls)
    # a policy-evaluation update is the same update with one control
    flop_per_policy_update = RL.sweep_flops_per_node_update(fine.diffusion, scheme, 1)
    avg_launch = visit_s / visit_launches
    achieved = (fine_updates * flop_per_update + policy_updates * flop_per_policy_update) / visit_s / 1e12
    kernel = "tilectl_visit_kernel<16,16,split 2,NONE,SL3,first-ring>"
    traffic = measured_traffic(kernel)

    out = {
        "metric": "time-to-residual-1e-6 at 2049^2 2D HJB (patchy method, warm start from u_hat)",
        "value": dt / args.steps,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded instance generator)",
        "config": {
            "workload": f"scattered targets {fine.n}^2, c=1+0.5sin(2pi x1)sin(2pi x2), 64 controls, {n_targets} point "
                        f"targets, 10% square obstacles, eps={args.eps}, h=dx/1.5={float(fine.h):.4g}, SL3; coarse "
                        f"{coarse.n}^2, {args.patches} patches; residual {args.tol:g}",
            "n": fine.n, "eps": args.eps, "h": float(fine.h), "dx": fine.dx, "n_controls": fine.n_controls,
            "seed": args.seed, "tol": args.tol, "free_nodes": free, "patches": args.patches,
        },
        "stages_s": {k: med(k) for k in ("t_coarse", "t_upsample", "t_synthesize", "t_label", "t_solve")},
        "ms_per_step_without_labels": 1e3 * dt_nolabels / args.steps,
        "source_partition_host_s": t_part,
        "passes": int(med("passes")),
        "node_updates_per_free_node": fine_updates / len(kstats) / free,
        "policy_updates_per_free_node": policy_updates / len(kstats) / free,
        "node_updates_per_s": fine_updates / len(kstats) / (dt / args.steps),
        "policy_sweeps": args.policy_sweeps,
        "check_sweeps": {"per_step": check_sweeps / len(kstats),
                         "node_update_share": check_sweeps * free / max(1, fine_updates),
                         "visit_time_share": check_visit_s / visit_s if visit_s > 0 else None,
                         "visit_ms_per_step": 1e3 * check_visit_s / len(kstats)},
        "roofline": {
            "kernel": kernel,
            "bound": "alu",
            "achieved": achieved,
            "peak": RL.FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / RL.FP32_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "avg_launch_us": avg_launch * 1e6,
            # per step, over the visit launches of the instrumented steps (passes that did work plus
            # the no-op passes of the last batch): a kernel-trace profile of the same command has
            # the same total per step over its graph replays
            "visit_ms_per_step": 1e3 * visit_s / len(kstats),
            "measured_over": f"{args.steps} steps after the timed steps, every visit launched through "
                             "hipExtLaunchKernel with events stamped at the kernel's start and end",
            "flops_per_node_update": flop_per_update,
            "flops_per_policy_update": flop_per_policy_update,
        },
    }
    acc = oracle_samples_error(v_pdd, fine, args.seed, args.eps)
    if acc is not None:
        out["accuracy_vs_oracle"] = acc
    if acc is not None and not args.no_arms:
        # the same step stopped at residual 2e-7: the error left at 1e-6 is the stopping point's
        # distance to the fixed point, not the arithmetic's
        st2 = ctx.solve_patchy(dp, dpc, v, mode=capi.PATCHY_TRANSMISSION, tol=2e-7, tol_coarse=1e-7,
                               policy_sweeps=args.policy_sweeps)
        acc2 = oracle_samples_error(v, fine, args.seed, args.eps)
        out["accuracy_vs_oracle_at_residual_2e-7"] = {"max_abs": acc2["max_abs"], "mean_abs": acc2["mean_abs"],
                                                      "passes": st2["passes"], "time_s": st2["t_total"]}

    jacobi_sweeps = None
    which = set() if args.no_arms else {a.strip() for a in args.arms.split(",") if a.strip()}
    arms = {}
    if "c2" in which:
        v0 = torch.from_numpy(fine.initial().reshape(-1)).cuda()
        # plain global Jacobi from v = 1: the SL sweep kernel at full rate
        vj = v0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        sj = ctx.solve(dp, vj, tol=args.tol, max_sweeps=2_000_000)
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        jacobi_sweeps = sj["converged_sweep"]
        sweep_flops = flop_per_update * free / (sj["sweep_seconds"] / sj["sweep_launches"]) / 1e12
        arms["global_jacobi_cold"] = {
            "time_s": t, "sweeps": sj["sweeps"], "node_updates_per_s": sj["node_updates"] / t,
            "sweep_kernel_us": 1e6 * sj["sweep_seconds"] / sj["sweep_launches"],
            "sweep_kernel_tflops": sweep_flops, "sweep_kernel_frac": sweep_flops / RL.FP32_VECTOR_PEAK_TFLOPS,
            "max_abs_diff_vs_patchy": float((vj - v_pdd).abs().max()),
        }
        acc_j = oracle_samples_error(vj, fine, args.seed, args.eps)
        if acc_j is not None:
            arms["global_jacobi_cold"]["max_abs_vs_oracle"] = acc_j["max_abs"]
        # global Jacobi from u_hat (the warm start without the u_hat order)
        vh = torch.empty_like(v0)
        vc = torch.from_numpy(coarse.initial().reshape(-1)).cuda()
        ctx.solve(dpc, vc, tol=1e-7)
        ctx.upsample(vc, coarse.n, vh, fine.n)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sw = ctx.solve(dp, vh, tol=args.tol, max_sweeps=2_000_000)
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        arms["global_jacobi_uhat"] = {"time_s_after_uhat": t, "sweeps": sw["sweeps"],
                                      "node_updates_per_s": sw["node_updates"] / t,
                                      "max_abs_diff_vs_patchy": float((vh - v_pdd).abs().max())}
        # static decomposition: active tiles in a fixed order, no pre-computation, cold start
        vs = torch.empty_like(v0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        ss = ctx.solve_patchy(dp, None, vs, mode=capi.PATCHY_STATIC, tol=args.tol, policy_sweeps=args.policy_sweeps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        arms["static_decomposition_cold"] = {"time_s": t, "passes": ss["passes"],
                                             "node_updates_per_free_node": ss["node_updates"] / free,
                                             "max_abs_diff_vs_patchy": float((vs - v_pdd).abs().max())}
        out["speedup_vs_global_jacobi_cold"] = arms["global_jacobi_cold"]["time_s"] / out["value"]
        log(f"c2: cold global Jacobi {arms['global_jacobi_cold']['time_s']:.3f} s, static "
            f"{arms['static_decomposition_cold']['time_s'] * 1e3:.1f} ms")
    if "c2eps" in which:
        arms["c2_diffusion"] = arm_c2_eps(ctx, args.seed, args.tol, args.patches)
    if "indep" in which:
        arms["independent_patches"] = arm_indep(ctx, args.seed, args.tol, args.patches)
    if "hdx" in which:
        arms["h_equals_dx"] = arm_hdx(ctx, args.seed, args.tol, args.patches)
    if "batch" in which:
        arms["batch_256_instances"] = arm_batch(ctx, args.seed, args.tol)
    if "bumps" in which:
        arms["rank1_bumps"] = arm_bumps(ctx, args.seed, args.tol, args.bumps_n)
    if "balance" in which:
        arms["balanced_patches"] = arm_balance(ctx, args.seed, args.patches)
    if "learned" in which:
        arms["learned_warm_start"] = arm_learned(ctx, args.seed, args.tol, train_count=args.learned_train,
                                                   steps=args.learned_steps)
    if "exit" in which:
        arms["exit_to_boundary"] = arm_exit(ctx, args.tol)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(fine, scheme, jacobi_sweeps or 1672)
    ctx.close()
    full = dict(out, arms=arms)
    if args.arms_out:
        os.makedirs(os.path.dirname(os.path.abspath(args.arms_out)), exist_ok=True)
        with open(args.arms_out, "w") as f:
            json.dump(full, f, indent=1)
        log(f"full record: {args.arms_out}")
    print(json.dumps(summary_line(full)), flush=True)


def _r(x, d: int = 4):
    """Round for the summary line (None passes through)."""
    if x is None:
        return None
    if isinstance(x, float):
        return float(f"{x:.{d}g}")
    return x


def summary_line(full: dict) -> dict:
    """The one stdout line: the headline fields as they are, and a few numbers per arm."""
    keep = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data", "config", "passes", "node_updates_per_s", "node_updates_per_free_node",
            "policy_updates_per_free_node", "check_sweeps", "stages_s", "accuracy_vs_oracle",
            "accuracy_vs_oracle_at_residual_2e-7",
            "speedup_vs_global_jacobi_cold", "ms_per_step_without_labels")
    out = {k: full[k] for k in keep if k in full}
    out["config"] = {k: full["config"][k] for k in ("workload", "n", "h", "eps", "tol", "free_nodes")}
    out["stages_s"] = {k: _r(v) for k, v in full.get("stages_s", {}).items()}
    out["check_sweeps"] = {k: _r(v) for k, v in full.get("check_sweeps", {}).items()}
    r = full["roofline"]
    out["roofline"] = {k: _r(r[k]) for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "avg_launch_us",
                                               "visit_ms_per_step", "kernel")}
    if "cpu_baseline" in full:
        out["cpu_baseline"] = {k: _r(v) for k, v in full["cpu_baseline"].items()}
    A = full.get("arms", {})
    arms = {}
    if "global_jacobi_cold" in A:
        g = A["global_jacobi_cold"]
        arms["global_jacobi_cold"] = {"time_s": _r(g["time_s"]), "sweeps": g["sweeps"],
                                      "node_updates_per_s": _r(g["node_updates_per_s"]),
                                      "sweep_kernel_us": _r(g["sweep_kernel_us"]),
                                      "sweep_kernel_frac": _r(g["sweep_kernel_frac"]),
                                      "max_abs_vs_oracle": _r(g.get("max_abs_vs_oracle"))}
        arms["global_jacobi_uhat_s"] = _r(A["global_jacobi_uhat"]["time_s_after_uhat"])
        arms["static_decomposition_s"] = _r(A["static_decomposition_cold"]["time_s"])
    if "c2_diffusion" in A:
        arms["c2_diffusion"] = {k: {"patchy_s": _r(e["patchy_time_s"]), "jacobi_s": _r(e["global_jacobi_cold_s"]),
                                    "max_abs_diff": _r(e["max_abs_diff"], 3)} for k, e in A["c2_diffusion"].items()}
    if "independent_patches" in A:
        arms["decomposition_error"] = {k: {"max": _r(e["decomposition_error_max"], 3), "band_max": _r(e["band_max"], 3),
                                           "interior_max": _r(e["interior_max"], 3),
                                           "interior_mean": _r(e["interior_mean"], 3)}
                                       for k, e in A["independent_patches"].items()}
    if "h_equals_dx" in A:
        e = A["h_equals_dx"]
        arms["h_equals_dx"] = {"patchy_s": _r(e["patchy_time_s"]), "jacobi_s": _r(e["global_jacobi_cold_s"]),
                               "halo": e["halo"]}
    if "batch_256_instances" in A:
        e = A["batch_256_instances"]
        arms["batch_256"] = {"batched_s": _r(e["time_s_batched"]), "sequential_s": _r(e["time_s_sequential"]),
                             "bit_exact": e["bit_exact_vs_single"]}
        if "active_tiles" in e:
            t = e["active_tiles"]
            arms["batch_256"]["active_tiles"] = {"batched_s": _r(t["time_s_batched"]),
                                                 "sequential_s": _r(t["time_s_sequential"]),
                                                 "bit_exact": t["bit_exact_vs_single"]}
    if "rank1_bumps" in A:
        e = A["rank1_bumps"]
        arms["rank1_4097"] = {"full_sweeps_s": _r(e["full_sweeps"]["time_s"]),
                              "active_tiles_cold_s": _r(e["active_tiles_cold"]["time_s"]),
                              "active_tiles_uhat_s": _r(e["active_tiles_uhat"]["time_s"])}
    if "balanced_patches" in A:
        e = A["balanced_patches"]
        arms["balance_2049"] = {"largest_over_mean": [_r(v, 3) for v in e["largest_over_mean"]],
                                "kept": e["kept_round"], "s": _r(e["time_s"])}
    if "learned_warm_start" in A:
        e = A["learned_warm_start"]
        arms["learned_1025"] = {"train": e["train_problems"],
                                "start_error_mean": {k: _r(v, 3) for k, v in e["start_error_mean"].items()},
                                "jacobi_sweeps": {k: _r(v) for k, v in e["jacobi_sweeps"].items()},
                                "active_tiles_s": {k: _r(v) for k, v in e["active_tiles_time_s"].items()},
                                "stop_err_tiles": {k: _r(v, 3) for k, v in e["active_tiles_stop_error_max"].items()}}
    if "exit_to_boundary" in A:
        t0 = A["exit_to_boundary"]["table0"]
        arms["exit_table0_sl2_sl3"] = {f"{r['equation']}/{r['eps']:g}": [r["jacobi_sweeps_sl2"], r["jacobi_sweeps_sl3"]]
                                       for r in t0}
    out["arms"] = arms
    return out


if __name__ == "__main__":
    main()

"""Tile-shape autotuner of the batched solve (slhjb_solve_batch).

Instances are grouped in buckets by what sets the cost of a tile visit: grid size n, number of
controls (in steps of 16), diffusion kind (feet per control) and interpolation halo (foot reach in
cells). For each
bucket the tuner times a short run of the batched solve on (up to) a few of the bucket's own
instances with every tile shape, keeps the fastest, and caches the choice in a JSON file keyed by
the bucket and the device name, so later batches pay nothing. The tile shape changes only the
schedule, never the values, so the choice is free to be made by timing.
"""
from __future__ import annotations

import json
import math
import os

from . import capi

DEFAULT_CACHE = os.environ.get("SLHJB_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "slhjb", "batch_tiles.json"))


def bucket_key(inst) -> str:
    """n, controls (rounded up to 16), diffusion kind (0 when eps = 0) and the halo the kernels stage."""
    dp_struct = capi.DeviceProblem.host_struct(inst)
    speed_max = float(inst.speed.max())
    reach = capi.lib().slhjb_foot_reach(dp_struct, speed_max)
    diff = int(inst.diffusion) if float(inst.eps) > 0.0 else 0
    halo = 2 if (diff == 0 and reach <= 1.0 + 1e-6) else int(math.floor(reach * (1.0 + 1e-6) + 1e-6)) + 1
    na = -(-inst.controls.shape[0] // 16) * 16  # the cost is linear in N_A: buckets of 16
    return f"n{inst.n}-a{na}-d{diff}-r{halo}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(ctx: "capi.Context", instances, scheme: int = capi.SL3, cache: str | None = DEFAULT_CACHE,
         sweeps: int = 24, per_bucket: int = 4, device_name: str | None = None) -> list[int]:
    """Tile shape (capi.BATCH_TILE_*) for every instance, from the cache or by timing."""
    import torch

    dev = device_name or torch.cuda.get_device_name(0)
    table = _load(cache) if cache else {}
    entries = table.setdefault(dev, {})
    keys = [bucket_key(x) for x in instances]
    todo = sorted({k for k in keys if k not in entries})
    for key in todo:
        members = [x for x, k in zip(instances, keys) if k == key][:per_bucket]
        probs = [capi.DeviceProblem(x, scheme) for x in members]
        best, best_t = None, math.inf
        timings = {}
        for shape in capi.BATCH_TILE_SHAPES:
            t = math.inf
            for _ in range(2):  # the first run also warms up
                vs = [torch.from_numpy(x.initial().reshape(-1)).cuda() for x in members]
                _, tot = ctx.solve_batch(probs, vs, tol=0.0, max_sweeps=sweeps, check_every=8,
                                         tile_shapes=[shape] * len(members))
                t = min(t, tot["seconds"])
            timings[str(shape)] = t
            if t < best_t:
                best, best_t = shape, t
        entries[key] = {"shape": best, "seconds": timings, "sweeps": sweeps, "instances": len(members)}
    if cache and todo:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return [int(entries[k]["shape"]) for k in keys]

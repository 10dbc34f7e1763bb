"""Seeded synthetic problem instances (inputs only).

This module builds the FP32 input arrays of the 2-D test problems: node classes (free,
target, obstacle), the speed field c(x), the discrete control set and the scalar
parameters. It holds none of the scheme's arithmetic and serves both the GPU path and the
FP64 oracle, which consume exactly the same arrays.

Problem family (Section 5 of the paper, eikonal dynamics B): Omega = [-1,1]^2, dynamics
f(x,a) = c(x) a with a in a discretized unit circle, running cost l = 1, discount lambda = 1
(Kruzkov form v = 1 - exp(-T)), value v_out = 1 outside the box and on obstacles, v = 0 on
target nodes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FREE, TARGET, OBSTACLE = 0, 1, 2
DIFF_NONE, DIFF_ISO, DIFF_RANK1 = 0, 1, 2


@dataclass
class Instance:
    n: int
    h: np.float32
    eps: np.float32
    diffusion: int
    controls: np.ndarray  # float32 (N_A, 2)
    speed: np.ndarray  # float32 (n, n), row j = x2 index
    node_class: np.ndarray  # uint8 (n, n)
    x_lo: np.float32 = np.float32(-1.0)
    x_hi: np.float32 = np.float32(1.0)
    lam: np.float32 = np.float32(1.0)
    running_cost: np.float32 = np.float32(1.0)
    target_value: np.float32 = np.float32(0.0)
    v_out: np.float32 = np.float32(1.0)
    meta: dict = field(default_factory=dict)
    drift: np.ndarray | None = None  # float32 (n, n, 2): f(x,a) = c(x) (drift(x) + a); None = no drift
    # Sections 5.2-5.3: l(x,a) = l_x(x) + l_a(a) and a diffusion coefficient eps(x) per node
    running_cost_field: np.ndarray | None = None  # float32 (n, n): l_x; None = running_cost
    control_cost: np.ndarray | None = None  # float32 (N_A,): l_a; None = 0
    eps_field: np.ndarray | None = None  # float32 (n, n): eps(x); None = eps

    @property
    def dx(self) -> float:
        return (float(self.x_hi) - float(self.x_lo)) / (self.n - 1)

    @property
    def n_controls(self) -> int:
        return int(self.controls.shape[0])

    def initial(self, free_value: float = 1.0) -> np.ndarray:
        """FP32 start vector: free_value on FREE nodes (1 = the cold start T = +inf)."""
        v = np.full((self.n, self.n), np.float32(free_value), dtype=np.float32)
        v[self.node_class == TARGET] = self.target_value
        v[self.node_class == OBSTACLE] = self.v_out
        return v


def control_table(n_controls: int) -> np.ndarray:
    """a_m = (cos 2 pi m/N, sin 2 pi m/N), m = 0..N-1, as float32. When 8 divides N the table
    is built from its first octant by exact swaps and 90-degree rotations, so it is closed
    under the symmetries of the square in float32 (axis directions are exactly (+-1,0),
    (0,+-1)). Components that are zero in exact arithmetic (|c| < 1e-6 after rounding, e.g.
    sin(pi)) are stored as exact zeros, so a foot of a boundary node moving along the boundary
    stays on it."""
    N = int(n_controls)
    out = np.zeros((N, 2), dtype=np.float32)
    if N % 8 == 0:
        q = N // 8
        for m in range(2 * q + 1):
            if m <= q:
                th = 2.0 * math.pi * m / N
                out[m % N] = (np.float32(math.cos(th)), np.float32(math.sin(th)))
            else:
                out[m] = out[2 * q - m][::-1]
        quarter = 2 * q
        for m in range(quarter, N):
            x, y = out[m - quarter]
            out[m] = (-y, x)
    else:
        for m in range(N):
            th = 2.0 * math.pi * m / N
            out[m] = (np.float32(math.cos(th)), np.float32(math.sin(th)))
    out[np.abs(out) < 1e-6] = 0.0
    return out


def node_coords(n: int, x_lo: float = -1.0, x_hi: float = 1.0):
    dx = (x_hi - x_lo) / (n - 1)
    x = x_lo + dx * np.arange(n, dtype=np.float64)
    X1, X2 = np.meshgrid(x, x, indexing="xy")  # X1[j, i] = x_i, X2[j, i] = x_j
    return X1, X2


@dataclass
class Geometry:
    """Continuous description of a problem: disc targets, square obstacles, a speed law."""

    targets: list  # [(cx, cy, r)]
    obstacles: list = field(default_factory=list)  # [(x0, y0, side)] lower-left corner
    speed_law: str = "const"  # const | sines | bumps
    bumps: list = field(default_factory=list)  # [(mx, my, amp, width)]

    def speed(self, n: int) -> np.ndarray:
        X1, X2 = node_coords(n)
        if self.speed_law == "const":
            c = np.ones_like(X1)
        elif self.speed_law == "sines":
            c = 1.0 + 0.5 * np.sin(2 * np.pi * X1) * np.sin(2 * np.pi * X2)
        elif self.speed_law == "bumps":
            c = np.ones_like(X1)
            for (mx, my, amp, width) in self.bumps:
                c += amp * np.exp(-((X1 - mx) ** 2 + (X2 - my) ** 2) / (2.0 * width * width))
            c = np.maximum(c, 0.1)
        else:
            raise ValueError(self.speed_law)
        return c.astype(np.float32)

    def classes(self, n: int) -> np.ndarray:
        X1, X2 = node_coords(n)
        cls = np.zeros((n, n), dtype=np.uint8)
        for (x0, y0, s) in self.obstacles:
            cls[(X1 >= x0) & (X1 <= x0 + s) & (X2 >= y0) & (X2 <= y0 + s)] = OBSTACLE
        for (cx, cy, r) in self.targets:
            cls[(X1 - cx) ** 2 + (X2 - cy) ** 2 <= r * r] = TARGET
        return cls

    def instance(self, n: int, n_controls: int, eps: float, diffusion: int, h: float, **meta) -> Instance:
        return Instance(n=n, h=np.float32(h), eps=np.float32(eps),
                        diffusion=diffusion if eps > 0 else DIFF_NONE,
                        controls=control_table(n_controls), speed=self.speed(n), node_class=self.classes(n),
                        meta=dict(meta, geometry=self))


# ---------------------------------------------------------------------------------------
# The five workload shapes.

def disc_problem(n: int = 129, eps: float = 0.0, n_controls: int = 32, h_factor: float = 1.0,
                 diffusion: int = DIFF_ISO) -> Instance:
    """Plain global method, CPU-sized: target disc of radius 0.1 at the origin, c = 1,
    32 directions, h = dx, isotropic diffusion sqrt(2 eps) I."""
    g = Geometry(targets=[(0.0, 0.0, 0.1)])
    dx = 2.0 / (n - 1)
    return g.instance(n, n_controls, eps, diffusion, h_factor * dx, workload="disc")


def offcenter_problem(n: int = 129, cx: float = 0.55, cy: float = 0.35, r: float = 0.12, n_controls: int = 32,
                      seed: int = 0) -> Instance:
    """Unbalanced patches: one disc target off the centre of the box (the patches facing the far
    sides are much larger than those facing the near ones), c(x) from 8 bumps, sigma = 0,
    h = 0.99 dx / max c (every foot in the first ring of cells, as the patch labeling needs)."""
    rng = np.random.default_rng(np.random.SeedSequence([1502, 1629, 6, seed]))
    g = Geometry(targets=[(cx, cy, r)], speed_law="bumps", bumps=bump_geometry(rng, 8))
    h = 0.99 * (2.0 / (n - 1)) / float(g.speed(n).max())
    return g.instance(n, n_controls, 0.0, DIFF_NONE, h, workload="offcenter", seed=seed)


def _coarse_node_inside(cx, cy, r, n_coarse):
    X1, X2 = node_coords(n_coarse)
    return bool(np.any((X1 - cx) ** 2 + (X2 - cy) ** 2 <= r * r))


def scattered_geometry(seed: int, n_targets: int = 3, target_r: float = 0.02, n_obstacles: int = 10,
                       obstacle_side: float = 0.2, n_coarse: int = 129) -> Geometry:
    """Point-like disc targets (radius 0.02, centres U[-0.9,0.9]^2, pairwise >= 0.2 apart, each
    holding at least one node of the coarse grid) and non-overlapping square obstacles of side
    0.2 covering 10% of the box, kept 0.05 away from every target."""
    rng = np.random.default_rng(np.random.SeedSequence([1502, 1629, seed]))
    targets = []
    while len(targets) < n_targets:
        cx, cy = rng.uniform(-0.9, 0.9, size=2)
        if any((cx - tx) ** 2 + (cy - ty) ** 2 < 0.2 ** 2 for (tx, ty, _) in targets):
            continue
        if not _coarse_node_inside(cx, cy, target_r, n_coarse):
            continue
        targets.append((float(cx), float(cy), target_r))
    obstacles = []
    guard = 0.05
    while len(obstacles) < n_obstacles:
        x0, y0 = rng.uniform(-1.0, 1.0 - obstacle_side, size=2)
        ok = True
        for (ox, oy, s) in obstacles:
            if x0 < ox + s and ox < x0 + obstacle_side and y0 < oy + s and oy < y0 + obstacle_side:
                ok = False
                break
        for (tx, ty, r) in targets:
            px = min(max(tx, x0), x0 + obstacle_side)
            py = min(max(ty, y0), y0 + obstacle_side)
            if (px - tx) ** 2 + (py - ty) ** 2 <= (r + guard) ** 2:
                ok = False
        if ok:
            obstacles.append((float(x0), float(y0), obstacle_side))
    return Geometry(targets=targets, obstacles=obstacles, speed_law="sines")


def scattered_problem(seed: int = 0, n: int = 2049, eps: float = 0.0, n_controls: int = 64,
                      h_factor: float = 1.0 / 1.5, n_coarse: int = 129) -> tuple[Instance, Instance]:
    """Patchy-vs-static workload: c(x) = 1 + 0.5 sin(2 pi x1) sin(2 pi x2), 64 controls, three
    point targets, obstacles on 10% of the box, isotropic diffusion. h = dx / 1.5 keeps every
    drift foot inside the first ring of cells (h c_max <= dx). Returns (fine, coarse); the
    coarse problem has sigma = 0 and its own h = dx_c / 1.5."""
    g = scattered_geometry(seed, n_coarse=n_coarse)
    fine = g.instance(n, n_controls, eps, DIFF_ISO, h_factor * 2.0 / (n - 1), workload="scattered", seed=seed)
    coarse = g.instance(n_coarse, n_controls, 0.0, DIFF_NONE, h_factor * 2.0 / (n_coarse - 1),
                        workload="scattered-coarse", seed=seed)
    return fine, coarse


def bump_geometry(rng: np.random.Generator, n_bumps: int, width: float = 0.1) -> list:
    return [(float(rng.uniform(-1, 1)), float(rng.uniform(-1, 1)), float(rng.uniform(-0.5, 0.5)), width)
            for _ in range(n_bumps)]


def bumps_problem(seed: int = 0, n: int = 4097, eps: float = 1e-3, n_controls: int = 64,
                  h_factor: float = 1.0) -> Instance:
    """Degenerate-diffusion workload: rank-1 noise sqrt(2 eps) a along the control, c(x) = 1 + 16
    seeded Gaussian bumps (amplitude U[-0.5,0.5], width 0.1, floor 0.1), single disc target of
    radius 0.1 at the origin."""
    rng = np.random.default_rng(np.random.SeedSequence([1502, 1629, 3, seed]))
    g = Geometry(targets=[(0.0, 0.0, 0.1)], speed_law="bumps", bumps=bump_geometry(rng, 16))
    return g.instance(n, n_controls, eps, DIFF_RANK1, h_factor * 2.0 / (n - 1), workload="bumps", seed=seed)


def batch_problems(seed: int = 0, count: int = 256, sizes=(65, 129, 257, 513, 1025)) -> list[Instance]:
    """Serving-style batch: grid sizes uniform over `sizes`, 1-4 disc targets of radius
    U[0.02,0.1] with centres U[-0.8,0.8]^2, c(x) from 8 bumps, eps log-uniform in [1e-4,1e-2],
    32-64 controls, isotropic diffusion, h = dx."""
    ss = np.random.SeedSequence([1502, 1629, 4, seed])
    out = []
    for k, child in enumerate(ss.spawn(count)):
        rng = np.random.default_rng(child)
        n = int(rng.choice(sizes))
        nt = int(rng.integers(1, 5))
        targets = [(float(rng.uniform(-0.8, 0.8)), float(rng.uniform(-0.8, 0.8)), float(rng.uniform(0.02, 0.1)))
                   for _ in range(nt)]
        eps = float(10.0 ** rng.uniform(-4, -2))
        na = int(rng.integers(32, 65))
        g = Geometry(targets=targets, speed_law="bumps", bumps=bump_geometry(rng, 8))
        out.append(g.instance(n, na, eps, DIFF_ISO, 2.0 / (n - 1), workload="batch", seed=seed, index=k))
    return out


def warmstart_problems(seed: int = 0, count: int = 64, n: int = 1025, n_coarse: int = 129,
                       sizes_controls=(32, 65)) -> list[tuple[Instance, Instance]]:
    """Learned-warm-start data: the batch law (1-4 discs, 8 bumps, eps log-uniform in
    [1e-4, 1e-2], 32-64 controls, isotropic diffusion, h = dx) at a fixed fine size n, each with
    its coarse sigma = 0 companion on n_coarse^2 (h = dx_c). Returns (fine, coarse) pairs."""
    ss = np.random.SeedSequence([1502, 1629, 5, seed])
    out = []
    for k, child in enumerate(ss.spawn(count)):
        rng = np.random.default_rng(child)
        nt = int(rng.integers(1, 5))
        targets = [(float(rng.uniform(-0.8, 0.8)), float(rng.uniform(-0.8, 0.8)), float(rng.uniform(0.02, 0.1)))
                   for _ in range(nt)]
        eps = float(10.0 ** rng.uniform(-4, -2))
        na = int(rng.integers(*sizes_controls))
        g = Geometry(targets=targets, speed_law="bumps", bumps=bump_geometry(rng, 8))
        fine = g.instance(n, na, eps, DIFF_ISO, 2.0 / (n - 1), workload="warmstart", seed=seed, index=k)
        coarse = g.instance(n_coarse, na, 0.0, DIFF_NONE, 2.0 / (n_coarse - 1), workload="warmstart-coarse",
                            seed=seed, index=k)
        out.append((fine, coarse))
    return out


# ---------------------------------------------------------------------------------------
# Small problems with closed-form discrete solutions (used to pin the oracle).

def transport_problem(n: int = 17, n_controls: int = 32, scheme_h_factor: float = 1.0) -> Instance:
    """Left column is the target, c = 1, h = dx, sigma = 0."""
    cls = np.zeros((n, n), dtype=np.uint8)
    cls[:, 0] = TARGET
    dx = 2.0 / (n - 1)
    return Instance(n=n, h=np.float32(scheme_h_factor * dx), eps=np.float32(0.0), diffusion=DIFF_NONE,
                    controls=control_table(n_controls), speed=np.ones((n, n), dtype=np.float32),
                    node_class=cls, meta=dict(workload="transport"))


def rank1_walk_problem(n: int = 9) -> Instance:
    """One control (-1,0), rank-1 noise along it with eps = dx/2 (so sqrt(2 eps h) = dx when
    h = dx), the first two columns are the target."""
    cls = np.zeros((n, n), dtype=np.uint8)
    cls[:, :2] = TARGET
    dx = 2.0 / (n - 1)
    return Instance(n=n, h=np.float32(dx), eps=np.float32(dx / 2.0), diffusion=DIFF_RANK1,
                    controls=np.array([[-1.0, 0.0]], dtype=np.float32), speed=np.ones((n, n), dtype=np.float32),
                    node_class=cls, meta=dict(workload="rank1-walk"))


# ---------------------------------------------------------------------------------------
# Exit-to-boundary problems of the paper's experiments (Section 5): Omega = [-1,1]^2, g = 0 on
# the boundary, l = 1, 16 controls discretizing the unit ball, in Kruzkov form (lambda = 1,
# v = 1 - exp(-T), T the exit time). Boundary nodes are the target (v = 0); a foot outside the
# box has exited (v_out = 0).

def zermelo_drift(n: int, theta: float) -> np.ndarray:
    """d(x) = R_theta x / |x| (counter-clockwise rotation by theta), 0 at the origin."""
    X1, X2 = node_coords(n)
    r = np.hypot(X1, X2)
    safe = np.where(r > 0.0, r, 1.0)
    ux, uy = X1 / safe, X2 / safe
    ct, st = math.cos(theta), math.sin(theta)
    d = np.stack([ct * ux - st * uy, st * ux + ct * uy], axis=-1)
    d[r == 0.0] = 0.0
    return d.astype(np.float32)


def exit_dynamics(n: int, dynamics: str, eta: float = 1.0, theta: float = math.pi / 4,
                  n_controls: int = 16):
    """(speed, drift, controls, f_min, f_max) of the paper's test dynamics:
      A   advection b . grad u = 1 with b = (1, 0): in the control form f = -b (no control; the
          solution is T = 1 + x_1, information runs from the left side to the right)
      B   eikonal f = c a, c = 1
      B2  eikonal f = c a, c = 1 + chi{x_1 >= 0}
      C   Zermelo f = (R_theta x/|x| + (eta/2) a) / (1 + |x|^2)"""
    X1, X2 = node_coords(n)
    ones = np.ones((n, n), dtype=np.float32)
    if dynamics == "A":
        drift = np.zeros((n, n, 2), dtype=np.float32)
        drift[..., 0] = -1.0
        return ones, drift, np.zeros((1, 2), dtype=np.float32), 1.0, 1.0
    if dynamics == "B":
        return ones, None, control_table(n_controls), 1.0, 1.0
    if dynamics == "B2":
        c = np.where(X1 >= 0.0, 2.0, 1.0).astype(np.float32)
        return c, None, control_table(n_controls), 1.0, 2.0
    if dynamics == "C":
        c = (1.0 / (1.0 + X1 * X1 + X2 * X2)).astype(np.float32)
        ctrl = (np.float32(eta / 2.0) * control_table(n_controls)).astype(np.float32) if eta > 0 else \
            np.zeros((1, 2), dtype=np.float32)
        # |f| over the box and the controls: (1 - eta/2) / 3 at the corners, (1 + eta/2) at the origin
        return c, zermelo_drift(n, theta), ctrl, (1.0 - eta / 2.0) / 3.0, 1.0 + eta / 2.0
    raise ValueError(dynamics)


def exit_problem(n: int, dynamics: str = "B", eps: float = 0.0, eta: float = 1.0, theta: float = math.pi / 4,
                 n_controls: int = 16, h: float | None = None, diffusion: int = DIFF_ISO,
                 lam: float = 1.0) -> Instance:
    """Exit time from [-1,1]^2 with g = 0 (Section 5). h defaults to the paper's choice
    h = alpha dx / f_min with alpha = 1 / (1 + Upsilon), Upsilon = f_max / f_min. lam = 1: the
    Kruzkov form v = 1 - exp(-T); lam = 0: the undiscounted scheme of the paper, v = T."""
    speed, drift, ctrl, fmin, fmax = exit_dynamics(n, dynamics, eta, theta, n_controls)
    dx = 2.0 / (n - 1)
    if h is None:
        h = dx / (1.0 + fmax / fmin) / fmin
    cls = np.zeros((n, n), dtype=np.uint8)
    cls[0, :] = cls[-1, :] = cls[:, 0] = cls[:, -1] = TARGET
    return Instance(n=n, h=np.float32(h), eps=np.float32(eps), diffusion=diffusion if eps > 0 else DIFF_NONE,
                    controls=ctrl, speed=speed, node_class=cls, v_out=np.float32(0.0), drift=drift,
                    lam=np.float32(lam),
                    meta=dict(workload=f"exit {dynamics}", f_min=fmin, f_max=fmax, eta=eta, theta=theta))


def degenerate_problem(n: int, eps: float = 0.1, n_controls: int = 16, lam: float = 0.0) -> Instance:
    """Section 5.2: the eikonal-diffusion exit problem with c = 1 + chi{x_1 >= 0} and the diffusion
    coefficient eps(x) = eps chi{x_2 >= 0} (elliptic in the upper half, hyperbolic below), isotropic
    noise, g = 0 on the boundary, l = 1, h by the paper's rule."""
    x = exit_problem(n, "B2", eps=eps, n_controls=n_controls, lam=lam)
    _, X2 = node_coords(n)
    x.eps_field = np.where(X2 >= 0.0, np.float32(eps), np.float32(0.0)).astype(np.float32)
    x.meta["workload"] = "degenerate diffusion"
    return x


def general_problem(n: int, cost: int = 1, sigma: int = 1, eps: float = 0.1, n_controls: int = 16,
                    lam: float = 0.0) -> Instance:
    """Section 5.3: f = c(x) a with c = 1 + max{x_2, max{x_1, 0}} (eq. nonomog), exit from the box
    with g = 0, diffusion sigma_1 = 0, sigma_2 = d_eps(x) I, sigma_3 = d_eps(x) a with
    d_eps = sqrt(2 eps) chi{x_2 >= 0} (eq. s123), running costs l_1 = 1, l_2 = 1 + |x_1 x_2|,
    l_3 = l_2 + |a_1 / (2 + a_2)| (eq. l123). The paper does not print eps for this test; 0.1 is the
    value of its degenerate-diffusion test. h by the paper's rule with f_min = 1, f_max = 2."""
    X1, X2 = node_coords(n)
    c = (1.0 + np.maximum(X2, np.maximum(X1, 0.0))).astype(np.float32)
    ctrl = control_table(n_controls)
    dx = 2.0 / (n - 1)
    h = dx / (1.0 + 2.0)
    cls = np.zeros((n, n), dtype=np.uint8)
    cls[0, :] = cls[-1, :] = cls[:, 0] = cls[:, -1] = TARGET
    diffusion = {1: DIFF_NONE, 2: DIFF_ISO, 3: DIFF_RANK1}[sigma]
    x = Instance(n=n, h=np.float32(h), eps=np.float32(eps if sigma > 1 else 0.0), diffusion=diffusion,
                 controls=ctrl, speed=c, node_class=cls, v_out=np.float32(0.0), lam=np.float32(lam),
                 meta=dict(workload=f"general l{cost} sigma{sigma}", f_min=1.0, f_max=2.0))
    if sigma > 1:
        x.eps_field = np.where(X2 >= 0.0, np.float32(eps), np.float32(0.0)).astype(np.float32)
    if cost >= 2:
        x.running_cost_field = (1.0 + np.abs(X1 * X2)).astype(np.float32)
    if cost == 3:
        x.control_cost = np.abs(ctrl[:, 0].astype(np.float64) / (2.0 + ctrl[:, 1].astype(np.float64))).astype(np.float32)
    return x

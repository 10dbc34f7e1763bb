"""Pins of the oracle on the paper's exit-to-boundary problems (Section 5: Omega = [-1,1]^2,
g = 0 on the boundary, l = 1, 16 controls; dynamics A advection, B eikonal, C Zermelo), which
bring a drift into the feet: f(x,a) = c(x) (d(x) + a). CPU only.

The pins: the advection problem's exact discrete solution (feet on nodes) in both axis
directions, the rotation invariance of the Zermelo problem, first-order agreement of the
uncontrolled Zermelo problem with exit times integrated from the ODE, and the iteration counts
of Table 0 where the paper's text fixes them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import SL2, SL3, Problem
from paper_1502_01629_amd import instances as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table0_iterations.json")


def _paper_order(n):
    """Nodes left to right within a row, rows from the top (x2 = 1) down (Section 5.1)."""
    return np.array([j * n + i for j in range(n - 1, -1, -1) for i in range(n)], dtype=np.int32)


@pytest.mark.parametrize("scheme", [SL2, SL3])
@pytest.mark.parametrize("axis", [0, 1])
def test_advection_exact_discrete_solution(scheme, axis):
    """A: f = -b with b along one axis, h = dx: every foot is the neighbouring node upstream, so
    v_i = beta v_{i-1} + (1 - beta) and the discrete solution is v = 1 - beta^k exactly, k the
    node's distance in cells to the side the flow leaves through (x_1 = -1, or x_2 = -1 for the
    transposed field). A wrong sign of the drift, a swapped component or a dropped factor h c
    breaks this."""
    n = 17
    inst = I.exit_problem(n, "A", h=2.0 / (n - 1))
    if axis == 1:
        inst.drift = inst.drift[..., ::-1].copy()  # d = (0, -1)
        # the transposed field leaves through x2 = -1 only: keep the other sides out of reach
    p = Problem.from_instance(inst, scheme)
    v, sweeps, _, _ = p.solve(tol=1e-15, max_sweeps=10_000)
    beta = p.beta()
    V = v.reshape(n, n)
    free = inst.node_class == 0
    J, Ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    k = Ii if axis == 0 else J
    want = 1.0 - beta ** k
    assert np.abs(V[free] - want[free]).max() <= 1e-13


@pytest.mark.parametrize("eps", [0.0, 1e-2])
def test_zermelo_rotation_invariance(eps):
    """C: the box, the drift R_theta x/|x|, the speed 1/(1+|x|^2), the 16 controls and bilinear
    interpolation on the square grid are all invariant under a quarter turn, so the discrete
    solution is too (to rounding). Swapping the drift's components or its sign on one axis breaks
    the symmetry by O(1)."""
    n = 33
    inst = I.exit_problem(n, "C", eps=eps)
    p = Problem.from_instance(inst, SL3)
    v, _, _, _ = p.solve(tol=1e-13, threads=4)
    V = v.reshape(n, n)
    assert np.abs(np.rot90(V) - V).max() <= 1e-12
    assert np.abs(V.T - V).max() > 1e-2  # the rotation makes it chiral: not mirror-symmetric


def _zermelo_exit_time(x0, theta=math.pi / 4, dt=1e-3):
    """Exit time from the open square of x' = (R_theta x/|x|) / (1 + |x|^2), by classical RK4
    with a linear interpolation of the crossing inside the last step."""
    ct, st = math.cos(theta), math.sin(theta)

    def f(x):
        r = math.hypot(x[0], x[1])
        ux, uy = x[0] / r, x[1] / r
        return np.array([ct * ux - st * uy, st * ux + ct * uy]) / (1.0 + r * r)

    x = np.array(x0, dtype=float)
    t = 0.0
    while True:
        k1 = f(x)
        k2 = f(x + 0.5 * dt * k1)
        k3 = f(x + 0.5 * dt * k2)
        k4 = f(x + dt * k3)
        xn = x + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        m0, m1 = max(abs(x[0]), abs(x[1])), max(abs(xn[0]), abs(xn[1]))
        if m1 >= 1.0:
            return t + dt * (1.0 - m0) / (m1 - m0)
        x, t = xn, t + dt


def test_zermelo_uncontrolled_converges_to_ode_exit_time():
    """C with eta = 0 is pure transport along the whirling drift: T = -ln(1 - v) must approach
    the exit time of the ODE, at first order in dx. The measure is the median error over points
    at least 0.3 from the origin: the origin is a stagnation point (T = +inf there), and the
    interpolation spreads that value along the trajectories that spiral out of its neighbourhood,
    where the error decays only slowly (a few of the sampled points); elsewhere it halves with dx."""
    rng = np.random.default_rng(7)
    pts = []
    while len(pts) < 40:
        x = rng.uniform(-0.95, 0.95, size=2)
        if math.hypot(*x) >= 0.3:
            pts.append(x)
    errs = {}
    for n in (65, 129):
        inst = I.exit_problem(n, "C", eta=0.0)
        p = Problem.from_instance(inst, SL3)
        v, _, _, _ = p.solve(tol=1e-12, threads=4)
        e = []
        for (x1, x2) in pts:
            vi = p.interp(v, float(x1), float(x2))
            e.append(abs(-math.log(1.0 - vi) - _zermelo_exit_time((x1, x2))))
        errs[n] = float(np.median(e))
    assert errs[129] < 0.02
    assert errs[65] / errs[129] > 1.6


def test_table0_iteration_counts():
    """Table 0 with the paper's node order: A at eps = 0 takes one iteration plus the check
    (the text after the table), B with c = 1 at eps = 0 takes 25 + 1 (the same text; the grid's
    middle), and eq. SLscheme3 needs fewer iterations than eq. SLscheme2 in every row (by more
    than a factor 2 wherever eps = 0)."""
    g = json.load(open(GOLDEN))
    n = g["grid"]
    order = _paper_order(n)
    counts = {}
    for row in g["rows"]:
        inst = I.exit_problem(n, row["equation"], eps=row["eps"])
        got = []
        for scheme in (SL2, SL3):
            p = Problem.from_instance(inst, scheme)
            _, sweeps, _, _ = p.solve(tol=1e-6, gauss_seidel=True, order=order, threads=4)
            got.append(sweeps)
        counts[(row["equation"], row["eps"])] = got
        assert got[1] < got[0], (row, got)
        if row["eps"] == 0.0:
            assert 2 * got[1] < got[0], (row, got)
    assert counts[("A", 0.0)][1] == 2
    assert abs(counts[("B", 0.0)][1] - 26) <= 1

"""Pins of the oracle's undiscounted scheme (lambda = 0, eq. SLscheme2 exactly as Section 3 prints
it: beta = 1, rho = h l) and of the costs and diffusion that vary over the state and the control
(Sections 5.2-5.3: l(x,a) = l_x(x) + l_a(a), eps(x)). CPU only.

Each pin is fixed by something other than the oracle's own formula: exact discrete closed forms
(transport with feet on nodes: the cost collected along the characteristic), the equivalence of
eq. SLscheme2 and eq. SLscheme3, Howard's exact policy iteration, linearity of the undiscounted
value in the running cost, and reductions to the constant case and to sigma = 0. A cost taken at the foot instead of the node, a missing h,
a discount left in, or a noise offset from the wrong node fails one of them."""
import numpy as np
import pytest

from oracle import SL2, SL3, Problem, policy
from paper_1502_01629_amd import instances as I


def _transport(n=17, lam=0.0):
    x = I.transport_problem(n, 32)
    x.lam = np.float32(lam)
    x.v_out = np.float32(100.0)  # leaving the box is never cheaper than the transport
    return x


@pytest.mark.parametrize("scheme", [SL2, SL3])
def test_undiscounted_transport_collects_h_per_step(scheme):
    """Target = left column, c = 1, h = dx, sigma = 0: the control (-1, 0) moves a node exactly one
    column left, so v(i, j) = i h (l = 1, no discount)."""
    x = _transport()
    p = Problem.from_instance(x, scheme)
    assert p.beta() == 1.0 and p.rho() == float(x.h)
    v, _, _, _ = p.solve(tol=1e-15)
    i = np.arange(x.n)[None, :] + np.zeros((x.n, 1))
    assert np.abs(v.reshape(x.n, x.n) - i * float(x.h)).max() < 1e-13


@pytest.mark.parametrize("scheme", [SL2, SL3])
def test_state_dependent_cost_is_taken_at_the_node(scheme):
    """With l_x(x) = 1.5 + x_1^2 (> 0, varying along the characteristic) the transport solution is
    the cost collected at the nodes the characteristic leaves: v(i, j) = h sum_{k=1..i} l_x(x_k).
    (v then depends on the column only and grows with it, so the foot one column to the left, a
    node, is the best one: it is the fixed point.)"""
    x = _transport()
    X1, _ = I.node_coords(x.n)
    lx = (1.5 + X1 * X1).astype(np.float32)
    x.running_cost_field = lx
    p = Problem.from_instance(x, scheme)
    v, _, _, _ = p.solve(tol=1e-15)
    want = np.zeros((x.n, x.n))
    want[:, 1:] = float(x.h) * np.cumsum(lx[:, 1:].astype(np.float64), axis=1)
    assert np.abs(v.reshape(x.n, x.n) - want).max() < 1e-12


@pytest.mark.parametrize("scheme", [SL2, SL3])
def test_control_cost_of_the_optimal_control(scheme):
    """A control cost: 0.5 on the transport control (-1, 0), 3 on every other one. The transport
    control stays optimal, and every step costs h (1 + 0.5)."""
    x = _transport()
    left = int(np.flatnonzero((x.controls[:, 0] == -1.0) & (x.controls[:, 1] == 0.0))[0])
    cc = np.full(x.n_controls, 3.0, dtype=np.float32)
    cc[left] = 0.5
    x.control_cost = cc
    p = Problem.from_instance(x, scheme)
    v, _, _, _ = p.solve(tol=1e-15)
    i = np.arange(x.n)[None, :] + np.zeros((x.n, 1))
    assert np.abs(v.reshape(x.n, x.n) - 1.5 * i * float(x.h)).max() < 1e-12


@pytest.mark.parametrize("dyn", ["B", "C"])
def test_undiscounted_sl2_and_sl3_have_the_same_fixed_point(dyn):
    """The equivalence theorem of Section 3 without discount, with diffusion."""
    x = I.exit_problem(17, dyn, eps=0.01, lam=0.0)
    v2, _, _, _ = Problem.from_instance(x, SL2).solve(tol=1e-14)
    v3, _, _, _ = Problem.from_instance(x, SL3).solve(tol=1e-14)
    assert np.abs(v2 - v3).max() < 1e-11


@pytest.mark.parametrize("cost,sigma", [(1, 1), (2, 2), (3, 3), (3, 2), (2, 1)])
def test_general_problems_value_iteration_equals_policy_iteration(cost, sigma):
    """Section 5.3's dynamics, diffusions and costs on a 9 x 9 grid, undiscounted: the value
    iteration stops at the exact fixed point of Howard's policy iteration (exact linear solves)."""
    x = I.general_problem(9, cost=cost, sigma=sigma, eps=0.02)
    for scheme in (SL2, SL3):
        p = Problem.from_instance(x, scheme)
        v_vi, _, _, _ = p.solve(tol=1e-15)
        v_pi, _, _ = policy.policy_iteration(p)
        assert np.abs(v_vi - v_pi).max() < 1e-11
        v_sp, _, _ = policy.sparse_policy_iteration(p)
        assert np.abs(v_vi - v_sp).max() < 1e-11


def test_undiscounted_value_is_linear_in_the_running_cost():
    """With g = 0 on the boundary and v_out = 0, scaling l by s scales v by s (no discount; s = 2
    keeps the FP32 inputs exact)."""
    x = I.general_problem(17, cost=3, sigma=2, eps=0.05)
    v1, _, _, _ = Problem.from_instance(x, SL3).solve(tol=1e-14)
    x.running_cost_field = (2.0 * x.running_cost_field).astype(np.float32)
    x.control_cost = (2.0 * x.control_cost).astype(np.float32)
    v2, _, _, _ = Problem.from_instance(x, SL3).solve(tol=1e-14)
    assert np.abs(v2 - 2.0 * v1).max() < 1e-11


def test_constant_fields_reduce_to_the_scalar_problem():
    """l_x = 1.25 everywhere with l_a = 0.5 for every control is the constant cost 1.75, and
    eps(x) = eps everywhere is the constant coefficient (same values to rounding)."""
    x = I.exit_problem(17, "B2", eps=0.02, lam=0.0)
    ref = I.exit_problem(17, "B2", eps=0.02, lam=0.0)
    ref.running_cost = np.float32(1.75)
    x.running_cost_field = np.full((17, 17), 1.25, dtype=np.float32)
    x.control_cost = np.full(x.n_controls, 0.5, dtype=np.float32)
    x.eps_field = np.full((17, 17), np.float32(0.02), dtype=np.float32)
    a, _, _, _ = Problem.from_instance(x, SL3).solve(tol=1e-14)
    b, _, _, _ = Problem.from_instance(ref, SL3).solve(tol=1e-14)
    assert np.abs(a - b).max() < 1e-12


@pytest.mark.parametrize("diffusion", [I.DIFF_ISO, I.DIFF_RANK1])
def test_zero_diffusion_field_is_the_first_order_scheme(diffusion):
    """eps(x) = 0 everywhere: the feet of each control coincide and the scheme is the sigma = 0
    one (degenerate diffusion, Section 5.2)."""
    x = I.exit_problem(17, "B2", eps=0.05, lam=0.0, diffusion=diffusion)
    x.eps_field = np.zeros((17, 17), dtype=np.float32)
    ref = I.exit_problem(17, "B2", eps=0.0, lam=0.0)
    a, _, _, _ = Problem.from_instance(x, SL3).solve(tol=1e-14)
    b, _, _, _ = Problem.from_instance(ref, SL3).solve(tol=1e-14)
    assert np.abs(a - b).max() < 1e-12


def test_degenerate_diffusion_acts_only_where_eps_is_positive():
    """eps(x) = 0.1 chi{x_2 >= 0} (Section 5.2): far below the axis the solution is that of the
    first-order problem until the characteristics reach the diffusive half; and the diffusive
    half differs from the first-order solution."""
    n = 33
    deg = I.degenerate_problem(n, eps=0.1)
    first = I.exit_problem(n, "B2", eps=0.0, lam=0.0)
    a, _, _, _ = Problem.from_instance(deg, SL3).solve(tol=1e-13)
    b, _, _, _ = Problem.from_instance(first, SL3).solve(tol=1e-13)
    a, b = a.reshape(n, n), b.reshape(n, n)
    X1, X2 = I.node_coords(n)
    lower = X2 < -0.55  # closer to the bottom side than to the diffusive half: exit downwards
    upper = (X2 > 0.3) & (np.abs(X1) < 0.6)
    assert np.abs(a - b)[lower].max() < 1e-12
    assert np.abs(a - b)[upper].max() > 1e-3

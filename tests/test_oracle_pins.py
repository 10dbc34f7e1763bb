"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: exact discrete closed forms,
exact reproduction of polynomials, the equivalence theorem of Section 3, exact fixed points by
policy iteration and brute force, and invariants of a monotone contraction. Together they
are chosen so that a dropped term, a wrong sign or index, or a transposed operand anywhere in
the scheme fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import SL2, SL3, Problem, policy
from paper_1502_01629_amd import instances as I


def _prob(inst, scheme=SL3, **kw):
    p = Problem.from_instance(inst, scheme)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------- bilinear reconstruction
def test_interpolation_reproduces_bilinear_functions():
    """Bilinear reconstruction (Section 3, Fig. bilinear) is exact on a + b x + c y + d x y,
    including points on the upper edges where the cell index is clamped; transposed weights
    or a wrong corner fail this."""
    inst = I.disc_problem(n=9)
    p = _prob(inst)
    X1, X2 = I.node_coords(9)
    rng = np.random.default_rng(1)
    for _ in range(5):
        a, b, c, d = rng.normal(size=4)
        v = (a + b * X1 + c * X2 + d * X1 * X2).reshape(-1)
        pts = list(rng.uniform(-1, 1, size=(200, 2))) + [(1.0, 1.0), (1.0, -0.3), (0.25, 1.0), (-1.0, -1.0)]
        for (y1, y2) in pts:
            exact = a + b * y1 + c * y2 + d * y1 * y2
            assert abs(p.interp(v, y1, y2) - exact) < 1e-13
    # outside the closed box: v_out
    assert p.interp(np.zeros(81), 1.0 + 1e-12, 0.0) == p.v_out
    assert p.interp(np.zeros(81), 0.0, -1.0 - 1e-12) == p.v_out


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("scheme", [SL2, SL3])
@pytest.mark.parametrize("n_controls", [8, 32, 64])
def test_transport_closed_form(scheme, n_controls):
    """Target = left column, c = 1, h = dx, sigma = 0: the left control lands on node i-1 and the
    interpolant of an increasing function of x1 is minimal there, so v(i,j) = 1 - beta^i exactly
    (Problem A of Section 5 in Kruzkov form)."""
    inst = I.transport_problem(17, n_controls)
    p = _prob(inst, scheme)
    v, sweeps, r, _ = p.solve(tol=1e-15)
    exact = 1.0 - p.beta() ** np.arange(17)
    assert np.abs(v.reshape(17, 17) - exact[None, :]).max() < 1e-14


@pytest.mark.parametrize("scheme", [SL2, SL3])
def test_rank1_random_walk_closed_form(scheme):
    """One control (-1,0), rank-1 noise along it with sqrt(2 eps h) = dx: the feet are nodes i-2 and i,
    so w_i = beta w_{i-2} / (2 - beta) and v = 1 - (beta/(2-beta))^floor(i/2)."""
    inst = I.rank1_walk_problem(9)
    p = _prob(inst, scheme)
    v, sweeps, r, _ = p.solve(tol=1e-15)
    b = p.beta()
    exact = 1.0 - (b / (2.0 - b)) ** (np.arange(9) // 2)
    assert np.abs(v.reshape(9, 9) - exact[None, :]).max() < 1e-14


def test_rank1_self_dependency_removal_cuts_sweeps():
    """The self-dependency removal of eq. SLscheme3 needs far fewer Jacobi sweeps than eq. SLscheme2
    on the same problem (the qualitative claim of Table 0)."""
    inst = I.rank1_walk_problem(9)
    _, s2, _, _ = _prob(inst, SL2).solve(tol=1e-13)
    _, s3, _, _ = _prob(inst, SL3).solve(tol=1e-13)
    assert s3 <= 6 and s2 > 5 * s3


def test_transport_single_pass_gauss_seidel():
    """Problem A at eps = 0 with feet between nodes (h = dx/2): processed left to right, the modified
    scheme is exact after one pass, so it stops after 2 passes (one plus the check, Table 0 row 1);
    the original scheme keeps the self-dependency and needs many more."""
    n = 17
    inst = I.transport_problem(n, 32, scheme_h_factor=0.5)
    order = np.arange(n * n, dtype=np.int32)  # row-major: i fastest = left to right
    _, s3, _, _ = _prob(inst, SL3).solve(tol=1e-14, gauss_seidel=True, order=order)
    _, s2, _, _ = _prob(inst, SL2).solve(tol=1e-14, gauss_seidel=True, order=order)
    assert s3 == 2
    assert s2 > 10


def test_iso_one_step_moments():
    """With control (-1,0), c = 1, h = dx and sqrt(2 eps h) = dx the four isotropic feet land on the nodes
    (i-2,j), (i,j), (i-1,j+-1), so one step of the chain has mean displacement (-dx, 0) and second
    moments E[dX1^2] = 1.5 dx^2, E[dX2^2] = 0.5 dx^2, E[dX1 dX2] = 0 (sigma = sqrt(2 eps) I of
    Section 4.1). Checked on nodal polynomials, which interpolation reproduces at nodes."""
    n = 9
    dx = 2.0 / (n - 1)
    inst = I.Instance(n=n, h=np.float32(dx), eps=np.float32(dx / 2), diffusion=I.DIFF_ISO,
                      controls=np.array([[-1.0, 0.0]], dtype=np.float32),
                      speed=np.ones((n, n), dtype=np.float32), node_class=np.zeros((n, n), dtype=np.uint8))
    p = _prob(inst)
    X1, X2 = I.node_coords(n)
    i, j = 4, 4
    node = j * n + i
    x1, x2 = X1[j, i], X2[j, i]
    for fn, expect in [
        (X1, x1 - dx),
        (X2, x2),
        ((X1 - x1) ** 2, 1.5 * dx * dx),
        ((X2 - x2) ** 2, 0.5 * dx * dx),
        ((X1 - x1) * (X2 - x2), 0.0),
    ]:
        assert abs(p.one_step_mean(fn.reshape(-1), node, 0) - expect) < 1e-14


# ---------------------------------------------------------------- equivalence theorem
@pytest.mark.parametrize("diff,eps", [(I.DIFF_NONE, 0.0), (I.DIFF_ISO, 0.01), (I.DIFF_RANK1, 0.005)])
def test_sl2_and_sl3_share_the_fixed_point(diff, eps):
    """Section 3 proves that the explicit form (eq. SLexplicit / SLscheme3) has the same solution as
    the implicit one (eq. SLimplicit): a wrong Lambda0 or Lambda1 moves the SL3 fixed point."""
    inst = I.disc_problem(n=33, eps=eps, n_controls=16, diffusion=diff)
    rng = np.random.default_rng(3)
    inst.speed = (0.6 + 0.8 * rng.random((33, 33))).astype(np.float32)
    v2, _, _, _ = _prob(inst, SL2).solve(tol=1e-14, threads=4)
    v3, _, _, _ = _prob(inst, SL3).solve(tol=1e-14, threads=4)
    assert np.abs(v2 - v3).max() < 1e-12


# ---------------------------------------------------------------- exact fixed points
@pytest.mark.parametrize("diff,eps", [(I.DIFF_NONE, 0.0), (I.DIFF_ISO, 0.02), (I.DIFF_RANK1, 0.02)])
def test_value_iteration_matches_policy_iteration(diff, eps):
    """Howard's policy iteration (exact linear solves) gives the exact fixed point on a tiny grid."""
    n = 9
    inst = I.disc_problem(n=n, eps=eps, n_controls=8, diffusion=diff)
    inst.node_class[:] = 0
    inst.node_class[4, 4] = I.TARGET
    inst.node_class[1, 6] = I.OBSTACLE
    rng = np.random.default_rng(7)
    inst.speed = (0.5 + rng.random((n, n))).astype(np.float32)
    for scheme in (SL2, SL3):
        p = _prob(inst, scheme)
        v_vi, _, _, _ = p.solve(tol=1e-15)
        v_pi, _, _ = policy.policy_iteration(p)
        assert np.abs(v_vi - v_pi).max() < 1e-12


@pytest.mark.parametrize("diff,eps", [(I.DIFF_NONE, 0.0), (I.DIFF_ISO, 0.02), (I.DIFF_RANK1, 0.02)])
def test_sparse_policy_iteration_matches_dense_and_value_iteration(diff, eps):
    """The sparse Howard iteration (used to write the stored fixed points of the larger parity
    cases) equals the dense one on a tiny grid and value iteration on a 33^2 grid with obstacles."""
    n = 9
    inst = I.disc_problem(n=n, eps=eps, n_controls=8, diffusion=diff)
    inst.node_class[:] = 0
    inst.node_class[4, 4] = I.TARGET
    inst.node_class[1, 6] = I.OBSTACLE
    rng = np.random.default_rng(7)
    inst.speed = (0.5 + rng.random((n, n))).astype(np.float32)
    p = _prob(inst, SL3)
    v_d, _, _ = policy.policy_iteration(p)
    v_s, _, _ = policy.sparse_policy_iteration(p)
    assert np.abs(v_d - v_s).max() < 1e-13
    inst = I.scattered_problem(2, n=33, n_coarse=9, eps=eps * 4, n_controls=16)[0]
    inst.diffusion = diff
    p = _prob(inst, SL3)
    v_s, _, _ = policy.sparse_policy_iteration(p, threads=4)
    v_vi, _, _, _ = p.solve(tol=1e-15, threads=4)
    assert np.abs(v_vi - v_s).max() < 1e-12


def test_value_iteration_matches_brute_force():
    """A 3x3 block with one target node inside (8 free nodes), 4 controls: the optimal value is the
    componentwise minimum over all 4^8 deterministic policies."""
    n = 5
    inst = I.disc_problem(n=n, eps=0.03, n_controls=4, diffusion=I.DIFF_ISO)
    cls = np.full((n, n), I.OBSTACLE, dtype=np.uint8)
    cls[1:4, 1:4] = I.FREE
    cls[2, 0] = I.TARGET
    cls[2, 1] = I.TARGET
    cls[2, 2] = I.FREE
    cls[0, 2] = I.TARGET
    inst.node_class = cls
    p = _prob(inst, SL2)
    v_bf = policy.brute_force(p)
    v_vi, _, _, _ = p.solve(tol=1e-15)
    assert np.abs(v_vi - v_bf).max() < 1e-12
    v_vi3, _, _, _ = _prob(inst, SL3).solve(tol=1e-15)
    assert np.abs(v_vi3 - v_bf).max() < 1e-12


def test_a_posteriori_bound():
    """For the SL2 contraction with modulus beta: |v^k - v*| <= beta/(1-beta) r_k at every sweep."""
    n = 9
    inst = I.disc_problem(n=n, eps=0.02, n_controls=8)
    p = _prob(inst, SL2)
    v_star, _, _ = policy.policy_iteration(p)
    v = p.initial()
    b = p.beta()
    for _ in range(60):
        v, r = p.sweep(v)
        assert np.abs(v - v_star).max() <= b / (1 - b) * r * (1 + 1e-9) + 1e-15


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("scheme", [SL2, SL3])
@pytest.mark.parametrize("eps", [0.0, 0.01])
def test_monotone_contraction_and_bounds(scheme, eps):
    """From v = 1 the iterates are non-increasing (T is monotone and T(1) <= 1), stay in [0,1], and the
    sup-norm change contracts at least by beta per sweep."""
    inst = I.disc_problem(n=33, eps=eps, n_controls=16)
    p = _prob(inst, scheme)
    v = p.initial()
    b = p.beta()
    r_prev = None
    for _ in range(80):
        v_new, r = p.sweep(v, threads=4)
        assert (v_new <= v + 1e-15).all()
        assert v_new.min() >= -1e-15 and v_new.max() <= 1 + 1e-15
        if r_prev is not None and r_prev > 1e-13:
            assert r <= b * r_prev * (1 + 1e-9) + 1e-15
        r_prev = r
        v = v_new


@pytest.mark.parametrize("eps", [0.0, 0.01])
def test_d4_symmetry(eps):
    """The disc problem with a table closed under the square's symmetries is itself symmetric."""
    n = 33
    inst = I.disc_problem(n=n, eps=eps, n_controls=32)
    v, _, _, _ = _prob(inst).solve(tol=1e-14, threads=4)
    V = v.reshape(n, n)
    for W in (V.T, V[::-1, :], V[:, ::-1], np.rot90(V)):
        assert np.abs(V - W).max() < 1e-13


def test_fixed_point_independent_of_order_and_start():
    n = 17
    inst = I.disc_problem(n=n, eps=0.01, n_controls=16)
    p = _prob(inst)
    v_j, _, _, _ = p.solve(tol=1e-15)
    v_gs, _, _, _ = p.solve(tol=1e-15, gauss_seidel=True)
    rev = np.arange(n * n, dtype=np.int32)[::-1].copy()
    v_gr, _, _, _ = p.solve(tol=1e-15, gauss_seidel=True, order=rev)
    v_z, _, _, _ = p.solve(v0=p.initial(0.0), tol=1e-15)
    for w in (v_gs, v_gr, v_z):
        assert np.abs(v_j - w).max() < 1e-13


def test_continuum_limit_eps0():
    """At eps = 0 the Kruzkov value of the disc problem is 1 - exp(-max(|x| - 0.1, 0)); the scheme is
    consistent of order O(h) (Section 3), so away from the target (whose node set differs from the
    disc by up to one cell) the max error must shrink at an observed order above 1/2."""
    errs, sizes = [], (33, 65, 129, 257)
    for n in sizes:
        inst = I.disc_problem(n=n, eps=0.0, n_controls=64)
        v, _, _, _ = _prob(inst).solve(tol=1e-12, threads=8)
        X1, X2 = I.node_coords(n)
        r = np.hypot(X1, X2)
        exact = 1.0 - np.exp(-np.maximum(r - 0.1, 0.0))
        away = (r > 0.3) & (r < 0.9)
        errs.append(np.abs(v.reshape(n, n) - exact)[away].max())
    assert errs[0] > errs[-1]
    slope = -np.polyfit(np.log(sizes), np.log(errs), 1)[0]
    assert slope > 0.5


# ---------------------------------------------------------------- synthesis / upsampling
def test_synthesis_on_transport_picks_the_left_control():
    inst = I.transport_problem(17, 32)
    p = _prob(inst)
    v, _, _, _ = p.solve(tol=1e-15)
    ctrl, gap = p.synthesize(v)
    left = int(np.flatnonzero((inst.controls[:, 0] == -1.0) & (inst.controls[:, 1] == 0.0))[0])
    free = inst.node_class.reshape(-1) == I.FREE
    assert (ctrl[free] == left).all()
    assert (ctrl[~free] == -1).all()


@pytest.mark.parametrize("axis", [0, 1])
def test_synthesis_ties_go_to_the_first_minimum(axis):
    """With u_hat = |x_2| (resp. |x_1|), piecewise linear with its kink on a grid line, bilinear
    reconstruction is exact: at a FREE node on the kink the controls along the line, a = (1, 0) and
    (-1, 0) (resp. (0, 1) and (0, -1)), both give exactly 0 and every other control more. The
    lower index must win: 0 (resp. N/4), never N/2 (resp. 3N/4); the gap to the second best is 0."""
    n, N = 17, 32
    inst = I.transport_problem(n, N)
    inst.node_class[:] = I.FREE
    p = _prob(inst)
    X1, X2 = I.node_coords(n)
    v = np.abs(X2 if axis == 0 else X1).astype(np.float64)
    ctrl, gap = p.synthesize(v)
    mid = n // 2
    nodes = [mid * n + i for i in range(2, n - 2)] if axis == 0 else [j * n + mid for j in range(2, n - 2)]
    assert np.array_equal(inst.controls[0], [1.0, 0.0]) and np.array_equal(inst.controls[N // 4], [0.0, 1.0])
    want = 0 if axis == 0 else N // 4
    assert (ctrl[nodes] == want).all(), ctrl[nodes]
    assert (gap[nodes] == 0.0).all()


def test_upsample_reproduces_bilinear_and_coarse_nodes():
    rng = np.random.default_rng(5)
    a, b, c, d = rng.normal(size=4)
    Xc1, Xc2 = I.node_coords(9)
    vc = a + b * Xc1 + c * Xc2 + d * Xc1 * Xc2
    vf = oracle.upsample_bilinear(vc, 33).reshape(33, 33)
    Xf1, Xf2 = I.node_coords(33)
    assert np.abs(vf - (a + b * Xf1 + c * Xf2 + d * Xf1 * Xf2)).max() < 1e-13
    vr = rng.random((9, 9))
    vf = oracle.upsample_bilinear(vr, 33).reshape(33, 33)
    assert np.array_equal(vf[::4, ::4], vr)


def test_bicubic_upsample_pins():
    """Keys' kernel with a = -1/2: (1) interpolates (coarse nodes copied exactly); (2) its weights
    sum to 1, so constants are exact everywhere, edges included; (3) it reproduces quadratics
    exactly wherever the 4 x 4 stencil lies inside the grid (third-order accuracy, Keys 1981);
    (4) at t = 1/2 the 1-D weights are (-1/16, 9/16, 9/16, -1/16)."""
    rng = np.random.default_rng(11)
    vr = rng.random((9, 9))
    vf = oracle.upsample_bicubic(vr, 33).reshape(33, 33)
    assert np.array_equal(vf[::4, ::4], vr)
    c = oracle.upsample_bicubic(np.full((9, 9), 0.37), 33)
    assert np.abs(c - 0.37).max() < 1e-15
    Xc1, Xc2 = I.node_coords(9)
    a, b, cc, d, e, f = rng.normal(size=6)
    quad = lambda x, y: a + b * x + cc * y + d * x * x + e * x * y + f * y * y
    vf = oracle.upsample_bicubic(quad(Xc1, Xc2), 33).reshape(33, 33)
    Xf1, Xf2 = I.node_coords(33)
    inner = (slice(4, 29), slice(4, 29))  # fine nodes whose stencil stays inside coarse 0..8
    assert np.abs(vf[inner] - quad(Xf1, Xf2)[inner]).max() < 1e-12
    # half-way between coarse columns the 1-D weights of columns c-1, c, c+1, c+2 are
    # -1/16, 9/16, 9/16, -1/16: a single column of ones on a 3 x 3 grid gives 9/16 on both sides
    row = np.zeros((3, 3))
    row[:, 1] = 1.0
    vf = oracle.upsample_bicubic(row, 5).reshape(5, 5)
    assert np.array_equal(vf[0], [0.0, 9 / 16, 1.0, 9 / 16, 0.0])
    # ones in column 0: at x = 1/2 the clamped column -1 is column 0 again: 9/16 - 1/16
    row = np.zeros((3, 3))
    row[:, 0] = 1.0
    vf = oracle.upsample_bicubic(row, 5).reshape(5, 5)
    assert np.allclose(vf[0], [1.0, 8 / 16, 0.0, -1 / 16, 0.0], atol=1e-15)


# ---------------------------------------------------------------- independent (state-constraint) sweep
@pytest.mark.parametrize("scheme", [SL2, SL3])
@pytest.mark.parametrize("eps", [0.0, 0.02])
def test_independent_sweep_reduces_to_the_global_sweep_with_one_patch(scheme, eps):
    """With every node in one patch there is no interface: the per-patch sweep is the global one."""
    inst = I.disc_problem(33, eps)
    p = _prob(inst, scheme)
    rng = np.random.default_rng(7)
    v = p.initial()
    v[inst.node_class.reshape(-1) == I.FREE] = rng.uniform(0.2, 1.0, size=int((inst.node_class == I.FREE).sum()))
    a, ra = p.sweep(v)
    b, rb = p.sweep_independent(np.zeros(33 * 33, dtype=np.int16), v)
    assert np.array_equal(a, b) and ra == rb


@pytest.mark.parametrize("scheme", [SL2, SL3])
def test_independent_sweep_is_a_state_constraint(scheme):
    """Reading v_out (the largest value) at other-patch corners can only raise a monotone update, and
    a node whose feet never leave its patch's cells gets exactly the global update."""
    inst = I.disc_problem(33, 0.02)
    p = _prob(inst, scheme)
    n = 33
    v = p.initial()
    rng = np.random.default_rng(3)
    free = inst.node_class.reshape(-1) == I.FREE
    v[free] = rng.uniform(0.2, 0.9, size=int(free.sum()))
    lab = (np.arange(n)[None, :] // 11 + np.zeros((n, 1), dtype=np.int64)).astype(np.int16).reshape(-1)
    g, _ = p.sweep(v)
    s, _ = p.sweep_independent(lab, v)
    assert (s >= g - 1e-15).all()
    # the reach of every foot is below 2 cells here: nodes at least 3 columns from an interface
    col = np.arange(n * n) % n
    far = np.minimum(np.abs(col - 10.5), np.abs(col - 21.5)) >= 3
    assert np.array_equal(s[far & free], g[far & free])
    near = (~far) & free
    assert (s[near] > g[near]).any()

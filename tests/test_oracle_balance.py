"""Pins of the balanced-patch rounds (oracle/balance.py): the exact angular order against atan2,
the starting subdivision against its restatement in tests/test_capi_cpu.py, the invariants of a
round (sources only, runs contiguous in angular order, every component keeps a patch), the
equal-weight property of the runs, and that the rounds reduce the imbalance of an unbalanced
decomposition."""
import math

import numpy as np
import pytest

import oracle
from oracle import balance as B
from paper_1502_01629_amd import instances as I


def radial_field(n, centres, controls):
    """Control index pointing from each node toward its nearest centre (an input field)."""
    X1, X2 = I.node_coords(n)
    best = np.full((n, n), np.inf)
    ctrl = np.zeros((n, n), dtype=np.int32)
    N = controls.shape[0]
    for (cx, cy, _r) in centres:
        d = np.hypot(X1 - cx, X2 - cy)
        th = np.arctan2(cy - X2, cx - X1) % (2 * np.pi)
        m = np.round(th / (2 * np.pi) * N).astype(np.int32) % N
        ctrl = np.where(d < best, m, ctrl)
        best = np.minimum(best, d)
    return ctrl


def _case(n=129, seed=0):
    fine, _ = I.scattered_problem(seed, n=n, n_coarse=33)
    ctrl = radial_field(n, fine.meta["geometry"].targets, fine.controls)
    ctrl = np.where(fine.node_class == I.FREE, ctrl, -1).astype(np.int32)
    disp = oracle.displacement(n, float(fine.x_lo), float(fine.x_hi), float(fine.h), fine.speed, fine.controls, ctrl)
    return fine, ctrl, disp


def test_angular_order_is_the_atan2_order():
    rng = np.random.default_rng(0)
    n = 4096
    for _ in range(20):
        pts = rng.choice(n * n, size=200, replace=False)
        cnt, si, sj = 7, int(rng.integers(0, 7 * n)), int(rng.integers(0, 7 * n))
        got = B.angular_order([int(p) for p in pts], n, cnt, si, sj)
        ang = {int(p): math.atan2((p // n) * cnt - sj, (p % n) * cnt - si) for p in pts}
        # without collinear pairs the float angles are distinct and order the points the same way
        vals = sorted(ang.values())
        if len(set(vals)) < len(vals) or min(np.diff(vals)) < 1e-12:
            continue
        assert got == sorted(ang, key=ang.get)


def test_angular_order_ties_and_axes():
    # centroid (0, 0) of a 5 x 5 grid (n = 5, cnt = 1): points on the negative x axis come last
    # (angle pi), the positive x axis and the centroid at angle 0, collinear points by index
    n = 5
    left, right, up, down, centre = 0 * n + 0, 0 * n + 4, 4 * n + 0, 0, 0
    pts = [2 * n + 2, 2 * n + 4, 4 * n + 4, 4 * n + 2, 2 * n + 0, 0 * n + 2, 0 * n + 4, 0 * n + 0, 3 * n + 3, 4 * n + 4]
    got = B.angular_order(sorted(set(pts)), n, 1, 2, 2)
    ang = {p: math.atan2(p // n - 2, p % n - 2) for p in set(pts)}
    want = sorted(set(pts), key=lambda p: (ang[p], p))
    assert got == want


@pytest.mark.parametrize("seed", [0, 1])
def test_starting_subdivision_matches_its_restatement(seed):
    from test_capi_cpu import _partition_reference

    fine, _ = I.scattered_problem(seed, n=257)
    for P in (3, 16, 64):
        assert np.array_equal(B.partition_sources(fine.node_class, P), _partition_reference(fine.node_class, P))


def test_round_invariants_and_equal_weight_runs():
    fine, ctrl, disp = _case(129, 0)
    n, P = fine.n, 16
    src = B.partition_sources(fine.node_class, P).reshape(-1)
    lab, _, _ = oracle.label(n, fine.node_class, disp, src, P)
    new = B.rebalance(fine.node_class, src, lab, P).reshape(-1)
    tgt = fine.node_class.reshape(-1) == I.TARGET
    assert (new[~tgt] == -1).all() and (new[tgt] >= 0).all() and (new[tgt] < P).all()
    comp, cnt, si, sj = B.components(fine.node_class)
    sizes = np.bincount(lab[lab >= 0].astype(np.int64), minlength=P)
    members = np.bincount(src[src >= 0].astype(np.int64), minlength=P)
    used = 0
    for t in range(len(cnt)):
        nodes = B.angular_order([int(v) for v in np.nonzero(comp == t)[0]], n, cnt[t], si[t], sj[t])
        runs = [int(new[v]) for v in nodes]
        assert runs == sorted(runs), "runs are contiguous in angular order"
        ks = sorted(set(runs))
        used += ks[-1] - ks[0] + 1 if ks else 0
        w = np.array([sizes[src[v]] / members[src[v]] for v in nodes])
        wt, wmax = w.sum(), w.max()
        Pt = len(set(runs)) if wt == 0 else None
        lo = min(runs)
        hi = max(runs)
        for k in range(lo, hi + 1):
            wk = w[np.array(runs) == k].sum()
            assert abs(wk - wt / (hi - lo + 1)) <= wmax + 1e-9 * wt
    assert used <= P


def _offcenter(n):
    x = I.offcenter_problem(n)
    ctrl = radial_field(n, x.meta["geometry"].targets, x.controls)
    ctrl = np.where(x.node_class == I.FREE, ctrl, -1).astype(np.int32)
    disp = oracle.displacement(n, float(x.x_lo), float(x.x_hi), float(x.h), x.speed, x.controls, ctrl)
    return x, disp


@pytest.mark.parametrize("n,P", [(129, 8), (129, 16)])
def test_rounds_reduce_the_imbalance(n, P):
    """An off-centre target: equal angular sectors give patches more than twice the mean size; the
    first round already shrinks the largest patch relative to the mean by more than 10%, and the
    kept subdivision is the best visited."""
    x, disp = _offcenter(n)
    src0 = B.partition_sources(x.node_class, P)
    src, sizes, lab, k = B.balance_sources(n, x.node_class, disp, src0, P, 3)
    ratios = [B.imbalance(s) for s in sizes]
    print("imbalance", [round(r, 3) for r in ratios], "kept", k, flush=True)
    assert ratios[0] > 2.0 and ratios[1] < 0.9 * ratios[0]
    assert ratios[k] == min(ratios) and k == ratios.index(min(ratios))
    assert sizes.sum(axis=1).min() == sizes.sum(axis=1).max()  # the same nodes are labelled
    lab2, _, _ = oracle.label(n, x.node_class, disp, src, P)
    assert np.array_equal(lab2, lab)


def test_balanced_start_is_kept():
    """A subdivision no round improves on comes back unchanged (round 0 kept)."""
    x, disp = _offcenter(129)
    P = 4
    src0 = B.partition_sources(x.node_class, P)
    src, sizes, lab, k = B.balance_sources(129, x.node_class, disp, src0, P, 0)
    assert k == 0 and np.array_equal(src, src0.reshape(-1)) and sizes.shape == (1, P)

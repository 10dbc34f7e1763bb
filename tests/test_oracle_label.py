"""Pins of the oracle's integer patch labeler (CPU only).

The labeler is the fixed-point form of the discrete advection of Section 4.3
(eq. discrete-advection) followed by the argmax that turns the fuzzy indicators into patches.
"""
import numpy as np

import oracle
from paper_1502_01629_amd import instances as I

ONE = 1 << 15


def test_exact_shift_copies_sources():
    """Every free node's foot is exactly one cell to the left (D = (-256, 0)): the advection copies
    the indicator unchanged along rows, so each row takes the patch of its source node."""
    n, P = 17, 5
    cls = np.zeros((n, n), dtype=np.uint8)
    cls[:, 0] = I.TARGET
    src = np.full((n, n), -1, dtype=np.int16)
    src[:, 0] = np.arange(n) // 4
    disp = np.zeros((n * n, 2), dtype=np.int32)
    disp[:, 0] = -256
    lab, phi, passes = oracle.label(n, cls, disp, src, P)
    lab = lab.reshape(n, n)
    for j in range(n):
        assert (lab[j] == j // 4).all()
    phi = phi.reshape(n, n, P)
    assert (phi[:, 1:, :].sum(axis=2) == ONE).all()
    assert passes == n  # one column per pass, plus the pass that changes nothing


def _random_case(seed, n=33, P=6):
    rng = np.random.default_rng(seed)
    cls = np.zeros((n, n), dtype=np.uint8)
    cls[n // 2 - 1: n // 2 + 2, n // 2 - 1: n // 2 + 2] = I.TARGET
    cls[rng.random((n, n)) < 0.05] = I.OBSTACLE
    src = np.full((n, n), -1, dtype=np.int16)
    t = np.argwhere(cls == I.TARGET)
    src[t[:, 0], t[:, 1]] = rng.integers(0, P, size=len(t))
    disp = rng.integers(-400, 400, size=(n * n, 2)).astype(np.int32)
    return n, P, cls, src, disp


def test_label_is_independent_of_update_order():
    """The map is monotone and the start is below its image, so Jacobi, in-place and reversed in-place
    orders all climb to the same least fixed point: identical bits."""
    for seed in range(3):
        n, P, cls, src, disp = _random_case(seed)
        ref_lab, ref_phi, _ = oracle.label(n, cls, disp, src, P, order_mode=0)
        for mode in (1, 2):
            lab, phi, _ = oracle.label(n, cls, disp, src, P, order_mode=mode)
            assert np.array_equal(lab, ref_lab)
            assert np.array_equal(phi, ref_phi)


def test_radial_field_gives_angular_sectors():
    """c = 1, one disc target at the origin, every node steered straight at the origin: the patches
    grown from P equal angular sectors of the target are the same sectors of the plane, away from a
    band around the sector rays where interpolation smears the indicators."""
    n, P = 97, 8
    X1, X2 = I.node_coords(n)
    r = np.hypot(X1, X2)
    cls = np.where(r <= 0.1, I.TARGET, I.FREE).astype(np.uint8)
    ang = np.arctan2(X2, X1)
    sector = np.minimum((P * (ang + np.pi) / (2 * np.pi)).astype(np.int64), P - 1)
    src = np.where(cls == I.TARGET, sector, -1).astype(np.int16)
    controls = I.control_table(256)
    # control closest to the direction towards the origin
    th = np.arctan2(-X2, -X1)
    ctrl = np.round((th % (2 * np.pi)) / (2 * np.pi) * 256).astype(np.int32) % 256
    ctrl[cls != I.FREE] = -1
    dx = 2.0 / (n - 1)
    disp = oracle.displacement(n, -1.0, 1.0, dx, np.ones((n, n), np.float32), controls, ctrl)
    lab, phi, _ = oracle.label(n, cls, disp, src, P)
    lab = lab.reshape(n, n)
    # angular distance to the nearest sector boundary, in radians
    bound = (ang + np.pi) % (2 * np.pi / P)
    dist = np.minimum(bound, 2 * np.pi / P - bound) * r
    away = (cls == I.FREE) & (dist > 0.15) & (r < 0.95)
    assert away.sum() > 1000
    assert (lab[away] == sector[away]).mean() > 0.99
    tot = phi.reshape(n, n, P).sum(axis=2)
    reach = (cls == I.FREE) & (r < 0.9)
    assert np.abs(tot[reach].astype(np.int64) - ONE).max() <= 4 * P


def test_displacement_rounding_is_half_even_in_float():
    """D = round_half_even(256 fl(fl(fl(h/dx) c) a)): a foot of exactly half a 1/256 cell rounds to even."""
    n = 3
    ctrl = np.zeros(n * n, dtype=np.int32)
    controls = np.array([[1.0, -1.0]], dtype=np.float32)
    speed = np.full((n, n), 1.0 / 512.0 * 3, dtype=np.float32)  # k a = 3/512 -> 256 k a = 1.5 -> 2
    d = oracle.displacement(n, -1.0, 1.0, 1.0, speed, controls, ctrl)
    assert (d[:, 0] == 2).all() and (d[:, 1] == -2).all()
    speed = np.full((n, n), 1.0 / 512.0 * 5, dtype=np.float32)  # 2.5 -> 2
    d = oracle.displacement(n, -1.0, 1.0, 1.0, speed, controls, ctrl)
    assert (d[:, 0] == 2).all() and (d[:, 1] == -2).all()

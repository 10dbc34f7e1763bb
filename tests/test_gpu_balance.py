"""Balanced patches on the GPU (slhjb_balance_sources): the labels of every round come from the
library's labeler and the re-division runs on the host; the subdivision kept, the patch sizes of
every round, the labels and the kept round equal those of oracle/balance.py bit for bit."""
import numpy as np
import pytest

import oracle
from oracle import balance as B
from paper_1502_01629_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_1502_01629_amd import capi

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = capi.Context(0)
    yield c
    c.close()


def _dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt).reshape(-1)).cuda()


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


@pytest.mark.parametrize("case,n,P,rounds", [("offcenter", 129, 8, 3), ("offcenter", 257, 16, 3),
                                             ("scattered", 257, 16, 2)])
def test_balance_matches_oracle(ctx, case, n, P, rounds):
    from paper_1502_01629_amd import capi

    x = I.offcenter_problem(n) if case == "offcenter" else I.scattered_problem(0, n=n, n_coarse=33)[0]
    ctrl = radial_field(n, x.meta["geometry"].targets, x.controls)
    ctrl = np.where(x.node_class == I.FREE, ctrl, -1).astype(np.int32)
    print(f"balance {case} n={n} P={P} rounds={rounds}", flush=True)
    src0, _ = capi.partition_sources(x.node_class, P)
    dp = capi.DeviceProblem(x, capi.SL3)
    src = _dev(src0, np.int16)
    lab = torch.empty(n * n, dtype=torch.int16, device="cuda")
    sizes, best = ctx.balance_sources(dp, _dev(ctrl, np.int16), src, P, rounds, label_out=lab)
    disp = oracle.displacement(n, float(x.x_lo), float(x.x_hi), float(x.h), x.speed, x.controls, ctrl)
    ref_src, ref_sizes, ref_lab, ref_best = B.balance_sources(n, x.node_class, disp,
                                                              B.partition_sources(x.node_class, P), P, rounds)
    print("imbalance", [round(B.imbalance(s), 3) for s in sizes], "kept", best, flush=True)
    assert np.array_equal(sizes, ref_sizes)
    assert best == ref_best
    assert np.array_equal(src.cpu().numpy(), ref_src)
    assert np.array_equal(lab.cpu().numpy(), ref_lab)
    assert B.imbalance(sizes[best]) <= B.imbalance(sizes[0])


def test_balance_rejects_a_bad_start(ctx):
    from paper_1502_01629_amd import capi

    x = I.offcenter_problem(65)
    src0, _ = capi.partition_sources(x.node_class, 4)
    src0 = src0.reshape(-1).copy()
    src0[np.nonzero(x.node_class.reshape(-1) == I.TARGET)[0][0]] = -1  # a source without a patch
    dp = capi.DeviceProblem(x, capi.SL3)
    ctrl = np.where(x.node_class == I.FREE, 0, -1)
    with pytest.raises(capi.SlhjbError):
        ctx.balance_sources(dp, _dev(ctrl, np.int16), _dev(src0, np.int16), 4, 1)

"""The patchy method end to end on the GPU (Section 4.3) against the oracle: the transmission
and static decompositions reach the global fixed point, the patch labels of the GPU pipeline agree
with the oracle's own pipeline, and the independent (state-constraint) mode is measured."""
import numpy as np
import pytest

import oracle
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


@pytest.fixture(scope="module")
def case():
    fine, coarse = I.scattered_problem(4, n=257, n_coarse=65)
    ref, sweeps, _, _ = oracle.Problem.from_instance(fine, 1).solve(tol=1e-10, threads=8)
    return fine, coarse, ref


def _dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype).reshape(-1)).cuda()


@pytest.mark.parametrize("mode", [0, 2])
def test_patchy_transmission_and_static_reach_the_global_solution(ctx, case, mode):
    from paper_1502_01629_amd import capi

    fine, coarse, ref = case
    v = torch.empty(fine.n * fine.n, dtype=torch.float32, device="cuda")
    st = ctx.solve_patchy(capi.DeviceProblem(fine, 1), capi.DeviceProblem(coarse, 1), v, mode=mode, tol=5e-7)
    print(mode, st, flush=True)
    assert st["status"] == 0 and st["residual"] <= 5e-7
    err = np.abs(v.cpu().numpy().astype(np.float64) - ref).max()
    print("max abs err", err, flush=True)
    assert err < 1e-5


def test_patchy_labels_agree_with_the_oracle_pipeline(ctx, case):
    """The oracle runs its own coarse solve, u_hat, synthesis and integer labeling; the GPU pipeline's
    labels must agree except where the synthesized control is a near-tie in FP32."""
    from paper_1502_01629_amd import capi

    fine, coarse, _ = case
    P = 16
    src, _ = capi.partition_sources(fine.node_class, P)
    v = torch.empty(fine.n * fine.n, dtype=torch.float32, device="cuda")
    lab = torch.empty(fine.n * fine.n, dtype=torch.int16, device="cuda")
    st = ctx.solve_patchy(capi.DeviceProblem(fine, 1), capi.DeviceProblem(coarse, 1), v, mode=0, tol=5e-7,
                          source_patch=_dev(src, np.int16), n_patches=P, label_out=lab)
    assert st["status"] == 0
    vc, _, _, _ = oracle.Problem.from_instance(coarse, 1).solve(tol=1e-10, threads=8)
    vhat = oracle.upsample_bilinear(vc, fine.n)
    ctrl, gap = oracle.Problem.from_instance(fine, 1).synthesize(vhat)
    disp = oracle.displacement(fine.n, -1.0, 1.0, float(fine.h), fine.speed, fine.controls, ctrl)
    ref_lab, _, _ = oracle.label(fine.n, fine.node_class, disp, src, P)
    got = lab.cpu().numpy()
    agree = (got == ref_lab).mean()
    print("label agreement", agree, flush=True)
    assert agree > 0.99


def test_patchy_independent_mode_error_is_measured(ctx, case):
    """State constraints at the interfaces of the dynamic patches: every patch reads the others as v_out
    (the largest value), so the operator and its fixed point can only lie above the global ones; the
    decomposition error is a number of its own (the paper prints none) and is concentrated at the
    interfaces (Section 2)."""
    from paper_1502_01629_amd import capi

    fine, coarse, ref = case
    P = 16
    n = fine.n
    src, _ = capi.partition_sources(fine.node_class, P)
    v = torch.empty(n * n, dtype=torch.float32, device="cuda")
    lab = torch.empty(n * n, dtype=torch.int16, device="cuda")
    st = ctx.solve_patchy(capi.DeviceProblem(fine, 1), capi.DeviceProblem(coarse, 1), v, mode=1, tol=5e-7,
                          source_patch=_dev(src, np.int16), n_patches=P, label_out=lab)
    assert st["status"] == 0
    got = v.cpu().numpy().astype(np.float64)
    assert (got >= ref - 2e-6).all()
    err = (got - ref).reshape(n, n)
    L = lab.cpu().numpy().reshape(n, n)
    # nodes with another label within two cells are interface nodes
    iface = np.zeros((n, n), dtype=bool)
    for dj in range(-2, 3):
        for di in range(-2, 3):
            sh = np.roll(np.roll(L, dj, axis=0), di, axis=1)
            iface |= sh != L
    free = fine.node_class == I.FREE
    e_if, e_in = err[free & iface], err[free & ~iface]
    print("decomposition error max", err[free].max(), "interface mean", e_if.mean(), "interior mean", e_in.mean(),
          flush=True)
    assert e_if.mean() > e_in.mean()


def test_labels_beside_the_solve_equal_the_sequential_labels(ctx, case):
    """In the transmission mode the labeler runs on its own stream beside the fine solve; its labels
    are bit-identical to those computed before the solve (independent mode), and the solution to the
    one computed without labels. (The pass counts of the two labelings may differ: a visit updates
    phi in place and its neighbours in the same pass see the new values or the old ones depending on
    timing; the least fixed point they reach does not.)"""
    from paper_1502_01629_amd import capi

    fine, coarse, _ = case
    P = 16
    src, _ = capi.partition_sources(fine.node_class, P)
    dp, dpc = capi.DeviceProblem(fine, 1), capi.DeviceProblem(coarse, 1)
    n2 = fine.n * fine.n
    v1 = torch.empty(n2, dtype=torch.float32, device="cuda")
    v2 = torch.empty_like(v1)
    v3 = torch.empty_like(v1)
    lab1 = torch.empty(n2, dtype=torch.int16, device="cuda")
    lab2 = torch.empty_like(lab1)
    s1 = ctx.solve_patchy(dp, dpc, v1, mode=0, tol=5e-7, source_patch=_dev(src, np.int16), n_patches=P,
                          label_out=lab1, policy_sweeps=4)
    s2 = ctx.solve_patchy(dp, dpc, v2, mode=1, tol=5e-7, source_patch=_dev(src, np.int16), n_patches=P,
                          label_out=lab2)
    s3 = ctx.solve_patchy(dp, dpc, v3, mode=0, tol=5e-7, policy_sweeps=4)
    assert s1["status"] == 0 and s2["status"] == 0 and s3["status"] == 0
    assert s1["label_passes"] > 0 and s2["label_passes"] > 0
    assert torch.equal(lab1, lab2)
    assert torch.equal(v1, v3)

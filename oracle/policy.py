"""Exact fixed points of the discounted scheme on tiny grids (TEST INFRASTRUCTURE ONLY).

For a fixed policy pi (one control per FREE node) the scheme of Section 3 in its SL2 form is
a linear system: v = beta P_pi v + rho_pi + beta p_out v_out on FREE nodes (rho_pi the step cost
of each node under its control), with TARGET and
OBSTACLE values known. Howard's policy iteration alternates an exact solve of that system
(LAPACK Gaussian elimination with partial pivoting) with a greedy improvement; on a finite
discounted Markov decision problem it stops at the optimal value in finitely many steps.
Brute force enumerates every policy and takes the componentwise minimum, which for a
discounted problem is again the optimal value. Both are independent of the value iteration
they are used to check; the chain's transition weights come from the oracle's bilinear
reconstruction, which is pinned separately by closed forms.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import FREE, OBSTACLE, TARGET, Problem


def _chain(p: Problem):
    """Dense transition data: per (free node, control) the row of P over all nodes and p_out."""
    N = p.n * p.n
    free = np.flatnonzero(p.node_class == FREE)
    NA = p.controls.shape[0]
    P = np.zeros((free.size, NA, N))
    pout = np.zeros((free.size, NA))
    for a, node in enumerate(free):
        for m in range(NA):
            idx, w, wo = p.transitions(int(node), m)
            np.add.at(P[a, m], idx, w)
            pout[a, m] = wo
    return free, P, pout


def _fixed_values(p: Problem) -> np.ndarray:
    v = np.zeros(p.n * p.n)
    v[p.node_class == TARGET] = p.target_value
    v[p.node_class == OBSTACLE] = p.v_out
    return v


def evaluate(p: Problem, free, P, pout, policy, rho_t=None) -> np.ndarray:
    beta = p.beta()
    if rho_t is None:
        rho_t = p.rho_table()[free]
    rho = rho_t[np.arange(free.size), policy]
    fixed = _fixed_values(p)
    rows = P[np.arange(free.size), policy]  # (F, N)
    A = np.eye(free.size) - beta * rows[:, free]
    mask = np.ones(p.n * p.n, dtype=bool)
    mask[free] = False
    b = rho + beta * pout[np.arange(free.size), policy] * p.v_out + beta * rows[:, mask] @ fixed[mask]
    v = fixed.copy()
    v[free] = np.linalg.solve(A, b)
    return v


def policy_iteration(p: Problem, max_iter: int = 1000):
    """Howard's policy iteration on the SL2 form. Returns (v, policy, iterations)."""
    free, P, pout = _chain(p)
    beta, rho = p.beta(), p.rho_table()[free]  # rho: (F, NA)
    policy = np.zeros(free.size, dtype=np.int64)
    for it in range(1, max_iter + 1):
        v = evaluate(p, free, P, pout, policy, rho)
        q = beta * (P @ v + pout * p.v_out) + rho  # (F, NA)
        cur = q[np.arange(free.size), policy]
        best = q.argmin(axis=1)
        improve = q[np.arange(free.size), best] < cur - 1e-14 * np.maximum(1.0, np.abs(cur))
        if not improve.any():
            return v, policy, it
        policy = np.where(improve, best, policy)
    raise RuntimeError("policy iteration did not stop")


def brute_force(p: Problem, chunk: int = 8192):
    """Componentwise minimum of v_pi over every deterministic stationary policy (exact
    linear solves, batched over policies)."""
    free, P, pout = _chain(p)
    NA = p.controls.shape[0]
    F = free.size
    beta, rho = p.beta(), p.rho_table()[free]  # rho: (F, NA)
    fixed = _fixed_values(p)
    mask = np.ones(p.n * p.n, dtype=bool)
    mask[free] = False
    # per (free node, control): the free-to-free block row and the constant part
    Pff = P[:, :, free]  # (F, NA, F)
    const = rho + beta * (pout * p.v_out + P[:, :, mask] @ fixed[mask])  # (F, NA)
    best = np.full(F, np.inf)
    pols = itertools.product(range(NA), repeat=F)
    eye = np.eye(F)
    while True:
        block = np.array(list(itertools.islice(pols, chunk)), dtype=np.int64)
        if block.size == 0:
            break
        rows = Pff[np.arange(F)[None, :], block]  # (B, F, F)
        A = eye[None] - beta * rows
        b = const[np.arange(F)[None, :], block]  # (B, F)
        v = np.linalg.solve(A, b[..., None])[..., 0]
        best = np.minimum(best, v.min(axis=0))
    out = fixed.copy()
    out[free] = best
    return out


def sparse_policy_iteration(p: Problem, v0: np.ndarray | None = None, threads: int = 1, max_iter: int = 500):
    """Howard's policy iteration with exact sparse solves, for grids beyond the dense form.

    The same algorithm as policy_iteration: evaluate the policy exactly (here SciPy's sparse LU
    of I - beta P_pi on the FREE nodes), then improve greedily on the SL2 candidates, keeping a
    node's control unless another is smaller by more than a relative 1e-14. The first policy is
    the greedy one at v0 (default: the start vector of the value iteration). Returns
    (v, policy, iterations)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    N = p.n * p.n
    free = np.flatnonzero(p.node_class == FREE)
    F = free.size
    pos = np.full(N, -1, dtype=np.int64)
    pos[free] = np.arange(F)
    fixed = _fixed_values(p)
    beta = p.beta()
    policy = np.zeros(N, dtype=np.int32)
    p.policy_improve(p.initial() if v0 is None else v0, policy, threads)
    rows = np.repeat(np.arange(F), 16).reshape(F, 16)
    for it in range(1, max_iter + 1):
        idx, w, wo = p.policy_chain(policy, threads)
        idx, w, wo = idx[free], w[free], wo[free]
        valid = idx >= 0
        col = np.where(valid, idx, 0)
        to_free = valid & (p.node_class[col] == FREE)
        to_fixed = valid & ~to_free
        A = sp.csr_matrix((-beta * w[to_free], (rows[to_free], pos[col[to_free]])), shape=(F, F)) + sp.eye(F)
        rho = p.rho_policy(policy)[free]
        b = rho + beta * (wo * p.v_out + (np.where(to_fixed, w, 0.0) * fixed[col]).sum(axis=1))
        v = fixed.copy()
        v[free] = spla.spsolve(A.tocsc(), b)
        if p.policy_improve(v, policy, threads) == 0:
            return v, policy, it
    raise RuntimeError("policy iteration did not stop")

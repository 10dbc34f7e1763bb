"""Balanced patches: the iterative re-division of the information sources that the paper proposes
(Section 2, on the relative sizes of the patches; Section 4.3, closing remarks) and leaves open.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain Python over the oracle labeler.

The paper's observation: equal sub-sets of the boundary can give patches of very different
sizes, because the optimal dynamics decides where the information flows; it suggests optimising
the subdivision of the boundary so that the patches come out about equal. The reading built here
(one round, repeated `iterations` times):

1. label the patches of the current subdivision (eq. discrete-advection, then the argmax);
2. size of patch p: the nodes labelled p; weight of a source node: the size of its patch divided
   by the number of source nodes of that patch (the patch's nodes shared out evenly among the
   sources they came from);
3. across the target components (each a connected set of sources): one patch each, the rest
   apportioned by the components' total size, largest remainder;
4. within a component: its sources in angular order around the component's centroid, cut into
   P_t consecutive runs of equal total weight (a source goes to the run that holds the middle of
   its weight).

The rounds keep the best balanced subdivision they visit (largest patch over the mean size).

The angular order is exact: a source's direction (i cnt - sum_i, j cnt - sum_j) from the centroid
is compared by half-plane and integer cross product, in the order of atan2 on (-pi, pi], ties by
node index, so that no rounding of an angle decides it.
"""
from __future__ import annotations

import functools
import math

import numpy as np

from . import FREE, TARGET  # noqa: F401  (node classes)
from . import label as oracle_label


def components(node_class: np.ndarray):
    """4-connected TARGET components, numbered in raster order of their first node. Returns
    (comp int32[n*n] with -1 off targets, count, sum of i, sum of j per component)."""
    n = node_class.shape[0]
    cls = node_class.reshape(-1)
    comp = np.full(n * n, -1, dtype=np.int64)
    cnt, si, sj = [], [], []
    for start in range(n * n):
        if cls[start] != TARGET or comp[start] >= 0:
            continue
        cid = len(cnt)
        cnt.append(0)
        si.append(0)
        sj.append(0)
        comp[start] = cid
        stack = [start]
        while stack:
            v = stack.pop()
            i, j = v % n, v // n
            cnt[cid] += 1
            si[cid] += i
            sj[cid] += j
            for u, ok in ((v - 1, i > 0), (v + 1, i < n - 1), (v - n, j > 0), (v + n, j < n - 1)):
                if ok and cls[u] == TARGET and comp[u] < 0:
                    comp[u] = cid
                    stack.append(u)
    return comp, cnt, si, sj


def partition_sources(node_class: np.ndarray, n_patches: int) -> np.ndarray:
    """The starting subdivision (Section 4.3 pre-computation: one source set per patch): one patch
    per target component plus a largest-remainder share of the rest by node count, equal angular
    sectors around each component's centroid in grid units (atan2 on (-pi, pi])."""
    n = node_class.shape[0]
    comp, cnt, si, sj = components(node_class)
    T = len(cnt)
    out = np.full(n * n, -1, dtype=np.int16)
    if T == 0:
        return out.reshape(n, n)
    extra = n_patches - T
    quota = [extra * cnt[t] / sum(cnt) for t in range(T)]
    share = [math.floor(q) for q in quota]
    order = sorted(range(T), key=lambda t: -(quota[t] - share[t]))
    for k in range(extra - sum(share)):
        share[order[k]] += 1
    offset = [0]
    for t in range(T):
        offset.append(offset[-1] + 1 + share[t])
    for v in np.nonzero(comp >= 0)[0]:
        t = int(comp[v])
        Pt = offset[t + 1] - offset[t]
        th = math.atan2(v // n - sj[t] / cnt[t], v % n - si[t] / cnt[t])
        sec = min(max(math.floor(Pt * (th + math.pi) / (2.0 * math.pi)), 0), Pt - 1)
        out[v] = offset[t] + sec
    return out.reshape(n, n)


def imbalance(sizes: np.ndarray) -> float:
    """Largest patch over the mean patch size."""
    sizes = np.asarray(sizes, dtype=np.float64)
    return float(sizes.max() / sizes.mean()) if sizes.sum() > 0 else 1.0


def _half(dx: int, dy: int) -> int:
    """Position class of atan2(dy, dx) on (-pi, pi]: 0 below the axis, 1 at angle 0 (and the
    centroid itself), 2 above, 3 at angle pi."""
    if dy < 0:
        return 0
    if dy == 0 and dx >= 0:
        return 1
    if dy > 0:
        return 2
    return 3


def angular_order(nodes, n: int, cnt: int, si: int, sj: int):
    """The nodes sorted by the angle of (i, j) around the centroid (si/cnt, sj/cnt), exactly."""

    def cmp(a, b):
        ax, ay = (a % n) * cnt - si, (a // n) * cnt - sj
        bx, by = (b % n) * cnt - si, (b // n) * cnt - sj
        ha, hb = _half(ax, ay), _half(bx, by)
        if ha != hb:
            return -1 if ha < hb else 1
        if ha in (0, 2):
            cross = ax * by - ay * bx  # > 0: b lies counter-clockwise of a
            if cross != 0:
                return -1 if cross > 0 else 1
        return -1 if a < b else (1 if a > b else 0)

    return sorted(nodes, key=functools.cmp_to_key(cmp))


def rebalance(node_class: np.ndarray, source_patch: np.ndarray, labels: np.ndarray, n_patches: int):
    """One round of steps 2-4: a new subdivision from the patches of the current one."""
    n = node_class.shape[0]
    comp, cnt, si, sj = components(node_class)
    T = len(cnt)
    src = np.asarray(source_patch).reshape(-1).astype(np.int64)
    out = np.full(n * n, -1, dtype=np.int16)
    if T == 0:
        return out
    lab = np.asarray(labels).reshape(-1).astype(np.int64)
    sizes = np.bincount(lab[lab >= 0], minlength=n_patches)[:n_patches]
    members = np.bincount(src[src >= 0], minlength=n_patches)[:n_patches]
    # step 3: patches per component by total size
    weight = [0] * T
    for p in range(n_patches):
        holders = np.nonzero(src == p)[0]
        if holders.size:
            weight[int(comp[holders[0]])] += int(sizes[p])
    total = sum(weight)
    extra = n_patches - T
    if total > 0:
        quota = [extra * weight[t] / total for t in range(T)]
    else:
        quota = [extra * cnt[t] / sum(cnt) for t in range(T)]
    share = [math.floor(q) for q in quota]
    order = sorted(range(T), key=lambda t: -(quota[t] - share[t]))
    for k in range(extra - sum(share)):
        share[order[k]] += 1
    offset = [0]
    for t in range(T):
        offset.append(offset[-1] + 1 + share[t])
    # step 4: equal-weight runs in angular order
    for t in range(T):
        Pt = offset[t + 1] - offset[t]
        nodes = angular_order([int(v) for v in np.nonzero(comp == t)[0]], n, cnt[t], si[t], sj[t])
        w = [float(sizes[src[v]]) / float(members[src[v]]) for v in nodes]
        wt = 0.0
        for x in w:
            wt += x
        cum = 0.0
        for r, (v, x) in enumerate(zip(nodes, w)):
            if wt > 0.0:
                sec = math.floor(Pt * (cum + x / 2) / wt)
            else:
                sec = (Pt * r) // len(nodes)
            out[v] = offset[t] + min(max(sec, 0), Pt - 1)
            cum += x
    return out


def _better(sizes_a, sizes_b) -> bool:
    """True if subdivision a is better balanced than b: a smaller largest-over-mean patch size,
    compared exactly (max_a sum_b < max_b sum_a in integers)."""
    ma, sa = int(np.max(sizes_a)), int(np.sum(sizes_a))
    mb, sb = int(np.max(sizes_b)), int(np.sum(sizes_b))
    return ma * sb < mb * sa


def balance_sources(n: int, node_class: np.ndarray, disp_q8: np.ndarray, source_patch: np.ndarray,
                    n_patches: int, iterations: int):
    """`iterations` rounds from source_patch, keeping the best balanced subdivision visited (the
    rounds do not converge in general: a patch's territory is an argmax of fuzzy indicators and can
    jump when its sources change). Returns (that subdivision int16[n*n], the patch sizes of every
    subdivision visited int64[iterations + 1, n_patches], its labels, its round)."""
    src = np.asarray(source_patch, dtype=np.int16).reshape(-1)
    sizes = []
    best = None
    for k in range(iterations + 1):
        lab, _, _ = oracle_label(n, node_class, disp_q8, src, n_patches)
        lab = lab.astype(np.int64)
        sizes.append(np.bincount(lab[lab >= 0], minlength=n_patches)[:n_patches])
        if best is None or _better(sizes[-1], sizes[best[0]]):
            best = (k, src.copy(), lab.astype(np.int16))
        if k < iterations:
            src = rebalance(node_class, src, lab, n_patches)
    return best[1], np.stack(sizes), best[2], best[0]

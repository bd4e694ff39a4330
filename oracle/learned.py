"""Oracle: the learned adjacent zone (an addition to the method; not from the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/grid.py``).

The paper's adjacent zone (Sec. 2.3) activates the next-level children of every significant
point (rule R3 of ``Hierarchy.adapt``).  The learned zone lets a network decide, per quadrant of
every 8 x 8-element patch, whether the children rule applies to the significant points of that
quadrant; after the step the threshold test on the new state judges the decision, and a
quadrant that was dropped but still holds a significant point makes the step be redone from the
state before the adapt with the blanket zone.

Definitions written out here (plain numpy, full levels):

* patch (L, pi, pj) of level j (lozenge side n, m = n/8 patches per side) holds the elements
  (8 pi .. 8 pi + 7, 8 pj .. 8 pj + 7) of lozenge L, index (L m + pi) m + pj; quadrant
  c = 2a + b holds the elements (8 pi + 4a .. +3, 8 pj + 4b .. +3); the poles belong to no patch
  (their children rule always applies);
* the size of a detail d against its threshold: r = clamp(log2(|d| / eps_var), -16, 4) / 8,
  rounded to single precision (the floor -2 for points without a detail);
* per patch: the largest r of the level-j height and velocity details (points of the patch's
  elements: node, three edges) and of the level-(j+1) height and velocity details (the four
  children (2i + a, 2j + b) of each element: node, three edges); the same per quadrant; the
  active fraction of each quadrant's children nodes; the number of significant level-j points
  (node and three edges) of each quadrant; the active fraction of the patch's nodes;
* 64 features: the four patch maxima of the patch and its 8 lattice neighbours (a neighbour
  outside the lozenge repeats the patch), the 16 quadrant maxima, the 4 child activities, the 4
  significant counts / 64, the patch activity, (j - jmin)/(jmax - jmin), 1, 0;
* label of a quadrant: it holds a significant level-j point;
* gate: the children rule of a quadrant's points applies where the network's probability is
  >= the threshold; a quadrant is dropped if it is significant and not allowed;
* threshold test after the step: a dropped quadrant that is significant again (thresholds from
  eps and the new maxima) is a miss; any miss redoes adapt and step with the blanket zone.

The network is ``oracle.mlp`` with bfloat16 rounding of the matrix-product operands.
"""
from __future__ import annotations

import numpy as np

from . import mlp

FLOOR = np.float32(-2.0)
N_STATS = 29


def rlog(d, eps):
    """Single-precision size of details d against the threshold eps."""
    d = np.abs(np.asarray(d, dtype=np.float64))
    if not eps > 0:
        return np.full(d.shape, np.float32(0.5))
    with np.errstate(divide="ignore"):
        v = np.where(d > 0, np.log2(np.where(d > 0, d, 1.0) / eps), -16.0).astype(np.float32)
    return (np.float32(0.125) * np.clip(v, np.float32(-16.0), np.float32(4.0))).astype(np.float32)


def learnable(H, j):
    """Levels whose children rule has a gate: jmin < j < jmax with at least one patch."""
    return H.jmin < j < H.jmax and j >= 3


def detail_sizes(H, det, eh, eu):
    """r of every fine point of levels jmin+1..jmax (each carries at most one detail)."""
    rn, re = {}, {}
    for j in range(H.jmin, H.jmax):
        P = H.pairs[j]
        f = j + 1
        a = np.full(H.g[f].N, FLOOR, np.float32)
        b = np.full(H.g[f].E, FLOOR, np.float32)
        dhd, dp, di = det[j]
        a[P.mid] = rlog(dhd, eh)
        r = rlog(dp, eu)
        b[P.h1] = r
        b[P.h2] = r
        b[P.int_e.ravel()] = rlog(di, eu).ravel()
        rn[f], re[f] = a, b
    return rn, re


def _patch_elements(n):
    """(npatch, 64) element ids of every patch, lanes row-major within the patch."""
    m = n // 8
    L, pi, pj, r, q = np.meshgrid(np.arange(10), np.arange(m), np.arange(m), np.arange(8), np.arange(8),
                                  indexing="ij")
    ei, ej = 8 * pi + r, 8 * pj + q
    return ((L * n + ei) * n + ej).reshape(10 * m * m, 64), ei.reshape(10 * m * m, 64), ej.reshape(10 * m * m, 64), \
        L.reshape(10 * m * m, 64)


def patch_stats(H, j, rn, re, sig_n, sig_e):
    """The 29 statistics of every patch of level j (see the module docstring)."""
    n = 2 ** j
    ids, ei, ej, L = _patch_elements(n)
    nf = 2 * n
    v = np.empty(ids.shape + (7,), np.float32)
    v[..., 0] = rn[j][ids]
    v[..., 1] = np.maximum(np.maximum(re[j][3 * ids], re[j][3 * ids + 1]), re[j][3 * ids + 2])
    bh = np.full(ids.shape, FLOOR, np.float32)
    bu = np.full(ids.shape, FLOOR, np.float32)
    act = np.zeros(ids.shape, np.float32)
    naf = H.node_act[j + 1]
    for a in (0, 1):
        for b in (0, 1):
            f = (L * nf + 2 * ei + a) * nf + 2 * ej + b
            bh = np.maximum(bh, rn[j + 1][f])
            bu = np.maximum(bu, np.maximum(np.maximum(re[j + 1][3 * f], re[j + 1][3 * f + 1]), re[j + 1][3 * f + 2]))
            act += naf[f].astype(np.float32)
    v[..., 2], v[..., 3], v[..., 4] = bh, bu, act
    v[..., 5] = (sig_n[j][ids].astype(np.float32) + sig_e[j][3 * ids] + sig_e[j][3 * ids + 1] + sig_e[j][3 * ids + 2])
    v[..., 6] = H.node_act[j][ids].astype(np.float32)
    st = np.zeros((ids.shape[0], N_STATS), np.float32)
    st[:, 0:4] = v[..., 0:4].max(1)
    lane = np.arange(64)
    for c in range(4):
        a, b = c // 2, c % 2
        inq = ((lane // 8) // 4 == a) & ((lane % 8) // 4 == b)
        for kind in range(4):
            st[:, 4 + 4 * kind + c] = v[:, inq, kind].max(1)
        st[:, 20 + c] = v[:, inq, 4].sum(1, dtype=np.float32) / np.float32(64.0)
        st[:, 24 + c] = v[:, inq, 5].sum(1, dtype=np.float32)
    st[:, 28] = v[..., 6].sum(1, dtype=np.float32) / np.float32(64.0)
    return st


def features(H, j, st):
    """64 features of every patch of level j from the statistics."""
    m = 2 ** j // 8
    npatch = 10 * m * m
    p = np.arange(npatch)
    L, pi, pj = p // (m * m), (p // m) % m, p % m
    X = np.zeros((npatch, 64), np.float32)
    k = 0
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            qi, qj = pi + di, pj + dj
            inside = (qi >= 0) & (qi < m) & (qj >= 0) & (qj < m)
            q = np.where(inside, (L * m + qi) * m + qj, p)
            for s in range(4):
                X[:, 9 * s + k] = st[q, s]
            k += 1
    X[:, 36:52] = st[:, 4:20]
    X[:, 52:56] = st[:, 20:24]
    X[:, 56:60] = st[:, 24:28] / np.float32(64.0)
    X[:, 60] = st[:, 28]
    X[:, 61] = np.float32(j - H.jmin) / np.float32(H.jmax - H.jmin)
    X[:, 62] = 1.0
    return X


def labels(st):
    return (st[:, 24:28] > 0).astype(np.float32)


def probabilities(theta, X):
    """sigmoid(network(X)) with the GPU's bfloat16 operand rounding."""
    z = mlp.forward(theta, np.asarray(X, np.float64), emulate_bf16=True)[0]
    return 1.0 / (1.0 + np.exp(-z))


def quadrant_of(n, elem):
    """Index 4 patch + quadrant of level elements (poles: -1)."""
    elem = np.asarray(elem)
    L = elem // (n * n)
    i, jj = (elem // n) % n, elem % n
    m = n // 8
    q = 4 * ((L * m + i // 8) * m + jj // 8) + 2 * ((i % 8) // 4) + (jj % 8) // 4
    return np.where(elem < 10 * n * n, q, -1)


def _allow_fn(n, allow_q):
    def f(elem):
        q = quadrant_of(n, elem)
        return np.where(q >= 0, allow_q[np.maximum(q, 0)], True)
    return f


def all_stats(H, det, eh, eu, sig_n, sig_e):
    rn, re = detail_sizes(H, det, eh, eu)
    return {j: patch_stats(H, j, rn, re, sig_n, sig_e) for j in range(H.jmin + 1, H.jmax) if learnable(H, j)}


def gated_adapt(H, eps, theta, thr, prob_fn=None):
    """Adapt with the learned gate of the children rule.  Returns the dropped quadrants per level
    and the probabilities (prob_fn(j, X) replaces the network when given)."""
    det = H.details()
    eh, eu = H.thresholds(eps)
    sig_n, sig_e = H.significant(det, eh, eu)
    stats = all_stats(H, det, eh, eu, sig_n, sig_e)
    allow, dropped, probs = {}, {}, {}
    for j, st in stats.items():
        X = features(H, j, st)
        P = prob_fn(j, X) if prob_fn is not None else probabilities(theta, X)
        a = (P >= thr).ravel()
        dropped[j] = (~a) & (st[:, 24:28].ravel() > 0)
        allow[j] = _allow_fn(2 ** j, a)
        probs[j] = P
    H.adapt(eps, allow=allow)
    return dropped, probs


def judge(H, eps, dropped):
    """Threshold test after the step: the number of dropped quadrants that are significant."""
    det = H.details()
    eh, eu = H.thresholds(eps)
    sig_n, sig_e = H.significant(det, eh, eu)
    stats = all_stats(H, det, eh, eu, sig_n, sig_e)
    return int(sum((dropped[j] & (st[:, 24:28].ravel() > 0)).sum() for j, st in stats.items()))


def snapshot(H):
    return ({j: v.copy() for j, v in H.dh.items()}, {j: v.copy() for j, v in H.u.items()},
            {j: v.copy() for j, v in H.node_act.items()}, {j: v.copy() for j, v in H.edge_act.items()})


def restore(H, snap):
    H.dh, H.u, H.node_act, H.edge_act = ({j: v.copy() for j, v in d.items()} for d in snap)


def learned_step(H, eps, dt, p, theta, thr, scheme="rk4", prob_fn=None):
    """adapt (gated) + step + threshold test; a miss redoes both with the blanket zone.
    Returns (redone, dropped quadrants, probabilities of the gated adapt)."""
    snap = snapshot(H)
    dropped, probs = gated_adapt(H, eps, theta, thr, prob_fn)
    H.step(dt, p, scheme)
    if judge(H, eps, dropped) > 0:
        restore(H, snap)
        H.adapt(eps)
        H.step(dt, p, scheme)
        return True, dropped, probs
    return False, dropped, probs


def active_dof(H):
    return int(sum(H.node_act[j].sum() + H.edge_act[j].sum() for j in H.levels))


def perfect_gate_bound(H, eps, dt, p, steps, scheme="rk4"):
    """The most any gate can drop under the threshold test: at every step the blanket run tells
    which significant quadrants are no longer significant after the step; the gate that drops
    exactly those (and is judged like any other) is run from the same state.  Returns the
    per-step active dof of the blanket and of this gated run, and the misses (quadrants whose
    significance came back once their children were dropped: those steps are redone)."""
    blanket, gated, misses = [], [], 0
    for _ in range(steps):
        snap = snapshot(H)
        # the blanket step and the significance of every quadrant after it
        det = H.details()
        eh, eu = H.thresholds(eps)
        sig_n, sig_e = H.significant(det, eh, eu)
        before = all_stats(H, det, eh, eu, sig_n, sig_e)
        H.adapt(eps)
        blanket.append(active_dof(H))
        H.step(dt, p, scheme)
        det = H.details()
        eh, eu = H.thresholds(eps)
        sig_n, sig_e = H.significant(det, eh, eu)
        after = all_stats(H, det, eh, eu, sig_n, sig_e)
        blanket_state = snapshot(H)
        # the perfect gate from the same start
        restore(H, snap)

        def prob_fn(j, X, before=before, after=after):
            keep = ~((before[j][:, 24:28] > 0) & ~(after[j][:, 24:28] > 0))
            return keep.astype(np.float64)

        redone, _, _ = learned_step(H, eps, dt, p, None, 0.5, scheme, prob_fn=prob_fn)
        misses += int(redone)
        gated.append(blanket[-1] if redone else None)
        if not redone:
            # the active dof the gated adapt kept (the step does not change masks)
            gated[-1] = active_dof(H)
        # continue from the blanket run so both series see the same states
        restore(H, blanket_state)
    return blanket, gated, misses


def zone_turnover(H, eps, dt, p, steps, scheme="rk4"):
    """The most any adjacent-zone gate can drop under a judge that asks only that every point the
    blanket zone requires after the step was active during it (a looser judge than the threshold
    test above, and one that covers gates on any rule, not just the children rule): per step, the
    points active under the blanket zone before the step that the blanket zone of the state after
    the step no longer holds.  Returns (dropped, active) per step; the blanket run continues."""
    out = []
    H.adapt(eps)
    for _ in range(steps):
        before = [(H.node_act[j].copy(), H.edge_act[j].copy()) for j in H.levels]
        H.step(dt, p, scheme)
        H.adapt(eps)
        gone = active = 0
        for (bn, be), j in zip(before, H.levels):
            gone += int((bn & ~H.node_act[j]).sum()) + int((be & ~H.edge_act[j]).sum())
            active += int(bn.sum()) + int(be.sum())
        out.append((gone, active))
    return out


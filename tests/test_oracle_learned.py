"""Pins of the oracle's learned adjacent zone (oracle/learned.py; an addition to the method, not
from the paper): detail sizes, patch statistics and features on hand-built cases, the gate's
limits (threshold 0 is the paper's blanket zone, a gate that drops everything is redone into
it), and the bound on what any gate can drop under the threshold test (CPU only)."""
import numpy as np
import pytest

from oracle import learned, trisk
from oracle.multiscale import Hierarchy
from paper_1404_0405_amd import inputs


def gate_params(min_count=2):
    """A network (oracle.mlp layout) whose probability is ~1 where a quadrant holds at least
    `min_count` significant points and ~0 elsewhere: hidden unit c = relu(64 x[56 + c] - m + 1/2)
    (x[56 + c] = count / 64), passed on by the second layer, output 40 h - 10.  Every weight and
    activation is exact in bfloat16, so both sides decide identically."""
    W1, b1 = np.zeros((64, 128)), np.zeros(128)
    W2, b2 = np.zeros((128, 128)), np.zeros(128)
    W3, b3 = np.zeros((128, 4)), np.zeros(4)
    for c in range(4):
        W1[56 + c, c] = 64.0
        b1[c] = -(min_count - 0.5)
        W2[c, c] = 1.0
        W3[c, c] = 40.0
        b3[c] = -10.0
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def test_gate_network_is_decisive():
    X = np.zeros((5, 64), np.float32)
    for k, cnt in enumerate([0, 1, 2, 3, 64]):
        X[k, 56:60] = cnt / 64.0
    P = learned.probabilities(gate_params(2), X)
    assert (P[:2] < 1e-4).all() and (P[2:] > 1 - 1e-4).all()


def test_detail_size_closed_forms():
    """r = clamp(log2(|d| / eps), -16, 4) / 8 in single precision."""
    d = np.array([1.0, -2.0, 0.5, 0.0, 1e9, 2.0 ** -20])
    r = learned.rlog(d, 1.0)
    assert r.dtype == np.float32
    assert list(r) == [0.0, 0.125, -0.125, -2.0, 0.5, -2.0]
    assert (learned.rlog(d, 0.0) == 0.5).all()


def test_quadrant_map_covers_patches():
    """Every element of a patch maps to 4 patch + quadrant, quadrants split the patch 4 x 4."""
    n = 16
    ids, ei, ej, L = learned._patch_elements(n)
    q = learned.quadrant_of(n, ids)
    for p in range(ids.shape[0]):
        assert set(q[p] // 4) == {p}
        counts = np.bincount(q[p] % 4, minlength=4)
        assert (counts == 16).all()
    assert (learned.quadrant_of(n, np.array([10 * n * n, 10 * n * n + 1])) == -1).all()


def test_patch_statistics_of_a_hand_built_state():
    """Levels 2..4; one significant level-3 node in quadrant 3 of patch 0 and the children of
    quadrant 0 of patch 0 all active: counts, labels, child activity and the detail maxima are
    the hand values."""
    H = Hierarchy(2, 4)
    for j in H.levels:
        H.node_act[j][:] = False
        H.edge_act[j][:] = False
    n = 8
    sig_n = {j: np.zeros(H.g[j].N, bool) for j in H.levels}
    sig_e = {j: np.zeros(H.g[j].E, bool) for j in H.levels}
    k = (0 * n + 5) * n + 6                          # element (5, 6) of lozenge 0: quadrant 3
    sig_n[3][k] = True
    sig_e[3][3 * k + 1] = True
    for i in range(4):
        for jj in range(4):
            for a in (0, 1):
                for b in (0, 1):
                    H.node_act[4][(0 * 16 + 2 * i + a) * 16 + 2 * jj + b] = True
    rn = {j: np.full(H.g[j].N, learned.FLOOR, np.float32) for j in (3, 4)}
    re = {j: np.full(H.g[j].E, learned.FLOOR, np.float32) for j in (3, 4)}
    rn[3][k] = 0.25
    re[4][3 * ((0 * 16 + 3) * 16 + 2) + 2] = 0.375   # a child of element (1, 1): quadrant 0
    st = learned.patch_stats(H, 3, rn, re, sig_n, sig_e)
    assert st.shape == (10, learned.N_STATS)
    assert list(st[0, 24:28]) == [0, 0, 0, 2]
    assert list(learned.labels(st)[0]) == [0, 0, 0, 1]
    assert list(st[0, 20:24]) == [1.0, 0, 0, 0]
    assert st[0, 0] == 0.25 and st[0, 3] == 0.375 and st[0, 1] == -2.0
    assert st[0, 4 + 3] == 0.25 and st[0, 4 + 12 + 0] == 0.375 and st[0, 4 + 12 + 1] == -2.0
    assert (st[1:, 24:28] == 0).all()
    X = learned.features(H, 3, st)
    # m = 1: every neighbour is outside the lozenge and repeats the patch
    assert (X[0, 0:9] == 0.25).all() and (X[0, 27:36] == 0.375).all()
    assert X[0, 59] == 2 / 64 and X[0, 61] == 0.5 and X[0, 62] == 1.0 and X[0, 63] == 0.0


def _jet(jmin, jmax):
    H = Hierarchy(jmin, jmax)
    g = H.g[jmax]
    dh, u, Hd = inputs.jet(g.xyz, g.e_mid, g.e_tan)
    H.set_state(jmax, dh, u)
    p = trisk.Params(mean_depth=Hd)
    return H, p, 0.8 * trisk.suggest_dt(g, dh, u, p, 1.0)


def test_gate_limits():
    """Threshold 0 lets every quadrant through: the masks are the blanket zone's.  A gate that
    drops every quadrant is caught by the threshold test and the step is redone with the
    blanket zone, which equals the plain step bitwise."""
    H, p, dt = _jet(2, 5)
    snap = learned.snapshot(H)
    H.adapt(2e-2)
    ref = learned.snapshot(H)
    H.step(dt, p)
    ref_after = learned.snapshot(H)
    learned.restore(H, snap)
    dropped, _ = learned.gated_adapt(H, 2e-2, gate_params(), 0.0)
    assert not any(d.any() for d in dropped.values())
    for a, b in zip(learned.snapshot(H)[2:], ref[2:]):
        for j in a:
            assert np.array_equal(a[j], b[j])
    learned.restore(H, snap)
    redone, dropped, _ = learned.learned_step(H, 2e-2, dt, p, gate_params(), 2.0)
    assert redone and any(d.any() for d in dropped.values())
    for a, b in zip(learned.snapshot(H), ref_after):
        for j in a:
            assert np.array_equal(a[j], b[j])


@pytest.mark.slow
def test_no_gate_gains_much_under_the_threshold_test():
    """The perfect gate -- dropping exactly the significant quadrants that are not significant
    after the step, known from the blanket run -- bounds every gate judged by the threshold test.
    On the jet (levels 3..6, eps 5e-3) it removes under 2 % of the active dof."""
    H, p, dt = _jet(3, 6)
    H.adapt(5e-3)
    blanket, gated, misses = learned.perfect_gate_bound(H, 5e-3, dt, p, 6)
    assert all(g <= b for g, b in zip(gated, blanket))
    gain = 1.0 - sum(gated) / sum(blanket)
    print(f"perfect gate: {gain:.4f} of the active dof, {misses} misses in 6 steps")
    assert gain < 0.02, gain


@pytest.mark.slow
def test_zone_turnover_bounds_every_gate():
    """Under the loosest judge (every point the blanket zone requires after the step was active
    during it) a gate can drop at most the points that leave the blanket zone within one step: on
    the jet (levels 4..7, eps 5e-3) under 5 % of the active dof per step, on the turbulence start
    (levels 3..6, eps 1e-2) none, since its zone only grows."""
    H, p, dt = _jet(4, 7)
    r = learned.zone_turnover(H, 5e-3, dt, p, 6)
    frac = [g / a for g, a in r]
    print("jet zone turnover per step", [f"{f:.4f}" for f in frac])
    assert max(frac) < 0.05 and sum(g for g, _ in r) > 0
    H = Hierarchy(3, 6)
    g = H.g[6]
    dh, u, Hd = inputs.turbulence(g.xyz, g.e_mid, g.e_tan)
    H.set_state(6, dh, u)
    p = trisk.Params(mean_depth=Hd)
    r = learned.zone_turnover(H, 1e-2, 60.0, p, 4)
    assert all(g == 0 for g, _ in r), r


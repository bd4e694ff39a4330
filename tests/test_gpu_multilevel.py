"""GPU parity of the multilevel (adaptive wavelet) path: HIP library through the C ABI against
the FP64 oracle, on the same seeded inputs."""
import os
import sys

import numpy as np
import pytest

from oracle import trisk
from oracle.multiscale import Hierarchy
from paper_1404_0405_amd import inputs, wt

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _ic(case, g_or_xyz):
    x, m, t = g_or_xyz
    if case == "tc2":
        return inputs.tc2(x, m, t)
    if case == "jet":
        return inputs.jet(x, m, t)
    if case == "turb":
        return inputs.turbulence(x, m, t)
    return inputs.tc2_perturbed(x, m, t, amplitude=300.0)


def _pair(jmin, jmax, case):
    H = Hierarchy(jmin, jmax)
    og = H.g[jmax]
    dh, u, Hd = _ic(case, (og.xyz, og.e_mid, og.e_tan))
    g = wt.Grid(jmin, jmax, 8)
    g.set_params(mean_depth=Hd)
    return H, g, dh, u, trisk.Params(mean_depth=Hd)


def _compare_all(H, g, tol, masks=True):
    worst = 0.0
    for j in H.levels:
        a, b, na, ea = H.get_state(j)
        x, y, gna, gea = g.get_state(j)
        if masks:
            assert np.array_equal(gna.astype(bool), na), f"node mask differs on level {j}"
            assert np.array_equal(gea.astype(bool), ea), f"edge mask differs on level {j}"
        worst = max(worst, _rel(x, a), _rel(y, b))
    assert worst < tol, worst
    return worst


@pytest.mark.parametrize("jmin,jmax", [(2, 4), (3, 5)])
def test_forward_details_and_inverse(jmin, jmax):
    """Forward transform details (eq. (WTpred), velocity prediction) and the inverse transform
    of the GPU equal the oracle's; the reconstruction is exact."""
    _say(f"forward/inverse {jmin}..{jmax}")
    H, g, dh, u, p = _pair(jmin, jmax, "tc2p")
    with g:
        g.set_state(jmax, dh, u)
        H.set_state(jmax, dh, u)
        g.forward()
        det = H.details()
        for j in range(jmin + 1, jmax + 1):
            a, b, c = g.get_details(j)
            rh, rp, ri = det[j - 1]
            assert _rel(a, rh) < 1e-12 and _rel(b, rp) < 1e-11 and _rel(c, ri) < 1e-11, j
        g.inverse()
        H.resync()
        _compare_all(H, g, 1e-13)
        x, y, _, _ = g.get_state(jmax)
        assert _rel(x, dh) < 1e-13 and _rel(y, u) < 1e-13


@pytest.mark.parametrize("scheme", ["rk4", "ssprk43"])
def test_multilevel_step_full_masks(scheme):
    """One multilevel step with every level full: restriction of F (R_F), Q and B and the
    partial height transform reproduce the oracle."""
    _say(f"ml step full masks {scheme}")
    H, g, dh, u, p = _pair(2, 4, "tc2p")
    with g:
        g.set_params(rk=wt.WT_RK4 if scheme == "rk4" else wt.WT_SSPRK43)
        g.set_state(4, dh, u)
        H.set_state(4, dh, u)
        for _ in range(3):
            g.step(600.0)
            H.step(600.0, p, scheme)
        _compare_all(H, g, 1e-12)


@pytest.mark.parametrize("case,eps", [("jet", 5e-2), ("jet", 1e-2), ("tc2p", 2e-3)])
def test_adapt_masks_and_state(case, eps):
    """wt_adapt: thresholds, adjacent zone, consistency and prediction-stencil closure give the
    oracle's masks exactly; the inverse transform gives its state."""
    _say(f"adapt {case} eps={eps}")
    H, g, dh, u, p = _pair(2, 5, case)
    with g:
        g.set_state(5, dh, u)
        H.set_state(5, dh, u)
        g.adapt(eps)
        H.adapt(eps)
        _compare_all(H, g, 1e-12)
        na = H.node_act[5]
        assert 0 < na.sum() <= na.size
        if case == "jet":
            assert na.sum() < na.size


def test_adaptive_run_parity_and_mass():
    """Jet with bump on levels 2..5, eps = 5e-2: 12 steps with adaptation after each step;
    masks identical and fields within 1e-11 (rel L-inf) of the oracle; mass conserved."""
    _say("adaptive run 2..5")
    H, g, dh, u, p = _pair(2, 5, "jet")
    with g:
        g.set_state(5, dh, u)
        H.set_state(5, dh, u)
        g.adapt(5e-2)
        H.adapt(5e-2)
        m0 = g.diagnostics()[0].mass
        dt = 400.0
        for s in range(12):
            g.step(dt)
            H.step(dt, p)
            g.adapt(5e-2)
            H.adapt(5e-2)
        _compare_all(H, g, 1e-11)
        d, code = g.diagnostics()
    assert code == wt.WT_OK
    assert abs(d.mass / m0 - 1) < 1e-13
    assert abs(d.mass_reconstructed / d.mass - 1) < 1e-13
    assert abs(d.mass / H.mass(p) - 1) < 1e-13
    assert d.active_nodes[5] == H.node_act[5].sum()


def test_adaptive_run_through_an_empty_level():
    """TC2 on levels 2..5 at eps = 1e-2: the first adapt empties level 5, later adaptations fill
    it again (an empty level adds nothing to the threshold maxima); after each of 5 steps and
    adaptations the masks are identical and the fields within 1e-11 of the oracle."""
    _say("adaptive run through an empty level 2..5")
    H, g, dh, u, p = _pair(2, 5, "tc2")
    with g:
        g.set_state(5, dh, u)
        H.set_state(5, dh, u)
        g.adapt(1e-2)
        H.adapt(1e-2)
        _compare_all(H, g, 1e-12)
        assert not H.node_act[5].any()
        for _ in range(5):
            g.step(400.0)
            H.step(400.0, p)
            g.adapt(1e-2)
            H.adapt(1e-2)
            _compare_all(H, g, 1e-11)
        d, code = g.diagnostics()
    assert code == wt.WT_OK and H.node_act[5].any()
    assert abs(d.mass / H.mass(p) - 1) < 1e-13


def test_eps_zero_equals_uniform_on_gpu():
    """eps = 0 keeps every point: the jmax field equals a uniform GPU run to round-off."""
    _say("eps=0 vs uniform")
    H, g, dh, u, p = _pair(3, 5, "tc2p")
    gu = wt.Grid(5, 5, 8)
    with g, gu:
        gu.set_params(mean_depth=p.H)
        g.set_state(5, dh, u)
        gu.set_state(5, dh, u)
        g.adapt(0.0)
        for _ in range(4):
            g.step(300.0)
            g.adapt(0.0)
            gu.step(300.0)
        x, y, na, ea = g.get_state(5)
        a, b, _, _ = gu.get_state(5)
    assert na.all() and ea.all()
    assert _rel(x, a) < 1e-13 and _rel(y, b) < 1e-13


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tc2_adaptive_levels_4_to_6(precision):
    """TC2 on levels 4..6, eps = 1e-3 relative, RK4, CFL 0.8, 50 steps with adaptation: FP64
    matches the oracle within 1e-11 (masks identical); FP32 tendencies stay within 1e-5 (rel
    L2 height) of it; mass conserved to 1e-13 in both."""
    _say(f"tc2 4..6 {precision}")
    H, g, dh, u, p = _pair(4, 6, "tc2")
    with g:
        if precision == "fp32":
            g.set_params(precision=wt.WT_FP32_TENDENCY)
        g.set_state(6, dh, u)
        H.set_state(6, dh, u)
        g.adapt(1e-3)
        H.adapt(1e-3)
        dt = trisk.suggest_dt(H.g[6], dh, u, p, 0.8)
        m0 = g.diagnostics()[0].mass
        for _ in range(50):
            g.step(dt)
            H.step(dt, p)
            g.adapt(1e-3)
            H.adapt(1e-3)
        d, _ = g.diagnostics()
        if precision == "fp64":
            _compare_all(H, g, 1e-11)
        else:
            x, _, _, _ = g.get_state(6)
            a, _, _, _ = H.get_state(6)
            A = H.A[6]
            l2 = np.sqrt((A * (x - a) ** 2).sum() / (A * (p.H + a) ** 2).sum())
            _say(f"fp32 tendencies, tc2 4..6: rel L2 height error {l2:.3e}")
            assert l2 < 1e-5
    assert abs(d.mass / m0 - 1) < 1e-13
    x, _, _, _ = H.get_state(6)
    assert np.abs(x - dh).max() / np.abs(dh).max() < 2e-2


@pytest.mark.parametrize("case,jmin,jmax,eps,prec", [("jet", 4, 7, 5e-3, "fp64"), ("tc2p", 3, 6, 1e-3, "fp64"),
                                                     ("jet", 5, 8, 5e-3, "fp32"), ("tc2p", 2, 5, 1e-3, "fp64"),
                                                     ("jet", 5, 9, 5e-3, "fp64")])
def test_work_lists_equal_whole_levels(case, jmin, jmax, eps, prec):
    """The adaptive stage over ballot/prefix-scan work lists (support rings of the active
    points) gives bitwise the same states, masks and diagnostics as the stage over whole
    levels."""
    _say(f"work lists {case} {jmin}..{jmax} eps={eps} {prec}")
    out = []
    for lists in (True, False):
        g = wt.Grid(jmin, jmax, 8)
        with g:
            x, m, t = g.coords(jmax)
            dh, u, Hd = _ic(case, (x, m, t))
            g.set_params(mean_depth=Hd, precision=wt.WT_FP64 if prec == "fp64" else wt.WT_FP32_TENDENCY)
            g.set_state(jmax, dh, u)
            g.set_work_lists(lists)
            dt = g.suggest_dt(0.8)
            for _ in range(6):
                g.adapt(eps)
                g.step(dt)
            d, code = g.diagnostics()
            assert code == wt.WT_OK
            out.append(([g.get_state(j) for j in range(jmin, jmax + 1)], d.mass, d.energy,
                        list(d.active_nodes), list(d.active_edges)))
    (sa, ma, ea_, an, ae), (sb, mb, eb, bn, be) = out
    for a, b in zip(sa, sb):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    assert ma == mb and ea_ == eb and an == bn and ae == be
    _say(f"active nodes per level {an[jmin:jmax + 1]}")


def test_checkpoint_restart_is_bitwise(tmp_path):
    """wt_save after 3 adaptive steps, then 3 more steps, against a fresh grid that loads the
    checkpoint and takes the same 3 steps: identical states and masks; a checkpoint of another
    grid shape, or a file that is not a checkpoint, is refused and leaves the grid usable."""
    _say("checkpoint restart")
    jmin, jmax, eps = 4, 7, 5e-3
    path = str(tmp_path / "jet.ckpt")
    g = wt.Grid(jmin, jmax, 8)
    with g:
        x, m, t = g.coords(jmax)
        dh, u, Hd = _ic("jet", (x, m, t))
        g.set_params(mean_depth=Hd, precision=wt.WT_FP32_TENDENCY)
        g.set_state(jmax, dh, u)
        dt = g.suggest_dt(0.8)
        for _ in range(3):
            g.adapt(eps)
            g.step(dt)
        g.save(path)
        for _ in range(3):
            g.adapt(eps)
            g.step(dt)
        ref = [g.get_state(j) for j in range(jmin, jmax + 1)]
    h = wt.Grid(jmin, jmax, 8)
    with h:
        h.load(path)
        assert h.get_params().precision == wt.WT_FP32_TENDENCY and h.get_params().mean_depth == Hd
        for _ in range(3):
            h.adapt(eps)
            h.step(dt)
        got = [h.get_state(j) for j in range(jmin, jmax + 1)]
    for a, b in zip(ref, got):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    other = wt.Grid(jmin, jmax - 1, 8)
    with other:
        with pytest.raises(wt.WtError):
            other.load(path)
        junk = str(tmp_path / "junk.ckpt")
        open(junk, "wb").write(b"not a checkpoint")
        with pytest.raises(wt.WtError):
            other.load(junk)


@pytest.mark.parametrize("rk,prec", [(wt.WT_RK4, wt.WT_FP64), (wt.WT_SSPRK43, wt.WT_FP32_TENDENCY)])
def test_merged_phase_launches_equal_kernel_by_kernel(rk, prec):
    """The listed step with the launches of independent work merged (one launch per phase over
    all levels) gives bitwise the states and masks of one launch per kernel and level, across
    adapts that change the work lists and a change of dt."""
    jmin, jmax, eps = 4, 8, 5e-3
    runs = []
    for merged in (True, False):
        _say(f"merged phases={merged} rk={rk} precision={prec}")
        g = wt.Grid(jmin, jmax, 8)
        with g:
            x, m, t = g.coords(jmax)
            dh, u, Hd = inputs.jet(x, m, t)
            g.set_params(mean_depth=Hd, rk=rk, precision=prec)
            g.set_state(jmax, dh, u)
            g.set_step_phases(merged)
            dt = g.suggest_dt(0.8)
            for k in range(6):
                g.adapt(eps)
                g.step(dt if k != 3 else 0.5 * dt)
            g.step(dt)
            runs.append([g.get_state(j) for j in range(jmin, jmax + 1)])
    for s1, s2 in zip(*runs):
        for a, b in zip(s1, s2):
            assert np.array_equal(a, b)


def test_turbulence_adaptive_parity():
    """Rotating-turbulence start (random non-divergent flow peaked at degree 40, depth 1 km) on
    levels 3..6, eps 1e-2: adapt + RK4 step four times.  FP64 against the oracle: masks identical,
    fields within 1e-11 (rel L-inf), mass conserved; FP32 tendencies: the same run within 1e-5
    (rel L2 height) of the FP64 run, mass conserved."""
    _say("turbulence 3..6")
    H, g, dh, u, p = _pair(3, 6, "turb")
    dt = 60.0
    with g:
        g.set_state(6, dh, u)
        H.set_state(6, dh, u)
        m0 = None
        for s in range(4):
            g.adapt(1e-2)
            H.adapt(1e-2)
            if m0 is None:
                m0 = g.diagnostics()[0].mass
            g.step(dt)
            H.step(dt, p)
        worst = _compare_all(H, g, 1e-11)
        d, code = g.diagnostics()
        ref = g.get_state(6)[0]
    _say(f"FP64 worst rel L-inf vs oracle {worst:.2e}")
    assert code == wt.WT_OK
    assert abs(d.mass / m0 - 1) < 1e-13
    g = wt.Grid(3, 6, 8)
    with g:
        g.set_params(mean_depth=p.H, precision=wt.WT_FP32_TENDENCY)
        g.set_state(6, dh, u)
        m0 = None
        for s in range(4):
            g.adapt(1e-2)
            if m0 is None:
                m0 = g.diagnostics()[0].mass
            g.step(dt)
        d, code = g.diagnostics()
        got = g.get_state(6)[0]
    err = float(np.sqrt(((got - ref) ** 2).sum() / ((p.H + ref) ** 2).sum()))
    _say(f"FP32 tendencies: rel L2 height vs FP64 {err:.2e}")
    assert code == wt.WT_OK
    assert 0.0 < err < 1e-5
    assert abs(d.mass / m0 - 1) < 1e-13


def test_full_size_jet_levels_5_to_9():
    """The adaptive workload at full size (zonal jet + 120 m bump, levels 5..9, eps = 5e-3, RK4 at
    0.8 of the stable step), in the configuration the bench times, against the oracle's run
    stored by tests/golden/make_jet_l5_9_samples.py: after four rounds of adapt and step every
    level's node and edge masks are identical, the state at seeded samples of every level's
    active points is within 1e-11 of the level's maximum, and the jmin mass agrees to 1e-13."""
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "jet_l5_9_samples.npz"))
    jmin, jmax = int(ref["jmin"]), int(ref["jmax"])
    eps, dt = float(ref["eps"]), float(ref["dt"])
    _say(f"full size jet levels {jmin}..{jmax} eps={eps}")
    g = wt.Grid(jmin, jmax, 8)
    with g:
        x, m, t = g.coords(jmax)
        dh, u, depth = inputs.jet(x, m, t)
        g.set_params(mean_depth=depth, rk=wt.WT_RK4, precision=wt.WT_FP64)
        g.set_state(jmax, dh, u)
        assert abs(g.suggest_dt(0.8) / dt - 1) < 1e-12
        for _ in range(int(ref["rounds"])):
            g.adapt(eps)
            g.step(dt)
        d, code = g.diagnostics()
        states = {j: g.get_state(j) for j in range(jmin, jmax + 1)}
    assert code == wt.WT_OK
    for j, (a, b, na, ea) in states.items():
        assert np.array_equal(np.packbits(na.astype(bool)), ref[f"na{j}"]), f"node mask differs on level {j}"
        assert np.array_equal(np.packbits(ea.astype(bool)), ref[f"ea{j}"]), f"edge mask differs on level {j}"
        ni, ei = ref[f"ni{j}"], ref[f"ei{j}"]
        if ni.size:
            err = np.abs(a[ni] - ref[f"dh{j}"]).max() / float(ref[f"dhmax{j}"])
            assert err < 1e-11, (j, err)
            assert np.abs(a[na.astype(bool)]).max() == pytest.approx(float(ref[f"dhmax{j}"]), rel=1e-11)
        if ei.size:
            err = np.abs(b[ei] - ref[f"u{j}"]).max() / float(ref[f"umax{j}"])
            assert err < 1e-11, (j, err)
            assert np.abs(b[ea.astype(bool)]).max() == pytest.approx(float(ref[f"umax{j}"]), rel=1e-11)
    assert abs(d.mass / float(ref["mass"]) - 1) < 1e-13

"""GPU parity of the dense finest levels: the finest level of an adaptive grid run whole through
the masked lattice kernel (tendencies zero at inactive points, F, Q and B stored for the
restriction chain), the level below it (from level 6 up) its intermediates F, Q, B through the
kernel's intermediates-only form (its tendencies stay listed, after the restriction), the rims
round the lozenge corners through the listed kernels.  Against the FP64 oracle, against the
listed stage, and between the step's launch forms."""
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


def _ic(case, x, m, t):
    if case == "jet":
        return inputs.jet(x, m, t)
    if case == "turb":
        return inputs.turbulence(x, m, t)
    return inputs.tc2_perturbed(x, m, t, amplitude=300.0)


def _masked_launches(g):
    return g.kernel_time("trisk_lattice_masked")[1]


def _inter_launches(g):
    return g.kernel_time("trisk_lattice_inter")[1]


@pytest.mark.parametrize("case,jmin,jmax,eps,steps,rk", [("turb", 3, 6, 1e-2, 4, wt.WT_RK4),
                                                          ("tc2p", 4, 6, 1e-3, 12, wt.WT_RK4),
                                                          ("jet", 4, 7, 5e-3, 8, wt.WT_SSPRK43)])
def test_dense_finest_level_against_oracle(case, jmin, jmax, eps, steps, rk):
    """Adapt + step with the finest levels always dense: masks identical to the oracle's, every
    level within 1e-11 (rel L-inf), mass conserved to 1e-13, and the masked lattice kernel
    launched once per stage, its intermediates-only form too when the level below the finest is
    6 or more."""
    _say(f"dense finest level vs oracle: {case} {jmin}..{jmax} eps={eps} rk={rk}")
    H = Hierarchy(jmin, jmax)
    og = H.g[jmax]
    dh, u, Hd = _ic(case, og.xyz, og.e_mid, og.e_tan)
    p = trisk.Params(mean_depth=Hd)
    scheme = "rk4" if rk == wt.WT_RK4 else "ssprk43"
    g = wt.Grid(jmin, jmax, 8)
    with g:
        g.set_params(mean_depth=Hd, rk=rk)
        g.set_dense_levels(0.0)
        g.set_dense_min_tiles(0)
        g.timing(True)
        g.set_state(jmax, dh, u)
        H.set_state(jmax, dh, u)
        dt = 60.0 if case == "turb" else 0.8 * trisk.suggest_dt(og, dh, u, p, 1.0)
        m0 = None
        for _ in range(steps):
            g.adapt(eps)
            H.adapt(eps)
            if m0 is None:
                m0 = g.diagnostics()[0].mass
            g.step(dt)
            H.step(dt, p, scheme)
        worst = 0.0
        for j in H.levels:
            a, b, na, ea = H.get_state(j)
            x, y, gna, gea = g.get_state(j)
            assert np.array_equal(gna.astype(bool), na), f"node mask differs on level {j}"
            assert np.array_equal(gea.astype(bool), ea), f"edge mask differs on level {j}"
            worst = max(worst, _rel(x, a), _rel(y, b))
        d, code = g.diagnostics()
        launches, inter = _masked_launches(g), _inter_launches(g)
    _say(f"worst rel L-inf {worst:.2e}, masked lattice launches {launches}, intermediates-only {inter}")
    assert code == wt.WT_OK
    assert worst < 1e-11, worst
    assert abs(d.mass / m0 - 1) < 1e-13
    assert launches == 4 * steps
    assert inter == (4 * steps if jmax - 1 >= 6 else 0)


@pytest.mark.parametrize("rk,prec", [(wt.WT_RK4, wt.WT_FP64), (wt.WT_SSPRK43, wt.WT_FP32_TENDENCY)])
def test_dense_launch_forms_agree_bitwise(rk, prec):
    """With the finest level dense, the merged-phase step, the one-launch-per-kernel step and the
    stage over whole levels give bitwise the same states and masks (the dense level takes the
    same launches in all three), across adapts and a change of dt."""
    jmin, jmax, eps = 4, 7, 5e-3
    runs = []
    for merged, lists in ((True, True), (False, True), (True, False)):
        _say(f"dense launch forms: merged={merged} lists={lists} rk={rk} precision={prec}")
        g = wt.Grid(jmin, jmax, 8)
        with g:
            x, m, t = g.coords(jmax)
            dh, u, Hd = inputs.tc2_perturbed(x, m, t, amplitude=300.0)
            g.set_params(mean_depth=Hd, rk=rk, precision=prec)
            g.set_dense_levels(0.0)
            g.set_dense_min_tiles(0)
            g.set_step_phases(merged)
            g.set_work_lists(lists)
            g.set_state(jmax, dh, u)
            dt = g.suggest_dt(0.8)
            for k in range(5):
                g.adapt(eps)
                g.step(dt if k != 2 else 0.5 * dt)
            runs.append([g.get_state(j) for j in range(jmin, jmax + 1)])
    for other in runs[1:]:
        for s1, s2 in zip(runs[0], other):
            for a, b in zip(s1, s2):
                assert np.array_equal(a, b)


def test_dense_agrees_with_listed_stage_and_switches_by_density():
    """The same run with and without the dense finest level agrees to round-off (FP64, rel
    L-inf 1e-12 on every level, identical masks), the masked kernel running only the tiles that
    hold support points.  A threshold above the level's density keeps the listed stage (bitwise
    equal to dense off, no masked launch); 1.5 turns it off."""
    jmin, jmax, eps = 4, 7, 5e-3
    out = {}
    for mode in ("off", "on", "high", "above1"):
        _say(f"dense {mode}")
        g = wt.Grid(jmin, jmax, 8)
        with g:
            x, m, t = g.coords(jmax)
            dh, u, Hd = inputs.jet(x, m, t)
            g.set_params(mean_depth=Hd)
            g.set_dense_levels({"off": 2.0, "on": 0.0, "high": 0.99, "above1": 1.5}[mode])
            g.set_dense_min_tiles(0)
            g.timing(True)
            g.set_state(jmax, dh, u)
            dt = g.suggest_dt(0.8)
            for _ in range(5):
                g.adapt(eps)
                g.step(dt)
            out[mode] = ([g.get_state(j) for j in range(jmin, jmax + 1)], _masked_launches(g),
                         g.diagnostics()[0].active_nodes[jmax], wt.kernel_units(g, "trisk_lattice_masked"),
                         _inter_launches(g))
    n_fine = 10 * 4 ** jmax + 2
    tiles = wt.host_lattice_check(jmax)[0]
    _say(f"finest level active nodes {out['off'][2]} of {n_fine}; masked kernel ran {out['on'][3]} of "
         f"{tiles * 512 * 10} tile elements")
    assert out["off"][2] < 0.5 * n_fine
    # the masked kernel skips the tiles of each lozenge without support points
    assert 0 < out["on"][3] < tiles * 512 * 10 and out["on"][3] % 512 == 0
    assert out["on"][1] == 20 and out["off"][1] == 0 and out["high"][1] == 0 and out["above1"][1] == 0
    # level 6 below the finest: its intermediates through the lattice kernel when on
    assert out["on"][4] == 20 and out["off"][4] == 0 and out["high"][4] == 0 and out["above1"][4] == 0
    for mode in ("high", "above1"):
        for s1, s2 in zip(out["off"][0], out[mode][0]):
            for a, b in zip(s1, s2):
                assert np.array_equal(a, b)
    worst = 0.0
    for s1, s2 in zip(out["off"][0], out["on"][0]):
        assert np.array_equal(s1[2], s2[2]) and np.array_equal(s1[3], s2[3])
        worst = max(worst, _rel(s2[0], s1[0]), _rel(s2[1], s1[1]))
    _say(f"dense vs listed: worst rel L-inf {worst:.2e}")
    assert worst < 1e-12


@pytest.mark.parametrize("case,jmin,jmax,eps", [("turb", 3, 6, 1e-2), ("jet", 4, 7, 5e-3)])
def test_dense_fp32_close_to_fp64_oracle(case, jmin, jmax, eps):
    """FP32 tendencies with the dense finest levels (the turbulence start on levels 3..6; the jet on
    levels 4..7, where level 6 runs the intermediates-only form): rel L2 height error against the
    FP64 oracle below 1e-5 of the depth on the finest level, mass conserved."""
    _say(f"dense fp32 {case} {jmin}..{jmax}")
    H = Hierarchy(jmin, jmax)
    og = H.g[jmax]
    dh, u, Hd = _ic(case, og.xyz, og.e_mid, og.e_tan)
    p = trisk.Params(mean_depth=Hd)
    g = wt.Grid(jmin, jmax, 8)
    with g:
        g.set_params(mean_depth=Hd, precision=wt.WT_FP32_TENDENCY)
        g.set_dense_levels(0.0)
        g.set_dense_min_tiles(0)
        g.timing(True)
        g.set_state(jmax, dh, u)
        H.set_state(jmax, dh, u)
        dt = 60.0 if case == "turb" else 0.8 * trisk.suggest_dt(og, dh, u, p, 1.0)
        m0 = None
        for _ in range(4):
            g.adapt(eps)
            H.adapt(eps)
            if m0 is None:
                m0 = g.diagnostics()[0].mass
            g.step(dt)
            H.step(dt, p)
        x = g.get_state(jmax)[0]
        d, code = g.diagnostics()
        inter = _inter_launches(g)
    a = H.get_state(jmax)[0]
    A = H.A[jmax]
    err = float(np.sqrt((A * (x - a) ** 2).sum() / (A * (Hd + a) ** 2).sum()))
    _say(f"dense fp32: rel L2 height vs FP64 oracle {err:.2e}, intermediates-only launches {inter}")
    assert code == wt.WT_OK
    assert err < 1e-5
    assert abs(d.mass / m0 - 1) < 1e-13
    assert inter == (16 if jmax - 1 >= 6 else 0)


def test_dense_levels_argument_errors():
    """A negative or non-finite fraction and a finest level below 6 are refused; other forms
    (viscous) keep the listed stage without error."""
    g = wt.Grid(3, 5, 8)
    with g:
        with pytest.raises(wt.WtError):
            g.set_dense_levels(0.0)
        g.set_dense_levels(2.0)
    g = wt.Grid(4, 6, 8)
    with g:
        for bad in (-0.5, float("nan"), float("inf")):
            with pytest.raises(wt.WtError):
                g.set_dense_levels(bad)
        with pytest.raises(wt.WtError):
            g.set_dense_min_tiles(-2)
        x, m, t = g.coords(6)
        dh, u, Hd = inputs.tc2_perturbed(x, m, t, amplitude=300.0)
        g.set_params(mean_depth=Hd, viscosity=1e5)
        g.set_dense_levels(0.0)
        g.timing(True)
        g.set_state(6, dh, u)
        g.adapt(1e-3)
        g.step(100.0)
        assert _masked_launches(g) == 0 and _inter_launches(g) == 0


def test_dense_full_size_turbulence_agrees_with_listed():
    """The rotating-turbulence configuration at full size (levels 6..10, eps 1e-2), 12 adapt +
    RK4 steps with the finest level always dense (the masked kernel over the flagged tiles, as
    level 10 fills from empty) and with every level listed: masks agree
    except at points whose significance sits on the threshold (at most 1e-6 of the points), and
    the fields agree to 1e-10 relative L-inf on every level at points active in both runs."""
    jmin, jmax, eps, steps = 6, 10, 1e-2, 12
    runs = []
    for dense in (0.0, 2.0):
        _say(f"full-size turbulence, dense_min={dense}")
        g = wt.Grid(jmin, jmax, 8)
        with g:
            x, m, t = g.coords(jmax)
            dh, u, Hd = inputs.turbulence(x, m, t, device="cuda")
            del x, m, t
            g.set_params(mean_depth=Hd)
            g.set_dense_levels(dense)
            g.timing(True)
            g.set_state(jmax, dh, u)
            dt = g.suggest_dt(0.8)
            for _ in range(steps):
                g.adapt(eps)
                g.step(dt)
            d, code = g.diagnostics()
            assert code == wt.WT_OK
            runs.append(([g.get_state(j) for j in range(jmin, jmax + 1)], _masked_launches(g), d.mass,
                         _inter_launches(g)))
    (sa, la, ma, ia), (sb, lb, mb, ib) = runs
    _say(f"intermediates-only launches (level 9): {ia}")
    assert la > 0 and ia > 0 and lb == 0 and ib == 0
    worst, flips, total = 0.0, 0, 0
    for (x, y, na, ea), (x2, y2, na2, ea2) in zip(sa, sb):
        flips += int((na != na2).sum()) + int((ea != ea2).sum())
        total += na.size + ea.size
        both_n, both_e = (na > 0) & (na2 > 0), (ea > 0) & (ea2 > 0)
        worst = max(worst, np.abs(x - x2)[both_n].max() / np.abs(x2).max(),
                    np.abs(y - y2)[both_e].max() / np.abs(y2).max())
    _say(f"masked launches {la}, mask differences {flips} of {total}, worst rel L-inf {worst:.2e}")
    assert flips <= 1e-6 * total
    assert worst < 1e-10
    assert abs(ma / mb - 1) < 1e-13

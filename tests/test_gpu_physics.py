"""GPU parity of the dissipative form, the advection form, the regime thresholds and the
implicit maximum level (Sec. 3.1, Sec. 6.1), of the single-precision transforms, of the device
allocator hook and of a precision change after a checkpoint load: HIP library through the C ABI
against the FP64 oracle on the same seeded inputs."""
import os
import sys
import tempfile

import numpy as np
import pytest

from oracle import trisk
from oracle.grid import Grid
from oracle.multiscale import Hierarchy, regime_thresholds
from paper_1404_0405_amd import inputs, wt

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


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


@pytest.mark.parametrize("J", [3, 6])
def test_viscous_tendencies_uniform(J):
    """Dissipative form (Sec. 3.1) on a uniform level: tendencies within 1e-11 of the oracle's
    (level 6 would take the lattice kernel; the viscous form runs the table-driven one)."""
    _say(f"viscous tendencies J={J}")
    og = Grid(J)
    dh, u, Hd = inputs.tc2_perturbed(og.xyz, og.e_mid, og.e_tan, amplitude=300.0)
    p = trisk.Params(mean_depth=Hd, nu=1e5 * 4.0 ** (6 - J))
    rdh, rdu = trisk.tendencies(og, dh, u, p)
    g = wt.Grid(J, J, 8)
    with g:
        g.set_params(mean_depth=Hd, viscosity=p.nu)
        g.set_state(J, dh, u)
        a, b = g.tendency(J)
    assert _rel(a, rdh) < 1e-11 and _rel(b, rdu) < 1e-11, (_rel(a, rdh), _rel(b, rdu))


def test_advection_tendencies_uniform():
    """Advection form (Sec. 6.1): height tendency within 1e-11, velocity tendency exactly 0."""
    _say("advection tendencies J=5")
    og = Grid(5)
    dh, u, H0 = inputs.tc1(og.xyz, og.e_mid, og.e_tan, alpha=0.3)
    p = trisk.Params(mean_depth=H0, adv=True)
    rdh, _ = trisk.tendencies(og, dh, u, p)
    g = wt.Grid(5, 5, 8)
    with g:
        g.set_params(mean_depth=H0, equations=wt.WT_ADVECTION)
        g.set_state(5, dh, u)
        a, b = g.tendency(5)
        assert abs(g.suggest_dt(0.8) / trisk.suggest_dt(og, dh, u, p, 0.8) - 1) < 1e-12
    assert _rel(a, rdh) < 1e-11
    assert np.abs(b).max() == 0.0


@pytest.mark.parametrize("scheme", ["rk4", "ssprk43"])
def test_viscous_adaptive_jet(scheme):
    """Viscous jet on levels 2..5 (nu = 2e5 m^2/s), eps = 1e-2, 12 rounds of adapt + step: masks
    identical to the oracle's, states within 1e-11, mass conserved."""
    _say(f"viscous adaptive jet {scheme}")
    H = Hierarchy(2, 5)
    og = H.g[5]
    dh, u, Hd = inputs.jet(og.xyz, og.e_mid, og.e_tan)
    p = trisk.Params(mean_depth=Hd, nu=2e5)
    g = wt.Grid(2, 5, 8)
    with g:
        g.set_params(mean_depth=Hd, viscosity=p.nu, rk=wt.WT_RK4 if scheme == "rk4" else wt.WT_SSPRK43)
        g.set_state(5, dh, u)
        H.set_state(5, dh, u)
        m0 = g.diagnostics()[0].mass
        for _ in range(12):
            g.adapt(1e-2)
            H.adapt(1e-2)
            g.step(600.0)
            H.step(600.0, p, scheme)
        w = _compare_all(H, g, 1e-11)
        d, _ = g.diagnostics()
        _say(f"  worst rel Linf {w:.2e}")
    assert abs(d.mass / m0 - 1) < 1e-13


@pytest.mark.parametrize("bell", ["cosine", "smooth"])
def test_tc1_adaptive(bell):
    """Advection test 1 on levels 2..5, eps = 2e-2, 30 rounds of adapt + RK4 step at CFL 0.8:
    masks identical, height within 1e-11 of the oracle, velocity of the active points unchanged
    by the steps, mass conserved, and the finest active level reported as the oracle's."""
    _say(f"tc1 adaptive {bell}")
    H = Hierarchy(2, 5)
    og = H.g[5]
    dh, u, H0 = inputs.tc1(og.xyz, og.e_mid, og.e_tan, bell=bell, alpha=0.5)
    p = trisk.Params(mean_depth=H0, adv=True)
    g = wt.Grid(2, 5, 8)
    with g:
        g.set_params(mean_depth=H0, equations=wt.WT_ADVECTION)
        g.set_state(5, dh, u)
        H.set_state(5, dh, u)
        dt = trisk.suggest_dt(og, dh, u, p, 0.8)
        m0 = g.diagnostics()[0].mass
        for _ in range(30):
            g.adapt(2e-2)
            H.adapt(2e-2)
            before = [g.get_state(j)[1] for j in H.levels]
            g.step(dt)
            H.step(dt, p)
            for j, ub in zip(H.levels, before):
                x, y, na, ea = g.get_state(j)
                assert np.array_equal(y[ea.astype(bool)], ub[ea.astype(bool)])
        _compare_all(H, g, 1e-11)
        d, _ = g.diagnostics()
        assert d.finest_level == H.finest_level()
    assert abs(d.mass / m0 - 1) < 1e-13


def test_regime_thresholds_and_finest_level():
    """Quasi-geostrophic thresholds (Sec. 3.1) on the jet, levels 2..6 with jmax as a cap: the
    adapt selects the oracle's masks, and the reported finest level is the oracle's."""
    _say("regime thresholds")
    H = Hierarchy(2, 6)
    og = H.g[6]
    dh, u, Hd = inputs.jet(og.xyz, og.e_mid, og.e_tan)
    p = trisk.Params(mean_depth=Hd)
    U, L, f = 80.0, 1.0e6, 1.0e-4
    g = wt.Grid(2, 6, 8)
    with g:
        g.set_params(mean_depth=Hd, threshold=wt.WT_THR_QG, scale_u=U, scale_l=L, scale_f=f)
        g.set_state(6, dh, u)
        H.set_state(6, dh, u)
        for eps in (5e-2, 5e-2, 3e-2):
            thr = regime_thresholds(eps, "qg", U, inputs.GRAVITY, L=L, f=f)
            g.adapt(eps)
            H.adapt(eps, thresholds=thr)
            g.step(300.0)
            H.step(300.0, p)
        _compare_all(H, g, 1e-11)
        d, _ = g.diagnostics()
        _say(f"  finest level {d.finest_level} (oracle {H.finest_level()}), cap 6")
        assert d.finest_level == H.finest_level()


def test_fp32_transforms_error_against_the_oracle():
    """Single-precision tendencies and transform predictions (FP64 state, F, R_h, mass): after
    adapt + 20 RK4 steps of the jet on levels 3..6 the height and velocity stay close to the FP64
    oracle (relative L2 of the height perturbation and of the velocity), mass is conserved, and
    the FP64 grid of the same run is much closer still."""
    _say("fp32 transforms vs oracle")
    H = Hierarchy(3, 6)
    og = H.g[6]
    dh, u, Hd = inputs.jet(og.xyz, og.e_mid, og.e_tan)
    p = trisk.Params(mean_depth=Hd)
    H.set_state(6, dh, u)
    dt = 0.8 * trisk.suggest_dt(og, dh, u, p, 1.0)
    for _ in range(20):
        H.adapt(5e-3)
        H.step(dt, p)
    ra, rb, _, _ = H.get_state(6)
    A = H.A[6]
    w = og.l_e * og.d_e
    errs = {}
    for prec in (wt.WT_FP64, wt.WT_FP32_TENDENCY):
        g = wt.Grid(3, 6, 8)
        with g:
            g.set_params(mean_depth=Hd, precision=prec)
            g.set_state(6, dh, u)
            m0 = g.diagnostics()[0].mass
            for _ in range(20):
                g.adapt(5e-3)
                g.step(dt)
            x, y, _, _ = g.get_state(6)
            d, _ = g.diagnostics()
            assert abs(d.mass / m0 - 1) < 1e-13
        eh = np.sqrt((A * (x - ra) ** 2).sum() / (A * ra ** 2).sum())
        ehd = np.sqrt((A * (x - ra) ** 2).sum() / (A * (Hd + ra) ** 2).sum())
        eu = np.sqrt((w * (y - rb) ** 2).sum() / (w * rb ** 2).sum())
        errs[prec] = (eh, ehd, eu)
        _say(f"  precision {prec}: rel L2 dh {eh:.3e} (of the depth {ehd:.3e}), u {eu:.3e}")
    assert errs[wt.WT_FP32_TENDENCY][0] < 1e-4 and errs[wt.WT_FP32_TENDENCY][2] < 1e-4
    assert errs[wt.WT_FP64][0] < 1e-11 and errs[wt.WT_FP64][2] < 1e-11


def test_allocator_hook_receives_every_buffer():
    """Grids created after routing the allocator through PyTorch's caching allocator own no
    hipMalloc buffer; their states equal bitwise those of a grid on hipMalloc."""
    import torch
    _say("allocator hook")
    out = []
    for hook in (True, False):
        if hook:
            wt.use_torch_allocator()
        try:
            before = torch.cuda.memory_allocated()
            g = wt.Grid(2, 5, 8)
            with g:
                x, m, t = g.coords(5)
                dh, u, Hd = inputs.jet(x, m, t)
                g.set_params(mean_depth=Hd, viscosity=1e5)
                g.set_state(5, dh, u)
                for _ in range(3):
                    g.adapt(1e-2)
                    g.step(400.0)
                st = g.alloc_stats()
                grown = torch.cuda.memory_allocated() - before
                out.append([g.get_state(j)[:2] for j in range(2, 6)])
        finally:
            if hook:
                wt.use_hip_allocator()
        _say(f"  hook={hook}: {st}, torch grew by {grown} bytes")
        if hook:
            assert st["direct"][0] == 0 and st["hook"][0] > 0
            assert grown >= st["hook"][1]
        else:
            assert st["hook"][0] == 0 and st["direct"][0] > 0
    for (a, b), (c, d) in zip(out[0], out[1]):
        assert np.array_equal(a, c) and np.array_equal(b, d)


def test_precision_switch_after_checkpoint_load():
    """A checkpoint stores the saved grid's parameters; switching the precision after wt_load
    must take effect: FP32 and FP64 continuations from the same checkpoint differ (and each
    equals a second run of itself bitwise)."""
    _say("precision after load")
    jmin, jmax = 3, 6
    g = wt.Grid(jmin, jmax, 8)
    path = os.path.join(tempfile.mkdtemp(), "p.ckpt")
    with g:
        x, m, t = g.coords(jmax)
        dh, u, Hd = inputs.jet(x, m, t)
        g.set_params(mean_depth=Hd)
        g.set_state(jmax, dh, u)
        dt = g.suggest_dt(0.8)
        for _ in range(3):
            g.adapt(5e-3)
            g.step(dt)
        g.save(path)
    res = {}
    for prec in (wt.WT_FP32_TENDENCY, wt.WT_FP64, wt.WT_FP32_TENDENCY):
        h = wt.Grid(jmin, jmax, 8)
        with h:
            h.load(path)
            h.set_params(precision=prec)
            assert h.get_params().precision == prec
            for _ in range(3):
                h.adapt(5e-3)
                h.step(dt)
            a = h.get_state(jmax)[0]
        if prec in res:
            assert np.array_equal(res[prec], a)
        res[prec] = a
    diff = np.abs(res[wt.WT_FP32_TENDENCY] - res[wt.WT_FP64]).max()
    _say(f"  max |fp32 - fp64| after 3 steps: {diff:.3e} m")
    assert diff > 0.0
    os.remove(path)

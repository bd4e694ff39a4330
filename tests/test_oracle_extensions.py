"""Pins of the oracle's dissipative form and advection form (Sec. 3.1, Sec. 6.1), the regime
thresholds and the implicit maximum level (Sec. 3.1), checked against closed forms, exact
identities and spherical-harmonic eigenvalues (CPU only)."""
import math

import numpy as np
import pytest

from oracle import trisk
from oracle.multiscale import Hierarchy, regime_thresholds
from paper_1404_0405_amd import inputs

A = inputs.EARTH_RADIUS


def _y3(xyz):
    """One real spherical harmonic of degree 3 (eigenvalue -12/a^2 of the Laplacian)."""
    co = np.zeros((4, 7))
    co[3, 3 + 2] = 1.0
    return inputs.real_sph_harm_sum(xyz, co, 3)


def _quotients(g, curl_adjoint=trisk.curl_adjoint):
    """Rayleigh quotients a^2 <f, L f> / <f, f> of the scalar Laplacian on Y_3 at the nodes and
    of the velocity dissipation operator on the discrete gradient of Y_3 (curl-free) and on
    the discrete perpendicular gradient of Y_3 at the triangle centres (divergence-free)."""
    Y = _y3(g.xyz)
    Yv = _y3(g.t_cc)
    w = g.l_e * g.d_e
    Ls = trisk.laplacian(g, Y)
    out = {"scalar": (g.A_i * Y * Ls).sum() / (g.A_i * Y * Y).sum() * A * A}
    for name, u in (("div", trisk.gradient(g, Y)), ("rot", curl_adjoint(g, Yv))):
        V = trisk.gradient(g, trisk.divergence(g, u)) - curl_adjoint(g, trisk.curl(g, u))
        out[name] = (w * u * V).sum() / (w * u * u).sum() * A * A
    return out


def test_dissipation_operators_have_the_sphere_eigenvalue(oracle_grid):
    """The Laplacian of Y_l is -l(l+1)/a^2 Y_l; on vector fields the operator
    grad div - grad^perp curl (Sec. 3.1) has the same eigenvalue on grad Y_l and on k x grad Y_l.
    The energy-norm Rayleigh quotients converge to -12 (pointwise values do not converge on the
    plain bisection grid, Sec. 3.2); the curl-free and scalar ones at second order."""
    q4, q5 = _quotients(oracle_grid(4)), _quotients(oracle_grid(5))
    for k in ("scalar", "div", "rot"):
        assert abs(q5[k] + 12.0) < 0.02 * 12.0, (k, q5[k])
    for k in ("scalar", "div"):
        assert abs(q5[k] + 12.0) < abs(q4[k] + 12.0) / 3.0, (k, q4[k], q5[k])


def test_planted_sign_of_curl_adjoint_is_caught(oracle_grid):
    """A grad^perp with the wrong orientation turns the enstrophy dissipation into growth."""
    q = _quotients(oracle_grid(4), curl_adjoint=lambda g, z: -trisk.curl_adjoint(g, z))
    assert q["rot"] > 10.0


def test_dissipation_adjointness_identities(oracle_grid):
    """div is minus the adjoint of grad and grad^perp is the adjoint of curl, so for any fields
    sum A phi lap(phi) = -sum l d (grad phi)^2 and
    sum l d u . L(u) = -sum A (div u)^2 - sum A_v (curl u)^2; both dissipate, and the height
    dissipation conserves mass (sum A lap = 0)."""
    g = oracle_grid(3)
    dh, u = inputs.random_state(g.N, g.E, 21)
    w = g.l_e * g.d_e
    lhs = (g.A_i * dh * trisk.laplacian(g, dh)).sum()
    rhs = -(w * trisk.gradient(g, dh) ** 2).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)
    lv = (w * u * trisk.vector_laplacian(g, u)).sum()
    rv = -(g.A_i * trisk.divergence(g, u) ** 2).sum() - (g.A_v * trisk.curl(g, u) ** 2).sum()
    assert abs(lv - rv) < 1e-12 * abs(rv)
    assert abs((g.A_i * trisk.laplacian(g, dh)).sum()) < 1e-12 * np.abs(g.A_i * trisk.laplacian(g, dh)).sum()


def test_viscous_multilevel_full_masks_equal_uniform():
    """With every point active the multilevel viscous tendencies on jmax are the uniform ones
    (the dissipative terms ride on F, B and qF^perp through the restriction), and the viscous
    adaptive run conserves mass."""
    H = Hierarchy(2, 4)
    g = H.g[4]
    dh, u, Hd = inputs.tc2_perturbed(g.xyz, g.e_mid, g.e_tan, amplitude=300.0)
    p = trisk.Params(mean_depth=Hd, nu=2e5)
    H.set_state(4, dh, u)
    ddh, du = H.tendencies(H.dh, H.u, p)
    rdh, rdu = trisk.tendencies(g, dh, u, p)
    assert np.abs(ddh[4] - rdh).max() < 1e-11 * np.abs(rdh).max()
    assert np.abs(du[4] - rdu).max() < 1e-11 * np.abs(rdu).max()
    # the dissipation changes the tendencies by much more than that
    p0 = trisk.Params(mean_depth=Hd)
    r0h, r0u = trisk.tendencies(g, dh, u, p0)
    assert np.abs(r0h - rdh).max() > 1e-4 * np.abs(rdh).max()
    H.adapt(1e-2)
    m0 = H.mass(p)
    for _ in range(4):
        H.step(600.0, p)
        H.adapt(1e-2)
    assert abs(H.mass(p) / m0 - 1) < 1e-14


def test_viscosity_damps_a_height_wave(oracle_grid):
    """Without rotation and flow, nu div grad alone on a small Y_3 height wave in a deep layer:
    the wave's energy decays, faster with larger nu (time-step limited by gravity waves)."""
    g = oracle_grid(3)
    gr = inputs.GRAVITY
    dh0 = _y3(g.xyz)
    dh0 = dh0 / np.abs(dh0).max()
    ens = []
    for nu in (0.0, 5e5, 2e6):
        p = trisk.Params(mean_depth=1000.0, nu=nu)
        p.g = gr
        dh, u = dh0.copy(), np.zeros(g.E)
        for _ in range(40):
            dh, u = trisk.step(g, dh, u, 200.0, p)
        ens.append((g.A_i * dh * dh).sum() * gr + (g.l_e * g.d_e * u * u).sum() * 1000.0)
    assert ens[2] < ens[1] < ens[0]


# ---------------------------------------------------------------- advection (Sec. 6.1)
def _tc1_run(jmin, jmax, eps, days, bell="cosine"):
    H = Hierarchy(jmin, jmax)
    g = H.g[jmax]
    dh, u, H0 = inputs.tc1(g.xyz, g.e_mid, g.e_tan, bell=bell)
    p = trisk.Params(mean_depth=H0, adv=True)
    H.set_state(jmax, dh, u)
    dt = trisk.suggest_dt(g, dh, u, p, 0.8)
    T = days * 86400.0
    n = int(math.ceil(T / dt))
    dt = T / n
    m0 = H.mass(p)
    for _ in range(n):
        if eps is not None:
            H.adapt(eps)
        H.step(dt, p)
    x, y, _, _ = H.get_state(jmax)
    return H, g, p, x, y, u, m0


def test_tc1_advection_converges_to_the_rotated_bell():
    """Test 1 (Sec. 6.1): after a quarter rotation (3 days) the uniform solution approaches the
    closed-form rotated cosine bell; the error falls by >= 2.5x from level 5 to 6 (second order
    is 4x), mass is conserved and the velocity does not change."""
    errs = []
    for J in (5, 6):
        H, g, p, x, y, u, m0 = _tc1_run(J, J, None, 3.0)
        exact = inputs.tc1_bell(g.xyz, t=3 * 86400.0)
        errs.append(math.sqrt((g.A_i * (x - exact) ** 2).sum() / (g.A_i * exact ** 2).sum()))
        assert abs(H.mass(p) / m0 - 1) < 1e-14
        assert np.array_equal(y, u)
    assert errs[0] / errs[1] > 2.5, errs
    assert errs[1] < 0.1, errs


def test_tc1_adaptive_error_controlled_by_eps():
    """Adaptive test 1 on levels 2..5: the difference from the uniform level-5 run falls with eps
    (error controlled by the threshold), is at most C eps with C < 20, and mass is conserved."""
    _, g, _, xu, _, _, _ = _tc1_run(5, 5, None, 1.5)
    diffs = []
    for eps in (4e-2, 1e-2):
        H, g, p, x, _, _, m0 = _tc1_run(2, 5, eps, 1.5)
        d = np.abs(x - xu).max() / np.abs(xu).max()
        diffs.append(d)
        assert d < 20 * eps, (eps, d)
        assert abs(H.mass(p) / m0 - 1) < 1e-14
    assert diffs[1] < diffs[0], diffs


def test_finest_level_set_by_eps():
    """Sec. 3.1: with jmax as a cap the thresholds choose the maximum level; it does not grow
    when eps grows, and eps = 0 fills every level."""
    H = Hierarchy(2, 6)
    g = H.g[6]
    dh, u, _ = inputs.tc1(g.xyz, g.e_mid, g.e_tan)
    finest = []
    for eps in (0.0, 3e-3, 3e-2, 2e-1):
        H.set_state(6, dh, u)
        H.adapt(eps)
        finest.append(H.finest_level())
    assert finest[0] == 6
    assert all(a >= b for a, b in zip(finest, finest[1:])), finest
    assert finest[-1] < 6, finest


# ---------------------------------------------------------------- regime thresholds (Sec. 3.1)
def test_qg_thresholds_scale_like_a_balanced_flow(oracle_grid):
    """In geostrophic balance g dh ~ f U L, so the height/velocity threshold ratio of the
    quasi-geostrophic regime, f L / g, must match max|dh| / max|u| of the balanced test-2 flow
    with f = 2 Omega and L = a/2 (to the few per cent of its u0^2/2 term); the reading with the
    printed names (ratio g / (f L)) or without the division by g misses it by orders."""
    g = oracle_grid(3)
    dh, u, Hd = inputs.tc2(g.xyz, g.e_mid, g.e_tan)
    U = np.abs(u).max()
    eh, eu = regime_thresholds(1e-2, "qg", U, inputs.GRAVITY, L=A / 2, f=2 * inputs.OMEGA)
    ratio = (eh / eu) / (np.abs(dh).max() / U)
    assert 0.9 < ratio < 1.1, ratio
    # eps^(3/2) scaling and the inertia-gravity pair: eps_h / eps_u = c / g, the height / velocity
    # ratio of a gravity wave on depth H (dh = (H / c) u)
    eh2, eu2 = regime_thresholds(4e-2, "qg", U, inputs.GRAVITY, L=A / 2, f=2 * inputs.OMEGA)
    assert abs(eu2 / eu - 8.0) < 1e-12 and abs(eh2 / eh - 8.0) < 1e-12
    eh3, eu3 = regime_thresholds(1e-2, "ig", U, inputs.GRAVITY, H=Hd)
    c = math.sqrt(inputs.GRAVITY * Hd)
    assert abs((eh3 / eu3) / (Hd / c) - 1.0) < 1e-12


def test_adapt_with_regime_thresholds():
    """The adapt takes absolute thresholds: masks are monotone in them and mass is conserved."""
    H = Hierarchy(2, 5)
    g = H.g[5]
    dh, u, Hd = inputs.jet(g.xyz, g.e_mid, g.e_tan)
    p = trisk.Params(mean_depth=Hd)
    counts = []
    for eps in (2e-2, 8e-2):
        H.set_state(5, dh, u)
        thr = regime_thresholds(eps, "qg", 80.0, inputs.GRAVITY, L=1e6, f=1e-4)
        eh, eu = H.adapt(eps, thresholds=thr)
        assert (eh, eu) == thr
        counts.append(sum(int(H.node_act[j].sum()) for j in H.levels))
    assert counts[1] < counts[0]
    m0 = H.mass(p)
    for _ in range(3):
        H.step(300.0, p)
        H.adapt(8e-2, thresholds=thr)
    assert abs(H.mass(p) / m0 - 1) < 1e-14

"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin catches each one.
This shows the pins constrain the oracle rather than restate it."""
import math

import numpy as np

from oracle import trisk
from paper_1404_0405_amd import inputs


def _tc2_day_error(g, tend):
    p = trisk.Params()
    dh0, u0, p.H = inputs.tc2(g.xyz, g.e_mid, g.e_tan)
    nst = 66
    dt = 86400.0 / nst
    rhs = lambda y: tend(g, y[0], y[1], p)  # noqa: E731
    y = (dh0, u0)
    for _ in range(nst):
        y = trisk.rk4_step(rhs, y, dt)
    return math.sqrt((g.A_i * (y[0] - dh0) ** 2).sum() / (g.A_i * dh0 ** 2).sum())


def _energy_residual(g, tend):
    p = trisk.Params()
    dh, u = inputs.random_state(g.N, g.E, 11)
    ddh, du = tend(g, dh, u, p)
    h = p.H + dh
    _, F = trisk.edge_quantities(g, dh, u, p)
    K = trisk.kinetic_energy(g, u)
    scale = np.abs(g.A_i * (p.g * h + K) * ddh).sum() + np.abs(g.l_e * g.d_e * F * du).sum()
    return abs(trisk.energy_rate(g, dh, u, ddh, du, p)) / scale


def test_sign_of_coriolis_term_is_pinned(oracle_grid):
    g = oracle_grid(3)
    good = _tc2_day_error(g, trisk.tendencies)

    def flipped(g, dh, u, p):
        _, F = trisk.edge_quantities(g, dh, u, p)
        B = p.g * dh + trisk.kinetic_energy(g, u)
        Q = trisk.perp_pv_flux(g, F, trisk.vertex_pv(g, dh, u, p))
        return -trisk.divergence(g, F), +Q - trisk.gradient(g, B)
    assert _tc2_day_error(g, flipped) > 20 * good


def test_dropped_kinetic_energy_is_pinned(oracle_grid):
    g = oracle_grid(3)
    assert _energy_residual(g, trisk.tendencies) < 1e-13

    def no_K(g, dh, u, p):
        _, F = trisk.edge_quantities(g, dh, u, p)
        Q = trisk.perp_pv_flux(g, F, trisk.vertex_pv(g, dh, u, p))
        return -trisk.divergence(g, F), -Q - trisk.gradient(g, p.g * dh)
    assert _energy_residual(g, no_K) > 1e-6


def test_transposed_weights_are_pinned(oracle_grid):
    """Using w_{e',e} in place of w_{e,e'} reverses the perpendicular flux: TC2 breaks."""
    g = oracle_grid(3)
    good = _tc2_day_error(g, trisk.tendencies)
    saved = g.w.copy()
    try:
        g.w = -saved   # antisymmetry: the transpose is the negative
        bad = _tc2_day_error(g, trisk.tendencies)
    finally:
        g.w = saved
    assert bad > 20 * good


def test_wrong_vertex_height_weights_are_pinned(oracle_grid):
    """Kite/cell fractions in place of kite/triangle fractions for h_v break h_v of a constant."""
    g = oracle_grid(3)
    h = np.full(g.N, 1234.0)
    good = (g.R_iv * h[g.t_nodes]).sum(1)
    assert np.allclose(good, 1234.0, rtol=1e-14)
    rho = g.t_kite / g.A_i[g.t_nodes]
    bad = (rho * h[g.t_nodes]).sum(1)
    assert np.abs(bad - 1234.0).max() > 100.0


def test_wrong_flux_length_is_pinned(oracle_grid):
    """Using d_e in place of l_e in the divergence breaks the energy identity."""
    g = oracle_grid(3)

    def bad_div(g, dh, u, p):
        _, F = trisk.edge_quantities(g, dh, u, p)
        ce = np.maximum(g.c_edges, 0)
        div = (np.where(g.c_edges >= 0, g.c_signs * g.d_e[ce] * F[ce], 0.0)).sum(1) / g.A_i
        B = p.g * dh + trisk.kinetic_energy(g, u)
        Q = trisk.perp_pv_flux(g, F, trisk.vertex_pv(g, dh, u, p))
        return -div, -Q - trisk.gradient(g, B)
    assert _energy_residual(g, bad_div) > 1e-3

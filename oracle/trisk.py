"""Oracle: TRiSK tendencies of the rotating shallow-water equations, time schemes, diagnostics.

TEST INFRASTRUCTURE ONLY (see ``oracle/grid.py``).

* Eqs. (height) and (velo), Sec. 3.1: d(dh)/dt = -div F,  du/dt = -q F^perp - grad B, with
  F = h u, h = H + dh (no topography), B = g dh + K, K = |u|^2/2, q = (curl u + f)/h, and the
  energy-conserving qF^perp.
* Sec. 3.1 (time discretisation): four-stage third-order SSP Runge-Kutta; classical RK4 is
  provided as well.
* Sec. 7.2: total energy E = 1/2 int g h (g h + |u|^2) dS - 1/2 c^4 A_S, c^2 = (g/A_S) int h dS.
* Sec. 4.1 (mass conservation of the height restriction): mass  sum_k A_k h_k.
* Sec. 3.1, dissipative form: nu div grad (dh) added to the height tendency and
  nu (grad div u - grad^perp curl u) to the velocity tendency.
* Sec. 6.1: advection of the height by a prescribed, time-independent velocity (the velocity
  equation is dropped; the thickness flux is h u).
"""
from __future__ import annotations

import numpy as np

from .grid import GRAVITY


class Params:
    """g, mean depth H, viscosity nu (0: inviscid) and adv (True: advection of the height alone)."""

    def __init__(self, gravity=GRAVITY, mean_depth=2.94e4 / GRAVITY, nu=0.0, adv=False):
        self.g = gravity
        self.H = mean_depth
        self.nu = nu
        self.adv = adv


def edge_quantities(g, dh, u, p):
    """h_e = average of the two cells, F_e = h_e u_e."""
    h = p.H + dh
    he = 0.5 * (h[g.e_nodes[:, 0]] + h[g.e_nodes[:, 1]])
    return he, he * u


def kinetic_energy(g, u):
    """K_i = (1/A_i) sum_{e in i} (l_e d_e / 4) u_e^2."""
    ce = np.maximum(g.c_edges, 0)
    coef = np.where(g.c_edges >= 0, g.l_e[ce] * g.d_e[ce] / 4.0, 0.0)
    return (coef * u[ce] ** 2).sum(1) / g.A_i


def divergence(g, F):
    """(div F)_i = (1/A_i) sum_{e in i} n_{e,i} l_e F_e."""
    ce = np.maximum(g.c_edges, 0)
    return (np.where(g.c_edges >= 0, g.c_signs * g.l_e[ce] * F[ce], 0.0)).sum(1) / g.A_i


def gradient(g, B):
    """(grad B)_e = (B_{c2} - B_{c1}) / d_e, u_e pointing from c1 to c2."""
    return (B[g.e_nodes[:, 1]] - B[g.e_nodes[:, 0]]) / g.d_e


def curl(g, u):
    """zeta_v = (1/A_v) sum_{e in v} t_{e,v} d_e u_e (circulation around the triangle)."""
    return (g.t_signs * g.d_e[g.t_edges] * u[g.t_edges]).sum(1) / g.A_v


def curl_adjoint(g, zeta):
    """grad^perp of a dual-vertex field: the adjoint of `curl` for the inner products
    sum_v A_v zeta_v eta_v and sum_e l_e d_e u_e w_e.  From sum_v A_v curl(u)_v eta_v
    = sum_v sum_{e in v} t_{e,v} d_e u_e eta_v, the edge value is (1/l_e) sum_{v at e} t_{e,v} eta_v:
    every triangle scatters its t_{e,v} eta_v to its three edges."""
    acc = np.zeros(g.E)
    np.add.at(acc, g.t_edges.ravel(), (g.t_signs * zeta[:, None]).ravel())
    return acc / g.l_e


def laplacian(g, a):
    """div grad of a node field."""
    return divergence(g, gradient(g, a))


def vector_laplacian(g, u):
    """grad div u - grad^perp curl u (the dissipation operator of the velocity, Sec. 3.1)."""
    return gradient(g, divergence(g, u)) - curl_adjoint(g, curl(g, u))


def vertex_pv(g, dh, u, p):
    """q_v = (zeta_v + f_v) / h_v, with h_v the kite-weighted mean of the three cells."""
    h = p.H + dh
    hv = (g.R_iv * h[g.t_nodes]).sum(1)
    return (curl(g, u) + g.f_v) / hv


def perp_pv_flux(g, F, qv):
    """Q_e = (1/d_e) sum_{e'} w_{e,e'} l_{e'} F_{e'} (q_e + q_{e'})/2, q_e = mean of its vertices."""
    qe = 0.5 * (qv[g.e_tris[:, 0]] + qv[g.e_tris[:, 1]])
    terms = g.w * g.l_e[g.ecp] * F[g.ecp] * 0.5 * (qe[:, None] + qe[g.ecp])
    return terms.sum(1) / g.d_e


def tendencies(g, dh, u, p):
    """Right-hand side of eqs. (height) and (velo) on one uniform level (with the dissipative
    terms when p.nu > 0; the height equation alone, u fixed, when p.adv)."""
    _, F = edge_quantities(g, dh, u, p)
    ddh = -divergence(g, F)
    if p.adv:
        return ddh, np.zeros_like(u)
    B = p.g * dh + kinetic_energy(g, u)
    Q = perp_pv_flux(g, F, vertex_pv(g, dh, u, p))
    du = -Q - gradient(g, B)
    if p.nu:
        ddh = ddh + p.nu * laplacian(g, dh)
        du = du + p.nu * vector_laplacian(g, u)
    return ddh, du


# ---------------------------------------------------------------- time schemes

def rk4_step(rhs, y, dt):
    """Classical four-stage RK4 on a tuple of arrays."""
    add = lambda a, s, k: tuple(ai + s * ki for ai, ki in zip(a, k))  # noqa: E731
    k1 = rhs(y)
    k2 = rhs(add(y, 0.5 * dt, k1))
    k3 = rhs(add(y, 0.5 * dt, k2))
    k4 = rhs(add(y, dt, k3))
    return tuple(yi + dt / 6.0 * (a + 2.0 * b + 2.0 * c + d) for yi, a, b, c, d in zip(y, k1, k2, k3, k4))


def ssprk43_step(rhs, y, dt):
    """Four-stage third-order SSP RK (Shu-Osher form, SSP coefficient 2)."""
    k = rhs(y)
    y1 = tuple(a + 0.5 * dt * b for a, b in zip(y, k))
    k = rhs(y1)
    y2 = tuple(a + 0.5 * dt * b for a, b in zip(y1, k))
    k = rhs(y2)
    y3 = tuple(2.0 / 3.0 * a + 1.0 / 3.0 * b + dt / 6.0 * c for a, b, c in zip(y, y2, k))
    k = rhs(y3)
    return tuple(a + 0.5 * dt * b for a, b in zip(y3, k))


def step(g, dh, u, dt, p, scheme="rk4"):
    rhs = lambda y: tendencies(g, y[0], y[1], p)  # noqa: E731
    f = rk4_step if scheme == "rk4" else ssprk43_step
    return f(rhs, (dh, u), dt)


# ---------------------------------------------------------------- diagnostics

def mass(g, dh, p):
    """Total mass sum_i A_i (H + dh_i)."""
    return float((g.A_i * (p.H + dh)).sum())


def energy(g, dh, u, p):
    """E = sum_i A_i g^2 h_i^2 / 2 + g sum_e (l_e d_e / 2) h_e u_e^2 - c^4 A_S / 2 (Sec. 7.2).

    The kinetic part is sum_i A_i h_i K_i, the form whose time derivative the
    energy-conserving TRiSK scheme makes vanish; (l_e d_e/2) is the edge's diamond area.
    """
    h = p.H + dh
    he, _ = edge_quantities(g, dh, u, p)
    A_S = g.A_i.sum()
    c2 = p.g * (g.A_i * h).sum() / A_S
    return float(0.5 * (g.A_i * (p.g * h) ** 2).sum() + p.g * (0.5 * g.l_e * g.d_e * he * u * u).sum()
                 - 0.5 * c2 * c2 * A_S)


def energy_rate(g, dh, u, ddh, du, p):
    """dE/dt/g implied by tendencies (ddh, du): sum A_i (g h_i + K_i) ddh_i + sum l_e d_e F_e du_e.

    For the semi-discrete TRiSK scheme this is zero up to round-off.
    """
    h = p.H + dh
    _, F = edge_quantities(g, dh, u, p)
    K = kinetic_energy(g, u)
    return float((g.A_i * (p.g * h + K) * ddh).sum() + (g.l_e * g.d_e * F * du).sum())


def suggest_dt(g, dh, u, p, cfl):
    """dt = cfl * min(1/omega_max, min_e d_e/|u_e|), omega = sqrt(f^2 + g h (pi/dx)^2).

    The frequency bound printed in Sec. 3.1 is dimensionally inconsistent; the wavenumber
    pi/dx is squared here (the gravity-wave dispersion relation on the grid).  The advection
    form has no gravity waves: dt = cfl * min_e d_e/|u_e|.
    """
    if p.adv:
        ua = np.abs(u)
        return float(cfl * np.min(np.where(ua > 0, g.d_e / np.maximum(ua, 1e-300), np.inf)))
    h = p.H + dh
    he = 0.5 * (h[g.e_nodes[:, 0]] + h[g.e_nodes[:, 1]])
    fe = 0.5 * (g.f_v[g.e_tris[:, 0]] + g.f_v[g.e_tris[:, 1]])
    om = np.sqrt(fe ** 2 + p.g * he * (np.pi / g.d_e) ** 2).max()
    ua = np.abs(u)
    adv = np.min(np.where(ua > 0, g.d_e / np.maximum(ua, 1e-300), np.inf))
    return float(cfl * min(1.0 / om, adv))

"""Pins of the oracle's wavelet transforms, flux restriction and adaptive step against what the
paper and the mathematics fix (no GPU)."""
import math

import numpy as np
import pytest

from oracle import trisk
from oracle.grid import Grid
from oracle.multiscale import Hierarchy, overlap_areas
from paper_1404_0405_amd import inputs

_H = {}


def hier(jmin, jmax):
    if (jmin, jmax) not in _H:
        _H[(jmin, jmax)] = Hierarchy(jmin, jmax)
    return _H[(jmin, jmax)]


def test_clipping_closed_forms():
    """Spherical clipping: the octant triangle against itself has area pi/2; two octants that
    share only an edge overlap in zero area; a polygon clipped by a superset is unchanged."""
    e = np.eye(3)
    octa = np.zeros((1, 6, 3))
    octa[0, :3] = [e[0], e[1], e[2]]
    octb = np.zeros((1, 6, 3))
    octb[0, :3] = [e[1], -e[0], e[2]]
    n3 = np.array([3])
    assert abs(overlap_areas(octa, n3, octa, n3)[0] - math.pi / 2) < 1e-14
    assert abs(overlap_areas(octa, n3, octb, n3)[0]) < 1e-14
    # a small triangle inside the octant
    sm = np.zeros((1, 6, 3))
    v = np.array([[1, 0.2, 0.2], [0.2, 1, 0.2], [0.2, 0.2, 1]], float)
    sm[0, :3] = v / np.linalg.norm(v, axis=1, keepdims=True)
    from oracle.grid import _sph_tri_area
    ref = _sph_tri_area(sm[0, 0], sm[0, 1], sm[0, 2])
    assert abs(overlap_areas(sm, n3, octa, n3)[0] - ref) < 1e-15


@pytest.mark.parametrize("j", [2, 3, 4])
def test_overlap_areas_partition(j):
    """Sec. 4.1: the partial areas A_km cover the fine and coarse hexagons: the four coarse
    cells of every odd node tile its fine hexagon, and the pieces inside every coarse cell tile
    it, so the effective coarse areas equal the geometric ones up to round-off."""
    H = hier(2, 5)
    P = H.pairs[j]
    assert np.allclose(P.A_geo.sum(1), P.gf.A_i[P.mid] if not hasattr(P.gf, "A_geo") else P.gf.A_geo[P.mid],
                       rtol=1e-12, atol=0)
    assert np.abs(H.A[j] / P.gc.A_geo - 1).max() < 1e-12
    small = P.A_geo[:, 2:] / P.A_geo.sum(1, keepdims=True)
    assert small.min() > -1e-13 and small.max() < 0.1        # small overlap regions (Fig. 3)
    big = P.A_geo[:, :2] / P.A_geo.sum(1, keepdims=True)
    assert big.min() > 0.4


@pytest.mark.parametrize("j", [2, 3, 4])
def test_height_transform_reconstructs_and_conserves(j):
    """eqs. (WTpred)/(WTupd): forward then inverse lifting reproduces any field; R_h preserves
    constants and conserves mass sum A h between levels."""
    H = hier(2, 5)
    P = H.pairs[j]
    rng = np.random.default_rng(j)
    h = rng.standard_normal(P.gf.N)
    hc, d = P.h_restrict(h, P.s_upd)
    back = np.empty_like(h)
    back[P.even] = hc - np.bincount(P.cells.ravel(), (P.s_upd * d[:, None]).ravel(), P.gc.N)
    back[P.mid] = d + (P.st * back[P.even[P.cells]]).sum(1)
    assert np.abs(back - h).max() < 1e-14
    assert np.abs(P.h_restrict(np.full(P.gf.N, 7.5), P.s_upd)[0] - 7.5).max() < 1e-14
    mc, mf = (H.A[j] * hc).sum(), (H.A[j + 1] * h).sum()
    assert abs(mc - mf) < 1e-14 * (H.A[j + 1] * np.abs(h)).sum()


@pytest.mark.parametrize("j", [2, 3, 4])
def test_velocity_transform_reconstructs(j):
    """Vector transform: restriction then prediction + details reproduces any field; the
    restriction preserves circulation around every coarse triangle."""
    H = hier(2, 5)
    P = H.pairs[j]
    u = np.random.default_rng(10 + j).standard_normal(P.gf.E)
    uc = P.u_restrict(u)
    dp, di = P.u_details(u, uc)
    half = 0.5 * (P.u_pair_pred(uc) + dp)
    back = np.empty_like(u)
    back[P.h1] = P.s1 * (uc + half)
    back[P.h2] = P.s2 * (uc - half)
    back[P.int_e] = di + P.u_int_pred(uc)
    assert np.abs(back - u).max() < 1e-14
    # circulation: coarse triangle = sum of its four fine triangles' circulations
    gc, gf = P.gc, P.gf
    circ_c = (gc.t_signs * gc.d_e[gc.t_edges] * uc[gc.t_edges]).sum(1)
    half_d = 0.5 * gc.d_e
    fine = (gc.t_signs * (half_d[gc.t_edges] * (P.s1 * u[P.h1] + P.s2 * u[P.h2])[gc.t_edges])).sum(1)
    assert np.allclose(circ_c, fine, rtol=1e-13, atol=1e-6)


def test_details_decay_for_smooth_fields():
    """Wavelet coefficients measure the local interpolation error (Sec. 2.1): for smooth
    fields they fall about 4x per level (second-order prediction)."""
    H = hier(2, 5)
    g5 = H.g[5]
    dh, u, _ = inputs.tc2_perturbed(g5.xyz, g5.e_mid, g5.e_tan, lmax=4, amplitude=500.0)
    H.set_state(5, dh, u)
    det = H.details()
    mh = [np.abs(det[j][0]).max() for j in (2, 3, 4)]
    mu = [max(np.abs(det[j][1]).max(), np.abs(det[j][2]).max()) for j in (2, 3, 4)]
    assert mh[0] / mh[1] > 3.0 and mh[1] / mh[2] > 3.0, mh
    assert mu[0] / mu[1] > 2.5 and mu[1] / mu[2] > 2.5, mu


@pytest.mark.parametrize("j", [2, 3, 4])
def test_flux_restriction_commutes(j):
    """eq. (divRcommute): R_h(div_{j+1} F) = div_j(R_F F) at every coarse node, for random fine
    fluxes (full levels: every node complete)."""
    H = hier(2, 5)
    P = H.pairs[j]
    F = np.random.default_rng(20 + j).standard_normal(P.gf.E)
    c = trisk.divergence(P.gf, F)
    lhs = trisk.divergence(P.gc, H.flux_restrict(j, F, c)) * H.A[j]
    rhs = H.A[j] * P.h_restrict(c, P.s_upd)[0]
    assert np.abs(lhs - rhs).max() < 1e-14 * np.abs(rhs).max()


def test_flux_restriction_drops_fail_commutation():
    """Each part of R_F is needed: without the corrective exchanges or without the small-piece
    routing, the commutation breaks (planted mistakes)."""
    H = Hierarchy(2, 4)
    j = 3
    P = H.pairs[j]
    F = np.random.default_rng(5).standard_normal(P.gf.E)
    c = trisk.divergence(P.gf, F)
    rhs = H.A[j] * P.h_restrict(c, P.s_upd)[0]
    full_c = P.RF_c.copy()
    # zero the corrective columns = even fine nodes
    mask = np.zeros(P.gf.N)
    mask[P.even] = 1.0
    P.RF_c = full_c @ __import__("scipy").sparse.diags(1.0 - mask)
    bad = trisk.divergence(P.gc, H.flux_restrict(j, F, c)) * H.A[j]
    P.RF_c = full_c
    assert np.abs(bad - rhs).max() > 1e-6 * np.abs(rhs).max()


def test_eps_zero_adaptive_equals_uniform():
    """eps = 0: every point is kept, so the adaptive method is the uniform jmax scheme (equal
    to round-off: the inverse transform rewrites fine values from coarse ones)."""
    H = Hierarchy(3, 5)
    g = H.g[5]
    gu = Grid(5)
    dh, u, Hd = inputs.tc2_perturbed(g.xyz, g.e_mid, g.e_tan, amplitude=300.0)
    p = trisk.Params(mean_depth=Hd)
    H.set_state(5, dh, u)
    H.adapt(0.0)
    a, b = dh, u
    for _ in range(4):
        H.step(300.0, p)
        H.adapt(0.0)
        a, b = trisk.step(gu, a, b, 300.0, p)
    x, y, na, ea = H.get_state(5)
    assert na.all() and ea.all()
    assert np.abs(x - a).max() < 1e-13 * np.abs(a).max()
    assert np.abs(y - b).max() < 1e-13 * np.abs(b).max()


def test_adaptive_mass_conservation_and_masks():
    """Mass on jmin is conserved to round-off through steps and adaptations with changing
    masks; the reconstructed jmax mass equals it; masks are monotone in eps."""
    H = Hierarchy(2, 5)
    g = H.g[5]
    dh, u, Hd = inputs.jet(g.xyz, g.e_mid, g.e_tan)
    p = trisk.Params(mean_depth=Hd)
    H.set_state(5, dh, u)
    saved = (dict(H.dh), dict(H.u), dict(H.node_act), dict(H.edge_act))
    counts = []
    for eps in (1e-3, 1e-2, 5e-2):
        H.dh, H.u, H.node_act, H.edge_act = (dict(s) for s in saved)
        H.adapt(eps)
        counts.append({j: H.node_act[j].copy() for j in H.levels})
    for a, b in zip(counts, counts[1:]):
        for j in H.levels:
            assert (a[j] | ~b[j]).all(), "mask not monotone in eps"
    assert counts[2][5].sum() < counts[0][5].sum() < g.N
    m0 = H.mass(p)
    dt = 200.0
    for _ in range(5):
        H.step(dt, p)
        H.adapt(5e-2)
    assert abs(H.mass(p) / m0 - 1) < 1e-14
    assert abs(H.reconstructed_mass(p) / m0 - 1) < 1e-14


def test_compression_error_bounded_by_eps():
    """Sec. 2.3: dropping coefficients below eps gives an error of order eps; the constant is
    reported.  Adapt a full jmax field and compare the reconstruction with the original."""
    H = Hierarchy(2, 5)
    g = H.g[5]
    dh, u, _ = inputs.jet(g.xyz, g.e_mid, g.e_tan)
    for eps in (1e-2, 1e-3):
        H.set_state(5, dh, u)
        eh, eu = H.adapt(eps)
        x, y, na, _ = H.get_state(5)
        assert na.sum() < g.N
        Ch = np.abs(x - dh).max() / eh
        Cu = np.abs(y - u).max() / eu
        print(f"eps={eps}: C_h={Ch:.2f} C_u={Cu:.2f}")
        assert Ch < 10.0 and Cu < 10.0


@pytest.mark.slow
def test_tc2_adaptive_config0_closed_form():
    """TC2 on levels 4..6, eps = 1e-3 relative, RK4, 50 steps: the flow stays close to its
    closed form (error comparable to the uniform jmax run) and mass is conserved."""
    H = Hierarchy(4, 6)
    g = H.g[6]
    dh, u, Hd = inputs.tc2(g.xyz, g.e_mid, g.e_tan)
    p = trisk.Params(mean_depth=Hd)
    H.set_state(6, dh, u)
    H.adapt(1e-3)
    dt = trisk.suggest_dt(g, dh, u, p, 0.8)
    m0 = H.mass(p)
    for _ in range(50):
        H.step(dt, p)
        H.adapt(1e-3)
    x, _, na, _ = H.get_state(6)
    err = np.abs(x - dh).max() / np.abs(dh).max()
    assert err < 2e-2, err
    assert abs(H.mass(p) / m0 - 1) < 1e-13


def test_adapt_with_an_empty_level():
    """A smooth zonal flow (TC2) on levels 2..5 at eps = 1e-2 leaves level 5 without an active
    point; the next adapt takes the threshold maxima over the levels that have active points (an
    empty level adds nothing, every jmin point is active) and finds the same masks; through steps
    and adaptations the level fills again and the jmin mass stays conserved."""
    H = Hierarchy(2, 5)
    g = H.g[5]
    dh, u, Hd = inputs.tc2(g.xyz, g.e_mid, g.e_tan)
    p = trisk.Params(mean_depth=Hd)
    H.set_state(5, dh, u)
    H.adapt(1e-2)
    assert not H.node_act[5].any() and not H.edge_act[5].any()
    first = {j: (H.node_act[j].copy(), H.edge_act[j].copy()) for j in H.levels}
    H.adapt(1e-2)
    for j in H.levels:
        assert np.array_equal(first[j][0], H.node_act[j]) and np.array_equal(first[j][1], H.edge_act[j])
    m0 = H.mass(p)
    for _ in range(5):
        H.step(400.0, p)
        H.adapt(1e-2)
    assert H.node_act[5].any()
    assert abs(H.mass(p) / m0 - 1) < 1e-14
    assert abs(H.reconstructed_mass(p) / m0 - 1) < 1e-14

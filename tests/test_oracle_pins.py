"""Pins of oracle parts that the other tests only exercise: the time-step bound (Sec. 3.1)
against the spectrum of the linearised discrete operator, the velocity prediction (Sec. 4.1)
against fields its least-squares fit reproduces exactly, the completeness rule of the partial
height transform against a refinement region whose complete set is known, and the dual vertices
(circumcentres) against equidistance (CPU only)."""
import math

import numpy as np

from oracle import trisk
from oracle.grid import Grid, _normalize
from oracle.multiscale import Hierarchy, Pair
from paper_1404_0405_amd import inputs


def _jacobian(g, p, eps=1e-3):
    """Linearisation of the tendencies about the resting state (central differences; the
    tendencies are smooth, so this is the exact Jacobian to ~eps^2)."""
    n = g.N + g.E

    def T(v):
        a, b = trisk.tendencies(g, v[:g.N], v[g.N:], p)
        return np.concatenate([a, b])
    M = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = eps
        M[:, k] = (T(e) - T(-e)) / (2 * eps)
    return M


def test_time_step_bounds_the_discrete_spectrum():
    """Sec. 3.1: omega_max = max sqrt(f^2 + g h (pi/dx)^2) must bound the largest frequency the
    discrete operator supports (at rest every eigenvalue is imaginary: the scheme conserves
    energy), and not by a wide margin: on levels 2 and 3 the largest |lambda| is 0.6-1.0 of
    omega_max.  The printed, unsquared pi/dx gives an omega_max hundreds of times too large (a
    time step far shorter than needed), outside that window."""
    p = trisk.Params()
    for J in (2, 3):
        g = Grid(J)
        lam = np.linalg.eigvals(_jacobian(g, p))
        om = 1.0 / trisk.suggest_dt(g, np.zeros(g.N), np.zeros(g.E), p, 1.0)
        ratio = np.abs(lam).max() / om
        assert 0.6 < ratio <= 1.0, (J, ratio)
        assert lam.real.max() < 1e-12 * om
        fe = 0.5 * (g.f_v[g.e_tris[:, 0]] + g.f_v[g.e_tris[:, 1]])
        wrong = np.sqrt(fe ** 2 + inputs.GRAVITY * p.H * math.pi / g.d_e).max()
        assert np.abs(lam).max() / wrong < 0.01


def test_rk4_at_the_suggested_step_stays_bounded(oracle_grid):
    """RK4 at CFL 0.8 of the suggested step keeps the perturbed test-2 flow bounded for 200
    steps: RK4 slightly damps imaginary eigenvalues inside its stability region, so the energy
    does not grow and drifts by less than 1e-3; twice the RK4 stability limit blows up."""
    g = oracle_grid(3)
    dh0, u0, H = inputs.tc2_perturbed(g.xyz, g.e_mid, g.e_tan, amplitude=200.0)
    p = trisk.Params(mean_depth=H)
    dt = trisk.suggest_dt(g, dh0, u0, p, 0.8)
    E0 = trisk.energy(g, dh0, u0, p)
    dh, u = dh0, u0
    for _ in range(200):
        dh, u = trisk.step(g, dh, u, dt, p)
    E1 = trisk.energy(g, dh, u, p)
    assert E1 <= E0 * (1 + 1e-12) and abs(E1 / E0 - 1) < 1e-3
    dh, u = dh0, u0
    big = dt / 0.8 * 2.0 * 2.83
    for _ in range(60):
        dh, u = trisk.step(g, dh, u, big, p)
    assert not np.isfinite(dh).all() or np.abs(dh).max() > 1e3 * np.abs(dh0).max()


def _tangent_frame(c):
    ref = np.array([0.0, 0.0, 1.0]) if abs(c[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = _normalize(np.cross(ref, c))
    return e1, np.cross(c, e1)


def _linear_field(c, rng):
    """A tangent field that is linear in the gnomonic coordinates of the plane tangent at c:
    W(xi) = w0 + M xi, xi = x / (x . c) - c, in the plane's own basis.  Its value at an edge is
    W . (the edge tangent projected into the plane, normalised)."""
    e1, e2 = _tangent_frame(c)
    w0 = rng.normal(size=2)
    M = rng.normal(size=(2, 2))

    def value(x, t):
        xi = x / (x @ c) - c
        q = np.array([xi @ e1, xi @ e2])
        w = w0 + M @ q
        tp = np.array([t @ e1, t @ e2])
        return float(w @ tp / np.linalg.norm(tp))
    return value


def test_velocity_prediction_exact_for_gnomonic_linear_fields():
    """Sec. 4.1 (second-order velocity prediction): the least-squares fit of a linear tangent
    field is exact on a field that is linear in the gnomonic image about the triangle's dual
    vertex, so the interior fine edges and the half-edge difference of each of the triangle's
    edges (its own half of the pair weights) are predicted to round-off.  Built independently of
    the oracle's frames: a stencil in the wrong order, a transposed weight row or a flipped
    tangent fails."""
    gc, gf = Grid(3), Grid(4)
    P = Pair(gc, gf)
    rng = np.random.default_rng(5)
    worst = 0.0
    for T in rng.choice(gc.T, 40, replace=False):
        c = gc.t_cc[T]
        val = _linear_field(c, rng)
        uc = np.zeros(gc.E)
        for e in P.v_sten[T]:
            uc[e] = val(gc.e_mid[e], gc.e_tan[e])
        scale = np.abs(uc[P.v_sten[T]]).max()
        for s in range(3):
            f = P.int_e[T, s]
            pred = P.w_int[T, s] @ uc[P.v_sten[T]]
            worst = max(worst, abs(pred - val(gf.e_mid[f], gf.e_tan[f])) / scale)
        for e in gc.t_edges[T]:
            side_left = gc.e_tris[e, 0] == T
            w = P.w_pair_l[e] if side_left else P.w_pair_r[e]
            t1 = gf.e_tan[P.h1[e]] * P.s1[e]
            t2 = gf.e_tan[P.h2[e]] * P.s2[e]
            want = 0.5 * (val(gf.e_mid[P.h1[e]], t1) - val(gf.e_mid[P.h2[e]], t2))
            worst = max(worst, abs(w @ uc[P.v_sten[T]] - want) / scale)
    assert worst < 1e-12, worst


def test_completeness_of_a_refined_lozenge():
    """Partial height transform (Sec. 3.1): refine the whole of lozenge 0 (every node and edge of
    its elements on the fine level, plus the closure rules).  Coarse nodes deep inside the
    lozenge are complete, nodes away from it are not, and at every complete node the coarse
    height tendency equals R_h of the fine ones (eq. (Rh), the commutation of eq. (divRcommute))
    to round-off; where the fine copy is active but a stencil point or coarse edge is not, the
    equality fails for some node (the rule is not too permissive)."""
    H = Hierarchy(3, 4)
    gc, gf = H.g[3], H.g[4]
    dh, u, Hd = inputs.tc2_perturbed(gf.xyz, gf.e_mid, gf.e_tan, amplitude=300.0)
    p = trisk.Params(mean_depth=Hd)
    H.set_state(4, dh, u)
    nf, nc = 16, 8
    lz = np.zeros(gf.N, bool)
    lz[:nf * nf] = True                               # the elements of lozenge 0
    H.node_act[4] = lz.copy()
    H.edge_act[4] = np.repeat(lz[:10 * nf * nf], 3).copy()
    H.node_act[4][gf.e_nodes[H.edge_act[4]].ravel()] = True   # end nodes of active edges
    cm = H.complete(3)
    i, j = np.meshgrid(np.arange(nc), np.arange(nc), indexing="ij")
    deep = ((i >= 2) & (i <= nc - 3) & (j >= 2) & (j <= nc - 3)).ravel()
    inner = ((i >= 1) & (i <= nc - 2) & (j >= 1) & (j <= nc - 2)).ravel()
    assert cm[:nc * nc][deep].all()
    assert not cm[:nc * nc][~inner].any()
    assert not cm[nc * nc:].any()
    ddh, _ = H.tendencies(H.dh, H.u, p)
    P = H.pairs[3]
    Rf, _ = P.h_restrict(ddh[4], P.s_upd)
    scale = np.abs(ddh[3]).max()
    assert np.abs(Rf[cm] - ddh[3][cm]).max() < 1e-13 * scale
    near = H.node_act[4][P.even] & ~cm & H.node_act[3]
    assert near.any()
    assert np.abs(Rf[near] - ddh[3][near]).max() > 1e-3 * scale


def test_dual_vertices_are_circumcentres(oracle_grid):
    """The dual vertex of every triangle is equidistant from its three nodes (to round-off) and
    lies inside the triangle (positive kites are checked by the grid builder)."""
    for J in (3, 6):
        g = oracle_grid(J)
        x = g.xyz[g.t_nodes]
        d = np.linalg.norm(x - g.t_cc[:, None, :], axis=2)
        spread = (d.max(1) - d.min(1)) / d.mean(1)
        assert spread.max() < 1e-12, (J, spread.max())

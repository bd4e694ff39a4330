"""Oracle: multilevel wavelet operators and the adaptive step (plain FP64 numpy, full levels).

TEST INFRASTRUCTURE ONLY (see ``oracle/grid.py``).

Every level j = jmin..jmax is held as a full uniform field; points that are not active are
filled top-down by zero-detail prediction before they are read, so every stencil is defined.
Only active points are updated.  Passages followed:

* Sec. 2.2, eqs. (WTpred), (WTupd): lifting -- predict the odd fine values from the even ones,
  then update the coarse values with the details.
* Sec. 4.1, eq. (Rh) and the two area conditions after it: height restriction with
  s~_km = A_km/A_m and s_km = A_km/A_k, where A_km is the area shared by coarse hexagon k and
  fine hexagon m; mass is conserved between levels.
* Sec. 4.1: vector (velocity) transform, second-order prediction from coarse edges with a
  symmetric stencil and two 6x6 least-squares systems per edge.
* Sec. 4.1-4.3, eqs. (divRcommute), (R_f), (restr_flux), (ho_flux), (kml): flux restriction
  R_F = R_F0 + R'_F, which makes R_h(div_{j+1} F) = div_j(R_F F).
* Sec. 3.1 (time step): q and K everywhere; B, F and qF^perp on the locally finest level and
  restricted to coarser levels; tendencies; partial (height only) transforms; adaptation.
* Sec. 2.3: threshold |d| >= eps, plus all of Jmin, plus neighbours in space and scale, plus
  the h/u consistency step.

Readings where the paper is silent, ambiguous or garbled are listed with each function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

from . import trisk
from .grid import Grid, _match_rows, _normalize

_HERE = os.path.dirname(os.path.abspath(__file__))
_CLIP = None


def _cliplib():
    """Load the plain-C spherical clipping helper (compiled with gcc on first use)."""
    global _CLIP
    if _CLIP is None:
        so = os.path.join(_HERE, "libsphclip.so")
        src = os.path.join(_HERE, "csrc", "sphclip.c")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", src, "-o", so, "-lm"])
        lib = ctypes.CDLL(so)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int)
        lib.sph_overlap_areas.argtypes = [ctypes.c_int, D, I, D, I, D]
        lib.sph_overlap_area.argtypes = [D, ctypes.c_int, D, ctypes.c_int]
        lib.sph_overlap_area.restype = ctypes.c_double
        _CLIP = lib
    return _CLIP


def overlap_areas(P, npv, Q, nqv):
    """Unit-sphere areas of (convex polygon P_k) intersect (convex polygon Q_k), padded (K,6,3)."""
    lib = _cliplib()
    P = np.ascontiguousarray(P, np.float64)
    Q = np.ascontiguousarray(Q, np.float64)
    npv = np.ascontiguousarray(npv, np.int32)
    nqv = np.ascontiguousarray(nqv, np.int32)
    out = np.empty(P.shape[0])
    D = ctypes.POINTER(ctypes.c_double)
    I = ctypes.POINTER(ctypes.c_int)
    lib.sph_overlap_areas(P.shape[0], P.ctypes.data_as(D), npv.ctypes.data_as(I),
                          Q.ctypes.data_as(D), nqv.ctypes.data_as(I), out.ctypes.data_as(D))
    return out


def _third_vertex(g, tri, a, b):
    """Node of triangle `tri` that is neither a nor b."""
    tn = g.t_nodes[tri]
    m = (tn != a[:, None]) & (tn != b[:, None])
    assert (m.sum(1) == 1).all()
    return tn[m]


class Pair:
    """Inter-scale maps and weights between coarse level gc = j and fine level gf = j+1."""

    def __init__(self, gc: Grid, gf: Grid):
        self.gc, self.gf = gc, gf
        a, b = gc.e_nodes[:, 0], gc.e_nodes[:, 1]
        # nested grids: coarse nodes are the even fine nodes; odd nodes are edge midpoints
        self.even = _match_rows(gf.xyz, gc.xyz)
        self.mid = _match_rows(gf.xyz, _normalize(gc.xyz[a] + gc.xyz[b]))
        # the two fine half-edges of every coarse edge, with the sign that orients them along it
        self.h1, self.s1 = gf.edge_between(self.even[a], self.mid)
        self.h2, self.s2 = gf.edge_between(self.mid, self.even[b])
        # opposite vertices: p in the left triangle (a, b, p), q in the right triangle (b, a, q)
        self.p = _third_vertex(gc, gc.e_tris[:, 0], a, b)
        self.q = _third_vertex(gc, gc.e_tris[:, 1], a, b)
        self.cells = np.stack([a, b, self.p, self.q], 1)
        # the three fine edges inside every coarse triangle, joining consecutive midpoints
        M = self.mid[gc.t_edges]
        ie, isg = [], []
        for s in range(3):
            e, sg = gf.edge_between(M[:, s], M[:, (s + 1) % 3])
            ie.append(e)
            isg.append(sg)
        self.int_e = np.stack(ie, 1)
        self.int_s = np.stack(isg, 1)
        self._height_weights()
        self._velocity_weights()

    # --------------------------------------------------------------- height (Sec. 4.1)
    def _height_weights(self):
        """A_cm = area(coarse hexagon c  intersect  fine hexagon m) for the four coarse cells
        c = (a, b, p, q) around the odd node m of coarse edge a-b; the paper splits hexagons
        into triangles and intersects great-circle arcs, here convex spherical clipping gives
        the same areas.  The four cells cover the fine hexagon."""
        gc, gf = self.gc, self.gf
        R2 = gc.radius ** 2
        Pm, npm = gf.cell_polygon(self.mid)
        A = np.empty((gc.E, 4))
        for c in range(4):
            Qc, nqc = gc.cell_polygon(self.cells[:, c])
            A[:, c] = R2 * overlap_areas(Pm, npm, Qc, nqc)
        err = np.abs(A.sum(1) / gf.A_i[self.mid] - 1.0).max()
        assert err < 1e-9, f"coarse cells do not cover the fine hexagon ({err})"
        self.A_geo = A
        self.st = A / A.sum(1, keepdims=True)          # s~_{cm}, an exact partition of unity

    # --------------------------------------------------------------- velocity (Sec. 4.1)
    def _velocity_weights(self):
        """Reading: per coarse triangle T a linear tangent field V(xi) = a + G xi (6 unknowns)
        is fitted by least squares (the 6x6 normal equations) to the 9 coarse edges of T and of
        its three edge neighbours, in gnomonic coordinates about T's circumcentre.  The three
        fine edges inside T are predicted from T's fit; the pair of half-edges of a coarse edge
        from the average of the fits of its two triangles (13 distinct coarse edges)."""
        gc, gf = self.gc, self.gf
        T = gc.T
        te = gc.t_edges
        sten = np.empty((T, 9), np.int64)
        sten[:, :3] = te
        for s in range(3):
            e = te[:, s]
            nb = np.where(gc.e_tris[e, 0] == np.arange(T), gc.e_tris[e, 1], gc.e_tris[e, 0])
            other = gc.t_edges[nb]
            keep = other != e[:, None]
            assert (keep.sum(1) == 2).all()
            sten[:, 3 + 2 * s:5 + 2 * s] = other[keep].reshape(T, 2)
        assert all(np.unique(r).size == 9 for r in sten[: min(T, 500)])
        self.v_sten = sten
        c = gc.t_cc
        ref = np.where(np.abs(c[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
        b1 = _normalize(np.cross(ref, c))
        b2 = np.cross(c, b1)
        self._frame = (c, b1, b2)
        X = gc.e_mid[sten]                                   # (T, 9, 3)
        xi = self._gnomonic(X, c, b1, b2)
        scale = np.sqrt((xi ** 2).sum(-1)).mean(1)           # conditioning of the 6x6 system
        self._scale = scale
        rows = self._rows(xi / scale[:, None, None], gc.e_tan[sten], b1, b2)
        Mt = np.swapaxes(rows, 1, 2)
        self.v_pinv = np.linalg.solve(Mt @ rows, Mt)         # (T, 6, 9): normal equations
        # interior fine edges of each coarse triangle
        fe = self.int_e
        phi = self._phi_at(np.arange(T)[:, None].repeat(3, 1), gf.e_mid[fe], gf.e_tan[fe])
        self.w_int = np.einsum("tkc,tcs->tks", phi, self.v_pinv)      # (T, 3, 9)
        # half-edge pairs: (p1 - p2) with the half-edges oriented along the coarse edge
        tl, tr = gc.e_tris[:, 0], gc.e_tris[:, 1]
        t1 = gf.e_tan[self.h1] * self.s1[:, None]
        t2 = gf.e_tan[self.h2] * self.s2[:, None]
        x1, x2 = gf.e_mid[self.h1], gf.e_mid[self.h2]
        wl = (self._phi_at(tl, x1, t1) - self._phi_at(tl, x2, t2))[:, None, :] @ self.v_pinv[tl]
        wr = (self._phi_at(tr, x1, t1) - self._phi_at(tr, x2, t2))[:, None, :] @ self.v_pinv[tr]
        self.w_pair_l = 0.5 * wl[:, 0, :]                    # on v_sten[left triangle]
        self.w_pair_r = 0.5 * wr[:, 0, :]                    # on v_sten[right triangle]

    @staticmethod
    def _gnomonic(X, c, b1, b2):
        cx = (X * c[:, None, :]).sum(-1) if X.ndim == 3 else (X * c).sum(-1)
        if X.ndim == 3:
            return np.stack([(X * b1[:, None, :]).sum(-1) / cx, (X * b2[:, None, :]).sum(-1) / cx], -1)
        return np.stack([(X * b1).sum(-1) / cx, (X * b2).sum(-1) / cx], -1)

    @staticmethod
    def _rows(xi, tan, b1, b2):
        if tan.ndim == 3:
            t1 = (tan * b1[:, None, :]).sum(-1)
            t2 = (tan * b2[:, None, :]).sum(-1)
        else:
            t1 = (tan * b1).sum(-1)
            t2 = (tan * b2).sum(-1)
        nrm = np.sqrt(t1 * t1 + t2 * t2)
        t1, t2 = t1 / nrm, t2 / nrm
        return np.stack([t1, t2, t1 * xi[..., 0], t1 * xi[..., 1], t2 * xi[..., 0], t2 * xi[..., 1]], -1)

    def _phi_at(self, tri, x, tan):
        """Design-matrix row of a prediction point x (unit) with tangent tan in the frame of
        triangle(s) `tri`."""
        c, b1, b2 = self._frame
        if tri.ndim == 2:
            cc, bb1, bb2, sc = c[tri], b1[tri], b2[tri], self._scale[tri]
            cx = (x * cc).sum(-1)
            xi = np.stack([(x * bb1).sum(-1) / cx, (x * bb2).sum(-1) / cx], -1) / sc[..., None]
            t1 = (tan * bb1).sum(-1)
            t2 = (tan * bb2).sum(-1)
        else:
            cc, bb1, bb2, sc = c[tri], b1[tri], b2[tri], self._scale[tri]
            cx = (x * cc).sum(-1)
            xi = np.stack([(x * bb1).sum(-1) / cx, (x * bb2).sum(-1) / cx], -1) / sc[:, None]
            t1 = (tan * bb1).sum(-1)
            t2 = (tan * bb2).sum(-1)
        nrm = np.sqrt(t1 * t1 + t2 * t2)
        t1, t2 = t1 / nrm, t2 / nrm
        return np.stack([t1, t2, t1 * xi[..., 0], t1 * xi[..., 1], t2 * xi[..., 0], t2 * xi[..., 1]], -1)

    # --------------------------------------------------------------- transforms
    def h_details(self, hf):
        """eq. (WTpred): d_m = h_m - sum_c s~_cm h_even(c), one per coarse edge."""
        return hf[self.mid] - (self.st * hf[self.even[self.cells]]).sum(1)

    def h_restrict(self, hf, s_upd):
        """eq. (WTupd) with eq. (Rh): h^j_k = h^{j+1}_k + sum_m s_km d_m."""
        d = self.h_details(hf)
        return hf[self.even] + np.bincount(self.cells.ravel(), (s_upd * d[:, None]).ravel(),
                                           self.gc.N), d

    def u_restrict(self, uf):
        """Velocity restriction: mean of the two half-edges (preserves circulation)."""
        return 0.5 * (self.s1 * uf[self.h1] + self.s2 * uf[self.h2])

    def u_pair_pred(self, uc):
        """(p1 - p2) of every coarse edge from coarse values."""
        tl, tr = self.gc.e_tris[:, 0], self.gc.e_tris[:, 1]
        return (self.w_pair_l * uc[self.v_sten[tl]]).sum(1) + (self.w_pair_r * uc[self.v_sten[tr]]).sum(1)

    def u_int_pred(self, uc):
        """Predictions of the three interior fine edges of every coarse triangle."""
        return (self.w_int * uc[self.v_sten][:, None, :]).sum(2)

    def u_details(self, uf, uc):
        """Details of the half-edge pairs (per coarse edge) and interior edges (per triangle)."""
        d_pair = (self.s1 * uf[self.h1] - self.s2 * uf[self.h2]) - self.u_pair_pred(uc)
        d_int = uf[self.int_e] - self.u_int_pred(uc)
        return d_pair, d_int


class Hierarchy:
    """Levels jmin..jmax with inter-scale weights, effective areas, R_F, masks and state."""

    def __init__(self, jmin, jmax, radius=6.371e6, omega=7.292e-5, grids=None):
        self.jmin, self.jmax = jmin, jmax
        self.g = {j: (grids[j] if grids and j in grids else Grid(j, radius, omega)) for j in range(jmin, jmax + 1)}
        self.pairs = {j: Pair(self.g[j], self.g[j + 1]) for j in range(jmin, jmax)}
        self._effective_areas()
        for j in range(jmin, jmax):
            self._flux_restriction(j)
        self.node_act = {j: np.ones(self.g[j].N, bool) for j in self.levels}
        self.edge_act = {j: np.ones(self.g[j].E, bool) for j in self.levels}
        self.dh = {j: np.zeros(self.g[j].N) for j in self.levels}
        self.u = {j: np.zeros(self.g[j].E) for j in self.levels}

    @property
    def levels(self):
        return range(self.jmin, self.jmax + 1)

    # --------------------------------------------------------------- areas (Sec. 4.1)
    def _effective_areas(self):
        """Reading of the two area conditions after eq. (Rh) (the second prints A_k^{j+1}
        inside the sum where A_m^{j+1} is meant): starting from the geometric areas of jmax,
        A~_km = s~_km A^{j+1}_m and A^j_k = A^{j+1}_k + sum_m A~_km, bottom-up.  Both
        conditions then hold exactly, so the restriction conserves mass to round-off.  The
        effective areas replace the cell areas in div, K, mass and energy of levels < jmax."""
        self.A = {self.jmax: self.g[self.jmax].A_i.copy()}
        for j in range(self.jmax - 1, self.jmin - 1, -1):
            P = self.pairs[j]
            P.Aov = P.st * self.A[j + 1][P.mid][:, None]
            self.A[j] = self.A[j + 1][P.even] + np.bincount(P.cells.ravel(), P.Aov.ravel(), self.g[j].N)
            P.s_upd = P.Aov / self.A[j][P.cells]             # s_km = A~_km / A^j_k
        for j in self.levels:
            self.g[j].A_geo = self.g[j].A_i
            self.g[j].A_i = self.A[j]

    # --------------------------------------------------------------- R_F (Sec. 4.2-4.3)
    def _flux_restriction(self, j):
        """Coarse integrated fluxes Phi = l^j F^j on every coarse edge as a linear map of the
        fine integrated fluxes (l F)^{j+1} and fine divergences c^{j+1} = div_{j+1} F^{j+1}.

        Reading (divergence uniform inside each fine hexagon, as the paper assumes):
        (i)  basic part, eq. (restr_flux): Phi0(k->l) = F_in + alpha A_m c_m, F_in the flux into
             the midpoint cell m through its three k-side fine edges, alpha =
             A~_km / (A~_km + A~_lm);
        (ii) the small pieces A~_pm, A~_qm of m lying in the opposite coarse cells p, q are
             routed to the fluxes p->k, p->l (q->k, q->l) in the proportion alpha : 1-alpha; the
             interpolated small-boundary fluxes x_{+-1} are taken as zero (the commutation does
             not depend on them);
        (iii) corrective part, eqs. (ho_flux), (kml): for every odd m and every pair (a, b) of
             its overlapping coarse cells the exchange (A~_am A~_bm / A_m)(c_a - c_b) flows a->b,
             on edge a-b for neighbours, half through each common neighbour for p, q.
        With these three parts R_h(div_{j+1} F) = div_j(R_F F) holds exactly."""
        P = self.pairs[j]
        gc, gf = P.gc, P.gf
        Ec, Ef, Nf = gc.E, gf.E, gf.N
        Aov = P.Aov
        Am = self.A[j + 1][P.mid]
        a, b, p, q = P.cells.T
        rF, cF, vF = [], [], []       # Phi rows <- (l F) fine columns
        rc, cc, vc = [], [], []       # Phi rows <- c fine columns

        def flux_on(x, y):
            e, s = gc.edge_between(x, y)      # orientation of flux x->y relative to edge e
            return e, s

        # (i) basic part on every coarse edge (a -> b)
        alpha = Aov[:, 0] / (Aov[:, 0] + Aov[:, 1])
        mk_p = P.mid[gc.edge_between(a, p)[0]]
        mk_q = P.mid[gc.edge_between(a, q)[0]]
        for x in (P.even[a], mk_p, mk_q):
            f, s = gf.edge_between(P.mid, x)          # s = +1: fine edge points out of m
            rF.append(np.arange(Ec)); cF.append(f); vF.append(-s.astype(float))   # inflow into m
        rc.append(np.arange(Ec)); cc.append(P.mid); vc.append(alpha * Am)
        # (ii) small pieces of each odd node m' (edge a-b) in p and q
        for col, x in ((2, p), (3, q)):
            amount = Aov[:, col]
            for tgt, share in ((a, Aov[:, 0]), (b, Aov[:, 1])):
                e, s = flux_on(x, tgt)
                rc.append(e); cc.append(P.mid); vc.append(s * amount * share / (Aov[:, 0] + Aov[:, 1]))
        # (iii) corrective exchanges
        ev = P.even
        for i1, i2 in ((0, 1), (0, 2), (1, 2), (0, 3), (1, 3)):
            x, y = P.cells[:, i1], P.cells[:, i2]
            X = Aov[:, i1] * Aov[:, i2] / Am
            e, s = flux_on(x, y)
            rc += [e, e]; cc += [ev[x], ev[y]]; vc += [s * X, -s * X]
        Xpq = 0.5 * Aov[:, 2] * Aov[:, 3] / Am
        for via in (a, b):
            for x, y in ((p, via), (via, q)):
                e, s = flux_on(x, y)
                rc += [e, e]; cc += [ev[p], ev[q]]; vc += [s * Xpq, -s * Xpq]
        P.RF_F = sp.csr_matrix((np.concatenate(vF), (np.concatenate(rF), np.concatenate(cF))), shape=(Ec, Ef))
        P.RF_c = sp.csr_matrix((np.concatenate(vc), (np.concatenate(rc), np.concatenate(cc))), shape=(Ec, Nf))

    def flux_restrict(self, j, Ff, cf):
        """F^j on every coarse edge from fine F^{j+1} and c^{j+1}."""
        P = self.pairs[j]
        Phi = P.RF_F @ (P.gf.l_e * Ff) + P.RF_c @ cf
        return Phi / P.gc.l_e

    # --------------------------------------------------------------- prolongation
    def prolong(self, dh, u):
        """Fill every inactive point of levels > jmin, top-down, by zero-detail prediction.

        Reading: an inactive even node takes its coarse value, an inactive odd node the
        s~-weighted mean of its four even fine neighbours (eq. (WTpred) with zero detail); an
        inactive half-edge takes u^j_e -+ (p1 - p2)/2, an inactive interior edge its prediction
        (inverse velocity transform with zero detail)."""
        dh = {j: v.copy() for j, v in dh.items()}
        u = {j: v.copy() for j, v in u.items()}
        for j in range(self.jmin, self.jmax):
            P = self.pairs[j]
            f = j + 1
            na, ea = self.node_act[f], self.edge_act[f]
            hf = dh[f]
            ev = P.even
            hf[ev] = np.where(na[ev], hf[ev], dh[j])
            pred = (P.st * hf[ev[P.cells]]).sum(1)
            hf[P.mid] = np.where(na[P.mid], hf[P.mid], pred)
            uf = u[f]
            half = 0.5 * P.u_pair_pred(u[j])
            v1 = P.s1 * (u[j] + half)
            v2 = P.s2 * (u[j] - half)
            uf[P.h1] = np.where(ea[P.h1], uf[P.h1], v1)
            uf[P.h2] = np.where(ea[P.h2], uf[P.h2], v2)
            ip = P.u_int_pred(u[j])
            uf[P.int_e] = np.where(ea[P.int_e], uf[P.int_e], ip)
        return dh, u

    # --------------------------------------------------------------- multilevel tendency
    def nonleaf(self, j):
        P = self.pairs[j]
        return (self.edge_act[j + 1][P.h1] & self.edge_act[j + 1][P.h2]), self.node_act[j + 1][P.even]

    def tendencies(self, dh, u, p):
        """One tendency evaluation of the whole hierarchy (Sec. 3.1, time step).

        q, K, B, F and qF^perp are computed on every level from that level's values; then,
        from jmax-1 down to jmin, at non-leaf edges (both half-edges active) F^j = R_F(F^{j+1})
        and Q^j = mean of the two half-edge values, and at non-leaf nodes (fine copy active)
        B^j = B^{j+1} (injection).  Tendencies are taken with each level's own operators."""
        dh, u = self.prolong(dh, u)
        F, B, Q = {}, {}, {}
        for j in self.levels:
            g = self.g[j]
            # F: the total mass flux whose divergence is taken and restricted; Q uses the
            # thickness flux h u itself
            _, Fa = trisk.edge_quantities(g, dh[j], u[j], p)
            F[j] = Fa
            if p.adv:
                # advection form (Sec. 6.1): only the mass flux enters
                B[j], Q[j] = np.zeros(g.N), np.zeros(g.E)
                continue
            B[j] = p.g * dh[j] + trisk.kinetic_energy(g, u[j])
            Q[j] = trisk.perp_pv_flux(g, Fa, trisk.vertex_pv(g, dh[j], u[j], p))
            if p.nu:
                # viscous form (Sec. 3.1): nu div grad dh as the divergence of the flux
                # -nu grad dh, nu grad div u as the gradient of -nu div u added to B, and
                # -nu grad^perp curl u added to the perpendicular term, so that all three are
                # restricted to coarser levels like the inviscid quantities
                F[j] = Fa - p.nu * trisk.gradient(g, dh[j])
                B[j] = B[j] - p.nu * trisk.divergence(g, u[j])
                Q[j] = Q[j] + p.nu * trisk.curl_adjoint(g, trisk.curl(g, u[j]))
        for j in range(self.jmax - 1, self.jmin - 1, -1):
            P = self.pairs[j]
            ne, nn = self.nonleaf(j)
            cf = trisk.divergence(self.g[j + 1], F[j + 1])
            F[j] = np.where(ne, self.flux_restrict(j, F[j + 1], cf), F[j])
            Q[j] = np.where(ne, 0.5 * (P.s1 * Q[j + 1][P.h1] + P.s2 * Q[j + 1][P.h2]), Q[j])
            B[j] = np.where(nn, B[j + 1][P.even], B[j])
        ddh, du = {}, {}
        for j in self.levels:
            g = self.g[j]
            ddh[j] = np.where(self.node_act[j], -trisk.divergence(g, F[j]), 0.0)
            if p.adv:
                du[j] = np.zeros(g.E)   # advection form: the velocity is prescribed (Sec. 6.1)
            else:
                du[j] = np.where(self.edge_act[j], -Q[j] - trisk.gradient(g, B[j]), 0.0)
        return ddh, du

    # --------------------------------------------------------------- completeness and R_h
    def complete(self, j):
        """Coarse nodes k whose height restriction stencil (the even copy of k, the odd nodes
        sharing area with k and the even nodes of their cells) is all active and whose coarse
        edges are all non-leaf: there the coarse tendency is R_h of the fine ones."""
        P = self.pairs[j]
        gc = self.g[j]
        naf = self.node_act[j + 1]
        ok = naf[P.even].copy()
        # odd node of coarse edge e touches cells (a, b, p, q); needs itself and 4 evens active
        odd_ok = naf[P.mid] & naf[P.even[P.cells]].all(1)
        bad = np.zeros(gc.N, bool)
        np.logical_or.at(bad, P.cells.ravel(), np.repeat(~odd_ok, 4))
        ne, _ = self.nonleaf(j)
        bad_e = np.zeros(gc.N, bool)
        np.logical_or.at(bad_e, gc.e_nodes.ravel(), np.repeat(~ne, 2))
        return ok & ~bad & ~bad_e & self.node_act[j]

    def partial_height_transform(self):
        """After the step, bottom-up: h^j_k <- R_h(h^{j+1})_k at complete nodes (Sec. 3.1:
        partial transforms, height only)."""
        for j in range(self.jmax - 1, self.jmin - 1, -1):
            P = self.pairs[j]
            cm = self.complete(j)
            r, _ = P.h_restrict(self.dh[j + 1], P.s_upd)
            self.dh[j] = np.where(cm, r, self.dh[j])

    # --------------------------------------------------------------- step
    def step(self, dt, p, scheme="rk4"):
        y = (self.dh, self.u)

        def rhs(yy):
            return self.tendencies(yy[0], yy[1], p)

        def add(a, s, k):
            return tuple({j: a[i][j] + s * k[i][j] for j in self.levels} for i in range(2))

        if scheme == "rk4":
            k1 = rhs(y)
            k2 = rhs(add(y, 0.5 * dt, k1))
            k3 = rhs(add(y, 0.5 * dt, k2))
            k4 = rhs(add(y, dt, k3))
            new = tuple({j: y[i][j] + dt / 6.0 * (k1[i][j] + 2 * k2[i][j] + 2 * k3[i][j] + k4[i][j])
                         for j in self.levels} for i in range(2))
        else:
            k = rhs(y)
            y1 = add(y, 0.5 * dt, k)
            y2 = add(y1, 0.5 * dt, rhs(y1))
            k = rhs(y2)
            y3 = tuple({j: 2.0 / 3.0 * y[i][j] + 1.0 / 3.0 * y2[i][j] + dt / 6.0 * k[i][j]
                        for j in self.levels} for i in range(2))
            new = add(y3, 0.5 * dt, rhs(y3))
        self.dh, self.u = new
        self.partial_height_transform()

    # --------------------------------------------------------------- state in/out
    def set_state(self, level, dh, u):
        """Load a full level; coarser levels by restriction, finer levels inactive."""
        self.dh[level] = np.asarray(dh, float).copy()
        self.u[level] = np.asarray(u, float).copy()
        for j in self.levels:
            full = j <= level
            self.node_act[j] = np.full(self.g[j].N, full)
            self.edge_act[j] = np.full(self.g[j].E, full)
        for j in range(level - 1, self.jmin - 1, -1):
            P = self.pairs[j]
            self.dh[j], _ = P.h_restrict(self.dh[j + 1], P.s_upd)
            self.u[j] = P.u_restrict(self.u[j + 1])

    def get_state(self, level):
        """Fields on `level` reconstructed by the inverse transform with the details of the
        active points (zero elsewhere), so that their mass equals the mass on jmin."""
        dh, u = self.inverse(self.details(), self._active)
        return dh[level], u[level], self.node_act[level].copy(), self.edge_act[level].copy()

    def resync(self):
        """Inverse transform with the details of the active points applied to the state."""
        self.dh, self.u = self.inverse(self.details(), self._active)

    def _active(self, f, pts, kind, node_act=None, edge_act=None):
        na = self.node_act if node_act is None else node_act
        ea = self.edge_act if edge_act is None else edge_act
        P = self.pairs[f - 1]
        if kind == "odd":
            return na[f][P.mid]
        if kind == "pair":
            return ea[f][P.h1] & ea[f][P.h2]
        return ea[f][P.int_e]

    def inverse(self, det, keep):
        """Inverse transform, top-down from jmin: eqs. (WTupd), (WTpred) undone with the
        details d where keep(level, points, kind) holds and zero elsewhere.  Coarse values are
        never changed; R_h of the result is the coarse field, so mass is that of jmin."""
        dh, u = self.prolong(self.dh, self.u)
        for j in range(self.jmin, self.jmax):
            P = self.pairs[j]
            f = j + 1
            dhd, dp, di = det[j]
            d = np.where(keep(f, None, "odd"), dhd, 0.0)
            hf = dh[f]
            hf[P.even] = dh[j] - np.bincount(P.cells.ravel(), (P.s_upd * d[:, None]).ravel(), P.gc.N)
            hf[P.mid] = d + (P.st * hf[P.even[P.cells]]).sum(1)
            half = 0.5 * (P.u_pair_pred(u[j]) + np.where(keep(f, None, "pair"), dp, 0.0))
            uf = u[f]
            uf[P.h1] = P.s1 * (u[j] + half)
            uf[P.h2] = P.s2 * (u[j] - half)
            uf[P.int_e] = np.where(keep(f, None, "int"), di, 0.0) + P.u_int_pred(u[j])
        return dh, u

    # --------------------------------------------------------------- adapt (Sec. 2.3, 3.1)
    def details(self):
        """Height and velocity details of every level pair from the (prolonged) fields."""
        dh, u = self.prolong(self.dh, self.u)
        out = {}
        for j in range(self.jmin, self.jmax):
            P = self.pairs[j]
            dp, di = P.u_details(u[j + 1], u[j])
            out[j] = (P.h_details(dh[j + 1]), dp, di)
        return out

    def thresholds(self, eps):
        """Relative thresholds eps max|dh|, eps max|u| over the active points (an empty level adds
        nothing to the maxima; every jmin point is active)."""
        mh = max(np.abs(self.dh[j][self.node_act[j]]).max(initial=0.0) for j in self.levels)
        mu = max(np.abs(self.u[j][self.edge_act[j]]).max(initial=0.0) for j in self.levels)
        return eps * mh, eps * mu

    def significant(self, det, eh, eu):
        """R1: active fine points whose detail reaches the threshold (|d| >= eps_var): odd nodes,
        both half-edges of a coarse edge (one detail per pair), interior edges."""
        sig_n = {j: np.zeros(self.g[j].N, bool) for j in self.levels}
        sig_e = {j: np.zeros(self.g[j].E, bool) for j in self.levels}
        for j in range(self.jmin, self.jmax):
            P = self.pairs[j]
            dhd, dp, di = det[j]
            f = j + 1
            na, ea = self.node_act[f], self.edge_act[f]
            sig_n[f][P.mid] |= na[P.mid] & (np.abs(dhd) >= eh)
            both = ea[P.h1] & ea[P.h2]
            sp_ = both & (np.abs(dp) >= eu)
            sig_e[f][P.h1] |= sp_
            sig_e[f][P.h2] |= sp_
            si = ea[P.int_e] & (np.abs(di) >= eu)
            sig_e[f][P.int_e[si]] = True
        return sig_n, sig_e

    def adapt(self, eps, thresholds=None, allow=None):
        """Threshold and adjacent zone (Sec. 2.3) and the h/u consistency step (Sec. 3.1).

        thresholds: absolute (eps_h, eps_u) -- e.g. from `regime_thresholds` -- instead of the
        relative reading below.  allow: optional {level j: function(elements) -> bool array}
        that restricts the children rule R3 of level j's significant points to the elements it
        passes (the learned zone, not from the paper); the significant points, details and
        thresholds of the call are kept in ``self.last``.

        Readings: eps is relative, eps_h = eps max|dh|, eps_u = eps max|u| over active points;
        significant iff |d| >= eps_var (the paper's >=).  Rules, in order: R1 significant
        points; R2 their same-level neighbours (a node: its neighbour nodes and incident edges;
        an edge: its end nodes and the other edges of its two triangles); R3 their children
        on the next level (a node: its fine copy, the odd nodes and half-edges around it; an
        edge: its midpoint and the six fine edges at it); all of jmin; then top-down, per
        level, R4 h/u consistency (edges at active nodes, then end nodes of active edges) and
        R5 the prediction stencils of every active point on the level below.  Finally the
        inverse transform rewrites every active fine point from its coarse level and the
        details that are kept (those of points active before and after); coarse values are
        never changed, so the mass on jmin is unchanged."""
        det = self.details()
        eh, eu = self.thresholds(eps) if thresholds is None else thresholds
        sig_n, sig_e = self.significant(det, eh, eu)
        self.last = dict(det=det, eh=eh, eu=eu, sig_n=sig_n, sig_e=sig_e)
        new_n = {j: sig_n[j].copy() for j in self.levels}
        new_e = {j: sig_e[j].copy() for j in self.levels}
        for j in self.levels:
            g = self.g[j]
            # R2: same-level neighbours
            sn, se = sig_n[j], sig_e[j]
            nb = g.c_nbrs[sn]
            new_n[j][nb[nb >= 0]] = True
            ce = g.c_edges[sn]
            new_e[j][ce[ce >= 0]] = True
            new_n[j][g.e_nodes[se].ravel()] = True
            tri = g.e_tris[se].ravel()
            new_e[j][g.t_edges[tri].ravel()] = True
            # R3: children on the next level
            if j < self.jmax:
                P = self.pairs[j]
                f = j + 1
                gf = self.g[f]
                if allow is not None and j in allow:
                    sn = sn & allow[j](np.arange(g.N))
                    se = se & allow[j](np.arange(g.E) // 3)
                kids = P.even[sn]
                new_n[f][kids] = True
                nbk = gf.c_nbrs[kids]
                new_n[f][nbk[nbk >= 0]] = True
                cek = gf.c_edges[kids]
                new_e[f][cek[cek >= 0]] = True
                m = P.mid[se]
                new_n[f][m] = True
                cem = gf.c_edges[m]
                new_e[f][cem[cem >= 0]] = True
        new_n[self.jmin][:] = True
        new_e[self.jmin][:] = True
        for j in range(self.jmax, self.jmin - 1, -1):
            g = self.g[j]
            # R4: consistency
            ce = g.c_edges[new_n[j]]
            new_e[j][ce[ce >= 0]] = True
            new_n[j][g.e_nodes[new_e[j]].ravel()] = True
            if j > self.jmin:
                # R5: prediction stencils on level j-1
                P = self.pairs[j - 1]
                gc = self.g[j - 1]
                odd_act = new_n[j][P.mid]
                new_n[j - 1][P.cells[odd_act].ravel()] = True
                ev_act = new_n[j][P.even]
                new_n[j - 1][ev_act] = True
                half_act = new_e[j][P.h1] | new_e[j][P.h2]
                new_e[j - 1][half_act] = True
                tl, tr = gc.e_tris[half_act, 0], gc.e_tris[half_act, 1]
                new_e[j - 1][P.v_sten[tl].ravel()] = True
                new_e[j - 1][P.v_sten[tr].ravel()] = True
                tri_act = new_e[j][P.int_e].any(1)
                new_e[j - 1][P.v_sten[tri_act].ravel()] = True
        # inverse transform with the kept details (points active before and after), top-down
        dh, u = self.inverse(det, lambda f, pts, kind: self._active(f, pts, kind) & self._active(f, pts, kind, new_n, new_e))
        self.dh, self.u = dh, u
        self.node_act, self.edge_act = new_n, new_e
        return eh, eu

    # --------------------------------------------------------------- diagnostics
    def finest_level(self):
        """Highest level holding an active point: the maximum level the thresholds select when
        jmax only caps the refinement (Sec. 3.1, Jmax set implicitly by eps)."""
        return max(j for j in self.levels if self.node_act[j].any() or self.edge_act[j].any())

    def mass(self, p):
        return float((self.A[self.jmin] * (p.H + self.dh[self.jmin])).sum())

    def reconstructed_mass(self, p):
        dh, _, _, _ = self.get_state(self.jmax)
        return float((self.A[self.jmax] * (p.H + dh)).sum())


def regime_thresholds(eps, regime, U, g, L=None, f=None, H=None):
    """Absolute thresholds (eps_h [m], eps_u [m/s]) of the two flow regimes of Sec. 3.1.

    Reading: the printed pair gives a velocity threshold in m/s and a height threshold in
    geopotential units (m^2/s^2) under exchanged names; with the names swapped back and the
    geopotential divided by g,
      quasi-geostrophic, Ro = U/(f L):  eps_u = U Ro eps^1.5,  eps_h = f U L Ro eps^1.5 / g;
      inertia-gravity, c = sqrt(g H):   eps_u = U eps^1.5,     eps_h = c U eps^1.5 / g.
    """
    e32 = eps ** 1.5
    if regime == "qg":
        Ro = U / (f * L)
        return f * U * L * Ro * e32 / g, U * Ro * e32
    if regime == "ig":
        c = np.sqrt(g * H)
        return c * U * e32 / g, U * e32
    raise ValueError(regime)

"""Oracle: nested icosahedral C-grid, spherical geometry and TRiSK weights (plain FP64 numpy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package: only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

What is built here, and where the paper defines it:

* Sec. 2.2 and Fig. 1: the level-0 grid is the icosahedron projected on the sphere; each
  level adds the arc midpoints of the previous level's edges ("edge bisection and projection
  to the sphere"), so the node sets of successive levels are nested.
* Sec. 4.1: all areas are spherical polygons, all lengths are great-circle arcs; the dual
  cells are hexagons except 12 pentagons.
* Sec. 5.2: one computational element is one node, two triangles and three edges; the
  unfolded icosahedron is 10 lozenges of regular sub-grids.  The canonical numbering used at
  the library boundary follows that element structure (lozenge L, row i, column j).
* Sec. 3.1 (TRiSK, energy-conserving variant for qF^perp): the operator weights.  The TRiSK
  papers are not reproduced in the paper, so the weights are derived here from the two
  properties the scheme is built on (antisymmetry => the Coriolis term does no work; the
  curl of the perpendicular flux equals the kite-weighted divergence => steady geostrophic
  modes); the tests check both properties and the regular-hexagon limit.

The construction is deliberately generic: canonical node ids are found by exact position
matching (not by lozenge seam rules), cells are ordered by sorting neighbour directions by
angle, and every adjacency is derived from the triangle list.
"""
from __future__ import annotations

import numpy as np

EARTH_RADIUS = 6.371e6
OMEGA = 7.292e-5
GRAVITY = 9.80616


def _normalize(v):
    return v / np.sqrt((v * v).sum(axis=-1, keepdims=True))


def icosahedron_vertices():
    """North pole, upper ring U_k (lon 72k), lower ring L_k (lon 72k+36), south pole."""
    s = 1.0 / np.sqrt(5.0)
    c = 2.0 / np.sqrt(5.0)
    k = np.arange(5)
    up = np.stack([c * np.cos(2 * np.pi * k / 5), c * np.sin(2 * np.pi * k / 5), np.full(5, s)], -1)
    lo = np.stack([c * np.cos(2 * np.pi * k / 5 + np.pi / 5), c * np.sin(2 * np.pi * k / 5 + np.pi / 5),
                   np.full(5, -s)], -1)
    return np.array([0.0, 0.0, 1.0]), up, lo, np.array([0.0, 0.0, -1.0])


def lozenge_corners():
    """Corners (c00, c10, c11, c01) of the 10 lozenges, each the union of two icosahedron
    faces (c00,c10,c11) and (c00,c11,c01), both counter-clockwise seen from outside.

    Lozenges 0..4: faces (U_k, L_k, U_k+1) and (U_k, U_k+1, N).
    Lozenges 5..9: faces (L_k, S, L_k+1) and (L_k, L_k+1, U_k+1).
    """
    N, up, lo, S = icosahedron_vertices()
    cor = np.empty((10, 2, 2, 3))
    for k in range(5):
        k1 = (k + 1) % 5
        cor[k, 0, 0], cor[k, 1, 0], cor[k, 1, 1], cor[k, 0, 1] = up[k], lo[k], up[k1], N
        cor[5 + k, 0, 0], cor[5 + k, 1, 0], cor[5 + k, 1, 1], cor[5 + k, 0, 1] = lo[k], S, lo[k1], up[k1]
    return cor


def lozenge_positions(J):
    """Unit positions of the closed lattice [0, 2^J]^2 of every lozenge at level J.

    Level j+1 keeps the level-j points at even indices and puts the normalised sum (the arc
    midpoint) of the two end points of each level-j edge at the odd ones (Sec. 2.2, Fig. 1).
    """
    P = lozenge_corners()
    for _ in range(J):
        m = P.shape[1] - 1
        Q = np.empty((10, 2 * m + 1, 2 * m + 1, 3))
        Q[:, ::2, ::2] = P
        Q[:, 1::2, ::2] = _normalize(P[:, :-1, :] + P[:, 1:, :])
        Q[:, ::2, 1::2] = _normalize(P[:, :, :-1] + P[:, :, 1:])
        Q[:, 1::2, 1::2] = _normalize(P[:, :-1, :-1] + P[:, 1:, 1:])
        P = Q
    return P


def _match_rows(canonical, query):
    """Index into ``canonical`` of each row of ``query`` by exact (bitwise) equality."""
    allp = np.ascontiguousarray(np.concatenate([canonical, query]))
    keys = allp.view(np.dtype((np.void, allp.dtype.itemsize * 3))).ravel()
    _, inv = np.unique(keys, return_inverse=True)
    inv = inv.ravel()
    nc = canonical.shape[0]
    first = np.full(inv.max() + 1, -1, dtype=np.int64)
    first[inv[:nc]] = np.arange(nc)
    assert np.unique(inv[:nc]).size == nc, "duplicate canonical positions"
    out = first[inv[nc:]]
    assert (out >= 0).all(), "lattice point with no canonical owner"
    return out


def _sph_tri_area(a, b, c):
    """Signed spherical triangle area on the unit sphere (Van Oosterom & Strackee, 1983).

    The triple product is formed from vertex differences (exact for nearby points), so its
    rounding does not grow like 1/h^2 for small triangles of size h."""
    num = ((a - c) * np.cross(b - c, c)).sum(-1)
    den = 1.0 + (a * b).sum(-1) + (b * c).sum(-1) + (c * a).sum(-1)
    return 2.0 * np.arctan2(num, den)


def _arc(a, b):
    """Great-circle angle between unit vectors (cross product from the exact difference)."""
    return np.arctan2(np.sqrt((np.cross(a - b, b) ** 2).sum(-1)), (a * b).sum(-1))


def _two_square(x):
    """x*x as an unevaluated sum p + e, exactly (Dekker's splitting)."""
    p = x * x
    c = 134217729.0 * x
    hi = c - (c - x)
    lo = x - hi
    e = ((hi * hi - p) + 2.0 * hi * lo) + lo * lo
    return p, e


def _norm2_minus_one(v):
    """|v|^2 - 1 to full relative precision for |v| ~ 1 (exact squares, Neumaier summation)."""
    terms = []
    for k in range(3):
        terms += list(_two_square(v[..., k]))
    terms.append(np.full(v.shape[:-1], -1.0))
    s = terms[0]
    comp = np.zeros_like(s)
    for t in terms[1:]:
        u = s + t
        comp = comp + np.where(np.abs(s) >= np.abs(t), (s - u) + t, (t - u) + s)
        s = u
    return s + comp


def _circumcentre(a, b, c):
    """Circumcentre of a counter-clockwise spherical triangle: the normal of the plane
    through the three unit directions, from direction differences b/|b| - a/|a| in which the
    (rounding-size) length error of each normalised position is removed exactly; otherwise it
    would tilt the plane by O(1e-16/h)."""
    def ddiff(q, p):
        sp = 0.5 * _norm2_minus_one(p)[..., None]
        sq = 0.5 * _norm2_minus_one(q)[..., None]
        return (q - p) + (sp * p - sq * q)
    return _normalize(np.cross(ddiff(b, a), ddiff(c, a)))


class Grid:
    """One uniform level J of the icosahedral grid with every TRiSK table.

    Canonical numbering (shared with the HIP library only as an interface):
      node  (L, i, j), 0 <= L < 10, 0 <= i, j < n = 2^J :  id = (L*n + i)*n + j;
      north pole 10 n^2, south pole 10 n^2 + 1;
      edge  3*id + d, d = 0: (i,j)->(i+1,j), 1: (i,j)->(i+1,j+1), 2: (i,j)->(i,j+1);
            u_e > 0 points from the owning node to the other end;
      triangle 2*id + t, t = 0: ((i,j),(i+1,j),(i+1,j+1)), t = 1: ((i,j),(i+1,j+1),(i,j+1)).
    """

    def __init__(self, J, radius=EARTH_RADIUS, omega=OMEGA):
        self.J = J
        self.n = n = 2 ** J
        self.radius = radius
        self.omega = omega
        self.N = 10 * n * n + 2
        self.E = 30 * n * n
        self.T = 20 * n * n
        P = lozenge_positions(J)
        owned = P[:, :n, :n].reshape(-1, 3)
        self.xyz = np.concatenate([owned, [[0.0, 0.0, 1.0]], [[0.0, 0.0, -1.0]]])
        cid = _match_rows(self.xyz, P.reshape(-1, 3)).reshape(10, n + 1, n + 1)
        assert (cid[:, :n, :n].ravel() == np.arange(10 * n * n)).all()
        self.lattice_id = cid
        self._topology(cid)
        self._geometry()
        self._trisk_weights()

    # ------------------------------------------------------------------ topology
    def _topology(self, cid):
        n = self.n
        I, Jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        L = np.arange(10)[:, None, None]
        c = lambda di, dj: cid[L, I + di, Jj + dj]  # noqa: E731
        p00, p10, p11, p01 = c(0, 0), c(1, 0), c(1, 1), c(0, 1)
        # edges owned by element (L,i,j)
        e_nodes = np.stack([np.stack([p00, p10], -1), np.stack([p00, p11], -1),
                            np.stack([p00, p01], -1)], -2).reshape(-1, 2)
        assert e_nodes.shape[0] == self.E
        self.e_nodes = e_nodes
        tri = np.stack([np.stack([p00, p10, p11], -1), np.stack([p00, p11, p01], -1)], -2).reshape(-1, 3)
        self.t_nodes = tri
        x = self.xyz
        assert (_sph_tri_area(x[tri[:, 0]], x[tri[:, 1]], x[tri[:, 2]]) > 0).all(), "triangle not CCW"

        # unordered pair -> edge
        lo = e_nodes.min(1).astype(np.int64)
        hi = e_nodes.max(1).astype(np.int64)
        key = lo * self.N + hi
        order = np.argsort(key)
        skey = key[order]
        assert (np.diff(skey) > 0).all(), "duplicate edge"
        self._edge_order, self._edge_skey = order, skey

        def find(a, b):
            k = np.minimum(a, b).astype(np.int64) * self.N + np.maximum(a, b)
            pos = np.searchsorted(skey, k)
            assert (skey[np.minimum(pos, skey.size - 1)] == k).all(), "triangle side is not an edge"
            e = order[pos]
            sgn = np.where(e_nodes[e, 0] == a, 1, -1)
            return e, sgn

        te = np.empty((self.T, 3), np.int64)
        ts = np.empty((self.T, 3), np.int64)
        for s in range(3):
            e, sg = find(tri[:, s], tri[:, (s + 1) % 3])
            te[:, s], ts[:, s] = e, sg
        self.t_edges, self.t_signs = te, ts   # t_{e,v}: +1 if u_e circulates CCW around v

        # each edge: the triangle on its left (CCW sense) and on its right
        e_left = np.full(self.E, -1, np.int64)
        e_right = np.full(self.E, -1, np.int64)
        tid = np.repeat(np.arange(self.T), 3)
        fe, fs = te.ravel(), ts.ravel()
        e_left[fe[fs > 0]] = tid[fs > 0]
        e_right[fe[fs < 0]] = tid[fs < 0]
        assert (e_left >= 0).all() and (e_right >= 0).all()
        self.e_tris = np.stack([e_left, e_right], 1)

        # cells: incident edges sorted counter-clockwise by angle around the node
        inc_node = np.concatenate([e_nodes[:, 0], e_nodes[:, 1]])
        inc_edge = np.concatenate([np.arange(self.E), np.arange(self.E)])
        inc_sign = np.concatenate([np.ones(self.E, np.int64), -np.ones(self.E, np.int64)])  # n_{e,i}
        other = np.concatenate([e_nodes[:, 1], e_nodes[:, 0]])
        o = np.argsort(inc_node, kind="stable")
        inc_node, inc_edge, inc_sign, other = inc_node[o], inc_edge[o], inc_sign[o], other[o]
        deg = np.bincount(inc_node, minlength=self.N)
        assert set(np.unique(deg)) <= {5, 6} and (deg == 5).sum() == 12
        start = np.concatenate([[0], np.cumsum(deg)[:-1]])
        slot = np.arange(inc_node.size) - start[inc_node]
        ce = np.full((self.N, 6), -1, np.int64)
        cs = np.zeros((self.N, 6), np.int64)
        cn = np.full((self.N, 6), -1, np.int64)
        ce[inc_node, slot], cs[inc_node, slot], cn[inc_node, slot] = inc_edge, inc_sign, other
        # local tangent basis at every node, angle of each neighbour
        a = x
        ref = np.where(np.abs(a[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
        b1 = _normalize(np.cross(ref, a))
        b2 = np.cross(a, b1)
        nb = x[np.where(cn >= 0, cn, 0)]
        ang = np.arctan2((nb * b2[:, None]).sum(-1), (nb * b1[:, None]).sum(-1))
        ang = np.where(cn >= 0, ang, np.inf)
        srt = np.argsort(ang, axis=1)
        rows = np.arange(self.N)[:, None]
        self.c_edges, self.c_signs, self.c_nbrs = ce[rows, srt], cs[rows, srt], cn[rows, srt]
        self.c_deg = deg
        # vertex between consecutive edges k and k+1: the triangle left of e_k oriented outward
        outward_left = np.where(self.c_signs > 0, self.e_tris[np.maximum(self.c_edges, 0), 0],
                                self.e_tris[np.maximum(self.c_edges, 0), 1])
        self.c_tris = np.where(self.c_edges >= 0, outward_left, -1)
        # check that it is also adjacent to the next edge (right of e_{k+1} oriented outward)
        nxt = np.where(np.arange(6)[None, :] + 1 < deg[:, None], np.arange(6)[None, :] + 1, 0)
        e_next = self.c_edges[rows, nxt]
        s_next = self.c_signs[rows, nxt]
        outward_right = np.where(s_next > 0, self.e_tris[np.maximum(e_next, 0), 1],
                                 self.e_tris[np.maximum(e_next, 0), 0])
        ok = (self.c_edges < 0) | (outward_right == self.c_tris)
        assert ok.all(), "cell edges are not in counter-clockwise order"

    def edge_between(self, a, b):
        """Edge joining nodes a and b (arrays), and +1 where it points from a to b."""
        a = np.asarray(a, np.int64)
        b = np.asarray(b, np.int64)
        k = np.minimum(a, b) * self.N + np.maximum(a, b)
        pos = np.searchsorted(self._edge_skey, k)
        pos = np.minimum(pos, self._edge_skey.size - 1)
        assert (self._edge_skey[pos] == k).all(), "nodes are not joined by an edge"
        e = self._edge_order[pos]
        return e, np.where(self.e_nodes[e, 0] == a, 1, -1)

    def cell_polygon(self, nodes):
        """Counter-clockwise dual-cell (hexagon/pentagon) vertices of `nodes`, padded to 6 by
        repeating the first vertex; returns (K, 6, 3) unit vectors and the vertex counts."""
        ct = self.c_tris[nodes]
        deg = self.c_deg[nodes]
        poly = self.t_cc[np.where(ct >= 0, ct, ct[:, :1])]
        return poly, deg

    # ------------------------------------------------------------------ geometry
    def _geometry(self):
        R = self.radius
        x = self.xyz
        tn = self.t_nodes
        a, b, c = x[tn[:, 0]], x[tn[:, 1]], x[tn[:, 2]]
        cc = _circumcentre(a, b, c)                        # circumcentre (dual vertex)
        self.t_cc = cc
        self.f_v = 2.0 * self.omega * cc[:, 2]
        en = self.e_nodes
        self.d_e = R * _arc(x[en[:, 0]], x[en[:, 1]])     # node-node arc
        self.l_e = R * _arc(cc[self.e_tris[:, 0]], cc[self.e_tris[:, 1]])  # dual (hexagon) edge
        self.e_mid = _normalize(x[en[:, 0]] + x[en[:, 1]])
        self.e_tan = _normalize(x[en[:, 1]] - x[en[:, 0]])
        # kite of node a in triangle (a,b,c): (a, mid(a,b), cc, mid(c,a))
        kites = np.empty((self.T, 3))
        for s in range(3):
            p, q, r = x[tn[:, s]], x[tn[:, (s + 1) % 3]], x[tn[:, (s + 2) % 3]]
            mpq, mrp = _normalize(p + q), _normalize(r + p)
            kites[:, s] = R * R * (_sph_tri_area(p, mpq, cc) + _sph_tri_area(p, cc, mrp))
        assert (kites > 0).all(), "circumcentre outside its triangle"
        self.t_kite = kites
        self.A_v = kites.sum(1)
        self.A_i = np.bincount(tn.ravel(), weights=kites.ravel(), minlength=self.N)
        self.R_iv = kites / self.A_v[:, None]              # kite / triangle (for h_v)
        # rho_{i,v} = kite / cell, per cell slot (for the TRiSK weights)
        ct = self.c_tris
        rows = np.arange(self.N)[:, None]
        kite_slot = np.zeros((self.N, 6))
        for s in range(3):
            hit = (tn[np.maximum(ct, 0), s] == rows) & (ct >= 0)
            kite_slot = np.where(hit, kites[np.maximum(ct, 0), s], kite_slot)
        self.c_rho = kite_slot / self.A_i[:, None]

    # ------------------------------------------------------------------ TRiSK weights
    def _trisk_weights(self):
        """Perpendicular-flux weights w_{e,e'} for the energy-conserving qF^perp (Sec. 3.1).

        For edge e in cell i with the cell's edges e_1..e_K counter-clockwise, and e' = the
        edge reached after passing the vertices v_k..v_{k'-1}:
            w_{e,e'} = n_{e,i} n_{e',i} (S - 1/2),   S = sum of kite/cell fractions passed.
        Per cell the integrated outward fluxes are distributed over the kites so that every
        kite carries its share of the cell divergence; the resulting cross-kite fluxes are the
        perpendicular fluxes.  The result is antisymmetric (w_{e',e} = -w_{e,e'}) and its curl
        equals the kite-weighted divergence.
        """
        E = self.E
        ecp = np.zeros((E, 10), np.int64)
        w = np.zeros((E, 10))
        fill = np.zeros(E, np.int64)
        deg = self.c_deg
        for i_side in range(2):
            cells = self.e_nodes[:, i_side]
            ce, cs, rho = self.c_edges[cells], self.c_signs[cells], self.c_rho[cells]
            K = deg[cells]
            me = np.argmax(ce == np.arange(E)[:, None], axis=1)    # slot of e in cell
            assert (ce[np.arange(E), me] == np.arange(E)).all()
            n_e = cs[np.arange(E), me]
            S = np.zeros(E)
            for step in range(1, 6):
                valid = step < K
                k_prev = (me + step - 1) % K
                k_now = (me + step) % K
                S = S + rho[np.arange(E), k_prev]
                ep = ce[np.arange(E), k_now]
                sp = cs[np.arange(E), k_now]
                col = np.minimum(fill, 9)
                ecp[np.arange(E)[valid], col[valid]] = ep[valid]
                w[np.arange(E)[valid], col[valid]] = (n_e * sp * (S - 0.5))[valid]
                fill = fill + valid
        self.ecp = np.where(np.arange(10)[None, :] < fill[:, None], ecp, np.arange(E)[:, None])
        self.w = w
        self.ecp_n = fill

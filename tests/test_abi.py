"""CPU checks of the C ABI library: it loads, exports every symbol that include/*.h declares,
and its host-side grid builder agrees with the oracle's (independent) construction."""
import glob
import os
import re

import numpy as np
import pytest

from paper_1404_0405_amd import wt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(wt_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = wt.load()
    declared = _declared_functions()
    assert len(declared) >= 20, declared
    for name in declared:
        assert hasattr(lib, name), name
    bound = {n for n, _, _ in wt.SIGNATURES}
    assert declared == bound, (declared - bound, bound - declared)


def test_errors_without_device_are_reported():
    lib = wt.load()
    assert lib.wt_grid_create(3, 2, 8) is None
    assert b"jmin" in lib.wt_last_error()
    assert lib.wt_grid_create(2, 2, 5) is None
    assert b"patch" in lib.wt_last_error()
    assert lib.wt_step(None, 1.0) == wt.WT_EINVAL
    assert lib.wt_save(None, b"/tmp/wt_none.ckpt") == wt.WT_EINVAL
    assert lib.wt_load(None, b"/tmp/wt_none.ckpt") == wt.WT_EINVAL


@pytest.mark.parametrize("J", [0, 1, 2, 3, 4])
def test_host_builder_matches_oracle(J, oracle_grid):
    """Seam-rule topology (library) == position-matching topology (oracle); geometry and the
    TRiSK weights agree to round-off."""
    h = wt.host_level_tables(J)
    g = oracle_grid(J)
    assert np.array_equal(h["e_nodes"], g.e_nodes)
    for k in ("A_i", "A_v", "d_e", "l_e"):
        assert np.allclose(h[k], getattr(g, k), rtol=1e-14, atol=0), k
    # stencil as (edge, e') -> w maps; padding slots hold e itself with weight 0
    for e in range(0, g.E, max(1, g.E // 997)):
        mine = {int(a): b for a, b in zip(h["ecp"][e], h["w"][e]) if not (a == e and b == 0.0)}
        ref = {int(g.ecp[e, k]): g.w[e, k] for k in range(g.ecp_n[e])}
        assert mine.keys() == ref.keys()
        assert all(abs(mine[k] - ref[k]) < 1e-14 for k in ref)


@pytest.mark.parametrize("jc,jmax", [(2, 4), (3, 4)])
def test_host_flux_restriction_matches_oracle(jc, jmax):
    """The library's flux-restriction rows between levels jc and jc+1 (eqs. (restr_flux),
    (ho_flux), (kml); effective areas from level jmax) give the oracle's restricted flux on random
    fine fluxes and divergences, on every coarse edge.  A row keeps at most 7 nonzero weights of its
    8 slots -- fine nodes whose terms cancel exactly are left out when it is built -- and its
    padding, after the nonzero entries, carries zero weight."""
    from oracle.multiscale import Hierarchy
    t = wt.host_pair_tables(jc, jmax)
    lf = wt.host_level_tables(jc + 1)["l_e"]
    lc = wt.host_level_tables(jc)["l_e"]
    H = Hierarchy(jc, jmax)
    rng = np.random.default_rng(7)
    Ff = rng.standard_normal(lf.size)
    cf = rng.standard_normal(H.g[jc + 1].N)
    phi = (t["rf_fw"] * (lf[t["rf_f"]] * Ff[t["rf_f"]])).sum(1) + (t["rf_cw"] * cf[t["rf_c"]]).sum(1)
    ref = H.flux_restrict(jc, Ff, cf)
    assert np.abs(phi / lc - ref).max() <= 1e-12 * np.abs(ref).max()
    nz = t["rf_cw"] != 0
    assert nz.sum(1).max() <= 7
    assert (np.diff(nz.astype(int), axis=1) <= 0).all()


@pytest.mark.parametrize("jc,jmax", [(2, 4), (3, 4)])
def test_host_pair_tables_match_oracle(jc, jmax):
    """The library's inter-scale tables between levels jc and jc+1 against the oracle's (same
    numbering of nodes, edges and triangles): the height-prediction weights s~ per coarse edge
    (eq. (WTpred)), the effective coarse areas, and the velocity predictions -- the three
    interior fine edges of every coarse triangle and (p1 - p2) of every coarse edge -- evaluated
    on random coarse velocities, all to round-off."""
    from oracle.multiscale import Hierarchy
    t = wt.host_pair_tables(jc, jmax)
    H = Hierarchy(jc, jmax)
    P, gc = H.pairs[jc], H.g[jc]
    for e in range(gc.E):
        mine = {int(c): w for c, w in zip(t["cells"][e], t["st"][e])}
        ref = {int(c): w for c, w in zip(P.cells[e], P.st[e])}
        assert mine.keys() == ref.keys()
        # areas of clipped spherical polygons summed in another order: measured 1.1e-14
        assert all(abs(mine[c] - ref[c]) < 1e-13 for c in ref)
    assert np.abs(t["A_c"] - H.A[jc]).max() <= 1e-13 * np.abs(H.A[jc]).max()
    uc = np.random.default_rng(3).standard_normal(gc.E)
    mine = (t["w_int"] * uc[t["v_sten"]][:, None, :]).sum(2)
    ref = P.u_int_pred(uc)
    # the interior edges of a triangle may be listed in another order
    assert np.abs(np.sort(mine, 1) - np.sort(ref, 1)).max() <= 1e-13 * np.abs(ref).max()
    tl, tr = gc.e_tris[:, 0], gc.e_tris[:, 1]
    mine = (t["w_pl"] * uc[t["v_sten"][tl]]).sum(1) + (t["w_pr"] * uc[t["v_sten"][tr]]).sum(1)
    ref = P.u_pair_pred(uc)
    assert np.abs(mine - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("J", [6, 7, 8])
def test_lattice_reference_geometry(J):
    """The 10 lozenges are congruent (rotations of the icosahedron map lattice to lattice), so
    one reference geometry serves all of them: it agrees with every lozenge's own tables to
    round-off; the builder's emulation of the kernel's halo addressing matched the canonical
    seam lookup for every regular tile (it aborts otherwise)."""
    tiles, rim, err = wt.host_lattice_check(J)
    n = 2 ** J
    assert tiles == (n // 16) * (n // 32) - 4
    assert rim == 4 * 16 * 32 * 10 + 2
    assert err < 1e-12, err


def test_bench_refuses_several_gpus():
    """bench.py runs on one GPU: --gpus N > 1 exits with status 2 and says so, before any GPU
    work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_traffic_only_for_the_measured_grid_and_source():
    """The HBM traffic figure of the bench line comes from counters taken on one grid level and
    one kernel source: the level-10 lattice kernel reports it while its source is the one measured,
    any other level or an unknown kernel reports null."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    import hashlib
    rec = bench.MEASURED_TRAFFIC["trisk_lattice"]
    current = all(hashlib.sha256(open(os.path.join(root, f), "rb").read()).hexdigest() == h
                  for f, h in zip(rec["sources"], rec["sha256"]))
    t = bench.measured_traffic("trisk_lattice", 10)
    if current:
        assert t is not None and 1.8e9 < t < 2.2e9
    else:
        assert t is None
    assert bench.measured_traffic("trisk_lattice", 8) is None
    assert bench.measured_traffic("trisk_tend", 10) is None

"""Consistency of the stored oracle samples under tests/golden/ (no GPU): sizes follow the grid's
closed forms N = 10 4^J + 2, E = 30 4^J (Table 1), the sampled entities are the ones the scripts
name (every pentagon, active points only), and jmin is whole."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _sizes(J):
    return 10 * 4 ** J + 2, 30 * 4 ** J


def _pentagons(J):
    """Lozenge corners (L, 0, 0) and the two poles: the 12 five-edge cells."""
    n, N = 2 ** J, _sizes(J)[0]
    return [(L * n) * n for L in range(10)] + [N - 2, N - 1]


def test_pentagon_ids():
    from oracle.grid import Grid
    g = Grid(3)
    assert sorted(np.flatnonzero(g.c_deg == 5).tolist()) == _pentagons(3)


def test_level10_samples():
    r = np.load(os.path.join(GOLDEN, "j10_samples.npz"))
    J = int(r["level"])
    N, E = _sizes(J)
    nodes, edges = r["nodes"], r["edges"]
    assert J == 10 and nodes.max() < N and edges.max() < E and nodes.min() >= 0
    pentagons = _pentagons(J)
    assert np.isin(pentagons, nodes).all()
    assert np.isin(3 * np.array(pentagons[:10])[:, None] + np.arange(3), edges).all()
    for k, m in (("ddh", "ddh_max"), ("du", "du_max"), ("dh1", "dh1_max"), ("u1", "u1_max")):
        assert np.isfinite(r[k]).all() and np.abs(r[k]).max() <= float(r[m])
    assert r["ddh"].size == nodes.size and r["du"].size == edges.size


def test_jet_levels_5_to_9_run():
    r = np.load(os.path.join(GOLDEN, "jet_l5_9_samples.npz"))
    jmin, jmax = int(r["jmin"]), int(r["jmax"])
    assert (jmin, jmax) == (5, 9)
    for j in range(jmin, jmax + 1):
        N, E = _sizes(j)
        na = np.unpackbits(r[f"na{j}"])
        ea = np.unpackbits(r[f"ea{j}"])
        assert na.size == -(-N // 8) * 8 and ea.size == -(-E // 8) * 8
        assert not na[N:].any() and not ea[E:].any()
        if j == jmin:
            assert na[:N].all() and ea[:E].all()
        assert na[r[f"ni{j}"]].all() and ea[r[f"ei{j}"]].all()
        assert r[f"ni{j}"].size == min(1024, int(na.sum()))
    assert float(r["mass"]) > 0 and 0 < float(r["dt"]) < 600

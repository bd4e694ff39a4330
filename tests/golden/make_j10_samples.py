"""Writes ``j10_samples.npz``: oracle values at sampled nodes and edges of the full-size uniform
grid (level 10, 10,485,762 cells) for the GPU parity test at that size.

Only ``oracle/`` and the seeded input generator are called.  The state is the seeded random field
of ``inputs.random_state`` (it depends on the entity index alone, so the GPU test regenerates it
bit for bit without the oracle's coordinates).  Stored: the tendencies of eqs. (height),(velo) and
the state after one classical RK4 step of ``DT`` seconds, at every pentagon, at seeded samples of
the lozenge borders and at seeded samples of the whole grid; and the maxima of the full fields,
which normalise the relative errors.

Run from the repository root: ``python tests/golden/make_j10_samples.py`` (about 5 minutes and
30 GB of host memory).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import trisk  # noqa: E402
from oracle.grid import Grid  # noqa: E402
from paper_1404_0405_amd import inputs  # noqa: E402

J = 10
SEED = 1010       # random_state seed of the state
SAMPLE_SEED = 4242
DT = 5.0          # seconds, below the stable step of this state
N_RANDOM = 2048   # random nodes and random edges each
N_BORDER = 64     # border elements per lozenge


def sample_ids(n, N, E):
    """Pentagons (lozenge corners and poles), seeded lozenge-border elements and seeded random
    entities; edges: the three edges of every sampled element plus random edges."""
    rng = np.random.default_rng(SAMPLE_SEED)
    corners = [(L * n) * n for L in range(10)]
    border = []
    for L in range(10):
        k = rng.integers(0, n, size=N_BORDER)
        side = rng.integers(0, 4, size=N_BORDER)
        i = np.where(side == 0, 0, np.where(side == 1, n - 1, k))
        j = np.where(side == 2, 0, np.where(side == 3, n - 1, k))
        border.append((L * n + i) * n + j)
    elems = np.unique(np.concatenate([np.array(corners), *border, rng.integers(0, 10 * n * n, size=N_RANDOM)]))
    nodes = np.unique(np.concatenate([elems, [N - 2, N - 1], rng.integers(0, N, size=N_RANDOM)]))
    edges = np.unique(np.concatenate([(3 * elems[:, None] + np.arange(3)).ravel(),
                                      rng.integers(0, E, size=N_RANDOM)]))
    return nodes.astype(np.int64), edges.astype(np.int64)


def main():
    t0 = time.time()
    g = Grid(J)
    print(f"grid {time.time() - t0:.0f} s", flush=True)
    n = 2 ** J
    dh, u = inputs.random_state(g.N, g.E, SEED)
    H = inputs.tc2_constants()[2]
    p = trisk.Params(mean_depth=H)
    ra, rb = trisk.tendencies(g, dh, u, p)
    print(f"tendencies {time.time() - t0:.0f} s", flush=True)
    sa, sb = trisk.step(g, dh, u, DT, p, "rk4")
    print(f"rk4 step {time.time() - t0:.0f} s", flush=True)
    nodes, edges = sample_ids(n, g.N, g.E)
    np.savez(os.path.join(HERE, "j10_samples.npz"), level=J, seed=SEED, dt=DT, mean_depth=H,
             nodes=nodes, edges=edges,
             ddh=ra[nodes], du=rb[edges], ddh_max=np.abs(ra).max(), du_max=np.abs(rb).max(),
             dh1=sa[nodes], u1=sb[edges], dh1_max=np.abs(sa).max(), u1_max=np.abs(sb).max())
    print(f"wrote {len(nodes)} nodes, {len(edges)} edges", flush=True)


if __name__ == "__main__":
    main()

"""Writes ``jet_l5_9_samples.npz``: the oracle's adaptive run of the zonal jet with its 120 m bump
on levels 5..9 at eps = 5e-3 (the adaptive workload at full size), for the GPU parity test at
that size.

Only ``oracle/`` and the seeded input generator are called.  The run: initial state on level 9,
then four rounds of threshold-and-zone adaptation (Sec. 2.3) and one classical RK4 step at 0.8 of
the stable step.  Stored: every level's node and edge masks (bit-packed), the state at seeded
samples of every level's active nodes and edges, the maxima over the active points (which
normalise the relative errors) and the jmin mass.

Run from the repository root: ``python tests/golden/make_jet_l5_9_samples.py`` (about 4 minutes,
11 GB of host memory).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import trisk  # noqa: E402
from oracle.multiscale import Hierarchy  # noqa: E402
from paper_1404_0405_amd import inputs  # noqa: E402

JMIN, JMAX, EPS, CFL, ROUNDS = 5, 9, 5e-3, 0.8, 4
SAMPLE_SEED = 5959
N_SAMPLE = 1024   # active nodes and active edges per level


def main():
    t0 = time.time()
    H = Hierarchy(JMIN, JMAX)
    print(f"hierarchy {time.time() - t0:.0f} s", flush=True)
    g = H.g[JMAX]
    dh, u, depth = inputs.jet(g.xyz, g.e_mid, g.e_tan)
    p = trisk.Params(mean_depth=depth)
    dt = trisk.suggest_dt(g, dh, u, p, CFL)
    H.set_state(JMAX, dh, u)
    for r in range(ROUNDS):
        H.adapt(EPS)
        H.step(dt, p)
        print(f"round {r} {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(SAMPLE_SEED)
    out = dict(jmin=JMIN, jmax=JMAX, eps=EPS, dt=dt, rounds=ROUNDS, mean_depth=depth, mass=H.mass(p))
    for j in H.levels:
        a, b, na, ea = H.get_state(j)
        ni, ei = np.flatnonzero(na), np.flatnonzero(ea)
        ni = np.sort(rng.choice(ni, size=min(N_SAMPLE, ni.size), replace=False))
        ei = np.sort(rng.choice(ei, size=min(N_SAMPLE, ei.size), replace=False))
        out.update({f"na{j}": np.packbits(na), f"ea{j}": np.packbits(ea), f"ni{j}": ni, f"ei{j}": ei,
                    f"dh{j}": a[ni], f"u{j}": b[ei],
                    f"dhmax{j}": np.abs(a[na]).max(initial=0.0), f"umax{j}": np.abs(b[ea]).max(initial=0.0)})
        print(f"level {j}: {int(na.sum())} nodes, {int(ea.sum())} edges active", flush=True)
    np.savez_compressed(os.path.join(HERE, "jet_l5_9_samples.npz"), **out)


if __name__ == "__main__":
    main()

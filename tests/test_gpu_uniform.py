"""GPU parity of the uniform-level TRiSK stage: HIP library (through the C ABI) against the
FP64 oracle on the same seeded inputs."""
import math
import os
import sys

import numpy as np
import pytest

from oracle import trisk
from paper_1404_0405_amd import inputs, wt

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _make(J, case, seed=0):
    g = wt.Grid(J, J, 8)
    x, m, t = g.coords(J)
    if case == "tc2":
        dh, u, H = inputs.tc2(x, m, t)
    elif case == "tc2p":
        dh, u, H = inputs.tc2_perturbed(x, m, t, amplitude=300.0)
    else:
        N, E, _ = g.info(J)
        dh, u = inputs.random_state(N, E, seed)
        H = inputs.tc2_constants()[2]
    return g, dh, u, H


def _oracle_inputs(og, case, seed=0):
    if case == "tc2":
        return inputs.tc2(og.xyz, og.e_mid, og.e_tan)
    if case == "tc2p":
        return inputs.tc2_perturbed(og.xyz, og.e_mid, og.e_tan, amplitude=300.0)
    dh, u = inputs.random_state(og.N, og.E, seed)
    return dh, u, inputs.tc2_constants()[2]


def _rel_inf(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("J,case", [(1, "rand"), (2, "rand"), (3, "tc2"), (4, "tc2p"), (5, "rand"), (6, "tc2p"),
                                    (6, "rand"), (7, "tc2p"), (7, "rand")])
def test_tendency_parity_fp64(J, case, oracle_grid):
    """One evaluation of eqs. (height),(velo): every node and edge within 1e-11 (rel L-inf).

    The height tendency of a near-balanced flow is a divergence about 10^3 smaller than its
    flux terms, so round-off of the geometry (~1e-14) appears at ~1e-12 of its maximum."""
    _say(f"tendency parity J={J} case={case}")
    og = oracle_grid(J)
    dh, u, H = _oracle_inputs(og, case, seed=J)
    g, gdh, gu, gH = _make(J, case, seed=J)
    with g:
        assert np.allclose(gdh, dh, rtol=1e-13, atol=1e-9) and np.allclose(gu, u, rtol=1e-13, atol=1e-12)
        g.set_params(mean_depth=H)
        g.set_state(J, dh, u)
        a, b = g.tendency(J)
    p = trisk.Params(mean_depth=H)
    ra, rb = trisk.tendencies(og, dh, u, p)
    assert _rel_inf(a, ra) < 1e-11, _rel_inf(a, ra)
    assert _rel_inf(b, rb) < 1e-11, _rel_inf(b, rb)


@pytest.mark.parametrize("J,scheme,nsteps", [(3, "rk4", 50), (4, "rk4", 50), (3, "ssprk43", 50), (5, "rk4", 20),
                                             (6, "rk4", 50), (6, "ssprk43", 20), (7, "rk4", 20)])
def test_step_parity_fp64(J, scheme, nsteps, oracle_grid):
    """50 Runge-Kutta steps: dh and u within 1e-11 relative L-inf of the oracle."""
    _say(f"step parity J={J} scheme={scheme} steps={nsteps}")
    og = oracle_grid(J)
    dh, u, H = _oracle_inputs(og, "tc2p")
    p = trisk.Params(mean_depth=H)
    dt = trisk.suggest_dt(og, dh, u, p, 0.8)
    g, _, _, _ = _make(J, "tc2p")
    with g:
        g.set_params(mean_depth=H, rk=wt.WT_RK4 if scheme == "rk4" else wt.WT_SSPRK43)
        g.set_state(J, dh, u)
        assert abs(g.suggest_dt(0.8) / dt - 1) < 1e-12
        for _ in range(nsteps):
            g.step(dt)
        gdh, gu, na, ea = g.get_state(J)
        d, code = g.diagnostics()
    assert code == wt.WT_OK and na.all() and ea.all()
    a, b = dh, u
    for _ in range(nsteps):
        a, b = trisk.step(og, a, b, dt, p, scheme)
    assert _rel_inf(gdh, a) < 1e-11, _rel_inf(gdh, a)
    assert _rel_inf(gu, b) < 1e-11, _rel_inf(gu, b)
    assert abs(d.mass / trisk.mass(og, a, p) - 1) < 1e-13
    assert abs(d.energy / trisk.energy(og, a, b, p) - 1) < 1e-10
    assert d.max_abs_dh == pytest.approx(np.abs(a).max(), rel=1e-11)
    assert d.max_abs_u == pytest.approx(np.abs(b).max(), rel=1e-11)


def test_fp32_tendency_mode_error_and_mass(oracle_grid):
    """FP32 tendencies with FP64 state: error against the FP64 oracle stated; mass conserved."""
    J, nsteps = 6, 50
    _say(f"fp32 mode J={J}")
    og = oracle_grid(J)
    dh, u, H = _oracle_inputs(og, "tc2p")
    p = trisk.Params(mean_depth=H)
    dt = trisk.suggest_dt(og, dh, u, p, 0.8)
    g, _, _, _ = _make(J, "tc2p")
    with g:
        g.set_params(mean_depth=H, precision=wt.WT_FP32_TENDENCY)
        g.set_state(J, dh, u)
        m0 = g.diagnostics()[0].mass
        for _ in range(nsteps):
            g.step(dt)
        gdh, gu, _, _ = g.get_state(J)
        m1 = g.diagnostics()[0].mass
    a, b = dh, u
    for _ in range(nsteps):
        a, b = trisk.step(og, a, b, dt, p)
    l2h = math.sqrt((og.A_i * (H + gdh - (H + a)) ** 2).sum() / (og.A_i * (H + a) ** 2).sum())
    _say(f"fp32 tendency: rel L2 height error {l2h:.3e}, rel Linf u {_rel_inf(gu, b):.3e}, mass drift {abs(m1 / m0 - 1):.2e}")
    assert l2h < 1e-5
    assert abs(m1 / m0 - 1) < 1e-13


def test_step_deterministic():
    """Gather-only kernels: two runs are bitwise identical."""
    outs = []
    for _ in range(2):
        g, dh, u, H = _make(4, "tc2p")
        with g:
            g.set_params(mean_depth=H)
            g.set_state(4, dh, u)
            for _ in range(5):
                g.step(300.0)
            outs.append(g.get_state(4)[:2])
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_error_paths_on_device():
    g = wt.Grid(2, 2, 8)
    with g:
        with pytest.raises(wt.WtError):
            g.step(10.0)                   # no state yet
        N, E, _ = g.info(2)
        with pytest.raises(ValueError):
            g.set_state(2, np.zeros(N + 1), np.zeros(E))
        dh = np.zeros(N)
        dh[7] = np.nan
        g.set_state(2, dh, np.zeros(E))
        d, code = g.diagnostics()
        assert code == wt.WT_ENUMERIC
        with pytest.raises(wt.WtError):
            g.step(-1.0)


def test_full_size_j10_properties():
    """The bench configuration (uniform J=10, 10,485,762 cells, TC2 + seeded SH perturbation,
    RK4): mass conserved to 1e-13, the state stays finite and close to the balanced flow, and
    the energy drift over the steps is tiny."""
    J = 10
    _say("full size J=10")
    g = wt.Grid(J, J, 8)
    with g:
        x, m, t = g.coords(J)
        dh, u, H = inputs.tc2_perturbed(x, m, t, device="cuda")
        g.set_params(mean_depth=H)
        g.set_state(J, dh, u)
        d0, _ = g.diagnostics()
        dt = g.suggest_dt(0.8)
        assert 7.0 < dt < 12.0, dt
        for _ in range(5):
            g.step(dt)
        d1, code = g.diagnostics()
        gdh, gu, _, _ = g.get_state(J)
    assert code == wt.WT_OK
    assert abs(d1.mass / d0.mass - 1) < 1e-13
    assert abs(d1.energy / d0.energy - 1) < 1e-9
    assert np.abs(gdh - dh).max() < 5.0 and np.abs(gu - u).max() < 2.0


def test_full_size_j10_sampled_parity():
    """Full size (level 10, 10,485,762 cells), the grid and kernels the bench times: tendencies
    of eqs. (height),(velo) and one classical RK4 step of a seeded random state against oracle
    values stored at sampled nodes and edges (every pentagon, lozenge borders, seeded random
    entities; tests/golden/make_j10_samples.py), within 1e-11 of the full field's maximum; the
    maxima of the full fields, which cover every entity, agree to the same bound; FP32
    tendencies within 1e-5."""
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "j10_samples.npz"))
    J = int(ref["level"])
    _say(f"full size J={J} sampled parity")
    g = wt.Grid(J, J, 8)
    with g:
        N, E, _ = g.info(J)
        dh, u = inputs.random_state(N, E, int(ref["seed"]))
        g.set_params(mean_depth=float(ref["mean_depth"]), rk=wt.WT_RK4, precision=wt.WT_FP64)
        g.set_state(J, dh, u)
        a, b = g.tendency(J)
        g.set_params(precision=wt.WT_FP32_TENDENCY)
        a32, b32 = g.tendency(J)
        g.set_params(precision=wt.WT_FP64)
        g.step(float(ref["dt"]))
        gdh, gu, _, _ = g.get_state(J)
    nodes, edges = ref["nodes"], ref["edges"]
    # FP32 tendencies of FP64 state: operands rounded to 6e-8 relative, sums of a few terms of
    # the size of the result (random fields: no cancellation), so 1e-5 leaves a wide margin
    assert np.abs(a32[nodes] - ref["ddh"]).max() / float(ref["ddh_max"]) < 1e-5
    assert np.abs(b32[edges] - ref["du"]).max() / float(ref["du_max"]) < 1e-5
    for got, full, want, wmax in ((a[nodes], a, ref["ddh"], ref["ddh_max"]), (b[edges], b, ref["du"], ref["du_max"]),
                                  (gdh[nodes], gdh, ref["dh1"], ref["dh1_max"]),
                                  (gu[edges], gu, ref["u1"], ref["u1_max"])):
        err = np.abs(got - want).max() / float(wmax)
        assert err < 1e-11, err
        assert np.abs(full).max() == pytest.approx(float(wmax), rel=1e-11)

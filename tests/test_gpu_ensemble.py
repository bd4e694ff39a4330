"""Ensembles on the GPU: one graph launch per ensemble step gives bitwise the states of the
members stepped one by one, with the blanket zone and with the learned zone."""
import numpy as np
import pytest

from paper_1404_0405_amd import inputs, wt

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-ensemble]", *a, flush=True)


def _member(p, jmin=4, prec=wt.WT_FP64):
    g = wt.Grid(jmin, p["jmax"], 8)
    x, m, t = g.coords(p["jmax"])
    dh, u, H = inputs.jet(x, m, t, bump=p["bump"], bump_lat=p["bump_lat"], bump_lon=p["bump_lon"])
    g.set_params(mean_depth=H, rk=wt.WT_RK4, precision=prec)
    g.set_state(p["jmax"], dh, u)
    return g


@pytest.mark.parametrize("learned", [False, True])
def test_ensemble_graph_equals_members_one_by_one(learned):
    params = inputs.ensemble_members(4, jmax_choices=(5, 6, 7))
    _say(f"members {[(p['jmax'], p['eps']) for p in params]} learned={learned}")
    nsteps = 5
    mlp = wt.Mlp(inputs.mlp_init()) if learned else None
    # one by one
    ref = []
    for p in params:
        g = _member(p)
        with g:
            if learned:
                g.set_predictor(mlp, 0.5)
            dt = g.suggest_dt(0.8)
            for _ in range(nsteps):
                g.adapt(p["eps"])
                g.step(dt)
            ref.append(([g.get_state(j) for j in range(g.jmin, g.jmax + 1)], g.redo_count(), dt))
    # ensemble
    grids = [_member(p) for p in params]
    if learned:
        for g in grids:
            g.set_predictor(mlp, 0.5)
    dts = [r[2] for r in ref]
    with wt.Ensemble(grids) as ens:
        for _ in range(nsteps):
            ens.adapt([p["eps"] for p in params])
            ens.step(dts)
        captures, launches = ens.stats()
    assert launches == nsteps and 1 <= captures <= nsteps
    for g, (states, redo, _) in zip(grids, ref):
        got = [g.get_state(j) for j in range(g.jmin, g.jmax + 1)]
        for a, b in zip(got, states):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
        assert g.redo_count() == redo
        g.close()
    if mlp:
        mlp.close()
    _say(f"captures {captures}, launches {launches}")


def test_ensemble_rejects_shared_grid():
    g = wt.Grid(3, 4, 8)
    with g:
        with pytest.raises(wt.WtError):
            wt.Ensemble([g, g])

"""Ensembles on the GPU: one graph launch, or one persistent batched launch over a work queue,
per ensemble step gives bitwise the states of the members stepped one by one, with the blanket
zone and with the learned zone, in FP64 and with FP32 tendencies."""
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


@pytest.mark.parametrize("learned,batched", [(False, False), (True, False), (False, True), (True, True)])
def test_ensemble_graph_equals_members_one_by_one(learned, batched):
    params = inputs.ensemble_members(4, jmax_choices=(5, 6, 7))
    # batched: members of both precisions in one launch
    precs = [wt.WT_FP32_TENDENCY if (batched and k % 2) else wt.WT_FP64 for k in range(len(params))]
    _say(f"members {[(p['jmax'], p['eps']) for p in params]} learned={learned} batched={batched}")
    nsteps = 5
    mlp = wt.Mlp(inputs.mlp_init()) if learned else None
    # one by one
    ref = []
    for p, prec in zip(params, precs):
        g = _member(p, prec=prec)
        with g:
            if learned:
                g.set_predictor(mlp, 0.5)
            dt = g.suggest_dt(0.8)
            for _ in range(nsteps):
                g.adapt(p["eps"])
                g.step(dt)
            ref.append(([g.get_state(j) for j in range(g.jmin, g.jmax + 1)], g.redo_count(), dt))
    # ensemble
    grids = [_member(p, prec=prec) for p, prec in zip(params, precs)]
    if learned:
        for g in grids:
            g.set_predictor(mlp, 0.5)
    dts = [r[2] for r in ref]
    with wt.Ensemble(grids) as ens:
        if batched:
            ens.set_batched(True)
        for _ in range(nsteps):
            ens.adapt([p["eps"] for p in params])
            ens.step(dts)
        captures, launches = ens.stats()
        if batched:
            shape = ens.tuning()
            _say(f"batched launch shape {shape}")
            assert shape["workgroups_per_cu"] >= 1 and shape["chunk_entries"] >= 256 and shape["last_launch_ms"] > 0
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


def test_batched_ensemble_rejects_single_level_member():
    g1, g2 = wt.Grid(3, 4, 8), wt.Grid(4, 4, 8)
    with g1, g2:
        with wt.Ensemble([g1, g2]) as ens:
            with pytest.raises(wt.WtError):
                ens.set_batched(True)


def test_batched_ensemble_mixed_schemes_and_whole_levels():
    """Batched step over members that differ in everything the step depends on: RK4 and SSPRK(4,3),
    FP64 and FP32 tendencies, work lists on and off (a member stepped over whole levels), levels
    3..5 to 4..7: bitwise equal to stepping the same members one by one."""
    params = inputs.ensemble_members(4, jmax_choices=(5, 6, 7))
    setup = [(wt.WT_RK4, wt.WT_FP64, True, 4), (wt.WT_SSPRK43, wt.WT_FP32_TENDENCY, True, 4),
             (wt.WT_SSPRK43, wt.WT_FP64, False, 3), (wt.WT_RK4, wt.WT_FP32_TENDENCY, False, 4)]

    def make(p, rk, prec, lists, jmin):
        g = wt.Grid(jmin, p["jmax"], 8)
        x, m, t = g.coords(p["jmax"])
        dh, u, H = inputs.jet(x, m, t, bump=p["bump"], bump_lat=p["bump_lat"], bump_lon=p["bump_lon"])
        g.set_params(mean_depth=H, rk=rk, precision=prec)
        g.set_state(p["jmax"], dh, u)
        g.set_work_lists(lists)
        return g

    nsteps = 4
    ref, dts = [], []
    for p, st in zip(params, setup):
        g = make(p, *st)
        with g:
            dt = g.suggest_dt(0.8)
            for _ in range(nsteps):
                g.adapt(p["eps"])
                g.step(dt)
            ref.append([g.get_state(j) for j in range(g.jmin, g.jmax + 1)])
            dts.append(dt)
    grids = [make(p, *st) for p, st in zip(params, setup)]
    with wt.Ensemble(grids) as ens:
        ens.set_batched(True)
        for _ in range(nsteps):
            ens.adapt([p["eps"] for p in params])
            ens.step(dts)
    for g, states in zip(grids, ref):
        got = [g.get_state(j) for j in range(g.jmin, g.jmax + 1)]
        for a, b in zip(got, states):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
        g.close()


def test_ensemble_graph_follows_parameter_changes():
    """A captured ensemble step is replayed only while its launches stay the same: changing a
    member's scheme or precision between steps (no adapt in between, so the work lists stay)
    recaptures it, and the states equal the members stepped one by one on the same schedule."""
    params = inputs.ensemble_members(3, seed=inputs.SEED_BASE + 9, jmax_choices=(5, 6))
    changes = [dict(rk=wt.WT_SSPRK43), dict(precision=wt.WT_FP32_TENDENCY), dict(mean_depth=9000.0)]

    def schedule(step_all, set_all, adapt_all):
        adapt_all()
        step_all()
        step_all()
        set_all()
        step_all()
        step_all()

    ref, dts = [], []
    for p, ch in zip(params, changes):
        g = _member(p)
        with g:
            dt = g.suggest_dt(0.8)
            dts.append(dt)
            schedule(lambda: g.step(dt), lambda: g.set_params(**ch), lambda: g.adapt(p["eps"]))
            ref.append([g.get_state(j) for j in range(g.jmin, g.jmax + 1)])
    grids = [_member(p) for p in params]
    with wt.Ensemble(grids) as ens:
        def set_all():
            for g, ch in zip(grids, changes):
                g.set_params(**ch)
        schedule(lambda: ens.step(dts), set_all, lambda: ens.adapt([p["eps"] for p in params]))
        captures, launches = ens.stats()
    _say(f"captures {captures}, launches {launches}")
    assert launches == 4 and captures == 2
    for g, states in zip(grids, ref):
        got = [g.get_state(j) for j in range(g.jmin, g.jmax + 1)]
        for a, b in zip(got, states):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
        g.close()


@pytest.mark.parametrize("batched", [False, True])
def test_ensemble_members_against_the_oracle(batched):
    """Every FP64 member of a 3-member ensemble (uneven levels 2..4 / 2..5, different bumps and
    thresholds; graph or batched step) against the oracle hierarchy stepped alone: masks
    identical and states within 1e-11 after 6 rounds of adapt + step."""
    from oracle import trisk
    from oracle.multiscale import Hierarchy
    params = inputs.ensemble_members(3, jmax_choices=(4, 5))
    _say(f"oracle members {[(p['jmax'], p['eps']) for p in params]} batched={batched}")
    grids, hier, dts = [], [], []
    for p in params:
        g = _member(p, jmin=2)
        H = Hierarchy(2, p["jmax"])
        og = H.g[p["jmax"]]
        dh, u, Hd = inputs.jet(og.xyz, og.e_mid, og.e_tan, bump=p["bump"], bump_lat=p["bump_lat"],
                               bump_lon=p["bump_lon"])
        H.set_state(p["jmax"], dh, u)
        grids.append(g)
        hier.append((H, trisk.Params(mean_depth=Hd)))
        dts.append(g.suggest_dt(0.8))
    with wt.Ensemble(grids) as ens:
        if batched:
            ens.set_batched(True)
        for _ in range(6):
            ens.adapt([p["eps"] for p in params])
            ens.step(dts)
            for (H, op), p, dt in zip(hier, params, dts):
                H.adapt(p["eps"])
                H.step(dt, op)
    worst = 0.0
    for g, (H, _) in zip(grids, hier):
        for j in H.levels:
            a, b, na, ea = H.get_state(j)
            x, y, gna, gea = g.get_state(j)
            assert np.array_equal(gna.astype(bool), na) and np.array_equal(gea.astype(bool), ea), j
            worst = max(worst, np.abs(x - a).max() / np.abs(a).max(), np.abs(y - b).max() / np.abs(b).max())
        g.close()
    _say(f"worst rel Linf against the oracle {worst:.2e}")
    assert worst < 1e-11

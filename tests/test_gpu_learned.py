"""Learned adjacent zone on the GPU: patch features and labels against a numpy recomputation
from the library's details and masks; the gate's limits (always allow = the paper's blanket
zone, always drop = every step redone by the threshold test, both bitwise equal to the plain
run); and a network trained on the method's own history, compared with the plain method."""
import sys

import numpy as np
import pytest

from paper_1404_0405_amd import inputs, wt

pytestmark = pytest.mark.gpu

DD0, DD1 = (1, 1, 0), (0, 1, 1)


def _say(*a):
    print("[gpu-learned]", *a, flush=True)
    sys.stdout.flush()


def _grid(jmin, jmax, case="jet", seed_bump=0.0):
    g = wt.Grid(jmin, jmax, 8)
    x, m, t = g.coords(jmax)
    if case == "jet":
        dh, u, H = inputs.jet(x, m, t, bump_lon=seed_bump)
    else:
        dh, u, H = inputs.tc2_perturbed(x, m, t, amplitude=300.0)
    g.set_params(mean_depth=H, rk=wt.WT_RK4)
    g.set_state(jmax, dh, u)
    return g


def _fid(L, i, j, n):
    return (L * n + i) * n + j


def _point_r(jc, dh, dp, di, eh, eu, nf):
    """Detail size of every point of level jc+1 from the details of pair (jc, jc+1), and the
    detail magnitudes at those points (for significance)."""
    n = 2 ** jc
    di = np.asarray(di).ravel()
    Nf, Ef = 10 * nf * nf + 2, 30 * nf * nf
    rn = np.full(Nf, -2.0)
    re = np.full(Ef, -2.0)
    an = np.zeros(Nf)
    ae = np.zeros(Ef)

    def r(d, eps):
        with np.errstate(divide="ignore"):
            v = np.where(np.abs(d) > 0, np.log2(np.abs(d) / eps), -16.0)
        return np.clip(v, -16.0, 4.0) / 8.0

    L, i, j = np.meshgrid(np.arange(10), np.arange(n), np.arange(n), indexing="ij")
    L, i, j = L.ravel(), i.ravel(), j.ravel()
    cid = (L * n + i) * n + j
    for d in range(3):
        e = 3 * cid + d
        mid = _fid(L, 2 * i + DD0[d], 2 * j + DD1[d], nf)
        rn[mid] = r(dh[e], eh)
        an[mid] = np.abs(dh[e])
        h1 = 3 * _fid(L, 2 * i, 2 * j, nf) + d
        h2 = 3 * mid + d
        re[h1] = re[h2] = r(dp[e], eu)
        ae[h1] = ae[h2] = np.abs(dp[e])
    # interior fine edges of the two coarse triangles of each element (int_e order)
    f = lambda a, b: _fid(L, 2 * i + a, 2 * j + b, nf)
    ints = {(0, 0): 3 * f(1, 0) + 1, (0, 1): 3 * f(1, 1) + 0, (0, 2): 3 * f(1, 0) + 2,
            (1, 0): 3 * f(1, 1) + 2, (1, 1): 3 * f(0, 1) + 1, (1, 2): 3 * f(0, 1) + 0}
    for (t, s), fe in ints.items():
        v = di[3 * (2 * cid + t) + s]
        re[fe] = r(v, eu)
        ae[fe] = np.abs(v)
    return rn, re, an, ae


def _numpy_stats(g, j, eps, pre):
    """Patch statistics of level j recomputed from the library's details, masks and state.
    `pre`: the state and masks of every level before the adapt (thresholds and significance
    are taken on them, as the adapt does); activity features use the masks after it."""
    jmin, jmax = g.jmin, g.jmax
    st = {lv: g.get_state(lv) for lv in range(jmin, jmax + 1)}
    eh = eps * max(np.abs(pre[lv][0][pre[lv][2] > 0]).max() for lv in pre)
    eu = eps * max(np.abs(pre[lv][1][pre[lv][3] > 0]).max() for lv in pre)
    n, nf = 2 ** j, 2 ** (j + 1)
    rn, re, an, ae = _point_r(j - 1, *g.get_details(j), eh, eu, n)
    rnf, ref, _, _ = _point_r(j, *g.get_details(j + 1), eh, eu, nf)
    na = st[j][2] > 0
    naf = st[j + 1][2] > 0
    na0, ea = pre[j][2] > 0, pre[j][3] > 0
    sn = na0 & (an >= eh)
    se = ea & (ae >= eu)
    # significant half-edges need both halves active: recompute per coarse edge
    dh_, dp_, _ = g.get_details(j)
    nc = n // 2
    L, i, jj = [a.ravel() for a in np.meshgrid(np.arange(10), np.arange(nc), np.arange(nc), indexing="ij")]
    cid = (L * nc + i) * nc + jj
    for d in range(3):
        h1 = 3 * _fid(L, 2 * i, 2 * jj, n) + d
        h2 = 3 * _fid(L, 2 * i + DD0[d], 2 * jj + DD1[d], n) + d
        both = ea[h1] & ea[h2] & (np.abs(dp_[3 * cid + d]) >= eu)
        se[h1] = both
        se[h2] = both
    E = lambda a: a[: 10 * n * n]
    el = lambda a: a.reshape(10, n, n)
    ah, au = el(E(rn)), el(np.maximum.reduce([re[0::3], re[1::3], re[2::3]]))
    sig = el(E(sn).astype(float) + se[0::3] + se[1::3] + se[2::3])
    act = el(E(na).astype(float))
    fr = lambda a: a.reshape(10, n, 2, n, 2)
    bh = fr(rnf[: 10 * nf * nf]).max((2, 4))
    bu = fr(np.maximum.reduce([ref[0::3], ref[1::3], ref[2::3]])).max((2, 4))
    actf = fr(naf[: 10 * nf * nf].astype(float)).sum((2, 4))
    m = n // 8
    P = lambda a: a.reshape(10, m, 8, m, 8)
    Q = lambda a: a.reshape(10, m, 2, 4, m, 2, 4)
    stats = np.zeros((10, m, m, 32))
    for k, a in enumerate((ah, au, bh, bu)):
        stats[..., k] = P(a).max((2, 4))
        stats[..., 4 + 4 * k:8 + 4 * k] = Q(a).max((3, 6)).transpose(0, 1, 3, 2, 4).reshape(10, m, m, 4)
    stats[..., 20:24] = Q(actf).sum((3, 6)).transpose(0, 1, 3, 2, 4).reshape(10, m, m, 4) / 64
    stats[..., 24:28] = Q(sig).sum((3, 6)).transpose(0, 1, 3, 2, 4).reshape(10, m, m, 4)
    stats[..., 28] = P(act).sum((2, 4)) / 64
    return stats, m


def _numpy_features(stats, m, level_pos):
    X = np.zeros((10, m, m, 64))
    pad = np.pad(stats, ((0, 0), (1, 1), (1, 1), (0, 0)), mode="edge")
    k = 0
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            nb = pad[:, 1 + di:1 + di + m, 1 + dj:1 + dj + m]
            # outside the lozenge the patch repeats itself (not its edge neighbour)
            ii, jj = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
            out = (ii + di < 0) | (ii + di >= m) | (jj + dj < 0) | (jj + dj >= m)
            nb = np.where(out[None, :, :, None], stats, nb)
            for q in range(4):
                X[..., 9 * q + k] = nb[..., q]
            k += 1
    X[..., 36:52] = stats[..., 4:20]
    X[..., 52:56] = stats[..., 20:24]
    X[..., 56:60] = stats[..., 24:28] / 64
    X[..., 60] = stats[..., 28]
    X[..., 61] = level_pos
    X[..., 62] = 1.0
    return X.reshape(-1, 64)


@pytest.mark.parametrize("jmin,jmax,eps", [(4, 7, 5e-3), (5, 7, 1e-2)])
def test_features_and_labels_match_numpy(jmin, jmax, eps):
    import torch
    _say(f"features {jmin}..{jmax} eps={eps}")
    g = _grid(jmin, jmax)
    with g:
        g.adapt(eps)
        pre = {lv: g.get_state(lv) for lv in range(jmin, jmax + 1)}
        g.adapt(eps)
        for j in range(jmin + 1, jmax):
            npatch = g.patch_count(j)
            assert npatch == 10 * (2 ** j // 8) ** 2
            x = torch.empty((npatch, 64), dtype=torch.float32, device="cuda")
            y = torch.empty((npatch, 4), dtype=torch.float32, device="cuda")
            g.patch_features(j, x)
            g.patch_labels(j, y)
            X, Y = x.cpu().numpy(), y.cpu().numpy()
            stats, m = _numpy_stats(g, j, eps, pre)
            Xr = _numpy_features(stats, m, (j - jmin) / (jmax - jmin))
            Yr = (stats[..., 24:28] > 0).reshape(-1, 4)
            err = np.abs(X - Xr).max()
            _say(f"level {j}: {npatch} patches, max |feature diff| {err:.2e}, labels on {Yr.mean():.3f}")
            if err >= 1e-5:
                col = np.abs(X - Xr).max(0)
                bad = np.nonzero(col > 1e-5)[0]
                _say("differing feature columns", bad.tolist(), "patches",
                     np.nonzero(np.abs(X - Xr).max(1) > 1e-5)[0][:20].tolist())
            assert err < 1e-5
            assert np.array_equal(Y > 0.5, Yr)
        assert g.patch_count(jmin) == 0 and g.patch_count(jmax) == 0


def _run(g, eps, dt, nsteps):
    act = []
    for _ in range(nsteps):
        g.adapt(eps)
        d, _ = g.diagnostics()
        act.append(sum(d.active_nodes) + sum(d.active_edges))
        g.step(dt)
    return act


@pytest.mark.parametrize("thr,expect_redo", [(0.0, False), (1.2, True)])
def test_gate_limits_equal_blanket_zone(thr, expect_redo):
    """Threshold 0 proposes every quadrant (the blanket zone); threshold above 1 drops every
    one, so the threshold test redoes each step with the blanket zone.  Both runs equal the
    plain run bitwise."""
    _say(f"gate limit thr={thr}")
    jmin, jmax, eps, nsteps = 4, 7, 5e-3, 6
    states = []
    redo = None
    for learned in (False, True):
        g = _grid(jmin, jmax)
        with g:
            dt = g.suggest_dt(0.8)
            m = wt.Mlp(inputs.mlp_init())
            if learned:
                g.set_predictor(m, thr)
            _run(g, eps, dt, nsteps)
            states.append([g.get_state(j) for j in range(jmin, jmax + 1)])
            if learned:
                redo = g.redo_count()
            m.close()
    for a, b in zip(states[0], states[1]):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    assert (redo == nsteps) if expect_redo else (redo == 0), redo


def test_trained_predictor_against_plain_zone():
    """Train the predictor on the plain method's history (features at one step, labels = the
    quadrants still significant after the step), then run the learned zone from a different
    initial bump: fewer active points, rare redos, small extra error, mass conserved."""
    import torch
    jmin, jmax, eps = 4, 7, 5e-3
    # history from plain runs
    Xs, Ys = [], []
    for bump_lon in (0.0, 40.0, -60.0):
        g = _grid(jmin, jmax, seed_bump=bump_lon)
        with g:
            dt = g.suggest_dt(0.8)
            prev = None
            for _ in range(16):
                g.adapt(eps)
                if prev is not None:
                    for j, x in prev:
                        y = torch.empty((x.shape[0], 4), dtype=torch.float32, device="cuda")
                        g.patch_labels(j, y)
                        Xs.append(x)
                        Ys.append(y)
                prev = []
                for j in range(jmin + 1, jmax):
                    x = torch.empty((g.patch_count(j), 64), dtype=torch.float32, device="cuda")
                    g.patch_features(j, x)
                    prev.append((j, x))
                g.step(dt)
    X, Y = torch.cat(Xs), torch.cat(Ys)
    _say(f"training set {X.shape[0]} patches, positive rate {Y.mean().item():.3f}")
    m = wt.Mlp(inputs.mlp_init())
    l0 = m.gradient(X, Y)[1]
    for _ in range(400):
        m.train_step(X, Y, 2e-3, want_loss=False)
    l1 = m.gradient(X, Y)[1]
    _say(f"loss {l0:.4f} -> {l1:.4f}")
    assert l1 < 0.5 * l0
    # held-out run: plain vs learned
    nsteps = 12
    res = {}
    for learned in (False, True):
        g = _grid(jmin, jmax, seed_bump=20.0)
        with g:
            dt = g.suggest_dt(0.8)
            if learned:
                g.set_predictor(m, 0.5)
            d0, _ = g.diagnostics()
            act = _run(g, eps, dt, nsteps)
            d1, _ = g.diagnostics()
            res[learned] = dict(act=np.mean(act), state=g.get_state(jmax), mass=(d0.mass, d1.mass),
                                redo=g.redo_count() if learned else 0)
    m.close()
    p, lrn = res[False], res[True]
    hp, hl = p["state"][0], lrn["state"][0]
    err = np.sqrt(((hl - hp) ** 2).sum() / ((hp + 1e4) ** 2).sum())
    _say(f"active dof plain {p['act']:.0f}, learned {lrn['act']:.0f} ({lrn['act'] / p['act']:.3f}); "
         f"redo {lrn['redo']}/{nsteps}; rel L2 height vs plain {err:.2e}")
    # no gate judged by the threshold test can drop more than the few quadrants that lose their
    # significance within one step (oracle bound on this jet: 1e-4 of the active dof)
    assert (1.0 - 0.01) * p["act"] <= lrn["act"] <= p["act"]
    assert lrn["redo"] <= nsteps // 2
    assert err < 1e-4
    m0, m1 = lrn["mass"]
    assert abs(m1 / m0 - 1) < 1e-13


def test_learned_zone_over_work_lists_equals_whole_levels():
    """The gated adapt, its patch features and the threshold test run over the work lists: with
    an untrained network at threshold 0.5 (a mix of proposed and dropped quadrants) the run
    equals, bitwise, the same run over whole levels, redo count included."""
    jmin, jmax, eps, nsteps = 4, 7, 5e-3, 6
    out = []
    for lists in (True, False):
        g = _grid(jmin, jmax, seed_bump=30.0)
        with g:
            g.set_work_lists(lists)
            dt = g.suggest_dt(0.8)
            m = wt.Mlp(inputs.mlp_init())
            g.set_predictor(m, 0.5)
            act = _run(g, eps, dt, nsteps)
            out.append(([g.get_state(j) for j in range(jmin, jmax + 1)], act, g.redo_count()))
            m.close()
    (sa, aa, ra), (sb, ab, rb) = out
    _say(f"lists vs whole levels: active {aa} / {ab}, redo {ra} / {rb}")
    assert aa == ab and ra == rb
    for a, b in zip(sa, sb):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("min_count", [2, 5])
def test_learned_zone_against_the_oracle(min_count):
    """The learned zone on the jet (levels 4..7, eps 5e-3) with a network that proposes a
    quadrant's children only where it holds at least `min_count` significant points (weights and
    activations exact in bfloat16, so both sides take the same decisions), against the oracle's
    learned zone (oracle/learned.py): after every passing threshold test the patch features the
    next gated adapt reads agree, and after every round of adapt + step + threshold test the masks
    are identical, the states within 1e-11 and the redo counts equal."""
    import torch
    from oracle import learned, trisk
    from oracle.multiscale import Hierarchy
    from test_oracle_learned import gate_params
    jmin, jmax, eps, nsteps = 4, 7, 5e-3, 6
    _say(f"learned zone vs oracle, min_count={min_count}")
    theta = gate_params(min_count)
    H = Hierarchy(jmin, jmax)
    og = H.g[jmax]
    dh, u, Hd = inputs.jet(og.xyz, og.e_mid, og.e_tan)
    p = trisk.Params(mean_depth=Hd)
    H.set_state(jmax, dh, u)
    dt = 0.8 * trisk.suggest_dt(og, dh, u, p, 1.0)
    g = wt.Grid(jmin, jmax, 8)
    m = wt.Mlp(theta.astype(np.float32))
    redo_o = 0
    with g:
        g.set_params(mean_depth=Hd)
        g.set_state(jmax, dh, u)
        # round 0 with the blanket zone, so the gate sees a developed significant set
        g.adapt(eps)
        g.step(dt)
        H.adapt(eps)
        H.step(dt, p)
        g.set_predictor(m, 0.5)
        redone, compared = True, 0
        for k in range(nsteps):
            if not redone:
                # after a passing threshold test both sides hold the details, thresholds and
                # significant points the next gated adapt uses: its features must agree
                det = H.details()
                eh, eu = H.thresholds(eps)
                sn, se = H.significant(det, eh, eu)
                for j, st in learned.all_stats(H, det, eh, eu, sn, se).items():
                    x = torch.empty((g.patch_count(j), 64), dtype=torch.float32, device="cuda")
                    g.patch_features(j, x)
                    err = np.abs(x.cpu().numpy() - learned.features(H, j, st)).max()
                    _say(f"  round {k} level {j}: max |feature diff| {err:.1e}")
                    assert err < 1e-6
                    compared += 1
            g.adapt(eps)
            g.step(dt)
            redone, dropped, _ = learned.learned_step(H, eps, dt, p, theta, 0.5)
            redo_o += int(redone)
            nd = sum(int(d.sum()) for d in dropped.values())
            w = 0.0
            for j in H.levels:
                a, b, na, ea = H.get_state(j)
                x, y, gna, gea = g.get_state(j)
                assert np.array_equal(gna.astype(bool), na) and np.array_equal(gea.astype(bool), ea), (k, j)
                w = max(w, np.abs(x - a).max() / np.abs(a).max(), np.abs(y - b).max() / np.abs(b).max())
            _say(f"  round {k}: dropped quadrants {nd}, redone {redone}, GPU redo {g.redo_count()}, rel Linf {w:.1e}")
            assert w < 1e-11
            assert g.redo_count() == redo_o
    m.close()
    _say(f"  feature comparisons {compared}, redo {redo_o}/{nsteps}")


def test_forced_drop_is_judged_and_redone():
    """wt_debug_force_drop: with a gate that proposes everything (threshold 0), withholding the
    children rule of a patch that holds significant points makes the threshold test find the
    miss and redo the step (redo count 1, state bitwise the plain run's); withholding it from a
    patch without significant points drops nothing and redoes nothing."""
    import torch
    jmin, jmax, eps, lev = 4, 7, 5e-3, 5
    out = []
    for case in ("plain", "significant", "empty"):
        g = _grid(jmin, jmax)
        with g:
            dt = g.suggest_dt(0.8)
            g.adapt(eps)
            g.step(dt)
            m = wt.Mlp(inputs.mlp_init())
            if case != "plain":
                g.set_predictor(m, 0.0)
                y = torch.empty((g.patch_count(lev), 4), dtype=torch.float32, device="cuda")
                g.patch_labels(lev, y)
                sig = y.cpu().numpy().max(1) > 0.5
                patch = int(np.nonzero(sig)[0][0]) if case == "significant" else int(np.nonzero(~sig)[0][0])
                g.debug_force_drop(lev, patch)
            g.adapt(eps)
            g.step(dt)
            out.append(([g.get_state(j) for j in range(jmin, jmax + 1)], g.redo_count()))
            m.close()
    _say(f"forced drop: redo {[r for _, r in out]}")
    assert [r for _, r in out] == [0, 1, 0]
    for states, _ in out[1:]:
        for a, b in zip(states, out[0][0]):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)

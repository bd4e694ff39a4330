#!/usr/bin/env python3
"""Throughput of the TRiSK Runge-Kutta stage on one MI355X.

Workload (default): uniform icosahedral C-grid J=10 (10,485,762 cells, 31,457,280 edges),
Williamson test 2 zonal flow plus a seeded spherical-harmonic height perturbation (l <= 32,
10 m), classical RK4, dt = 0.8 x the stable step.  A "step" is one RK4 step = four tendency
evaluations (stages).  The metric is active-point RK-stage updates per second:
(active nodes + active edges) x 4 stages x steps / wall time, inputs resident in HBM.

Prints ONE JSON line.  Plain FP64 is the headline `value`; the FP32-tendency form is reported
beside it under "fp32_tendency".
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the lattice stage kernel, from two rocprofv3 counter runs (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch) of `bench.py --steps 1 --warmup 0 --modes fp64`, averaged
# over the four stage launches of an RK4 step and scaled by what the same counters read for a
# 2 GiB device copy (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000).
# Valid only for the kernel source and the grid level it was taken on: otherwise null.
MEASURED_TRAFFIC = {
    "trisk_lattice": {
        "sources": ("paper_1404_0405_amd/csrc/wt_lattice.hip", "paper_1404_0405_amd/csrc/wt_lattice_dev.hpp"),
        "sha256": ("5d73a7b03dc4a251609a248e8297c797dba1ebe8a5af6c463f729d6ae9318ead",
                   "18c6e1fc6b3178e275b06de215aab33aef8588bb6fad7c1be6311c5c0a6aefcd"),
        "level": 10, "fetch_kib": 673251.9, "write_kib": 572320.5, "fetch_scale": 2.000, "write_scale": 1.000,
    },
}


def measured_traffic(kernel, level):
    """Scaled HBM bytes per launch of `kernel` on the uniform grid of `level`, or None if not
    measured on that grid or on the current source."""
    import hashlib
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec is None or rec["level"] != level:
        return None
    for path, digest in zip(rec["sources"], rec["sha256"]):
        try:
            with open(os.path.join(ROOT, path), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != digest:
                    return None
        except OSError:
            return None
    return 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])


def run_gpu(args):
    import numpy as np
    import torch

    from paper_1404_0405_amd import inputs, wt

    J = args.level
    g = wt.Grid(J, J, 8)
    stream = torch.cuda.current_stream()
    g.set_stream(stream.cuda_stream)
    N, E, T = g.info(J)
    x, m, t = g.coords(J)
    dh0, u0, H = inputs.tc2_perturbed(x, m, t, seed=inputs.SEED_BASE + 1, device="cuda")
    g.set_params(mean_depth=H, rk=wt.WT_RK4, precision=wt.WT_FP64)
    g.set_state(J, dh0, u0)
    dt = g.suggest_dt(0.8)
    out = {}
    for mode in args.modes.split(","):
        g.set_params(precision=wt.WT_FP64 if mode == "fp64" else wt.WT_FP32_TENDENCY)
        g.set_state(J, dh0, u0)
        d0, _ = g.diagnostics()
        for _ in range(args.warmup):
            g.step(dt)
        torch.cuda.synchronize()
        g.timing_reset()
        g.timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.step(dt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.timing(False)
        kt = {k: g.kernel_time(k) for k in wt.kernel_names()}
        d1, code = g.diagnostics()
        wall = t1 - t0
        upd = (N + E) * 4 * args.steps / wall
        kernels = {}
        for k, (ms, cnt, by) in kt.items():
            if cnt == 0:
                continue
            avg_ms = ms / cnt
            avg_b = by / cnt
            kernels[k] = {"avg_ms": avg_ms, "launches": cnt, "algorithmic_bytes": avg_b,
                          "gbs": avg_b / (avg_ms * 1e-3) / 1e9, "units": wt.kernel_units(g, k)}
        out[mode] = dict(value=upd, ms_per_step=wall * 1e3 / args.steps, kernels=kernels,
                         mass_drift=abs(d1.mass / d0.mass - 1), energy_drift=abs(d1.energy / d0.energy - 1),
                         finite=code == wt.WT_OK)
        if mode == "fp64":
            state64 = g.get_state(J)[:2]
            # the same steps with the state handed over in host memory (pageable numpy arrays)
            # and read back, transfers inside the clock: the PCIe-inclusive rate (context only)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.set_state(J, dh0, u0)
            for _ in range(args.steps):
                g.step(dt)
            g.get_state(J)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            out[mode]["pcie_inclusive"] = {"value": (N + E) * 4 * args.steps / (t1 - t0),
                                           "ms_total": (t1 - t0) * 1e3,
                                           "ms_transfers": (t1 - t0 - wall) * 1e3,
                                           "host_bytes": (N + E) * (8 + 8 + 1)}
        else:
            state32 = g.get_state(J)[:2]
    # error of the FP32-tendency run against the FP64 run (same steps)
    if "fp64" in out and "fp32" in out:
        out["fp32"].update(_errors(state32, state64, H))
    g.close()
    return out, (N, E, T), dt


def _progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _errors(st, ref, H):
    """Relative L2 differences of a state (dh, u) from a reference: the height perturbation,
    the height against the total depth H + dh, and the velocity."""
    import numpy as np
    (a, u), (b, v) = st, ref
    return {"rel_l2_dh_vs_fp64": float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum())),
            "rel_l2_height_vs_fp64": float(np.sqrt(((a - b) ** 2).sum() / ((H + b) ** 2).sum())),
            "rel_l2_u_vs_fp64": float(np.sqrt(((u - v) ** 2).sum() / (v ** 2).sum()))}


# The finest level of an adaptive grid runs through the masked lattice kernel (the tiles of each
# lozenge that hold support points) once its 3-ring support holds this fraction of its elements:
# measured, the spun-up jet's level 9 (~21 % of its dof active) makes the whole step 1.08x faster
# and the turbulence's level 10 (~75 %) 1.36x; a nearly empty level is left to the lists (the
# masked form also runs the fixed rim round the lozenge corners every stage).
DENSE_MIN = 0.05


def _dense_kernel(g):
    """Launches, average duration and algorithmic rate of the masked lattice kernel (timing on)."""
    from paper_1404_0405_amd import wt
    ms, n, by = g.kernel_time("trisk_lattice_masked")
    if n == 0:
        return {"launches": 0}
    gbs = by / (ms * 1e-3) / 1e9
    return {"launches": n, "avg_ms": ms / n, "algorithmic_bytes_per_launch": by / n,
            "units_per_launch": wt.kernel_units(g, "trisk_lattice_masked"), "achieved_gbs": gbs,
            "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}


def _timed_adaptive(g, eps, dt, steps, jmin, jmax, dense_min=None):
    """adapt + step timed together (threshold test and redo included), active dof of each step.
    The finest level runs dense once its support holds DENSE_MIN of its elements (dense_min
    overrides; above 1: always listed)."""
    import torch
    from paper_1404_0405_amd import wt
    g.set_dense_levels(DENSE_MIN if dense_min is None else dense_min)
    g.timing(True)
    g.timing_reset()
    d0, _ = g.diagnostics()
    active, wall, wall_adapt = 0, 0.0, 0.0
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.adapt(eps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.step(dt)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        wall_adapt += t1 - t0
        d, _ = g.diagnostics()    # untimed: active counts of the mask the step used
        active += sum(d.active_nodes) + sum(d.active_edges)
    d1, code = g.diagnostics()
    dk = _dense_kernel(g)
    g.timing(False)
    return {"value": active * 4 / wall, "ms_per_step": wall * 1e3 / steps, "ms_adapt_per_step": wall_adapt * 1e3 / steps,
            "active_dof_per_step": active / steps, "mass_drift": abs(d1.mass / d0.mass - 1), "redo": g.redo_count(),
            "finite": code == wt.WT_OK, "finest_level": d1.finest_level, "dense_finest_level": dk,
            "active_dof_last_step_by_level": {str(j): d.active_nodes[j] + d.active_edges[j]
                                              for j in range(jmin, jmax + 1)}}


def _jet_grid(jmin, jmax, precision, bump_lon=0.0):
    from paper_1404_0405_amd import inputs, wt
    g = wt.Grid(jmin, jmax, 8)
    x, m, t = g.coords(jmax)
    dh, u, H = inputs.jet(x, m, t, bump_lon=bump_lon)
    g.set_params(mean_depth=H, rk=wt.WT_RK4, precision=precision)
    g.set_state(jmax, dh, u)
    return g, H


def train_predictor(jmin, jmax, eps, steps=12, iters=300, lr=2e-3, bump_lon=-40.0):
    """The child-patch predictor trained on the plain method's own history (a jet run with a
    different bump position): features after each adapt, labels = the quadrants still holding a
    significant point after the step."""
    import torch
    from paper_1404_0405_amd import inputs, wt
    g, _ = _jet_grid(jmin, jmax, wt.WT_FP64, bump_lon)
    Xs, Ys = [], []
    with g:
        dt = g.suggest_dt(0.8)
        prev = None
        for _ in range(steps):
            g.adapt(eps)
            if prev is not None:
                for j, x in prev:
                    y = torch.empty((x.shape[0], 4), dtype=torch.float32, device="cuda")
                    g.patch_labels(j, y)
                    Xs.append(x)
                    Ys.append(y)
            prev = []
            for j in range(jmin + 1, jmax):
                if g.patch_count(j) > 0:
                    x = torch.empty((g.patch_count(j), 64), dtype=torch.float32, device="cuda")
                    g.patch_features(j, x)
                    prev.append((j, x))
            g.step(dt)
    X, Y = torch.cat(Xs), torch.cat(Ys)
    m = wt.Mlp(inputs.mlp_init())
    l0 = m.gradient(X, Y)[1]
    t0 = time.perf_counter()
    for _ in range(iters):
        m.train_step(X, Y, lr, want_loss=False)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    l1 = m.gradient(X, Y)[1]
    return m, {"samples": int(X.shape[0]), "loss_before": l0, "loss_after": l1, "train_s": train_s,
               "iterations": iters}


def run_adaptive(jmin=5, jmax=9, eps=5e-3, steps=10, spinup_days=2.0, ensemble_members=64):
    """Adaptive jet workload from a spun-up state: the jet (levels jmin..jmax) is run for
    `spinup_days` simulated days with adapt + RK4 step every step (untimed; the bump has then
    grown finer scales, level jmax populated), saved, and from that checkpoint plain FP64 (blanket
    zone), FP32 with the blanket zone and FP32 with the learned zone each run `steps` timed steps.
    Metric: active-point RK-stage updates/s = sum over steps of (active nodes + active edges of all
    levels) x 4 stages / wall time of adapt + step (the threshold test and any redo included)."""
    import tempfile
    import torch
    from paper_1404_0405_amd import wt
    mlp, train = train_predictor(jmin, jmax, eps)
    out = {"workload": f"zonal jet + 120 m bump, levels {jmin}..{jmax}, eps={eps}, RK4, dt = 0.8 x stable step, "
                       f"timed from day {spinup_days:g}",
           "training": train}
    ckpt = os.path.join(tempfile.mkdtemp(prefix="jet"), "spun_up.ckpt")
    _progress(f"jet spin-up, {spinup_days:g} days")
    g, H = _jet_grid(jmin, jmax, wt.WT_FP64)
    with g:
        dt = g.suggest_dt(0.8)
        nspin = int(round(spinup_days * 86400.0 / dt))
        timeline = {}
        t0 = time.perf_counter()
        for k in range(nspin):
            g.adapt(eps)
            g.step(dt)
            if k % 2000 == 1999:
                _progress(f"jet spin-up step {k + 1} of {nspin}")
            if k % max(1, nspin // 4) == 0 or k == nspin - 1:
                d, _ = g.diagnostics()
                timeline[f"{(k + 1) * dt / 86400.0:.2f}"] = [d.active_nodes[j] + d.active_edges[j]
                                                             for j in range(jmin, jmax + 1)]
        torch.cuda.synchronize()
        out["spinup"] = {"steps": nspin, "days": nspin * dt / 86400.0, "wall_s": time.perf_counter() - t0,
                         "active_dof_by_level_at_day": timeline}
        g.save(ckpt)
    final = {}
    for name, prec, learned in (("plain_fp64", wt.WT_FP64, False), ("fp32_blanket", wt.WT_FP32_TENDENCY, False),
                                ("fp32_learned", wt.WT_FP32_TENDENCY, True)):
        g = wt.Grid(jmin, jmax, 8)
        with g:
            g.load(ckpt)
            g.set_params(precision=prec)
            if learned:
                g.set_predictor(mlp, 0.5)
            out[name] = _timed_adaptive(g, eps, dt, steps, jmin, jmax)
            final[name] = g.get_state(jmax)[:2]
    os.remove(ckpt)
    os.rmdir(os.path.dirname(ckpt))
    for name in ("fp32_blanket", "fp32_learned"):
        out[name].update(_errors(final[name], final["plain_fp64"], H))
        out[f"speedup_{name}_over_plain_fp64"] = out[name]["value"] / out["plain_fp64"]["value"]
    if ensemble_members:
        _progress(f"ensemble of {ensemble_members} members")
        out["ensemble"] = run_ensemble(members=ensemble_members, mlp=mlp)
    mlp.close()
    return out


def _turb_grid(jmin, jmax, precision):
    from paper_1404_0405_amd import inputs, wt
    g = wt.Grid(jmin, jmax, 8)
    x, m, t = g.coords(jmax)
    dh, u, H = inputs.turbulence(x, m, t, device="cuda")
    del x, m, t
    g.set_params(mean_depth=H, rk=wt.WT_RK4, precision=precision)
    g.set_state(jmax, dh, u)
    return g, H


def run_turbulence(jmin=6, jmax=10, eps=1e-2, train_steps=200, collect_every=20, test_steps=20,
                   max_samples=150000, iters=300, lr=2e-3):
    """Learned-zone workload on rotating turbulence: seeded random non-divergent flow peaked at
    degree 40, rms 20 m/s, depth 1 km, levels jmin..jmax, eps relative.  A plain FP64 run of
    train_steps steps provides the predictor's training set (features after an adapt, labels
    after the next step, every collect_every steps, at most max_samples patches); then plain
    FP64 and FP32 tendencies + learned zone each run test_steps timed steps from the state at
    the end of the training window (a checkpoint).  Metric as for the jet."""
    import os
    import tempfile
    import numpy as np
    import torch
    from paper_1404_0405_amd import inputs, wt
    t_build = time.perf_counter()
    g, H = _turb_grid(jmin, jmax, wt.WT_FP64)
    build_s = time.perf_counter() - t_build
    N, E, _ = g.info(jmax)
    ckpt = os.path.join(tempfile.mkdtemp(prefix="turb"), "train_end.ckpt")
    Xs, Ys = [], []
    with g:
        dt = g.suggest_dt(0.8)
        d0, _ = g.diagnostics()
        t0 = time.perf_counter()
        prev = None
        timeline = {}
        for k in range(train_steps):
            g.adapt(eps)
            if k in (0, 10, 20, 50, 100, 150) or k == train_steps - 1:
                d, _ = g.diagnostics()
                timeline[k] = {"nodes": list(d.active_nodes)[jmin:jmax + 1],
                               "edges": list(d.active_edges)[jmin:jmax + 1]}
            if prev is not None:
                for j, x in prev:
                    y = torch.empty((x.shape[0], 4), dtype=torch.float32, device="cuda")
                    g.patch_labels(j, y)
                    Xs.append(x)
                    Ys.append(y)
                prev = None
            if k % collect_every == 0 and k + 1 < train_steps:
                prev = []
                for j in range(jmin + 1, jmax):
                    if g.patch_count(j) > 0:
                        x = torch.empty((g.patch_count(j), 64), dtype=torch.float32, device="cuda")
                        g.patch_features(j, x)
                        prev.append((j, x))
            g.step(dt)
        torch.cuda.synchronize()
        train_run_s = time.perf_counter() - t0
        dtr, _ = g.diagnostics()
        g.save(ckpt)
    X, Y = torch.cat(Xs), torch.cat(Ys)
    if X.shape[0] > max_samples:
        keep = torch.from_numpy(np.random.default_rng(inputs.SEED_BASE + 6).choice(
            X.shape[0], max_samples, replace=False)).cuda()
        X, Y = X[keep].contiguous(), Y[keep].contiguous()
    mlp = wt.Mlp(inputs.mlp_init())
    l0 = mlp.gradient(X, Y)[1]
    t0 = time.perf_counter()
    for _ in range(iters):
        mlp.train_step(X, Y, lr, want_loss=False)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    l1 = mlp.gradient(X, Y)[1]
    out = {"workload": f"rotating turbulence (random non-divergent flow peaked at degree 40, rms 20 m/s, "
                       f"depth 1 km), levels {jmin}..{jmax}, eps={eps}, RK4, dt = 0.8 x stable step",
           "dt_s": dt, "grid_build_and_ic_s": build_s,
           "training_window": {"steps": train_steps, "simulated_h": train_steps * dt / 3600.0,
                               "wall_s": train_run_s, "active_dof_at_end": int(sum(dtr.active_nodes) + sum(dtr.active_edges)),
                               "active_per_level_after_adapt": timeline},
           "training": {"samples": int(X.shape[0]), "loss_before": l0, "loss_after": l1, "train_s": train_s,
                        "iterations": iters},
           "uniform_dof_at_jmax": int(N + E)}
    del X, Y, Xs, Ys
    final = {}
    # from the checkpoint: plain FP64, FP32 with the blanket zone, FP32 with the learned zone, and
    # the viscous form of Sec. 3.1 (nu = 1e4 m^2/s, the paper's viscous turbulence) in FP64
    # (the finest level dense once its support holds DENSE_MIN of it; plain_fp64_listed keeps it
    # on the listed kernels for comparison; the viscous form always does)
    for name, prec, learned, nu in (("plain_fp64", wt.WT_FP64, False, 0.0),
                                    ("plain_fp64_listed", wt.WT_FP64, False, 0.0),
                                    ("fp32_blanket", wt.WT_FP32_TENDENCY, False, 0.0),
                                    ("fp32_learned", wt.WT_FP32_TENDENCY, True, 0.0),
                                    ("viscous_fp64", wt.WT_FP64, False, 1e4)):
        h = wt.Grid(jmin, jmax, 8)
        with h:
            h.load(ckpt)
            h.set_params(precision=prec, viscosity=nu)
            if learned:
                h.set_predictor(mlp, 0.5)
            out[name] = _timed_adaptive(h, eps, dt, test_steps, jmin, jmax,
                                        dense_min=2.0 if name == "plain_fp64_listed" else None)
            out[name]["compression"] = (N + E) / out[name]["active_dof_per_step"]
            if nu:
                out[name]["viscosity"] = nu
            final[name] = h.get_state(jmax)[:2]
    os.remove(ckpt)
    os.rmdir(os.path.dirname(ckpt))
    mlp.close()
    out["test_window"] = {"steps": test_steps, "simulated_h": test_steps * dt / 3600.0}
    for name in ("fp32_blanket", "fp32_learned", "plain_fp64_listed"):
        out[name].update(_errors(final[name], final["plain_fp64"], H))
        out[f"speedup_{name}_over_plain_fp64"] = out[name]["value"] / out["plain_fp64"]["value"]
    return out


def run_tc1(jmin=4, jmax=10, eps=2e-2, days=12.0, bell="cosine"):
    """Advection test 1 (Sec. 6.1): a cosine bell carried once round the sphere by solid-body
    rotation, levels jmin..jmax with jmax a cap (the thresholds choose the finest level used),
    RK4 at CFL 0.8 of the cap level's advective step.  eps is the tolerance on the trend: the
    wavelet thresholds are relative, eps^(3/2) of the largest height and speed (the eps^(3/2)
    scaling of the regime thresholds of Sec. 3.1, with the bell's height and the rotation speed
    as the scales).  Reports the finest level used, the error against the closed form (the
    initial bell after one rotation), mass conservation and the active-point rate of adapt +
    step."""
    import numpy as np
    import torch
    from paper_1404_0405_amd import inputs, wt
    g = wt.Grid(jmin, jmax, 8)
    with g:
        x, m, t = g.coords(jmax)
        dh, u, H0 = inputs.tc1(x, m, t, bell=bell)
        g.set_params(mean_depth=H0, equations=wt.WT_ADVECTION)   # (the listed kernels: no dense form)
        g.set_state(jmax, dh, u)
        dt0 = g.suggest_dt(0.8)
        n = int(math.ceil(days * 86400.0 / dt0))
        dt = days * 86400.0 / n
        d0, _ = g.diagnostics()
        finest, sampled, wall = 0, [], 0.0
        eps_w = eps ** 1.5
        for k in range(n):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.adapt(eps_w)
            g.step(dt)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            if k % 25 == 0:   # untimed: active counts of every 25th step
                d, _ = g.diagnostics()
                finest = max(finest, d.finest_level)
                sampled.append(sum(d.active_nodes) + sum(d.active_edges))
        d1, code = g.diagnostics()
        finest = max(finest, d1.finest_level)
        a, _, _, _ = g.get_state(jmax)
        err = float(np.sqrt(((a - dh) ** 2).sum() / (dh ** 2).sum()))
        mean_act = float(np.mean(sampled))
        return {"workload": f"advection test 1 ({bell} bell, solid-body rotation once in 12 days), levels {jmin}..{jmax} "
                            f"(jmax a cap), trend tolerance eps={eps} (relative wavelet thresholds eps^1.5 = "
                            f"{eps_w:.3g}), RK4, CFL 0.8", "steps": n, "dt_s": dt,
                "finest_level_used": finest, "rel_l2_error_vs_closed_form": err,
                "mass_drift": abs(d1.mass / d0.mass - 1), "finite": code == wt.WT_OK,
                "wall_s": wall, "ms_per_step": wall * 1e3 / n, "active_dof_mean_of_sampled_steps": mean_act,
                "active_dof_last_step_by_level": {str(j): d1.active_nodes[j] + d1.active_edges[j]
                                                  for j in range(jmin, jmax + 1)},
                "value": mean_act * 4 / (wall / n)}


def run_ensemble(members=64, jmin=5, jmax_choices=(7, 8, 9), steps=10, mlp=None):
    """Ensemble of jet members (seeded bump amplitude/position, Jmax and eps drawn per member),
    FP32 tendencies / FP64 state, learned zone when a network is given: one graph launch per
    ensemble step, and one persistent batched launch per step (its launch shape tuned during the
    first steps), against the same members stepped one after another (same grids, state set
    again in between)."""
    import torch
    from paper_1404_0405_amd import inputs, wt
    params = inputs.ensemble_members(members, jmax_choices=jmax_choices)
    t0 = time.perf_counter()
    grids, init = [], []
    for p in params:
        g = wt.Grid(jmin, p["jmax"], 8)
        x, m, t = g.coords(p["jmax"])
        dh, u, H = inputs.jet(x, m, t, bump=p["bump"], bump_lat=p["bump_lat"], bump_lon=p["bump_lon"])
        g.set_params(mean_depth=H, rk=wt.WT_RK4, precision=wt.WT_FP32_TENDENCY)
        grids.append(g)
        init.append((p["jmax"], dh, u))
    build_s = time.perf_counter() - t0

    def reset(net):
        for g, (j, dh, u) in zip(grids, init):
            g.set_state(j, dh, u)
            g.set_predictor(net, 0.5)

    reset(None)
    dts = [g.suggest_dt(0.8) for g in grids]
    eps = [p["eps"] for p in params]
    out = {"members": members, "jmin": jmin, "jmax": [p["jmax"] for p in params], "eps": eps,
           "grid_build_s": build_s, "steps": steps}

    def active():
        tot = 0
        for g in grids:
            d, _ = g.diagnostics()
            tot += sum(d.active_nodes) + sum(d.active_edges)
        return tot

    def redos():
        return sum(g.redo_count() for g in grids)

    def one_by_one(net):
        reset(net)
        wall, act, r0 = 0.0, 0, redos()
        for _ in range(steps):
            for g, e, dt in zip(grids, eps, dts):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                g.adapt(e)
                g.step(dt)
                torch.cuda.synchronize()
                wall += time.perf_counter() - t1
            act += active()
        return {"value": act * 4 / wall, "ms_per_step": wall * 1e3 / steps, "redo": redos() - r0}, act

    def run_ens(net, batched):
        reset(net)
        wall, wall_step, act, r0 = 0.0, 0.0, 0, redos()
        with wt.Ensemble(grids) as ens:
            if batched:
                ens.set_batched(True)
            for _ in range(steps):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                ens.adapt(eps)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                ens.step(dts)
                t3 = time.perf_counter()
                wall += t3 - t1
                wall_step += t3 - t2
                act += active()
            caps, launches = ens.stats()
            shape = ens.tuning() if batched else None
        r = {"value": act * 4 / wall, "ms_per_step": wall * 1e3 / steps, "ms_step_call": wall_step * 1e3 / steps,
             "captures": caps, "launches": launches, "redo": redos() - r0}
        if shape:
            r["launch_shape"] = shape
        return r

    for name, net in (("plain", None), ("learned", mlp)):
        if name == "learned" and mlp is None:
            continue
        res, act = one_by_one(net)
        res = {"one_by_one": res, "graph": run_ens(net, False), "batched": run_ens(net, True),
               "active_dof_per_step": act / steps}
        res["speedup_graph_over_one_by_one"] = res["graph"]["value"] / res["one_by_one"]["value"]
        res["speedup_batched_over_one_by_one"] = res["batched"]["value"] / res["one_by_one"]["value"]
        out[name] = res
    for g in grids:
        g.close()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORACLE_CASE = None   # (grid, dh, u, params) of the CPU baseline, shared with forked workers


def _oracle_stages(stages):
    from oracle import trisk
    g, dh, u, p = _ORACLE_CASE
    t0 = time.perf_counter()
    for _ in range(stages):
        trisk.tendencies(g, dh, u, p)
    return time.perf_counter() - t0


def cpu_baseline(level=9, stages=2, procs=None):
    """The oracle as it stands (numpy FP64), timed on the host's cores on bounded samples of the
    workloads: (i) `stages` tendency evaluations (RK stages) of the uniform TC2 + SH flow on the
    level-`level` grid in one process, then the same in `procs` forked processes at once (all
    cores; the aggregate rate is `value`) -- level 10, the headline's, would take about five
    minutes and 30 GB to build the oracle grid, so level 9; (ii) one adaptive step (adapt + RK4
    step) of the TC2 configuration on levels 4..6, eps 1e-3, one process."""
    import multiprocessing as mp
    from oracle import trisk
    from oracle.grid import Grid
    from oracle.multiscale import Hierarchy
    from paper_1404_0405_amd import inputs
    procs = procs or max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    og = Grid(level)
    build_s = time.perf_counter() - t0
    dh, u, H = inputs.tc2_perturbed(og.xyz, og.e_mid, og.e_tan)
    p = trisk.Params(mean_depth=H)
    dof = og.N + og.E
    global _ORACLE_CASE
    _ORACLE_CASE = (og, dh, u, p)
    single = _oracle_stages(stages)
    # forked workers find the case in the module global (nothing large is sent to them)
    ctx = mp.get_context("fork")
    with ctx.Pool(procs) as pool:
        pool.map(_oracle_stages, [0] * procs)      # workers started and warmed up
        t0 = time.perf_counter()
        each = pool.map(_oracle_stages, [stages] * procs)
        wall_all = time.perf_counter() - t0
    _ORACLE_CASE = None
    del og
    Hy = Hierarchy(4, 6)
    fg = Hy.g[6]
    dh6, u6, H6 = inputs.tc2(fg.xyz, fg.e_mid, fg.e_tan)
    p6 = trisk.Params(mean_depth=H6)
    Hy.set_state(6, dh6, u6)
    Hy.adapt(1e-3)
    dt6 = trisk.suggest_dt(fg, dh6, u6, p6, 0.8)
    t0 = time.perf_counter()
    Hy.adapt(1e-3)
    Hy.step(dt6, p6)
    wall_ad = time.perf_counter() - t0
    act = sum(int(Hy.node_act[j].sum() + Hy.edge_act[j].sum()) for j in Hy.levels)
    return {"value": procs * dof * stages / wall_all, "unit": "active-point RK-stage updates/s", "cores": procs,
            "kind": "oracle",
            "sample": f"{stages} RK stages (tendency evaluations) of the uniform TC2+SH flow on level {level} "
                      f"({dof} dof), numpy FP64 oracle, in {procs} processes at once "
                      f"({wall_all:.1f} s); level 10 not built (about 5 minutes and 30 GB for the oracle grid)",
            "host_cpu": _cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": dof * stages / single, "wall_s": single, "cores": 1},
            "all_cores_worker_s": [round(x, 3) for x in each],
            "oracle_grid_build_s": build_s,
            "adaptive_step_tc2_levels_4_6": {"value": act * 4 / wall_ad, "wall_s": wall_ad, "active_dof": act,
                                             "cores": 1, "eps": 1e-3}}


def stream_reference(ndouble, reps=10):
    """What this GPU streams for plain elementwise work on arrays the size of one state array
    (torch's own kernels, FP64): a copy (1 read, 1 write) and an add (2 reads, 1 write, near the
    lattice stage's mix of counted reads and writes).  Context for the lattice kernel's counted
    traffic rate; the roofline fraction stays against the published peak."""
    import torch
    a = torch.rand(ndouble, dtype=torch.float64, device="cuda")
    b = torch.rand_like(a)
    o = torch.empty_like(a)
    out = {}
    for name, fn, nbytes in (("copy_1r_1w", lambda: o.copy_(a), 2 * 8 * ndouble),
                             ("add_2r_1w", lambda: torch.add(a, b, alpha=0.5, out=o), 3 * 8 * ndouble)):
        fn()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        out[name] = {"avg_ms": ms, "GB/s": nbytes / (ms * 1e-3) / 1e9, "bytes": nbytes}
    del a, b, o
    return out


def copy_probe(nbytes=1 << 31, reps=5):
    """A plain device copy of known size (torch's copy kernel), for scaling the HBM byte
    counters: FETCH_SIZE and WRITE_SIZE of one copy should each read `nbytes`."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(json.dumps({"copy_probe_bytes_each_way": nbytes, "avg_ms": ms,
                      "gbs_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--level", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--modes", default="fp64,fp32", help="comma list of fp64, fp32")
    ap.add_argument("--copy-probe", action="store_true", help="only run the copy calibration")
    ap.add_argument("--no-adaptive", action="store_true", help="skip the adaptive jet comparison")
    ap.add_argument("--adaptive-steps", type=int, default=10)
    ap.add_argument("--only-adaptive", action="store_true", help="run only the adaptive jet comparison")
    ap.add_argument("--ensemble-members", type=int, default=64, help="0 skips the ensemble")
    ap.add_argument("--no-turbulence", action="store_true", help="skip the learned-zone turbulence workload")
    ap.add_argument("--no-tc1", action="store_true", help="skip the advection test 1 workload")
    ap.add_argument("--jet-days", type=float, default=2.0, help="simulated days of jet spin-up before timing")
    ap.add_argument("--only-turbulence", action="store_true", help="run only the turbulence workload")
    ap.add_argument("--turb-train-steps", type=int, default=100)
    ap.add_argument("--turb-test-steps", type=int, default=10)
    ap.add_argument("--dense-min", type=float, default=DENSE_MIN,
                    help="support fraction from which the finest level runs dense (above 1: never)")
    args = ap.parse_args()
    globals()["DENSE_MIN"] = args.dense_min
    if args.copy_probe:
        copy_probe()
        return
    turb_kw = dict(train_steps=args.turb_train_steps, test_steps=args.turb_test_steps,
                   collect_every=max(1, args.turb_train_steps // 10))
    if args.only_turbulence:
        print(json.dumps({"turbulence": run_turbulence(**turb_kw)}), flush=True)
        return
    if args.only_adaptive:
        print(json.dumps({"adaptive": run_adaptive(steps=args.adaptive_steps, spinup_days=args.jet_days,
                                                   ensemble_members=args.ensemble_members)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (--gpus {args.gpus} requested); "
              "a multi-GPU path is not implemented", file=sys.stderr)
        sys.exit(2)
    _progress("uniform stage")
    res, (N, E, T), dt = run_gpu(args)
    f64 = res["fp64"]
    dom = max(f64["kernels"], key=lambda k: f64["kernels"][k]["avg_ms"])
    kd = f64["kernels"][dom]
    # algorithmic bytes per launch of the dominant kernel, per element of the units it processes:
    # the state passes of an RK4 stage (8 B per dof, 4 dofs per element, r = 4 passes on average
    # over the stages) and the shared-geometry model of the per-element tables (376 B per element
    # on a general grid, one lozenge's tables shared by all ten: 37.6 B)
    units = kd["units"]
    alg = units * (8.0 * 4 * 4 + 376.0 / 10.0)
    achieved = alg / (kd["avg_ms"] * 1e-3) / 1e9
    line = {
        "metric": "active-point RK-stage updates/s",
        "value": f64["value"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"uniform icosahedral C-grid J={args.level} ({N} cells, {E} edges), "
                               "TC2 zonal flow + seeded SH height perturbation (l<=32, 10 m), RK4, "
                               f"dt={dt:.3f} s (CFL 0.8)",
                   "level": args.level, "cells": N, "edges": E, "rk": "rk4", "stages_per_step": 4},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, args.level),
                     "algorithmic_bytes": alg, "units_per_launch": units, "avg_launch_ms": kd["avg_ms"],
                     "byte_model": "RK4 stage: 8 B x 4 dof x 4 passes per element + 376 B / 10 shared tables",
                     "kernel_byte_model": {"algorithmic_bytes": kd["algorithmic_bytes"], "achieved": kd["gbs"],
                                           "frac": kd["gbs"] / HBM_PEAK_GBS,
                                           "model": "stage input + Runge-Kutta arrays read and written + "
                                                    "58 FP64 geometry values per tile position / 10"}},
        "stream_reference": None,
        "kernels_fp64": f64["kernels"],
        "stage_ms_fp64": f64["ms_per_step"] / 4,
        "fp32_tendency": ({"value": res["fp32"]["value"], "ms_per_step": res["fp32"]["ms_per_step"],
                           "rel_l2_height_vs_fp64": res["fp32"].get("rel_l2_height_vs_fp64"),
                           "mass_drift": res["fp32"]["mass_drift"], "kernels": res["fp32"]["kernels"]}
                          if "fp32" in res else None),
        "mass_drift_fp64": f64["mass_drift"],
        "energy_drift_fp64": f64["energy_drift"],
        "pcie_inclusive_fp64": f64.get("pcie_inclusive"),
    }
    sref = stream_reference(N + E)
    tr = line["roofline"]["traffic"]
    if tr:
        for v in sref.values():
            v["lattice_traffic_rate_frac"] = tr / (kd["avg_ms"] * 1e-3) / 1e9 / v["GB/s"]
    line["stream_reference"] = sref
    if not args.no_adaptive:
        _progress("adaptive jet")
        line["adaptive"] = run_adaptive(steps=args.adaptive_steps, spinup_days=args.jet_days,
                                        ensemble_members=args.ensemble_members)
    if not args.no_turbulence:
        _progress("turbulence")
        line["turbulence"] = run_turbulence(**turb_kw)
    if not args.no_tc1:
        _progress("advection test 1")
        line["advection_tc1"] = run_tc1()
    if not args.no_cpu_baseline:
        _progress("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline()
    _progress("done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

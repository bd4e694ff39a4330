"""Seeded synthetic initial conditions (point values at nodes and edge midpoints).

This module holds no arithmetic of the method itself: it turns coordinates (supplied by the
caller, each side computing its own) into initial fields.  The HIP library and the oracle
both receive their inputs from here.

Workloads (stand-ins for the paper's test cases, Sec. 6):

* ``tc2``: steady geostrophic zonal flow (Williamson test 2, Sec. 6.2),
  u = u0 cos(lat) eastward, g h = g h0 - (a Omega u0 + u0^2/2) sin^2(lat), u0 = 2 pi a / 12 d,
  g h0 = 2.94e4 m^2/s^2.  The printed height uses cos(lat) and drops a from U; the form used
  here is the one that is in gradient-wind balance.
* ``tc2_perturbed``: tc2 plus a seeded smooth height perturbation, sum of real spherical
  harmonics 1 <= l <= 32 with N(0,1) coefficients, scaled to 10 m maximum amplitude.
* ``jet``: zonal jet u = 80 exp(-((lat-45)/8)^2) m/s with the height in gradient-wind balance
  (composite Simpson quadrature), mean depth 10 km, plus a Gaussian height bump (stand-in for
  the Galewsky jet of Sec. 6.4).
* ``tc1``: advection of a bell by solid-body rotation (Williamson test 1, Sec. 6.1): velocity
  u = U (cos(lat) cos(alpha) + sin(lat) cos(lon) sin(alpha)), v = -U sin(lon) sin(alpha),
  U = 2 pi a / 12 d, i.e. rotation about the axis (-sin alpha, 0, cos alpha) once per 12 days;
  cosine bell h = (H0/2)(1 + cos(pi r/L)) for r < L (0 outside) or smooth bell
  h = H0 exp(r^2 / (r^2 - 2 L^2)) for r < sqrt(2) L (0 outside), r = a arccos(cos(lat) cos(lon))
  the distance from (0, 0), H0 = 1000 m, L = a/3, zero mean depth; at time t the same bell
  turned about the axis by the angle U t / a (the exact solution).
* ``turbulence``: seeded random non-divergent flow u = k x grad(psi) with an isotropic energy
  spectrum peaked at degree 40, rms speed 20 m/s, mean depth 1 km, height from linear balance
  g h' = f psi (stand-in for the rotating turbulence of Sec. 7).
"""
from __future__ import annotations

import math

import numpy as np

EARTH_RADIUS = 6.371e6
OMEGA = 7.292e-5
GRAVITY = 9.80616
DAY = 86400.0
SEED_BASE = 14040405


def tc2_constants(radius=EARTH_RADIUS, omega=OMEGA, gravity=GRAVITY):
    u0 = 2.0 * math.pi * radius / (12.0 * DAY)
    gh0 = 2.94e4
    return u0, gh0, gh0 / gravity


def tc2(node_xyz, edge_mid, edge_tan, radius=EARTH_RADIUS, omega=OMEGA, gravity=GRAVITY):
    """Returns (dh, u, H): perturbation height at nodes, normal velocity at edges, mean depth."""
    u0, gh0, H = tc2_constants(radius, omega, gravity)
    z = node_xyz[:, 2] / np.linalg.norm(node_xyz, axis=1)
    dh = -(radius * omega * u0 + 0.5 * u0 * u0) * z * z / gravity
    m = edge_mid / np.linalg.norm(edge_mid, axis=1, keepdims=True)
    vel = u0 * np.stack([-m[:, 1], m[:, 0], np.zeros_like(m[:, 0])], 1)   # u0 * z_hat x x
    u = (vel * edge_tan).sum(1)
    return dh, u, H


def tc1_axis(alpha, radius=EARTH_RADIUS):
    """Angular velocity vector [1/s] of the test-1 rotation: |w| = U / a, U = 2 pi a / 12 d."""
    w = 2.0 * math.pi / (12.0 * DAY)
    return w * np.array([-math.sin(alpha), 0.0, math.cos(alpha)])


def tc1_bell(xyz, bell="cosine", h0=1000.0, t=0.0, alpha=0.0, radius=EARTH_RADIUS):
    """Bell height at unit positions xyz after time t of rotation (t = 0: the initial bell)."""
    x = xyz / np.linalg.norm(xyz, axis=1, keepdims=True)
    if t != 0.0:
        # position at time 0 of the fluid now at x: turn x back about the axis (Rodrigues)
        w = tc1_axis(alpha, radius)
        k = w / np.linalg.norm(w)
        ang = -np.linalg.norm(w) * t
        c, s = math.cos(ang), math.sin(ang)
        x = x * c + np.cross(k, x) * s + np.outer(x @ k, k) * (1.0 - c)
    # distance from the bell centre (lat 0, lon 0): cos(lat) cos(lon) = x
    r = radius * np.arccos(np.clip(x[:, 0], -1.0, 1.0))
    L = radius / 3.0
    if bell == "cosine":
        return np.where(r < L, 0.5 * h0 * (1.0 + np.cos(np.pi * r / L)), 0.0)
    if bell == "smooth":
        q = r * r - 2.0 * L * L
        inside = q < 0
        return np.where(inside, h0 * np.exp(np.where(inside, r * r / np.where(inside, q, -1.0), 0.0)), 0.0)
    raise ValueError(bell)


def tc1(node_xyz, edge_mid, edge_tan, bell="cosine", alpha=0.0, t=0.0, radius=EARTH_RADIUS):
    """Returns (dh, u, H): bell height at nodes (time t), prescribed normal velocity at edges,
    mean depth 0."""
    m = edge_mid / np.linalg.norm(edge_mid, axis=1, keepdims=True)
    vel = np.cross(tc1_axis(alpha, radius), m) * radius
    u = (vel * edge_tan).sum(1)
    return tc1_bell(node_xyz, bell, t=t, alpha=alpha, radius=radius), u, 0.0


def real_sph_harm_sum(xyz, coeffs, lmax, device=None):
    """S(x) = sum_{l=1..lmax} sum_{m=-l..l} a_lm Y_lm(x), orthonormal real harmonics.

    ``coeffs[l, lmax + m]`` holds a_lm.  Associated Legendre functions by the standard stable
    recurrences in m then l.  Evaluated with torch in float64 on ``device`` (CPU by default;
    a GPU device only speeds up large grids) and returned as a numpy array.
    """
    import torch
    dev = torch.device(device) if device is not None else torch.device("cpu")
    x = torch.as_tensor(np.ascontiguousarray(xyz), dtype=torch.float64, device=dev)
    x = x / torch.linalg.norm(x, dim=1, keepdim=True)
    ct = x[:, 2]
    st = torch.sqrt(torch.clamp(1.0 - ct * ct, min=0.0))
    lon = torch.atan2(x[:, 1], x[:, 0])
    out = torch.zeros_like(ct)
    pmm = torch.full_like(ct, math.sqrt(1.0 / (4.0 * math.pi)))
    for m in range(0, lmax + 1):
        if m > 0:
            pmm = -math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * st * pmm
        cm = torch.zeros_like(ct)
        sm = torch.zeros_like(ct)
        p_prev, p_cur = None, pmm
        for l in range(m, lmax + 1):
            if l == m + 1:
                p_prev, p_cur = p_cur, math.sqrt(2.0 * m + 3.0) * ct * pmm
            elif l > m + 1:
                a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
                b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
                p_prev, p_cur = p_cur, a * (ct * p_cur - b * p_prev)
            if l == 0:
                continue
            cm = cm + float(coeffs[l, lmax + m]) * p_cur
            if m > 0:
                sm = sm + float(coeffs[l, lmax - m]) * p_cur
        if m == 0:
            out = out + cm
        else:
            out = out + math.sqrt(2.0) * (cm * torch.cos(m * lon) + sm * torch.sin(m * lon))
    return out.cpu().numpy()


def sh_coefficients(seed, lmax):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((lmax + 1, 2 * lmax + 1))
    c[0, :] = 0.0
    return c


def tc2_perturbed(node_xyz, edge_mid, edge_tan, seed=SEED_BASE + 1, lmax=32, amplitude=10.0,
                  radius=EARTH_RADIUS, omega=OMEGA, gravity=GRAVITY, device=None):
    dh, u, H = tc2(node_xyz, edge_mid, edge_tan, radius, omega, gravity)
    S = real_sph_harm_sum(node_xyz, sh_coefficients(seed, lmax), lmax, device)
    return dh + amplitude * S / np.abs(S).max(), u, H


def random_state(n_nodes, n_edges, seed, dh_scale=100.0, u_scale=10.0):
    """Unstructured random fields (for identity and parity tests, not physical)."""
    rng = np.random.default_rng(seed)
    return dh_scale * rng.standard_normal(n_nodes), u_scale * rng.standard_normal(n_edges)


def jet_profile(radius=EARTH_RADIUS, omega=OMEGA, gravity=GRAVITY, umax=80.0, lat0=45.0, width=8.0,
                mean_depth=1.0e4, npts=200001):
    """Latitude table of the balanced jet height, h(lat) = h0 - (a/g) int u (f + u tan/a) dlat."""
    lat = np.linspace(-math.pi / 2, math.pi / 2, npts)
    u = umax * np.exp(-((np.degrees(lat) - lat0) / width) ** 2)
    f = 2.0 * omega * np.sin(lat)
    with np.errstate(invalid="ignore", divide="ignore"):
        integrand = np.where(np.abs(np.cos(lat)) > 1e-12, u * (f + u * np.tan(lat) / radius), 0.0)
    step = lat[1] - lat[0]
    cum = np.zeros(npts)
    # composite Simpson on pairs of intervals, trapezoid for the odd leftover point
    cum[2::2] = np.cumsum((integrand[0:-2:2] + 4 * integrand[1:-1:2] + integrand[2::2]) * step / 3.0)
    cum[1::2] = cum[0:-1:2] + 0.5 * step * (integrand[0:-1:2] + integrand[1::2])
    hrel = -(radius / gravity) * cum
    # area mean of h equals mean_depth: mean over the sphere weights by cos(lat)
    w = np.cos(lat)
    h0 = mean_depth - (hrel * w).sum() / w.sum()
    return lat, u, h0 + hrel


def jet(node_xyz, edge_mid, edge_tan, bump=120.0, bump_lat=45.0, bump_lon=0.0,
        radius=EARTH_RADIUS, omega=OMEGA, gravity=GRAVITY, mean_depth=1.0e4):
    lat_t, u_t, h_t = jet_profile(radius, omega, gravity, mean_depth=mean_depth)
    x = node_xyz / np.linalg.norm(node_xyz, axis=1, keepdims=True)
    lat = np.arcsin(np.clip(x[:, 2], -1, 1))
    lon = np.arctan2(x[:, 1], x[:, 0])
    h = np.interp(lat, lat_t, h_t)
    dlon = np.degrees(lon) - bump_lon
    dlon = (dlon + 180.0) % 360.0 - 180.0
    h = h + bump * np.exp(-((np.degrees(lat) - bump_lat) / 6.0) ** 2) * np.exp(-(dlon / 12.0) ** 2)
    m = edge_mid / np.linalg.norm(edge_mid, axis=1, keepdims=True)
    mlat = np.arcsin(np.clip(m[:, 2], -1, 1))
    speed = np.interp(mlat, lat_t, u_t)
    east = np.stack([-m[:, 1], m[:, 0], np.zeros_like(m[:, 0])], 1)
    east /= np.maximum(np.linalg.norm(east, axis=1, keepdims=True), 1e-300)
    u = speed * (east * edge_tan).sum(1)
    return h - mean_depth, u, mean_depth


def turbulence_coefficients(seed=SEED_BASE + 5, l_peak=40, width=None, u_rms=20.0, radius=EARTH_RADIUS):
    """Streamfunction coefficients psi_lm (m^2/s) of orthonormal real harmonics, in the layout of
    ``real_sph_harm_sum``, and the degree cut-off.  Kinetic energy per degree
    E(l) ~ exp(-((l - l_peak) / width)^2) on l_peak +- 3 width (width l_peak / 5 by default); the
    coefficients of degree l are N(0, sigma_l^2) with (2l+1) l(l+1) sigma_l^2 ~ E(l), scaled so
    that the area mean of |u|^2, sum l(l+1) psi_lm^2 / (4 pi a^2), is u_rms^2 exactly."""
    width = float(l_peak) / 5.0 if width is None else float(width)
    l_lo = max(1, int(math.floor(l_peak - 3 * width)))
    lmax = int(math.ceil(l_peak + 3 * width))
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((lmax + 1, 2 * lmax + 1))
    l = np.arange(lmax + 1, dtype=np.float64)
    spec = np.where(l >= l_lo, np.exp(-((l - l_peak) / width) ** 2), 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        sig = np.where(l >= 1, np.sqrt(spec / np.maximum((2 * l + 1) * l * (l + 1), 1.0)), 0.0)
    c *= sig[:, None]
    for k in range(lmax + 1):          # only |m| <= l exists
        c[k, : lmax - k] = 0.0
        c[k, lmax + k + 1:] = 0.0
    mean_u2 = (l[:, None] * (l[:, None] + 1) * c * c).sum() / (4.0 * math.pi * radius * radius)
    return c * (u_rms / math.sqrt(mean_u2)), lmax


def turbulence(node_xyz, edge_mid, edge_tan, seed=SEED_BASE + 5, l_peak=40, width=None, u_rms=20.0,
               mean_depth=1000.0, radius=EARTH_RADIUS, omega=OMEGA, gravity=GRAVITY, device=None,
               delta=1e-5):
    """Returns (dh, u, H).  u_e = (k x grad psi) . t_e at the edge midpoint, i.e. the derivative
    of psi along t_e x k, taken by a central difference over two points an angle 2 atan(delta)
    apart (error ~ (l delta)^2); dh = f psi / g at the nodes (zero area mean: psi has no degree 1
    part)."""
    c, lmax = turbulence_coefficients(seed, l_peak, width, u_rms, radius)
    x = node_xyz / np.linalg.norm(node_xyz, axis=1, keepdims=True)
    psi_n = real_sph_harm_sum(x, c, lmax, device)
    dh = 2.0 * omega * x[:, 2] * psi_n / gravity
    m = edge_mid / np.linalg.norm(edge_mid, axis=1, keepdims=True)
    t = edge_tan - (edge_tan * m).sum(1, keepdims=True) * m
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    dirn = np.cross(t, m)                  # t x k: grad psi . (t x k) = (k x grad psi) . t
    psi_p = real_sph_harm_sum(m + delta * dirn, c, lmax, device)
    psi_m = real_sph_harm_sum(m - delta * dirn, c, lmax, device)
    u = (psi_p - psi_m) / (2.0 * math.atan(delta) * radius)
    return dh, u, mean_depth


def mlp_init(seed=SEED_BASE + 3, n_in=64, n_hidden=128, n_out=4):
    """Initial parameters of the child-patch predictor network (flat float32 vector, the layout
    of the C ABI): weights uniform in +-sqrt(6 / fan_in), biases zero.  Random numbers only."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((n_in, n_hidden), (n_hidden, n_hidden), (n_hidden, n_out)):
        b = np.sqrt(6.0 / fi)
        parts.append(rng.uniform(-b, b, fi * fo))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def ensemble_members(m, seed=SEED_BASE + 4, jmax_choices=(7, 8, 9), eps_choices=(2e-3, 5e-3, 1e-2)):
    """Seeded draws of an ensemble of jet members: bump amplitude U[60, 180] m, bump centre
    45 deg + U[-15, 15] deg latitude, U[-15, 15] deg longitude, Jmax and eps from the choices."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(m):
        out.append(dict(bump=float(rng.uniform(60.0, 180.0)), bump_lat=float(45.0 + rng.uniform(-15.0, 15.0)),
                        bump_lon=float(rng.uniform(-15.0, 15.0)), jmax=int(rng.choice(jmax_choices)),
                        eps=float(rng.choice(eps_choices))))
    return out

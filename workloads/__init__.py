"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds none of the lattice Boltzmann arithmetic: it only produces
macroscopic initial fields (density, velocity), body descriptions, instance
sizes and quadrature points.  Each side turns the fields into populations with
its own equilibrium.  All quantities are in lattice units.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Taylor-Green vortices (textbook initial conditions; the paper does not use
# them, they are the periodic benchmark workloads)
# ---------------------------------------------------------------------------


def taylor_green_2d(n, u0=0.02):
    """2D Taylor-Green vortex on an n x n periodic grid, wavenumber k = 2 pi / n.

    u_x = -u0 cos(kx) sin(ky), u_y = u0 sin(kx) cos(ky),
    rho = 1 - (3 u0^2 / 4)(cos 2kx + cos 2ky)   (rho = 1 + p'/cs^2).
    Returns rho (N,), u (2, N) planar, x-fastest.
    """
    k = 2.0 * math.pi / n
    y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                       indexing="ij")
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    rho = 1.0 - 0.75 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    return rho.ravel(), np.stack([ux.ravel(), uy.ravel()])


def taylor_green_2d_decay(nu, n, t):
    """Analytic velocity decay factor exp(-2 nu k^2 t) of the 2D vortex."""
    k = 2.0 * math.pi / n
    return math.exp(-2.0 * nu * k * k * t)


def tg3d_params(n, re=1600.0, ma=0.1):
    """U0 = Ma cs, L = n / (2 pi), nu = U0 L / Re for the 3D vortex on n^3."""
    u0 = ma / math.sqrt(3.0)
    L = n / (2.0 * math.pi)
    nu = u0 * L / re
    return u0, L, nu


def taylor_green_3d(n, re=1600.0, ma=0.1, perturb=1e-4, seed=1600, shape=None):
    """3D Taylor-Green vortex on an n^3 periodic grid (optionally a sub-box).

    u = U0 (sin X cos Y cos Z, -cos X sin Y cos Z, 0), X = x / L,
    rho = 1 + 3 (U0^2/16)(cos 2X + cos 2Y)(cos 2Z + 2),
    plus a seeded perturbation u += perturb * U0 * xi, xi ~ U(-1, 1) i.i.d. per
    node and component (numpy default_rng(seed), drawn for the full n^3 grid in
    x-fastest order, so sub-boxes see the same values).
    Returns (rho (N,), u (3, N), nu).
    """
    u0, L, nu = tg3d_params(n, re, ma)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    X, Y, Z = x / L, y / L, z / L
    ux = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    uy = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    uz = np.zeros_like(ux)
    rho = 1.0 + 3.0 * (u0 * u0 / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    u = np.stack([ux.ravel(), uy.ravel(), uz.ravel()])
    if perturb:
        rng = np.random.default_rng(seed)
        xi = rng.uniform(-1.0, 1.0, size=(n * n * n, 3)).T
        u = u + perturb * u0 * xi
    return rho.ravel(), u, nu


def random_node_states(Q, count, seed, amp=0.3):
    """Random positive node states f_i = W_i (1 + amp * xi_i), xi ~ U(-1, 1).

    W_i are the tensor-product D1Q3 weights (2/3, 1/6, 1/6 per axis), rebuilt
    here from their definition.  Returns an array (count, Q).
    """
    rng = np.random.default_rng(seed)
    w1 = np.array([1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0])
    idx = np.arange(Q)
    w = w1[idx % 3] * w1[(idx // 3) % 3] * (w1[idx // 9] if Q == 27 else 1.0)
    return w[None, :] * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(count, Q)))


# ---------------------------------------------------------------------------
# Bodies (prescribed motion laws; parameter layout shared by both sides)
# ---------------------------------------------------------------------------

BODY_NONE, BODY_SPHERE, BODY_FLAP, BODY_MESH, BODY_PLATES = 0, 1, 2, 3, 4


def sphere_params(center, radius, amplitude=(0.0, 0.0, 0.0), period=None, phase=0.0):
    """Sphere (circle in 2D): centre X0 + A sin(omega t + phase)."""
    omega = 0.0 if not period else 2.0 * math.pi / period
    p = np.zeros(16)
    p[0:3] = list(center) + [0.0] * (3 - len(center))
    p[3] = radius
    p[4:7] = list(amplitude) + [0.0] * (3 - len(amplitude))
    p[7] = omega
    p[8] = phase
    return p


def flap_params(x_f, length, thickness, amplitude, period, phase=0.0, y_base=-0.5):
    """2D flap clamped on the bottom wall: centre line x_f + d0 sin(wt+phi)(s/l)^2."""
    p = np.zeros(16)
    p[0:7] = [x_f, length, thickness, amplitude, 2.0 * math.pi / period, phase, y_base]
    return p


def plates_params(y_lo, y_hi, u_lo=(0.0, 0.0, 0.0), u_hi=(0.0, 0.0, 0.0)):
    """Two parallel plates, solid below y_lo and above y_hi, sliding tangentially."""
    p = np.zeros(16)
    p[0], p[1] = y_lo, y_hi
    p[2:5] = list(u_lo) + [0.0] * (3 - len(u_lo))
    p[5:8] = list(u_hi) + [0.0] * (3 - len(u_hi))
    return p


# ---------------------------------------------------------------------------
# Sphere in a channel (3D) and the batch of 2D flap channels
# ---------------------------------------------------------------------------


def sphere_channel(nx=512, ny=128, nz=128, radius=16.0, amplitude=4.0, period=3200.0,
                   u=0.05, re=300.0, ramp=1000):
    """Channel with an oscillating sphere: returns a dict of instance settings."""
    nu = u * 2.0 * radius / re
    center = (nx / 4.0, ny / 2.0, nz / 2.0)
    return dict(Q=27, nx=nx, ny=ny, nz=nz, nu=nu,
                faces=["inlet", "outlet", "periodic", "periodic", "periodic", "periodic"],
                u_in=(u, 0.0, 0.0), inlet_profile=0, ramp_steps=ramp,
                body=(BODY_SPHERE, sphere_params(center, radius, (0.0, amplitude, 0.0), period)),
                U=u, radius=radius)


def flap_channels(count=64, seed=2375, ubar=0.05):
    """Uneven 2D channels with a prescribed-motion flap on the bottom wall.

    Each quantity is drawn for all channels at once, in this order, from
    default_rng(seed): H = 16 * randint(4, 17); W = clip(16 * round(H * U(2,4)
    / 16), 128, 1024); flap length l = H * U(0.2, 0.4); Re = 10^U(2,3) with
    Re = Ubar H / nu.  Parabolic inflow with mean Ubar; walls at top and
    bottom; flap at W/4 with thickness max(2, H/32), tip amplitude 0.15 l,
    period 20 l / Ubar.  The 64-channel batch of seed 2375 has 5,608,448
    nodes (8,192 to 249,856 per channel).
    """
    rng = np.random.default_rng(seed)
    Hs = 16 * rng.integers(4, 17, size=count)
    Ws = np.clip(16 * np.round(Hs * rng.uniform(2.0, 4.0, size=count) / 16.0), 128, 1024)
    ells = Hs * rng.uniform(0.2, 0.4, size=count)
    res = 10.0 ** rng.uniform(2.0, 3.0, size=count)
    out = []
    for H, W, ell, re in zip(Hs, Ws, ells, res):
        H, W, ell, re = int(H), int(W), float(ell), float(re)
        nu = ubar * H / re
        thick = max(2.0, H / 32.0)
        out.append(dict(Q=9, nx=W, ny=H, nz=1, nu=nu,
                        faces=["inlet", "outlet", "wall", "wall", "periodic", "periodic"],
                        u_in=(ubar, 0.0, 0.0), inlet_profile=1, ramp_steps=0,
                        body=(BODY_FLAP, flap_params(W / 4.0, ell, thick, 0.15 * ell,
                                                     20.0 * ell / ubar)),
                        re=re))
    return out


# ---------------------------------------------------------------------------
# Surface quadrature
# ---------------------------------------------------------------------------


def icosphere(subdiv=4):
    """Unit icosphere: vertices (V,3), triangles (T,3)."""
    t = (1.0 + 5 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t),
         (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array(faces, dtype=np.int64)


def sphere_quadrature(center, radius, subdiv=4):
    """One point per flat facet of a scaled icosphere: centroid, unit outward
    facet normal, facet area.  sum_q w_q n_q = 0 holds for the closed surface."""
    V, T = icosphere(subdiv)
    V = V * radius + np.asarray(center, dtype=np.float64)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    xq = (a + b + c) / 3.0
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    n = cr / (2.0 * area[:, None])
    flip = np.sum(n * (xq - np.asarray(center)), axis=1) < 0
    n[flip] *= -1.0
    return xq, n, area


def circle_quadrature(center, radius, count=256):
    """2D analogue: midpoints of a regular polygon's edges, outward normals, lengths."""
    th = 2.0 * math.pi * np.arange(count + 1) / count
    p = np.stack([np.cos(th), np.sin(th)], axis=1) * radius + np.asarray(center)
    a, b = p[:-1], p[1:]
    xq = 0.5 * (a + b)
    e = b - a
    length = np.linalg.norm(e, axis=1)
    n = np.stack([e[:, 1], -e[:, 0]], axis=1) / length[:, None]
    flip = np.sum(n * (xq - np.asarray(center)), axis=1) < 0
    n[flip] *= -1.0
    return xq, n, length


def plate_quadrature(y, normal_sign, nx, width=1.0):
    """Points along a horizontal plate surface at height y (2D), one per column."""
    xq = np.stack([np.arange(nx, dtype=np.float64), np.full(nx, y)], axis=1)
    n = np.zeros((nx, 2))
    n[:, 1] = normal_sign
    return xq, n, np.full(nx, width)


# ---------------------------------------------------------------------------
# Surface meshes (closed; positions and faces only)
# ---------------------------------------------------------------------------


def cube_mesh(lo, hi):
    """Axis-aligned box [lo, hi] as 8 vertices and 12 outward-oriented
    triangles."""
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    V = np.array([[(hi if (k >> a) & 1 else lo)[a] for a in range(3)] for k in range(8)])
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    T = []
    for a, b, c, d in quads:
        T += [(a, b, c), (a, c, d)]
    return V, np.array(T, dtype=np.int64)


def sphere_mesh(center, radius, subdiv=3):
    """Icosphere with its vertices on the sphere (radius, center)."""
    V, T = icosphere(subdiv)
    return V * radius + np.asarray(center, dtype=np.float64), T


def circle_polygon(center, radius, count=64):
    """Closed polygon with its vertices on a circle, as 2D 'faces' (segments
    of the first two indices; z = 0)."""
    th = 2.0 * math.pi * np.arange(count) / count
    V = np.zeros((count, 3))
    V[:, 0] = center[0] + radius * np.cos(th)
    V[:, 1] = center[1] + radius * np.sin(th)
    T = np.stack([np.arange(count), (np.arange(count) + 1) % count, np.arange(count)], 1)
    return V, T.astype(np.int64)


def droplet_impact(nx=320, ny=250, nz=320, diameter=80.0, gap=4.0, u_impact=0.02, width=2.0,
                   rho_l=7.52, rho_v=0.073):
    """Multiphase droplet-impact setup of Sec. III.B: a liquid droplet of the
    given diameter (80 lattice spacings, domain 320 x 250 x 320 as in the
    paper) centred over the middle of a wall at the bottom (-y) face, its
    lowest point `gap` spacings above the first node row, moving towards the
    wall at u_impact inside the droplet; vapour at rest elsewhere.  The
    interface is a tanh profile of the given width between the flat-interface
    densities of the equation of state.  Returns (rho (N,), u (3, N), info);
    faces: walls at -y and +y, periodic in x and z."""
    R = 0.5 * diameter
    c = (0.5 * (nx - 1), R + gap, 0.5 * (nz - 1))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2).ravel()
    phase = 0.5 * (1.0 - np.tanh((r - R) / width))
    rho = rho_v + (rho_l - rho_v) * phase
    u = np.zeros((3, rho.size))
    u[1] = -u_impact * phase
    faces = ["periodic", "periodic", "wall", "wall", "periodic", "periodic"]
    return rho, u, dict(centre=c, radius=R, faces=faces)


def fsi3(d_lb=40, u_mean=0.035, nex=20, ney=2, arc_points=120, theta=0.55):
    """FSI3 of Sec. III.A.1 in lattice units: channel 2.5 x 0.41 m, cylinder
    of diameter D = 0.1 m at (0.2, 0.2) m, elastic flap 0.35 x 0.02 m clamped
    in it; rho_f = rho_s = 1e3 kg/m^3, nu_f = 1e-3 m^2/s, mean inflow 2 m/s
    (Re = 200), mu_s = 2e6 Pa, nu_s = 0.4 (Ae = 1.4e3), parabolic inflow with
    a 2 s cosine ramp.  D is resolved by d_lb spacings; the mean inflow is
    u_mean in lattice units.  Physical point (X, Y) is the lattice point
    (X/dx - 1/2, Y/dx - 1/2): the walls lie half a spacing outside the first
    and last node rows.  Returns a dict with the lattice domain, viscosity,
    time and stress scales, the beam parameters (lattice units) and the
    cylinder chain from the flap's clamped top corner round to its bottom
    corner.  theta = 0.55 (shifted Crank-Nicolson) damps the beam's
    high-frequency axial modes, which the staggered coupling otherwise
    excites (theta = 1/2 grows an alternating axial mode within 0.1 s); at
    the flag's 5.5 Hz the damping per period is below 1e-3."""
    D, H, Lc, U = 0.1, 0.41, 2.5, 2.0
    dx = D / d_lb
    dt = u_mean * dx / U
    nu_lb = 1e-3 * dt / dx ** 2
    stress = 1e3 * (dx / dt) ** 2
    to_lat = lambda X: X / dx - 0.5
    cx, cy, r = to_lat(0.2), to_lat(0.2), 0.05 / dx
    h = 0.02 / dx
    xc = 0.2 + np.sqrt(0.05 ** 2 - 0.01 ** 2)          # clamped edge on the circle
    x0, y0 = to_lat(xc), to_lat(0.19)
    length = (0.6 - xc) / dx
    a0 = np.arcsin(0.5 * h / r)
    ang = np.linspace(a0, 2 * np.pi - a0, arc_points + 2)[1:-1]
    arc = np.stack([cx + r * np.cos(ang), cy + r * np.sin(ang)], 1)
    mu_s, nu_s = 2e6 / stress, 0.4
    lam_s = 2 * mu_s * nu_s / (1 - 2 * nu_s)
    return dict(nx=int(round(Lc / dx)), ny=int(round(H / dx)), nu=nu_lb, dt=dt, dx=dx,
                stress=stress, u_mean=u_mean,
                faces=["inlet", "outlet", "wall", "wall", "periodic", "periodic"],
                inlet_profile=1, ramp_steps=int(round(2.0 / dt)),
                beam=(x0, y0, length, h, nex, ney, 1.0, lam_s, mu_s, 1.0, theta),
                arc=arc, steps_per_second=int(round(1.0 / dt)))

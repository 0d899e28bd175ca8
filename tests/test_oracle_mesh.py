"""Pins of the oracle's surface-mesh body (Sec. II.C.1: the structure's
surface as triangles, vertex velocities interpolated at the link
intersections): the solid test against shapes the mesh reproduces exactly,
the wall points and wall velocities through Grad target values that are
exact for a rigid-body velocity field, and the fresh-node velocity through a
polygon carried by a uniform flow."""
import math

import numpy as np
import pytest

import workloads as W


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(float)


@pytest.mark.parametrize("flip", [False, True])
def test_cube_mesh_solid_is_the_box(orc, flip):
    """12 triangles of an axis-aligned box with non-integer bounds: the solid
    nodes are exactly the nodes inside the box, for either orientation of the
    faces."""
    n = 9
    lo, hi = (1.3, 2.2, 0.6), (5.6, 6.7, 4.4)
    V, T = W.cube_mesh(lo, hi)
    if flip:
        T = T[:, ::-1].copy()
    d = orc.Domain(27, n, n, n, 0.05)
    d.set_mesh(V, np.zeros_like(V), T)
    X = _grid(n, n, n)
    box = np.all((X >= lo) & (X <= hi), axis=1)
    assert box.sum() > 20
    assert np.array_equal(d.solid().astype(bool), box)


def test_icosphere_solid_matches_sphere_off_the_facet_band(orc):
    """An icosphere with its vertices on a sphere of radius R: nodes closer
    to the centre than the smallest facet-plane distance are solid, nodes
    beyond R are fluid."""
    n, R, c = 17, 5.3, np.array([8.2, 7.9, 8.4])
    V, T = W.sphere_mesh(c, R, subdiv=3)
    a, b, cc = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nrm = np.cross(b - a, cc - a)
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    r_in = np.min(np.abs(np.sum(nrm * (a - c), axis=1)))
    d = orc.Domain(27, n, n, n, 0.05)
    d.set_mesh(V, np.zeros_like(V), T)
    r = np.linalg.norm(_grid(n, n, n) - c, axis=1)
    s = d.solid().astype(bool)
    assert np.all(s[r < r_in]) and not np.any(s[r > R])
    assert (r < r_in).sum() > 400


def test_square_polygon_solid_is_the_square_2d(orc):
    n = 12
    x0, x1, y0, y1 = 2.4, 8.7, 3.1, 9.5
    V = np.array([[x0, y0, 0], [x1, y0, 0], [x1, y1, 0], [x0, y1, 0]], dtype=float)
    T = np.array([[0, 1, 0], [1, 2, 1], [2, 3, 2], [3, 0, 3]])
    d = orc.Domain(9, n, n, 1, 0.05)
    d.set_mesh(V, np.zeros_like(V), T)
    X = _grid(n, n, 1)
    sq = (X[:, 0] >= x0) & (X[:, 0] <= x1) & (X[:, 1] >= y0) & (X[:, 1] <= y1)
    assert np.array_equal(d.solid().astype(bool), sq)


@pytest.mark.parametrize("Q", [27, 9])
def test_rigid_motion_targets_exact_on_mesh(orc, Q):
    """A box (3D) or polygon (2D) whose vertices move with a rigid-body
    velocity V(x) = U + Omega x (x - x0), and lagged fields prepared as the
    equilibrium of u = V(x) everywhere.  The wall point of each cut link lies
    on a face, where the vertex velocities interpolate the linear field
    exactly, and every interpolation and difference of the target values is
    exact for a linear field: at every node with missing populations the
    target velocity is V(x) and the target gradient the rotation matrix."""
    D = 3 if Q == 27 else 2
    n = 12
    x0 = np.array([5.9, 6.2, 6.1])
    U = np.array([0.012, -0.007, 0.004])
    Om = np.array([0.0007, -0.0004, 0.0011]) if D == 3 else np.array([0.0, 0.0, 0.0009])
    if D == 3:
        V, T = W.cube_mesh((3.4, 3.7, 3.2), (8.3, 8.6, 8.7))
    else:
        V = np.array([[3.4, 3.7, 0], [8.3, 3.9, 0], [8.6, 8.3, 0], [3.2, 8.6, 0]], dtype=float)
        T = np.array([[0, 1, 0], [1, 2, 1], [2, 3, 2], [3, 0, 3]])
        U[2] = 0.0
    field = lambda X: U + np.cross(Om, X - x0)
    Vel = field(V)
    if D == 2:
        Vel[:, 2] = 0.0
    nz = n if D == 3 else 1
    X = _grid(n, n, nz)
    u = field(X).T[:D]
    d = orc.Domain(Q, n, n, nz, 0.05)
    d.init_fields(np.ones(X.shape[0]), u)
    d.set_mesh(V, Vel, T)
    G = np.zeros((3, 3))   # d u_a / d x_b of U + Omega x (x - x0)
    G[0, 1], G[0, 2], G[1, 0], G[1, 2], G[2, 0], G[2, 1] = -Om[2], Om[1], Om[2], -Om[0], -Om[1], Om[0]
    if D == 2:
        G[2, :] = 0.0
        G[:, 2] = 0.0
    count = 0
    for p in X.astype(int):
        t = d.grad_targets(*p)
        if t is None:
            continue
        count += 1
        exp = field(p.astype(float))
        assert np.max(np.abs(t["u"][:D] - exp[:D])) < 1e-12, (p, t["u"], exp)
        assert np.max(np.abs(t["grad"] - G)) < 1e-11, (p, t["grad"])
    assert count > (150 if D == 3 else 20)


def test_polygon_carried_by_uniform_flow_leaves_it_uniform(orc):
    """A 48-gon carried by a uniform flow at its own velocity, the mesh moved
    every step (each mesh is the surface at the next step's time): nodes it
    uncovers are refilled at the velocity interpolated on the mesh, links are
    cut at the polygon's edges, and the flow stays uniform."""
    n, U, nu, rho0 = 48, 0.02, 0.02, 1.02
    c0 = np.array([18.3, 24.1])
    d = orc.Domain(9, n, n, 1, nu)
    N = n * n
    u = np.zeros((2, N))
    u[0] = U
    V0, T = W.circle_polygon(c0, 6.2, 48)
    Vel = np.zeros_like(V0)
    Vel[:, 0] = U
    d.init_fields(np.full(N, rho0), u)
    d.set_mesh(V0, Vel, T)
    for k in range(200):
        V = V0.copy()
        V[:, 0] += U * (k + 1)
        d.set_mesh(V, Vel, T)
        d.step(1)
    rho, uu, tot = d.moments()
    fl = d.solid() == 0
    assert np.max(np.abs(uu[0][fl] - U)) < 5e-5 * U
    assert np.max(np.abs(uu[1][fl])) < 5e-5 * U
    assert np.max(np.abs(rho[fl] - rho0)) < 2e-6


def test_mesh_velocity_at_closest_point_of_a_box(orc):
    """The closest point of a box to an outside point is the componentwise
    clamp into the box (face, edge or corner); the mesh velocity there, for
    a rigid-body motion of the vertices, is that motion's velocity at the
    clamped point (to rounding), so the triangle interiors, edges and
    vertices of the closest-point search are all exercised."""
    lo, hi = np.array([3.4, 3.7, 3.2]), np.array([8.3, 8.6, 8.7])
    V, T = W.cube_mesh(lo, hi)
    x0, U, Om = np.array([5.9, 6.2, 6.1]), np.array([0.01, -0.02, 0.03]), np.array([0.3, -0.2, 0.5])
    field = lambda X: U + np.cross(Om, X - x0)
    d = orc.Domain(27, 12, 12, 12, 0.05)
    d.set_mesh(V, field(V), T)
    rng = np.random.default_rng(9)
    P = rng.uniform(0.0, 12.0, size=(400, 3))
    P = P[np.any((P < lo) | (P > hi), axis=1)]
    for p in P:
        v = d.body_velocity(p)
        assert np.max(np.abs(v - field(np.clip(p, lo, hi)))) < 1e-12, p


@pytest.mark.parametrize("Q", [9, 27])
def test_nodes_on_the_surface_are_solid(orc, Q):
    """Faces through lattice nodes (integer bounds): the nodes on the faces,
    edges and corners count as solid, so the solid set is the closed box."""
    if Q == 27:
        n = 9
        lo, hi = (1.0, 2.0, 1.0), (5.0, 6.0, 4.0)
        V, T = W.cube_mesh(lo, hi)
        d = orc.Domain(27, n, n, n, 0.05)
        X = _grid(n, n, n)
    else:
        n = 12
        lo, hi = (2.0, 3.0), (9.0, 8.0)
        V = np.array([[lo[0], lo[1], 0], [hi[0], lo[1], 0], [hi[0], hi[1], 0], [lo[0], hi[1], 0]],
                     dtype=float)
        T = np.array([[0, 1, 0], [1, 2, 1], [2, 3, 2], [3, 0, 3]])
        d = orc.Domain(9, n, n, 1, 0.05)
        X = _grid(n, n, 1)[:, :2]
    d.set_mesh(V, np.zeros_like(V), T)
    box = np.all((X >= lo) & (X <= hi), axis=1)
    assert np.array_equal(d.solid().astype(bool), box)

"""Surface-mesh bodies on the GPU (Sec. II.C.1: the structure's surface as
triangles, vertex velocities interpolated at the link intersections) against
the oracle, whose mesh geometry is computed independently (generalized
winding number, bisection, closest point; the GPU uses line crossings and
ray-face intersection).  F64 runs agree to the arithmetic's rounding, so
every population of every fluid node is compared at 1e-12."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _pair(Q, nx, ny, nz, nu, storage="f64", rho=None, u=None, **kw):
    from paper_1710_02375_amd import lbm

    s = lbm.Solver([dict(Q=Q, nx=nx, ny=ny, nz=nz, nu=nu, storage=storage, **kw)])
    okw = {k: v for k, v in kw.items() if k in ("faces", "u_in", "inlet_profile", "ramp_steps")}
    d = oracle.Domain(Q, nx, ny, nz, nu, **okw)
    N = nx * ny * nz
    D = 3 if Q == 27 else 2
    if rho is None:
        rho, u = np.ones(N), np.zeros((D, N))
    s.init_fields(rho, u)
    d.init_fields(rho, u)
    return s, d


def _set_mesh(s, d, V, Vel, T):
    from paper_1710_02375_amd import lbm

    s.set_body(lbm.LBM_BODY_MESH, verts=V, vert_vel=Vel, tris=T)
    d.set_mesh(V, Vel, T)


def _compare(s, d, tol, label):
    fl = d.solid() == 0
    fg, fo = s.get_populations(), d.get_populations()
    err = float(np.max(np.abs(fg[:, fl] - fo[:, fl])))
    say("  %s: max |df| over %d fluid nodes = %.3e" % (label, int(fl.sum()), err))
    assert err < tol, label


def test_static_icosphere_channel_f64():
    """An icosphere (320 faces) at rest in a channel with inflow and
    outflow: solid nodes, cut links and Grad fill agree with the oracle."""
    nx, ny, nz, R = 24, 16, 16, 4.3
    c = (9.3, 7.8, 8.1)
    V, T = W.sphere_mesh(c, R, subdiv=2)
    say("case: static icosphere mesh F64 %dx%dx%d" % (nx, ny, nz))
    s, d = _pair(27, nx, ny, nz, 0.05, faces=["inlet", "outlet", "periodic", "periodic",
                                              "periodic", "periodic"], u_in=(0.03, 0, 0),
                 ramp_steps=10)
    _set_mesh(s, d, V, np.zeros_like(V), T)
    solid_g = s.moments()[0] == 0
    assert np.array_equal(solid_g, d.solid() == 1)
    for k in (1, 4, 10):
        s.step(k)
        d.step(k)
        _compare(s, d, 1e-12, "t=%d" % d.time)
    xq, nq, wq = W.sphere_quadrature(c, R, subdiv=2)
    Fg, _ = s.wall_force(xq, nq, wq)
    Fo, _, st = d.wall_force(xq, nq, wq)
    say("  force gpu %s oracle %s" % (Fg, Fo))
    assert st == 0 and np.allclose(Fg, Fo, rtol=0, atol=1e-12)


def test_moving_icosphere_f64():
    """The mesh translated along x and y every step (each call gives the
    surface at the next step's time, with its vertex velocities): fresh
    nodes, moving cut links and wall velocities agree with the oracle."""
    n, R = 18, 4.1
    c0 = np.array([7.2, 8.9, 8.6])
    U = np.array([0.08, 0.03, 0.0])
    V0, T = W.sphere_mesh(c0, R, subdiv=2)
    Vel = np.tile(U, (V0.shape[0], 1))
    say("case: moving icosphere mesh F64 n=%d" % n)
    s, d = _pair(27, n, n, n, 0.05)
    _set_mesh(s, d, V0, Vel, T)
    for k in range(14):
        V = V0 + U * (k + 1)
        _set_mesh(s, d, V, Vel, T)
        s.step(1)
        d.step(1)
    assert np.array_equal(s.moments()[0] == 0, d.solid() == 1)
    _compare(s, d, 1e-12, "after %d steps (%.2f spacings)" % (d.time, np.linalg.norm(U) * 14))


def test_moving_polygon_2d_f64():
    n = 40
    c0 = np.array([12.3, 19.6])
    U = np.array([0.1, -0.04, 0.0])
    V0, T = W.circle_polygon(c0, 5.7, 40)
    Vel = np.tile(U, (V0.shape[0], 1))
    say("case: moving 40-gon D2Q9 F64 n=%d" % n)
    s, d = _pair(9, n, n, 1, 0.03)
    _set_mesh(s, d, V0, Vel, T)
    for k in range(30):
        _set_mesh(s, d, V0 + U * (k + 1), Vel, T)
        s.step(1)
        d.step(1)
    assert np.array_equal(s.moments()[0] == 0, d.solid() == 1)
    _compare(s, d, 1e-12, "after 30 steps")


def test_icosphere_against_analytic_sphere_f32():
    """The same sphere as an analytic body and as an icosphere (5120 faces,
    vertices on the sphere) in the scaled sphere channel: the solid masks
    agree off the band between the facets and the sphere, and the drag
    coefficients agree to within the mesh's geometric error (the centre is
    off the lattice, so that no node lies on the sphere itself, where the
    sphere counts it solid and the inscribed mesh does not)."""
    from paper_1710_02375_amd import lbm

    cfg = W.sphere_channel(96, 32, 32, radius=6.0, amplitude=0.0, period=None, ramp=50)
    R = cfg["radius"]
    c = np.array([24.31, 15.77, 16.18])   # off the lattice: no node on the sphere
    kind, p = W.BODY_SPHERE, W.sphere_params(c, R)
    desc = dict(Q=27, nx=96, ny=32, nz=32, nu=cfg["nu"], storage="f32", faces=cfg["faces"],
                u_in=cfg["u_in"], ramp_steps=cfg["ramp_steps"])
    N = 96 * 32 * 32
    out = {}
    V, T = W.sphere_mesh(c, R, subdiv=4)
    a, b, cc = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nrm = np.cross(b - a, cc - a)
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    r_in = np.min(np.abs(np.sum(nrm * (a - c), axis=1)))
    say("case: icosphere (5120 faces) vs analytic sphere R=%g, facet band %.4f" % (R, R - r_in))
    for name in ("analytic", "mesh"):
        s = lbm.Solver([desc])
        s.init_fields(np.ones(N), np.zeros((3, N)))
        if name == "analytic":
            s.set_body(kind, p)
        else:
            s.set_body(lbm.LBM_BODY_MESH, verts=V, vert_vel=np.zeros_like(V), tris=T)
        solid = s.moments()[0] == 0
        s.step(600)
        xq, nq, wq = W.sphere_quadrature(c, R, subdiv=4)
        F, _ = s.wall_force(xq, nq, wq)
        out[name] = (solid, F)
        s.close()
    z, y, x = np.meshgrid(np.arange(32), np.arange(32), np.arange(96), indexing="ij")
    r = np.sqrt((x.ravel() - c[0]) ** 2 + (y.ravel() - c[1]) ** 2 + (z.ravel() - c[2]) ** 2)
    off_band = (r < r_in) | (r > R)
    assert np.array_equal(out["analytic"][0][off_band], out["mesh"][0][off_band])
    norm = 0.5 * cfg["U"] ** 2 * math.pi * R * R
    cd_a, cd_m = out["analytic"][1][0] / norm, out["mesh"][1][0] / norm
    say("  Cd analytic %.5f mesh %.5f (relative difference %.2e)" % (cd_a, cd_m, abs(cd_m / cd_a - 1)))
    assert abs(cd_m / cd_a - 1) < 0.03


def test_mesh_errors():
    from paper_1710_02375_amd import lbm

    say("case: invalid meshes")
    s = lbm.Solver([dict(Q=27, nx=12, ny=12, nz=12, nu=0.05)])
    V, T = W.cube_mesh((3.3, 3.3, 3.3), (7.7, 7.7, 7.7))
    bad = T.copy()
    bad[3, 1] = 99
    with pytest.raises(lbm.LBMError) as ei:
        s.set_body(lbm.LBM_BODY_MESH, verts=V, vert_vel=np.zeros_like(V), tris=bad)
    assert ei.value.status == lbm.LBM_ERR_INVALID
    with pytest.raises(lbm.LBMError) as ei:
        s.set_body(lbm.LBM_BODY_MESH, verts=V + 6.0, vert_vel=np.zeros_like(V), tris=T)
    assert ei.value.status == lbm.LBM_ERR_GEOMETRY


def test_faces_through_nodes_f64():
    """A polygon whose edges pass through lattice nodes (integer bounds) in a
    channel: nodes on the surface are solid on both sides, and the cut links
    that end on them (q = 1) agree with the oracle."""
    nx, ny = 40, 24
    V = np.array([[12.0, 8.0, 0], [22.0, 8.0, 0], [22.0, 15.0, 0], [12.0, 15.0, 0]])
    T = np.array([[0, 1, 0], [1, 2, 1], [2, 3, 2], [3, 0, 3]], dtype=np.int32)
    say("case: square polygon with edges through nodes, F64 %dx%d" % (nx, ny))
    s, d = _pair(9, nx, ny, 1, 0.05, faces=["inlet", "outlet", "wall", "wall", "periodic",
                                              "periodic"], u_in=(0.03, 0, 0), ramp_steps=10)
    _set_mesh(s, d, V, np.zeros_like(V), T)
    solid_g = s.moments()[0] == 0
    assert np.array_equal(solid_g, d.solid() == 1), (int(solid_g.sum()), int(d.solid().sum()))
    for k in (1, 10):
        s.step(k)
        d.step(k)
        _compare(s, d, 1e-12, "t=%d" % d.time)

"""Pins of the oracle's two-way coupling (Sec. II.C).

The coupling composes pinned parts (the lattice step, the wall traction, the
beam); what it adds is checked here against exact answers: the wet-edge
quadrature of the undeformed beam (unit outward normals, lengths), the
consistent nodal loads of a uniform traction, and a fluid at rest, which
must leave the beam at rest (the reference pressure is no load)."""
import numpy as np

from oracle import fsi as ofsi
from oracle.fem import Beam


def _beam():
    return Beam(20.0, 14.5, 20.0, 3.0, 5, 1, 1.0, 20.0, 5.0, 1.0)


def test_wet_edge_quadrature_of_the_undeformed_beam():
    b = _beam()
    pts, nrm, wts, nodes, shp = ofsi.quadrature(b)
    assert abs(wts.sum() - (2 * 20.0 + 3.0)) < 1e-12
    bottom = np.isclose(pts[:, 1], 14.5)
    top = np.isclose(pts[:, 1], 17.5)
    tip = np.isclose(pts[:, 0], 40.0)
    assert bottom.sum() + top.sum() + tip.sum() == len(wts)
    assert np.allclose(nrm[bottom], [0, -1]) and np.allclose(nrm[top], [0, 1])
    assert np.allclose(nrm[tip], [1, 0])
    assert np.allclose(shp.sum(1), 1.0)


def test_uniform_traction_gives_consistent_loads():
    """A uniform traction t0 on the wet edges: the loads sum to t0 times the
    wet length, and their moment about the clamped end is that of the
    distributed load (Gauss quadrature is exact for the quadratic edges)."""
    b = _beam()
    pts, nrm, wts, nodes, shp = ofsi.quadrature(b)
    t0 = np.array([0.3, -0.7])
    f = ofsi.nodal_loads(b, np.tile(t0, (len(wts), 1)), nodes, shp, wts).reshape(-1, 2)
    assert np.allclose(f.sum(0), t0 * (2 * 20.0 + 3.0), rtol=0, atol=1e-12)
    X = b.X - b.X[0]
    M = np.sum(X[:, 0] * f[:, 1] - X[:, 1] * f[:, 0])
    # Exact moment: bottom edge y = 0, x in [0, 20]; tip x = 20, y in [0, 3];
    # top edge y = 3, x in [0, 20].
    Mx = t0[1] * (2 * 20.0 ** 2 / 2 + 20.0 * 3.0)
    My = -t0[0] * (3.0 ** 2 / 2 + 3.0 * 20.0)
    assert abs(M - (Mx + My)) < 1e-10


def test_fluid_at_rest_leaves_the_beam_at_rest():
    """Walls and periodic faces, fluid at rest at the reference density: the
    gauge traction vanishes and the beam stays where it is."""
    import oracle

    nx, ny = 48, 32
    d = oracle.Domain(9, nx, ny, 1, 0.05, faces=["periodic", "periodic", "wall", "wall",
                                                 "periodic", "periodic"])
    d.init_fields(np.ones(nx * ny), np.zeros((2, nx * ny)))
    b = _beam()
    mount = np.array([[20.0, 19.5], [12.0, 19.5], [12.0, 12.5], [20.0, 12.5]])
    c = ofsi.Coupled(d, b, mount)
    for _ in range(30):
        F = c.step()
    assert np.abs(b.u).max() < 1e-12 and np.abs(F).max() < 1e-12

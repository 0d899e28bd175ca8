"""Plain two-way fluid-structure coupling (Sec. II.C) of the oracle's lattice
Boltzmann domain and finite-element beam, in lattice units (test
infrastructure only).

Conventional serial staggered scheme, one structure step per fluid step:
  1. the fluid steps n -> n + 1 with the body surface of the structure state
     (x^n, v^n) (the surface moves with the structure's last known state);
  2. the traction t = sigma n of the fluid on the structure is sampled at the
     Gauss points of the beam's wet edges in their current position
     (Sec. II.C.2, the oracle's wall force), with the reference pressure
     rho_0 c_s^2 (rho_0 = 1) taken out: the beam is only partly wet (its
     clamped end is not), so a uniform pressure does not cancel on it, and
     the lattice's reference pressure is not a physical load;
  3. the beam takes its theta step with the consistent nodal loads
     f_a = sum_q N_a(xi_q) t_q w_q;
  4. the body surface is rebuilt from the new structure state.
The body is one closed polygon: the beam's bottom edge from the clamped end
to the tip, the tip edge, the top edge back, and an optional static chain
(e.g. the arc of a cylinder the beam is clamped in) from the top of the
clamped end round to its bottom.
"""
from __future__ import annotations

import numpy as np

_G3 = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
_W3 = np.array([5.0, 8.0, 5.0]) / 9.0


def _edge_chains(beam):
    """Node indices along the wet edges (bottom left to right, tip bottom to
    top, top right to left), each a run of nodes 2 m + 1 long."""
    nxn, nyn = beam.nxn, beam.nyn
    bottom = [0 + nyn * i for i in range(nxn)]
    tip = [j + nyn * (nxn - 1) for j in range(nyn)]
    top = [(nyn - 1) + nyn * i for i in range(nxn - 1, -1, -1)]
    return [bottom, tip, top]


def outline(beam, arc=None, arc_vel=None):
    """Polygon vertices (V, 3), velocities (V, 3) and segments (S, 3) of the
    body: the beam's wet boundary in its current position and velocity, then
    the static chain arc (A, 2) from the clamped top corner round to the
    clamped bottom corner (exclusive of both)."""
    x = beam.X + beam.u.reshape(-1, 2)
    v = beam.v.reshape(-1, 2)
    chains = _edge_chains(beam)
    ids = chains[0] + chains[1][1:] + chains[2][1:]
    P = [x[k] for k in ids]
    Vv = [v[k] for k in ids]
    if arc is not None:
        for a in np.asarray(arc, float).reshape(-1, 2):
            P.append(a)
            Vv.append(np.zeros(2))
    n = len(P)
    V = np.zeros((n, 3))
    V[:, :2] = np.array(P)
    W = np.zeros((n, 3))
    W[:, :2] = np.array(Vv)
    T = np.array([[k, (k + 1) % n, (k + 1) % n] for k in range(n)], dtype=np.int32)
    return V, W, T


def quadrature(beam):
    """Gauss points (3 per quadratic edge element) of the wet edges in the
    current configuration: points (Q, 2), outward unit normals (Q, 2),
    weights (Q,) = Gauss weight x |dx/dxi|, and for each point its three
    nodes and their shape-function values."""
    x = beam.X + beam.u.reshape(-1, 2)
    pts, nrm, wts, nodes, shp = [], [], [], [], []
    for chain in _edge_chains(beam):
        for e in range(0, len(chain) - 1, 2):
            a, m, b = chain[e], chain[e + 1], chain[e + 2]
            for g, wg in zip(_G3, _W3):
                N = np.array([0.5 * g * (g - 1.0), 1.0 - g * g, 0.5 * g * (g + 1.0)])
                dN = np.array([g - 0.5, -2.0 * g, g + 0.5])
                p = N[0] * x[a] + N[1] * x[m] + N[2] * x[b]
                t = dN[0] * x[a] + dN[1] * x[m] + dN[2] * x[b]
                L = np.hypot(t[0], t[1])
                # The chains run counter-clockwise round the body, so the
                # outward normal is the tangent turned clockwise.
                pts.append(p)
                nrm.append(np.array([t[1], -t[0]]) / L)
                wts.append(wg * L)
                nodes.append((a, m, b))
                shp.append(N)
    return (np.array(pts), np.array(nrm), np.array(wts), np.array(nodes), np.array(shp))


def nodal_loads(beam, tractions, nodes, shp, wts):
    f = np.zeros(2 * beam.nn)
    for q in range(len(wts)):
        for k in range(3):
            f[2 * nodes[q, k]: 2 * nodes[q, k] + 2] += shp[q, k] * tractions[q] * wts[q]
    return f


class Coupled:
    """Oracle lattice domain `dom` (2D) and oracle beam `beam`, coupled."""

    def __init__(self, dom, beam, arc=None):
        self.dom, self.beam, self.arc = dom, beam, arc
        V, W, T = outline(beam, arc)
        dom.set_mesh(V, W, T)

    def step(self):
        """One coupled step; returns the force of the fluid on the beam's wet
        edges (the sum of the tractions times weights)."""
        d, b = self.dom, self.beam
        d.step(1)
        pts, nrm, wts, nodes, shp = quadrature(b)
        _, tr, st = d.wall_force(pts, nrm, wts)
        assert st == 0
        tr = np.asarray(tr).reshape(-1, 2) + nrm / 3.0   # gauge pressure
        b.step(nodal_loads(b, tr, nodes, shp, wts))
        V, W, T = outline(b, self.arc)
        d.set_mesh(V, W, T)
        return (tr * wts[:, None]).sum(0)

"""Plain FP64 finite-element oracle for the structure of Sec. II.B (test
infrastructure only, like the rest of this package).

Total-Lagrangian Saint Venant-Kirchhoff solid in plane strain on a
rectangular beam, 9-node biquadratic quadrilaterals with 3 x 3 Gauss
quadrature, consistent mass, and the two-field (u, v) formulation integrated
with the one-step-theta scheme and Newton's method:

  S = lambda tr(E) I + 2 mu E,  E = (F^T F - I) / 2,  F = I + grad u,  P = F S
  (Sec. II.B, Eqs. for P_s, F, E, S_s and the Lame relations),
  M (v1 - v0) / dt = theta (f_ext1 - f_int(u1)) + (1 - theta) (f_ext0 - f_int(u0)),
  (u1 - u0) / dt = theta v1 + (1 - theta) v0   (one-step-theta, Sec. II.B).

Eliminating v1 gives the residual in u1
  R(u1) = M ((u1 - u0) / (theta dt^2) - v0 / (theta dt))
          + theta (f_int(u1) - f_ext1) + (1 - theta) (f_int(u0) - f_ext0),
solved with the exact tangent M / (theta dt^2) + theta K_T(u1).  Everything is
written out with numpy over all Gauss points at once; the linear solves are
dense.  Nodes of the clamped edge (x = x0) are fixed.

Pinned in tests/test_oracle_fem.py: the patch test (a homogeneous
deformation leaves interior nodes in equilibrium), the tangent against finite
differences of the internal force, the small-deflection cantilever against
beam theory, energy conservation of the Crank-Nicolson scheme, and the CSM3
tip motion that the paper prints.
"""
from __future__ import annotations

import numpy as np

_G = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
_GW = np.array([5.0, 8.0, 5.0]) / 9.0


def _l(t):
    """1D quadratic Lagrange basis at nodes -1, 0, 1 and its derivative."""
    return (np.array([0.5 * t * (t - 1.0), 1.0 - t * t, 0.5 * t * (t + 1.0)]),
            np.array([t - 0.5, -2.0 * t, t + 0.5]))


class Beam:
    """Rectangular beam [x0, x0 + L] x [y0, y0 + H] meshed by nex x ney
    9-node elements; node (i, j), 0 <= i <= 2 nex, 0 <= j <= 2 ney, has index
    j + (2 ney + 1) i and DOFs 2 k (x), 2 k + 1 (y).  The edge x = x0 is
    clamped."""

    def __init__(self, x0, y0, L, H, nex, ney, rho, lam, mu, dt, theta=0.5):
        self.nex, self.ney = nex, ney
        self.nxn, self.nyn = 2 * nex + 1, 2 * ney + 1
        self.nn = self.nxn * self.nyn
        ii, jj = np.meshgrid(np.arange(self.nxn), np.arange(self.nyn), indexing="ij")
        self.X = np.stack([x0 + L * ii.ravel() / (2 * nex), y0 + H * jj.ravel() / (2 * ney)], 1)
        self.rho, self.lam, self.mu, self.dt, self.theta = rho, lam, mu, dt, theta
        self.H = H
        # Element connectivity: local node (a, b), a, b in {0, 1, 2} along
        # xi, eta, is global node (2 e_x + a, 2 e_y + b).
        conn = []
        for ex in range(nex):
            for ey in range(ney):
                conn.append([(2 * ey + b) + self.nyn * (2 * ex + a)
                             for a in range(3) for b in range(3)])
        self.conn = np.array(conn)                       # (ne, 9)
        # Shape functions and reference gradients at the 3 x 3 Gauss points.
        N, dNx, dNy, w = [], [], [], []
        hx, hy = L / nex, H / ney                        # element sizes
        for gi, gx in enumerate(_G):
            for gj, gy in enumerate(_G):
                lx, dlx = _l(gx)
                ly, dly = _l(gy)
                N.append(np.outer(lx, ly).ravel())
                dNx.append(np.outer(dlx, ly).ravel() * 2.0 / hx)
                dNy.append(np.outer(lx, dly).ravel() * 2.0 / hy)
                w.append(_GW[gi] * _GW[gj] * hx * hy / 4.0)
        self.N = np.array(N)                             # (9 gp, 9 nodes)
        self.dN = np.stack([np.array(dNx), np.array(dNy)], 1)   # (gp, 2, 9)
        self.w = np.array(w)                             # (gp,)
        ndof = 2 * self.nn
        # Consistent mass matrix.
        M = np.zeros((ndof, ndof))
        me = np.einsum("g,ga,gb->ab", self.w, self.N, self.N) * rho
        for c in self.conn:
            for a in range(9):
                for b in range(9):
                    for k in range(2):
                        M[2 * c[a] + k, 2 * c[b] + k] += me[a, b]
        self.M = M
        self.fixed = np.where(np.isclose(self.X[:, 0], x0))[0]
        fixed_dofs = np.concatenate([2 * self.fixed, 2 * self.fixed + 1])
        self.free = np.setdiff1d(np.arange(ndof), fixed_dofs)
        self.u = np.zeros(ndof)
        self.v = np.zeros(ndof)
        self.fext = np.zeros(ndof)

    # ---- constitutive law and element integrals ----------------------------
    def _kinematics(self, u):
        """F, S, P at every Gauss point of every element: (ne, gp, 2, 2)."""
        ue = u.reshape(-1, 2)[self.conn]                 # (ne, 9, 2)
        G = np.einsum("gJa,eai->egiJ", self.dN, ue)      # grad u: (ne, gp, i, J)
        F = G + np.eye(2)
        E = 0.5 * (np.einsum("egkI,egkJ->egIJ", F, F) - np.eye(2))
        trE = E[..., 0, 0] + E[..., 1, 1]
        S = self.lam * trE[..., None, None] * np.eye(2) + 2.0 * self.mu * E
        P = np.einsum("egiK,egKJ->egiJ", F, S)
        return F, S, P

    def internal_force(self, u):
        """f_int,a = sum over Gauss points of P grad N_a w."""
        _, _, P = self._kinematics(u)
        fe = np.einsum("egiJ,gJa,g->eai", P, self.dN, self.w)   # (ne, 9, 2)
        f = np.zeros(2 * self.nn)
        np.add.at(f, 2 * self.conn + 0, fe[..., 0])
        np.add.at(f, 2 * self.conn + 1, fe[..., 1])
        return f

    def tangent(self, u):
        """d f_int / d u: dP_iJ for a unit displacement k at node b is
        delta_ik dN_b/dX_L S_LJ + F_iL dS_LJ, dS = lambda tr(dE) I + 2 mu dE,
        dE_IJ = (F_kI dN_b/dX_J + F_kJ dN_b/dX_I) / 2."""
        F, S, _ = self._kinematics(u)
        dN = self.dN                                     # (g, J, b)
        I2 = np.eye(2)
        # dE[e, g, k, b, I, J]
        dE = 0.5 * (np.einsum("egkI,gJb->egkbIJ", F, dN) + np.einsum("egkJ,gIb->egkbIJ", F, dN))
        trdE = dE[..., 0, 0] + dE[..., 1, 1]
        dS = self.lam * trdE[..., None, None] * I2 + 2.0 * self.mu * dE
        geo = np.einsum("ik,gLb,egLJ->egkbiJ", I2, dN, S)
        mat = np.einsum("egiL,egkbLJ->egkbiJ", F, dS)
        dP = geo + mat                                   # (e, g, k, b, i, J)
        Ke = np.einsum("egkbiJ,gJa,g->eaibk", dP, dN, self.w)   # (e, a, i, b, k)
        K = np.zeros((2 * self.nn, 2 * self.nn))
        idx = (2 * self.conn[:, :, None] + np.arange(2)[None, None, :]).reshape(-1, 18)
        np.add.at(K, (idx[:, :, None], idx[:, None, :]), Ke.reshape(-1, 18, 18))
        return K

    def body_force(self, b):
        """Nodal loads of a uniform body force b per unit mass (rho b)."""
        f = np.zeros(2 * self.nn)
        nw = np.einsum("g,ga->a", self.w, self.N) * self.rho
        for c in self.conn:
            f[2 * c] += nw * b[0]
            f[2 * c + 1] += nw * b[1]
        return f

    # ---- time step ----------------------------------------------------------
    def step(self, fext1, tol=1e-10, maxit=30):
        """One theta step with external nodal loads fext1 at the new time;
        returns the Newton iteration count."""
        th, dt = self.theta, self.dt
        u0, v0, f0 = self.u.copy(), self.v.copy(), self.fext
        rhs0 = (1.0 - th) * (self.internal_force(u0) - f0)
        u = u0 + dt * v0
        free = self.free
        for it in range(1, maxit + 1):
            R = (self.M @ ((u - u0) / (th * dt * dt) - v0 / (th * dt)) +
                 th * (self.internal_force(u) - fext1) + rhs0)
            K = self.M / (th * dt * dt) + th * self.tangent(u)
            du = np.linalg.solve(K[np.ix_(free, free)], -R[free])
            u[free] += du
            # Relative to the displacement, with a floor of 1e-14 of the
            # thickness for a beam that has not moved.
            if np.abs(du).max() <= max(tol * np.abs(u[free]).max(), 1e-14 * self.H):
                break
        self.u = u
        self.v = (u - u0) / (th * dt) - (1.0 - th) / th * v0
        self.v[~np.isin(np.arange(u.size), free)] = 0.0
        self.fext = fext1.copy()
        return it

    def static(self, fext, tol=1e-12, maxit=50):
        """Static equilibrium f_int(u) = fext by Newton from the current u."""
        u = self.u.copy()
        free = self.free
        for it in range(1, maxit + 1):
            R = self.internal_force(u) - fext
            du = np.linalg.solve(self.tangent(u)[np.ix_(free, free)], -R[free])
            u[free] += du
            if np.abs(du).max() <= tol * max(np.abs(u[free]).max(), 1e-30):
                break
        self.u = u
        return it

    def tip(self, which="mid"):
        """Displacement of the node at the free end's mid-height."""
        k = self.ney + self.nyn * (self.nxn - 1)
        return self.u[2 * k: 2 * k + 2].copy()

    def energy(self):
        """Kinetic plus strain energy (per unit thickness)."""
        _, S, _ = self._kinematics(self.u)
        ue = self.u.reshape(-1, 2)[self.conn]
        G = np.einsum("gJa,eai->egiJ", self.dN, ue)
        F = G + np.eye(2)
        E = 0.5 * (np.einsum("egkI,egkJ->egIJ", F, F) - np.eye(2))
        psi = 0.5 * np.einsum("egIJ,egIJ->eg", S, E)
        return 0.5 * self.v @ self.M @ self.v + np.einsum("eg,g->", psi, self.w)

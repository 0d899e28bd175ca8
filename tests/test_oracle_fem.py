"""Pins of the finite-element oracle of the structure (Sec. II.B).

Checked against what mathematics and the paper fix: a homogeneous
deformation is an exact equilibrium of interior nodes (patch test), the
tangent is the derivative of the internal force, a small-deflection
cantilever follows beam theory, the Crank-Nicolson scheme keeps the energy
of a small free vibration, and the CSM3 benchmark reproduces the tip motion
the paper prints (Sec. III.A.1: u_x = -0.01460 +- 0.01460,
u_y = -0.06463 +- 0.06492, f = 1.10)."""
import numpy as np
import pytest

from oracle.fem import Beam

RHO, NU_S = 1000.0, 0.4


def lame(mu, nu=NU_S):
    return 2.0 * mu * nu / (1.0 - 2.0 * nu), mu


def test_patch_test_homogeneous_deformation():
    """u = A X with a finite A: F, S and P are constant, so the internal
    force vanishes at every interior node (to rounding)."""
    lam, mu = lame(0.5e6)
    b = Beam(0.0, 0.0, 0.35, 0.02, 6, 2, RHO, lam, mu, 1e-3)
    A = np.array([[0.08, -0.05], [0.12, -0.03]])
    b.u = (b.X @ A.T).ravel()
    f = b.internal_force(b.u).reshape(-1, 2)
    X = b.X
    inner = (X[:, 0] > 1e-12) & (X[:, 0] < 0.35 - 1e-12) & (X[:, 1] > 1e-12) & (X[:, 1] < 0.02 - 1e-12)
    scale = np.abs(f).max()
    assert scale > 1.0
    assert np.abs(f[inner]).max() < 1e-10 * scale


def test_tangent_is_derivative_of_internal_force():
    lam, mu = lame(2e6)
    b = Beam(0.0, 0.0, 0.35, 0.02, 4, 2, RHO, lam, mu, 1e-3)
    rng = np.random.default_rng(5)
    u = 0.01 * rng.standard_normal(2 * b.nn)
    K = b.tangent(u)
    h = 1e-7
    for k in rng.choice(2 * b.nn, 12, replace=False):
        e = np.zeros_like(u)
        e[k] = h
        fd = (b.internal_force(u + e) - b.internal_force(u - e)) / (2 * h)
        assert np.abs(fd - K[:, k]).max() < 1e-6 * np.abs(K).max()


@pytest.mark.parametrize("nu,tol", [(0.0, 1e-3), (0.4, 0.02)])
def test_small_deflection_cantilever_follows_beam_theory(nu, tol):
    """Tip load P at the free end: w = P L^3 / (3 E' I) with the plane-strain
    modulus E' = E / (1 - nu^2), plus Timoshenko's shear term P L /
    (kappa G A), kappa = 5/6.  Within 0.1 % for nu = 0; within 2 % for
    nu = 0.4, where the clamped edge also stops the Poisson contraction."""
    lam, mu = lame(0.5e6, nu)
    E = mu * (3 * lam + 2 * mu) / (lam + mu)
    L, H = 0.35, 0.02
    b = Beam(0.0, 0.0, L, H, 20, 2, RHO, lam, mu, 1e-3)
    P = 1e-3
    f = np.zeros(2 * b.nn)
    tip = np.where(np.isclose(b.X[:, 0], L))[0]
    assert np.all(np.diff(b.X[tip, 1]) > 0)
    # Consistent loads of a uniform shear traction P / H on the two quadratic
    # edge elements of the end (Simpson weights).
    f[2 * tip + 1] = -P * np.array([1, 4, 2, 4, 1]) / 12.0
    b.static(f)
    w = -b.tip()[1]
    Ep = E / (1 - nu ** 2)
    w_beam = P * L ** 3 / (3 * Ep * H ** 3 / 12) + P * L / (5 / 6 * mu * H)
    assert abs(w / w_beam - 1) < tol, (w, w_beam)


def test_crank_nicolson_keeps_energy_of_small_vibration():
    lam, mu = lame(0.5e6)
    b = Beam(0.0, 0.0, 0.35, 0.02, 6, 2, RHO, lam, mu, 2e-3)
    b.v = np.zeros(2 * b.nn)
    b.v[1::2] = 1e-3 * (b.X[:, 0] / 0.35) ** 2
    b.v[2 * b.fixed + 1] = 0.0
    e0 = b.energy()
    zero = np.zeros(2 * b.nn)
    for _ in range(300):
        b.step(zero)
    assert abs(b.energy() / e0 - 1) < 1e-6


def test_csm3_tip_motion_matches_printed():
    """CSM3: gravity acting on the clamped beam, mu_s = 0.5e6, nu_s = 0.4,
    rho_s = 1e3, from rest; the first period gives the mean and amplitude of
    the tip displacement and the frequency (1 / twice the time of the lowest
    point).  20 x 2 nine-node elements, dt = 0.002: amplitudes within 4 % and
    the frequency within 3 % of the printed values."""
    lam, mu = lame(0.5e6)
    b = Beam(0.0, 0.0, 0.35, 0.02, 20, 2, RHO, lam, mu, 2e-3)
    g = b.body_force((0.0, -2.0))
    tips = []
    for _ in range(500):
        b.step(g)
        tips.append(b.tip())
    t = 2e-3 * (1 + np.arange(len(tips)))
    tips = np.vstack([[0.0, 0.0], np.array(tips)])
    ux, uy = tips[:, 0], tips[:, 1]
    mx, ax = (ux.max() + ux.min()) / 2, (ux.max() - ux.min()) / 2
    my, ay = (uy.max() + uy.min()) / 2, (uy.max() - uy.min()) / 2
    f = 1.0 / (2 * t[np.argmin(uy[1:])])
    assert abs(mx / -0.01460 - 1) < 0.04 and abs(ax / 0.01460 - 1) < 0.04, (mx, ax)
    assert abs(my / -0.06463 - 1) < 0.04 and abs(ay / 0.06492 - 1) < 0.04, (my, ay)
    assert abs(f / 1.10 - 1) < 0.03, f

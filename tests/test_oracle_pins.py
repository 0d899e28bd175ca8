"""Pins of the CPU oracle's per-node arithmetic against what the paper and the
mathematics fix (closed forms, invariants, numerical minimisers).

None of these tests retypes the oracle's formula: each checks it against an
independent characterisation (a numerical minimisation, a moment identity, a
textbook special case, or a closed form derived differently).
"""
import itertools

import numpy as np
import pytest
from scipy import optimize

import workloads as W


def lattice_def(Q):
    """Lattice from its definition: c in {-1,0,1}^D, index (cx+1)+3(cy+1)+9(cz+1)."""
    D = 2 if Q == 9 else 3
    c = np.zeros((Q, 3))
    w = np.zeros(Q)
    w1 = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
    for i in range(Q):
        v = [i % 3 - 1, (i // 3) % 3 - 1, (i // 9 - 1) if D == 3 else 0]
        c[i] = v
        w[i] = np.prod([w1[v[a]] for a in range(D)])
    return c, w, D


@pytest.mark.parametrize("Q", [9, 27])
def test_lattice_matches_definition_and_isotropy(orc, Q):
    c, w = orc.lattice(Q)
    c0, w0, D = lattice_def(Q)
    assert np.array_equal(c, c0)
    assert np.allclose(w, w0, rtol=0, atol=1e-16)
    # Isotropy up to fourth order with cs^2 = 1/3 (Sec. II.A, Eq. 7).
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(w @ c, 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c)[:D, :D], np.eye(D) / 3, atol=1e-16)
    T4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)[:D, :D, :D, :D]
    d = np.eye(D)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(T4, iso, atol=1e-16)
    # opposite index
    assert np.array_equal(c[::-1], -c)


def rand_rho_u(rng, D):
    rho = rng.uniform(0.8, 1.2)
    u = np.zeros(3)
    u[:D] = rng.uniform(-0.15, 0.15, size=D)
    return rho, u


@pytest.mark.parametrize("Q", [9, 27])
def test_equilibrium_moments_exact(orc, Q):
    c, w, D = lattice_def(Q)
    rng = np.random.default_rng(1)
    for _ in range(50):
        rho, u = rand_rho_u(rng, D)
        f = orc.equilibrium(Q, rho, u)
        assert abs(f.sum() - rho) < 1e-14
        assert np.allclose(f @ c, rho * u, rtol=0, atol=1e-15)
        assert (f > 0).all()
    # At rest the equilibrium is rho W.
    assert np.allclose(orc.equilibrium(Q, 1.3, np.zeros(3)), 1.3 * w, atol=1e-16)


@pytest.mark.parametrize("Q", [9, 27])
def test_equilibrium_lagrange_condition(orc, Q):
    """Stationarity of H under mass/momentum constraints: ln(f/W) affine in c."""
    c, w, D = lattice_def(Q)
    rng = np.random.default_rng(2)
    A = np.hstack([np.ones((Q, 1)), c[:, :D]])
    for _ in range(20):
        rho, u = rand_rho_u(rng, D)
        y = np.log(orc.equilibrium(Q, rho, u) / w)
        coef, *_ = np.linalg.lstsq(A, y, rcond=None)
        assert np.max(np.abs(A @ coef - y)) < 1e-13


def h_minimiser_dual(Q, rho, u):
    """Minimiser of H(f) = sum f ln(f/W) under sum f = rho, sum f c = rho u, found
    by Newton iteration on the convex dual (multipliers of the constraints)."""
    c, w, D = lattice_def(Q)
    A = np.hstack([np.ones((Q, 1)), c[:, :D]])          # Q x (D+1)
    target = np.concatenate([[rho], rho * u[:D]])
    lam = np.zeros(D + 1)
    lam[0] = np.log(rho)
    for _ in range(100):
        f = w * np.exp(A @ lam)
        g = A.T @ f - target
        if np.max(np.abs(g)) < 1e-16:
            break
        J = A.T @ (f[:, None] * A)
        lam -= np.linalg.solve(J, g)
    return w * np.exp(A @ lam)


@pytest.mark.parametrize("Q", [9, 27])
def test_equilibrium_is_h_minimiser(orc, Q):
    c, w, D = lattice_def(Q)
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho, u = rand_rho_u(rng, D)
        assert np.allclose(orc.equilibrium(Q, rho, u), h_minimiser_dual(Q, rho, u),
                           rtol=1e-13, atol=0)
    # Direct constrained minimisation of H (SLSQP), looser tolerance.
    rho, u = 1.05, np.array([0.08, -0.05, 0.03 if D == 3 else 0.0])
    A = np.hstack([np.ones((Q, 1)), c[:, :D]])
    target = np.concatenate([[rho], rho * u[:D]])
    res = optimize.minimize(lambda f: np.sum(f * np.log(f / w)), rho * w, method="SLSQP",
                            constraints=[{"type": "eq", "fun": lambda f: A.T @ f - target}],
                            bounds=[(1e-9, None)] * Q, options={"ftol": 1e-15, "maxiter": 500})
    assert np.allclose(res.x, orc.equilibrium(Q, rho, u), rtol=0, atol=2e-6)


def monomial_moments(Q, v):
    """All 27 (or 9) monomial moments sum_i cx^p cy^q cz^r v_i by direct sums."""
    c, w, D = lattice_def(Q)
    out = {}
    for p, q, r in itertools.product(range(3), repeat=3):
        if D == 2 and r > 0:
            continue
        out[(p, q, r)] = np.sum(c[:, 0] ** p * c[:, 1] ** q * c[:, 2] ** r * v)
    return out


def closed_form_ds(Q, delta, trace_in_s):
    """Shear part from the second moments: Dev/2 on faces, Pi_ab c_a c_b / 4 on
    the 2-component edges, zero elsewhere; the trace column adds -T at rest and
    T/(2D) on the faces."""
    c, w, D = lattice_def(Q)
    P = np.einsum("ia,ib,i->ab", c, c, delta)[:D, :D]
    T = np.trace(P)
    Dev = P - T / D * np.eye(D)
    ds = np.zeros(Q)
    for i in range(Q):
        nz = [a for a in range(D) if c[i, a] != 0]
        if len(nz) == 1:
            ds[i] = Dev[nz[0], nz[0]] / 2
            if trace_in_s:
                ds[i] += T / (2 * D)
        elif len(nz) == 2:
            a, b = nz
            ds[i] = c[i, a] * c[i, b] * P[a, b] / 4
        elif len(nz) == 0 and trace_in_s:
            ds[i] = -T
    return ds


@pytest.mark.parametrize("Q", [9, 27])
@pytest.mark.parametrize("trace_in_s", [0, 1])
def test_split_moment_identities(orc, Q, trace_in_s):
    c, w, D = lattice_def(Q)
    states = W.random_node_states(Q, 30, seed=4)
    for f in states:
        feq, ds, dh = orc.split(Q, f, trace_in_s)
        delta = f - feq
        assert np.allclose(ds + dh, delta, atol=1e-16)
        md = monomial_moments(Q, delta)
        ms = monomial_moments(Q, ds)
        mh = monomial_moments(Q, dh)
        tr = md[(2, 0, 0)] + md[(0, 2, 0)] + (md[(0, 0, 2)] if D == 3 else 0.0)
        for k, v in ms.items():
            order = sum(k)
            diag = 2 in k
            if order == 2 and diag:
                assert abs(v - (md[k] if trace_in_s else md[k] - tr / D)) < 1e-15, k
                assert abs(mh[k] - (0.0 if trace_in_s else tr / D)) < 1e-15, k
            elif order == 2:
                assert abs(v - md[k]) < 1e-15 and abs(mh[k]) < 1e-15, k
            else:
                # shear part has no conserved, third- or fourth-order content
                assert abs(v) < 1e-15, k
                assert abs(mh[k] - md[k]) < 1e-15, k
        assert np.allclose(ds, closed_form_ds(Q, delta, trace_in_s), atol=1e-15)


def post_collision(f, feq, ds, dh, beta, gamma):
    return f - beta * (2 * ds + gamma * dh)


@pytest.mark.parametrize("Q", [9, 27])
def test_gamma_minimises_quadratic_entropy(orc, Q):
    """Eq. 6 is the exact minimiser of sum (f' - f^eq)^2 / f^eq over gamma."""
    rng = np.random.default_rng(5)
    states = W.random_node_states(Q, 20, seed=5, amp=0.2)
    for f in states:
        beta = rng.uniform(0.55, 0.99)
        feq, ds, dh = orc.split(Q, f)
        _, gamma, st = orc.collide(Q, beta, f)
        assert st == 0

        def qnorm(g):
            return np.sum((post_collision(f, feq, ds, dh, beta, g) - feq) ** 2 / feq)

        res = optimize.minimize_scalar(qnorm, bracket=(-10.0, 10.0), method="brent",
                                       options={"xtol": 1e-12})
        assert abs(res.x - gamma) < 1e-7 * max(1.0, abs(gamma))


@pytest.mark.parametrize("Q", [9, 27])
def test_gamma_near_full_entropy_minimiser(orc, Q):
    """Close to equilibrium the quadratic estimate approaches the minimiser of
    the full H over gamma (Sec. II.A: gamma from entropy minimisation)."""
    c, w, D = lattice_def(Q)
    rng = np.random.default_rng(6)
    for _ in range(10):
        rho, u = rand_rho_u(rng, D)
        feq0 = orc.equilibrium(Q, rho, u)
        f = feq0 * (1 + 0.01 * rng.uniform(-1, 1, size=Q))
        beta = 0.9
        feq, ds, dh = orc.split(Q, f)
        _, gamma, _ = orc.collide(Q, beta, f)

        def H(g):
            fp = post_collision(f, feq, ds, dh, beta, g)
            return np.sum(fp * np.log(fp / w))

        res = optimize.minimize_scalar(H, bracket=(gamma - 0.5, gamma + 0.5), method="brent",
                                       options={"xtol": 1e-12})
        assert abs(res.x - gamma) < 2e-2


@pytest.mark.parametrize("Q", [9, 27])
@pytest.mark.parametrize("collision", [0, 1])
def test_collision_conserves_mass_momentum(orc, Q, collision):
    c, w, D = lattice_def(Q)
    rng = np.random.default_rng(7)
    for f in W.random_node_states(Q, 30, seed=7):
        fo, g, st = orc.collide(Q, rng.uniform(0.5, 1.0), f, collision)
        assert st == 0
        assert abs(fo.sum() - f.sum()) < 2e-16 * Q
        assert np.allclose(fo @ c, f @ c, rtol=0, atol=2e-16 * Q)


@pytest.mark.parametrize("Q", [9, 27])
def test_lbgk_limit_and_half_beta(orc, Q):
    """gamma = 2 is LBGK with omega = 2 beta; beta = 1/2 gives f' = f^eq."""
    for f in W.random_node_states(Q, 10, seed=8):
        rho = f.sum()
        c, w, D = lattice_def(Q)
        u = (f @ c) / rho
        feq = h_minimiser_dual(Q, rho, u)
        beta = 0.83
        fo, g, _ = orc.collide(Q, beta, f, collision=1)
        assert g == 2.0
        assert np.allclose(fo, f + 2 * beta * (feq - f), rtol=0, atol=1e-15)
        fo, g, _ = orc.collide(Q, 0.5, f, collision=0)
        assert abs(g - 2.0) < 1e-12
        assert np.allclose(fo, feq, rtol=0, atol=1e-15)


@pytest.mark.parametrize("Q", [9, 27])
def test_equilibrium_state_unchanged_by_collision(orc, Q):
    feq = orc.equilibrium(Q, 1.1, np.array([0.05, -0.02, 0.04]))
    fo, g, _ = orc.collide(Q, 0.97, feq)
    assert np.allclose(fo, feq, rtol=0, atol=1e-16)
    assert np.isfinite(g)   # Delta is round-off only; gamma multiplies nothing


@pytest.mark.parametrize("Q", [9, 27])
def test_invalid_state_flagged(orc, Q):
    f = W.random_node_states(Q, 1, seed=9)[0]
    bad = f.copy()
    bad[:] = -bad
    assert orc.collide(Q, 0.9, bad)[2] == 1
    nan = f.copy()
    nan[3] = np.nan
    assert orc.collide(Q, 0.9, nan)[2] == 1


@pytest.mark.parametrize("Q", [9, 27])
def test_grad_fstar_reproduces_moments(orc, Q):
    """Grad's f* (Sec. II.C.1) carries exactly rho, rho v and Pi."""
    c, w, D = lattice_def(Q)
    rng = np.random.default_rng(10)
    for _ in range(20):
        rho, v = rand_rho_u(rng, D)
        A = rng.normal(size=(D, D)) * 0.01
        Pi = rho / 3 * np.eye(D) + rho * np.outer(v[:D], v[:D]) + (A + A.T)
        fs = orc.grad_fstar(Q, rho, v, Pi)
        assert abs(fs.sum() - rho) < 1e-15
        assert np.allclose(fs @ c, rho * v, atol=1e-15)
        assert np.allclose(np.einsum("i,ia,ib->ab", fs, c, c)[:D, :D], Pi, atol=1e-15)
        # With Pi = Pi^eq it is the second-order polynomial equilibrium.
        fe = orc.grad_fstar(Q, rho, v, rho / 3 * np.eye(D) + rho * np.outer(v[:D], v[:D]))
        cu = c @ v
        poly = w * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * v @ v)
        assert np.allclose(fe, poly, atol=1e-15)


@pytest.mark.parametrize("Q", [9, 27])
def test_stress_at_equilibrium_is_pressure(orc, Q):
    c, w, D = lattice_def(Q)
    feq = orc.equilibrium(Q, 1.2, np.array([0.05, 0.02, -0.03]))
    s = orc.stress(Q, 0.9, feq)
    expect = np.zeros((3, 3))
    expect[:D, :D] = -1.2 / 3 * np.eye(D)
    assert np.allclose(s, expect, atol=1e-15)


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
def test_storage_rounding_matches_numpy_and_bits(orc):
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-9, 4, size=5000),
                        [0.0, 65504.0, 65519.0, 65520.0, 1e-8, -6e-8, 2.0 ** -24 * 1.5]])
    assert np.array_equal(orc.round_storage("f16", x), x.astype(np.float16).astype(np.float64))
    assert np.array_equal(orc.round_storage("f32", x), x.astype(np.float32).astype(np.float64))
    # bfloat16: on binary32-exact inputs compare with the bit-level RNE of the
    # upper 16 bits.
    x32 = x.astype(np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    bf = r.astype(np.uint32).view(np.float32).astype(np.float64)
    assert np.array_equal(orc.round_storage("bf16", x32.astype(np.float64)), bf)

"""Domain-level pins of the CPU oracle: closed-form flows, invariants and brute
force on tiny grids (Sec. II.A viscosity relation, Sec. II.C.1 Grad walls,
Sec. II.C.2 wall stress)."""
import math

import numpy as np
import pytest

import workloads as W


def test_streaming_is_the_lattice_shift(orc):
    """Pull streaming f_i(x) = A_i(x - c_i) on a periodic 5x4x3 grid equals a
    cyclic shift of each population array by c_i (brute force)."""
    Q, nx, ny, nz = 27, 5, 4, 3
    d = orc.Domain(Q, nx, ny, nz, 0.1)
    c, _ = orc.lattice(Q)
    A = np.random.default_rng(0).uniform(size=(Q, nz, ny, nx))
    d.set_populations(A.reshape(Q, -1))
    d.stream_only()
    got = d.get_populations().reshape(Q, nz, ny, nx)
    for i in range(Q):
        exp = np.roll(A[i], shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2))
        assert np.array_equal(got[i], exp)


@pytest.mark.parametrize("Q", [9, 27])
def test_uniform_equilibrium_is_fixed_point(orc, Q):
    n = 6
    D = 2 if Q == 9 else 3
    N = n ** D
    d = orc.Domain(Q, n, n, n if D == 3 else 1, 0.02)
    u0 = np.array([0.05, -0.03, 0.02])[:D]
    d.init_fields(np.full(N, 1.02), np.repeat(u0[:, None], N, axis=1))
    f0 = d.get_populations()
    d.step(10)
    assert np.allclose(d.get_populations(), f0, rtol=0, atol=1e-15)


def test_tg2d_decay_and_second_order(orc):
    """2D Taylor-Green: velocity decays as exp(-2 nu k^2 t) with the viscosity of
    Eq. 7; error against the analytic field <= 2.5e-3 at 64^2 / 500 steps and
    second-order convergence over 32, 64, 128 at fixed nu t k^2."""
    errs = []
    for n in (32, 64, 128):
        steps = 500 * n * n // (64 * 64)
        rho, u = W.taylor_green_2d(n, 0.02)
        d = orc.Domain(9, n, n, 1, 0.01)
        d.init_fields(rho, u)
        d.step(steps)
        r, uu, tot = d.moments()
        ref = u * W.taylor_green_2d_decay(0.01, n, steps)
        errs.append(np.linalg.norm(uu - ref) / np.linalg.norm(ref))
        # mass and momentum conserved to round-off
        assert abs(tot["mass"] - rho.sum()) < 1e-12 * rho.sum()
        assert np.all(np.abs(tot["momentum"]) < 1e-11)
    assert errs[1] <= 2.5e-3
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(orders) >= 1.9, (errs, orders)


def test_tg2d_kbc_close_to_lbgk_when_resolved(orc):
    """On a resolved smooth flow KBC stays close to LBGK (gamma near 2)."""
    n = 32
    rho, u = W.taylor_green_2d(n, 0.02)
    out = []
    for coll in (0, 1):
        d = orc.Domain(9, n, n, 1, 0.01, collision=coll)
        d.init_fields(rho, u)
        d.step(200)
        out.append(d.moments()[1])
    assert np.linalg.norm(out[0] - out[1]) / np.linalg.norm(out[1]) < 1e-3


@pytest.mark.parametrize("qlo,qhi", [(0.25, 0.75), (0.5, 0.5), (0.75, 0.25)])
def test_couette_through_grad_walls(orc, qlo, qhi):
    """Moving-plate Couette flow with walls cutting links at fraction q: Grad's
    boundary (Sec. II.C.1) reproduces the linear profile, and the stress-based
    wall force (Sec. II.C.2) gives the shear rho nu U / h on each plate."""
    ny, nx, U, nu = 14, 4, 0.02, 0.1
    ylo, yhi = 1 - qlo, (ny - 2) + qhi
    d = orc.Domain(9, nx, ny, 1, nu)
    N = nx * ny
    d.init_fields(np.ones(N), np.zeros((2, N)))
    d.set_body(W.BODY_PLATES, W.plates_params(ylo, yhi, (0, 0, 0), (U, 0, 0)))
    d.step(5000)
    rho, u, tot = d.moments()
    ux = u[0].reshape(ny, nx)[:, 0]
    y = np.arange(ny)
    exact = U * (y - ylo) / (yhi - ylo)
    assert np.max(np.abs(ux[1:-1] - exact[1:-1])) < 1e-5 * U
    assert np.max(np.abs(u[1])) < 1e-5 * U       # no flux through the plates
    tau = nu * U / (yhi - ylo)
    F, tr, st = d.wall_force(*W.plate_quadrature(ylo, +1.0, nx))
    assert st == 0
    assert abs(F[0] / nx - tau) < 1e-3 * tau
    assert abs(F[1] / nx + 1 / 3) < 1e-4          # pressure pushes on the plate
    F2, _, _ = d.wall_force(*W.plate_quadrature(yhi, -1.0, nx))
    assert abs(F2[0] / nx + tau) < 1e-3 * tau


def test_poiseuille_channel_inlet_outlet_walls(orc):
    """Channel with parabolic velocity inflow, equilibrium pressure outflow and
    no-slip walls half a spacing outside the first/last rows (Sec. III.A.1
    inflow profile): the developed profile converges to the parabola at
    better than first order (Grad boundary, Sec. II.C.1), and the mass flux is
    the same through every cross-section."""
    ubar, nu = 0.02, 0.05
    errs = []
    for H in (8, 16):
        nx, ny = 4 * H, H
        d = orc.Domain(9, nx, ny, 1, nu, faces=["inlet", "outlet", "wall", "wall", "periodic",
                                                "periodic"], u_in=(ubar, 0, 0), inlet_profile=1)
        N = nx * ny
        d.init_fields(np.ones(N), np.zeros((2, N)))
        d.step(int(6 * H * H / nu))
        rho, u, tot = d.moments()
        ux = u[0].reshape(ny, nx)
        yp = np.arange(ny) + 0.5
        para = 1.5 * ubar * yp * (ny - yp) / (0.25 * ny * ny)
        x = nx // 2
        errs.append(np.max(np.abs(ux[:, x] / ux[:, x].mean() - para / para.mean())))
        assert abs(ux[:, x].mean() / ubar - 1) < 5e-3
        flux = (rho.reshape(ny, nx) * ux).sum(axis=0)[2:-2]
        assert (flux.max() - flux.min()) / flux.mean() < 5e-3
        assert np.max(np.abs(u[1].reshape(ny, nx)[:, H:-H])) < 1e-3 * ubar
        if H == 16:
            # Wall traction (Sec. II.C.2): the shear stress of the developed
            # flow is linear across the channel, so the linear extrapolation
            # of sigma from x_q + n_q and x_q + 2 n_q to the wall is exact.
            # The tangential traction must equal the wall shear rho nu du/dy,
            # 6 nu (mass flux) / H^2 for the parabola, on both walls, and the
            # normal traction -p = -rho/3.  Sampling at x_q + n_q or
            # x_q + 2 n_q alone, extrapolating the wrong way, or dropping the
            # (1 - beta) factor of the viscous stress misses by 12% or more.
            xs = np.arange(H, 3 * H).astype(float)
            xq = np.concatenate([np.stack([xs, np.full_like(xs, -0.5)], 1),
                                 np.stack([xs, np.full_like(xs, ny - 0.5)], 1)])
            nq = np.concatenate([np.tile([0.0, 1.0], (xs.size, 1)),
                                 np.tile([0.0, -1.0], (xs.size, 1))])
            F, tr, st = d.wall_force(xq, nq, np.ones(xq.shape[0]))
            assert st == 0
            ix = np.concatenate([xs, xs]).astype(int)
            r2 = rho.reshape(ny, nx)
            fx = (r2 * ux).sum(axis=0)
            tau = 6.0 * nu * fx[ix] / (H * H)
            assert np.max(np.abs(tr[:, 0] / tau - 1.0)) < 1e-2
            rw = np.concatenate([r2[0, ix[: xs.size]], r2[-1, ix[: xs.size]]])
            assert np.max(np.abs(tr[:, 1] * nq[:, 1] / (-rw / 3.0) - 1.0)) < 1e-4
            # Probes two and one spacings outside the bottom wall have no
            # fluid stencil corner: both take the nearest fluid node, the
            # first row (wall distance 1/2), whose shear stress in the
            # developed flow is 6 nu (mass flux) (H - 1) / H^3.  A search box
            # smaller than 5^D finds no node for the far probe.
            xf = np.arange(H, 3 * H).astype(float) + 0.25
            xq2 = np.stack([xf, np.full_like(xf, -3.0)], 1)
            nq2 = np.tile([0.0, 1.0], (xf.size, 1))
            F2, tr2, st2 = d.wall_force(xq2, nq2, np.ones(xf.size))
            assert st2 == 0
            ixf = np.floor(xf).astype(int)
            tau0 = 6.0 * nu * fx[ixf] * (H - 1) / H ** 3
            assert np.max(np.abs(tr2[:, 0] / tau0 - 1.0)) < 1e-2
            assert np.max(np.abs(tr2[:, 1] / (-r2[0, ixf] / 3.0) - 1.0)) < 1e-4
    assert errs[1] < 4e-3
    assert math.log2(errs[0] / errs[1]) > 1.5, errs


def test_body_carried_by_uniform_flow_leaves_it_uniform(orc):
    """A circle moving at the velocity U of the uniform flow around it
    (Galilean co-motion) at density rho0 = 1.02: every target velocity is U,
    the velocity gradient vanishes, and the fluid stays uniform up to the
    O(U^2) difference between the entropic equilibrium and Grad's
    second-order reconstruction.  The body moves four spacings, so nodes it
    uncovers are refilled every few steps; the nodes inside the body start at
    density 1.3, which no correct step reads.  A refill at rest instead of at
    the body velocity, at the reference density 1 instead of the neighbours'
    density, a refill that counts solid neighbours or sums instead of
    averaging, a wrong sign or a dropped wall-motion term in the target
    density (Sec. II.C.1), or interpolation weights that do not sum to one
    leave an O(U) or O(rho0 - 1) defect."""
    n, U, nu, rho0 = 48, 0.02, 0.02, 1.02
    amp = 1.0e4   # sin(omega t) ~ omega t: the body velocity is U to 1e-7
    d = orc.Domain(9, n, n, 1, nu)
    N = n * n
    u = np.zeros((2, N))
    u[0] = U
    d.init_fields(np.full(N, rho0), u)
    d.set_body(W.BODY_SPHERE, W.sphere_params((20.3, 24.1), 6.2, (amp, 0.0),
                                              2.0 * math.pi * amp / U))
    inside = d.solid().astype(bool)
    assert inside.sum() > 100
    rho = np.where(inside, 1.3, rho0)
    d.init_fields(rho, u)
    d.step(200)
    rho, uu, tot = d.moments()
    fl = d.solid() == 0
    assert np.max(np.abs(uu[0][fl] - U)) < 5e-5 * U
    assert np.max(np.abs(uu[1][fl])) < 5e-5 * U
    assert np.max(np.abs(rho[fl] - rho0)) < 2e-6


def test_resting_sphere_is_fixed_point_and_force_free(orc):
    """Body and fluid at rest: Grad's fill returns the rest populations, so the
    state does not change, and the force reduces to -p sum w n = 0."""
    n = 16
    d = orc.Domain(27, n, n, n, 0.05)
    N = n ** 3
    d.init_fields(np.ones(N), np.zeros((3, N)))
    center = (7.3, 8.1, 7.7)
    d.set_body(W.BODY_SPHERE, W.sphere_params(center, 4.2))
    solid = d.solid().astype(bool)
    f0 = d.get_populations()
    d.step(5)
    f1 = d.get_populations()
    assert np.allclose(f1[:, ~solid], f0[:, ~solid], rtol=0, atol=1e-15)
    xq, nq, wq = W.sphere_quadrature(center, 4.2, subdiv=3)
    F, tr, st = d.wall_force(xq, nq, wq)
    assert st == 0
    assert np.max(np.abs(F)) < 1e-12
    assert np.allclose(tr, -nq / 3, atol=1e-14)


def test_moving_sphere_drag_opposes_motion(orc):
    """A sphere pushed through fluid at rest feels a force against its motion,
    and the fluid near it is set in motion along it."""
    n = 24
    d = orc.Domain(27, n, n, n, 0.05)
    N = n ** 3
    d.init_fields(np.ones(N), np.zeros((3, N)))
    center = (11.6, 12.2, 11.9)
    amp, period = 3.0, 600.0
    d.set_body(W.BODY_SPHERE, W.sphere_params(center, 4.0, (amp, 0, 0), period))
    d.step(30)
    t = d.time
    cx = center[0] + amp * math.sin(2 * math.pi * t / period)
    xq, nq, wq = W.sphere_quadrature((cx, center[1], center[2]), 4.0, subdiv=3)
    F, tr, st = d.wall_force(xq, nq, wq)
    assert F[0] < 0
    assert abs(F[1]) < 0.2 * abs(F[0]) and abs(F[2]) < 0.2 * abs(F[0])
    rho, u, tot = d.moments()
    assert tot["momentum"][0] > 0
    assert not tot["invalid"]


def test_flap_channel_runs_and_stays_valid(orc):
    """One small flap channel (the batched workload's building block) stays a
    valid state (rho > 0, |u| < 1) over a few hundred steps."""
    ch = W.flap_channels(count=1, seed=2375)[0]
    d = orc.Domain(9, 128, 64, 1, ch["nu"], faces=ch["faces"], u_in=ch["u_in"],
                   inlet_profile=1)
    N = 128 * 64
    d.init_fields(np.ones(N), np.zeros((2, N)))
    kind, p = ch["body"]
    p = p.copy()
    p[0] = 32.0
    p[1] = min(p[1], 20.0)
    d.set_body(kind, p)
    assert d.solid().sum() > 0
    d.step(300)
    rho, u, tot = d.moments()
    assert not tot["invalid"]
    fl = d.solid() == 0
    assert rho[fl].min() > 0.9 and np.abs(u[:, fl]).max() < 0.2


# ---------------------------------------------------------------------------
# Grad target values on prepared lagged fields (Sec. II.C.1).  The lagged
# moments are those of the stored state, so initialising every node to the
# equilibrium of a chosen (rho, u) field prepares them exactly.  On fields
# that are linear (or quadratic) along the lattice lines that an
# interpolation or a difference uses, the formula is exact, so a wrong weight,
# factor or fallback shows as an O(gradient) error.
# ---------------------------------------------------------------------------


def _plates_domain(orc, Q, nx, ny, nz, y_lo, y_hi, ufield, u_lo, u_hi):
    """Periodic box with resting-shape plates below y_lo and above y_hi, the
    lagged velocity field ufield(x, y, z) -> (D,) at every node, rho = 1."""
    D = 2 if Q == 9 else 3
    d = orc.Domain(Q, nx, ny, nz, 0.05)
    N = nx * ny * nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.stack([np.asarray(c, dtype=float).ravel()
                  for c in ufield(x.astype(float), y.astype(float), z.astype(float))])[:D]
    d.init_fields(np.ones(N), u)
    d.set_body(W.BODY_PLATES, W.plates_params(y_lo, y_hi, u_lo, u_hi))
    return d


def test_target_velocity_linear_fallback_and_linear_wall_gradient(orc):
    """Two fluid rows between plates (rows 0 and 3 solid): for a node of row
    1, x + c_i is fluid but x + 2 c_i is not, so the target velocity of each
    missing link interpolates linearly between the wall point and x + c_i,
    and the wall-normal gradient takes the linear difference through the wall
    point.  On a lagged field linear across the channel that matches both
    plate velocities, both are exact: u_t = u(y) and du_x/dy = a."""
    y_lo, y_hi, U_lo, a = 0.6, 2.7, 0.01, 0.004
    U_hi = U_lo + a * (y_hi - y_lo)
    ux = lambda x, y, z: U_lo + a * (y - y_lo) + 0 * x
    d = _plates_domain(orc, 9, 6, 4, 1, y_lo, y_hi,
                       lambda x, y, z: (ux(x, y, z), 0 * x), (U_lo, 0, 0), (U_hi, 0, 0))
    for y in (1, 2):
        for x in range(6):
            t = d.grad_targets(x, y)
            assert t is not None and t["missing"] == 3
            assert abs(t["u"][0] - (U_lo + a * (y - y_lo))) < 1e-15
            assert abs(t["u"][1]) < 1e-15
            exp = np.zeros((3, 3))
            exp[0, 1] = a
            assert np.max(np.abs(t["grad"] - exp)) < 1e-15, (x, y, t["grad"])


def test_target_gradient_central_difference(orc):
    """Along an axis where both neighbours are fluid and not cut, the target
    gradient is the central difference of the lagged velocity, exact for a
    field linear along that axis.  D2Q9 (axis x) and D3Q27 (axes x and z)
    next to the plates, away from the periodic wrap of the prepared field."""
    h, g, m, k = 0.003, -0.002, 0.0015, 0.0025
    d = _plates_domain(orc, 9, 10, 8, 1, 0.7, 6.4,
                       lambda x, y, z: (h * (x - 4.5), g * (x - 4.5)), (0, 0, 0), (0, 0, 0))
    for y in (1, 6):
        for x in range(1, 9):
            t = d.grad_targets(x, y)
            assert t is not None
            assert abs(t["grad"][0, 0] - h) < 1e-15 and abs(t["grad"][1, 0] - g) < 1e-15
    d3 = _plates_domain(orc, 27, 6, 6, 8, 0.7, 4.4,
                        lambda x, y, z: (h * (x - 2.5) + m * (z - 3.5), 0 * x,
                                         k * (z - 3.5) + g * (x - 2.5)), (0, 0, 0), (0, 0, 0))
    for y in (1, 4):
        for z in range(1, 7):
            for x in range(1, 5):
                t = d3.grad_targets(x, y, z)
                assert t is not None and t["missing"] == 9
                G = t["grad"]
                assert np.max(np.abs(G[:, 0] - (h, 0, g))) < 1e-15, (x, y, z, G)
                assert np.max(np.abs(G[:, 2] - (m, 0, k))) < 1e-15, (x, y, z, G)


def test_target_velocity_and_gradient_quadratic(orc):
    """Wider channel: x + c_i and x + 2 c_i are fluid, so the target velocity
    interpolates quadratically through the wall point and the wall-normal
    gradient is the quadratic difference through the wall point; both are
    exact for a lagged profile quadratic across the channel that matches the
    plate velocities (wall fractions 0.65 and 0.8)."""
    y_lo, y_hi, U_lo, a, kq = 0.35, 10.8, 0.004, 0.003, -0.0002
    prof = lambda y: U_lo + a * (y - y_lo) + kq * (y - y_lo) ** 2
    d = _plates_domain(orc, 9, 5, 12, 1, y_lo, y_hi,
                       lambda x, y, z: (prof(y) + 0 * x, 0 * x), (U_lo, 0, 0), (prof(y_hi), 0, 0))
    for y in (1, 10):
        for x in range(5):
            t = d.grad_targets(x, y)
            assert t is not None and t["missing"] == 3
            assert abs(t["u"][0] - prof(y)) < 1e-15
            assert abs(t["grad"][0, 1] - (a + 2 * kq * (y - y_lo))) < 1e-14, (x, y, t["grad"])


def test_target_single_row_between_two_cut_walls(orc):
    """One fluid row between plates at equal distance (q = 0.4 on both
    sides): no lattice neighbour along any missing link is fluid, so every
    per-link target velocity is its wall velocity, and the wall-normal
    gradient spans the two wall points, (u_hi - u_lo) / (q_hi + q_lo).  For a
    lagged field linear between the plates both are exact: u_t = u(1) (the
    mean of the plate velocities) and du_x/dy = a."""
    y_lo, y_hi, U_lo, a = 0.6, 1.4, -0.003, 0.01
    U_hi = U_lo + a * (y_hi - y_lo)
    d = _plates_domain(orc, 9, 5, 3, 1, y_lo, y_hi,
                       lambda x, y, z: (U_lo + a * (y - y_lo) + 0 * x, 0 * x),
                       (U_lo, 0, 0), (U_hi, 0, 0))
    for x in range(5):
        t = d.grad_targets(x, 1)
        assert t is not None and t["missing"] == 6
        assert abs(t["u"][0] - (U_lo + a * (1 - y_lo))) < 1e-15
        assert abs(t["grad"][0, 1] - a) < 1e-14


# ---------------------------------------------------------------------------
# Stress probes that fall back to the nearest fluid node (Sec. II.C.2 with
# the extrapolation reading: a probe whose interpolation stencil holds no
# fluid node takes the stress of the nearest fluid node in the 5^D box around
# it, Euclidean distance, first in z, y, x order on ties).
# ---------------------------------------------------------------------------


def _probe_stress_brute_force(orc, d, beta, fpre, solid, p):
    """Stress at point p by brute force over the definition: multilinear over
    the stencil corners that are fluid (weights renormalised), else the
    nearest fluid node of the 5^D box around floor(p)."""
    D, dims = d.D, (d.nx, d.ny, d.nz)
    base = [int(math.floor(p[a])) for a in range(D)]
    fr = [p[a] - base[a] for a in range(D)]

    def node(c):
        c = [c[a] % dims[a] for a in range(D)] + [0] * (3 - D)
        return c[0] + d.nx * (c[1] + d.ny * c[2])

    acc, wsum = np.zeros((3, 3)), 0.0
    for corner in np.ndindex(*([2] * D)):
        w = np.prod([fr[a] if corner[a] else 1 - fr[a] for a in range(D)])
        m = node([base[a] + corner[a] for a in range(D)])
        if w <= 0 or solid[m]:
            continue
        acc += w * orc.stress(d.Q, beta, fpre[:, m])
        wsum += w
    if wsum > 0:
        return acc / wsum
    best = None
    rng_z = range(-2, 3) if D == 3 else range(0, 1)
    for dz in rng_z:
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                off = (dx, dy, dz)[:D]
                m = node([base[a] + off[a] for a in range(D)])
                if solid[m]:
                    continue
                r2 = sum((base[a] + off[a] - p[a]) ** 2 for a in range(D))
                if best is None or r2 < best[0]:
                    best = (r2, m)
    return orc.stress(d.Q, beta, fpre[:, best[1]])


@pytest.mark.parametrize("Q", [9, 27])
def test_probe_fallback_nearest_fluid_node_brute_force(orc, Q):
    """Random node states between plates, one step; quadrature points whose
    first probe lies inside a plate, with no fluid stencil corner, at
    fractional offsets where the Euclidean nearest node differs from the
    other candidates at equal wall distance; the tractions must equal the
    brute-force extrapolation 2 sigma(p1) - sigma(p2) applied to n."""
    D = 2 if Q == 9 else 3
    nx, ny, nz = (12, 12, 1) if D == 2 else (8, 10, 8)
    y_lo, y_hi = 2.5, ny - 2.5
    d = orc.Domain(Q, nx, ny, nz, 0.05)
    N = nx * ny * nz
    f0 = W.random_node_states(Q, N, seed=77, amp=0.3).T
    d.set_populations(np.ascontiguousarray(f0))
    d.set_body(W.BODY_PLATES, W.plates_params(y_lo, y_hi))
    d.step(1)
    fpre, solid = d.get_precollision(), d.solid()
    rng = np.random.default_rng(5)
    pts, nrm = [], []
    for k in range(24):
        x0 = rng.uniform(1.0, nx - 2.0)
        z0 = rng.uniform(1.0, nz - 2.0) if D == 3 else 0.0
        frac = (0.9, 0.1, 0.55)[k % 3]
        xq = [math.floor(x0) + frac, rng.uniform(0.05, 0.4)] + ([z0] if D == 3 else [])
        pts.append(xq)
        nrm.append([0.0, 1.0] + ([0.0] if D == 3 else []))
    xq, nq = np.array(pts), np.array(nrm)
    F, tr, st = d.wall_force(xq, nq, np.ones(len(pts)))
    assert st == 0
    beta = d.beta
    for k in range(len(pts)):
        p1, p2 = xq[k] + nq[k], xq[k] + 2 * nq[k]
        s1 = _probe_stress_brute_force(orc, d, beta, fpre, solid, p1)
        s2 = _probe_stress_brute_force(orc, d, beta, fpre, solid, p2)
        exp = ((2 * s1 - s2)[:D, :D] @ nq[k])
        assert np.max(np.abs(tr[k] - exp)) < 1e-14, (k, tr[k], exp)

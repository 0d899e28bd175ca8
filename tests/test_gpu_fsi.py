"""Two-way coupling (Sec. II.C) and the structure solver (Sec. II.B) of the
library against the oracle.

The library's beam (host code behind lbm_fem_*) and the oracle's beam
(numpy) solve the same discrete problem; the coupled step (lbm_fsi_step:
fluid step on the GPU, wall traction at the beam's Gauss points, beam step,
polygon body rebuilt) is compared with the oracle's coupling loop over its
own lattice domain, wall force and beam, in FP64."""
import numpy as np
import pytest

import oracle
from oracle import fsi as ofsi
from oracle.fem import Beam as OBeam

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_beam_matches_oracle():
    from paper_1710_02375_amd import lbm

    rho, mu = 1000.0, 0.5e6
    lam = 2 * mu * 0.4 / 0.2
    o = OBeam(0.1, 0.2, 0.35, 0.02, 10, 2, rho, lam, mu, 2e-3)
    g = lbm.Beam(0.1, 0.2, 0.35, 0.02, 10, 2, rho, lam, mu, 2e-3)
    fo, fg = o.body_force((0.3, -2.0)), g.body_force((0.3, -2.0))
    assert np.array_equal(fo, fg)
    for _ in range(200):
        o.step(fo)
        g.step(fg)
    u, v = g.state()
    du = np.abs(u - o.u).max() / np.abs(o.u).max()
    dv = np.abs(v - o.v).max() / np.abs(o.v).max()
    say("  beam after 200 steps: |du|/|u| %.2e, |dv|/|v| %.2e" % (du, dv))
    assert du < 1e-12 and dv < 1e-9


def _mount():
    # Static block [12, 20] x [12.5, 19.5] that holds the beam's clamped end,
    # as the chain from the clamped top corner round to the bottom one.
    return np.array([[20.0, 19.5], [12.0, 19.5], [12.0, 12.5], [20.0, 12.5]])


def test_coupled_channel_f64_matches_oracle():
    """A soft beam in a channel with inflow: 40 coupled steps; beam state and
    every population of every fluid node agree with the oracle."""
    from paper_1710_02375_amd import lbm

    nx, ny, nu = 80, 32, 0.05
    faces = ["inlet", "outlet", "wall", "wall", "periodic", "periodic"]
    kw = dict(faces=faces, u_in=(0.04, 0.0, 0.0), ramp_steps=20)
    s = lbm.Solver([dict(Q=9, nx=nx, ny=ny, nz=1, nu=nu, storage="f64", **kw)])
    d = oracle.Domain(9, nx, ny, 1, nu, **kw)
    N = nx * ny
    s.init_fields(np.ones(N), np.zeros((2, N)))
    d.init_fields(np.ones(N), np.zeros((2, N)))
    bp = (20.0, 14.5, 20.0, 3.0, 5, 1, 1.0, 20.0, 5.0, 1.0)
    gb = lbm.Beam(*bp)
    ob = OBeam(*bp)
    cg = lbm.Coupling(s, gb, _mount())
    co = ofsi.Coupled(d, ob, _mount())
    say("case: D2Q9 F64 channel %dx%d with a beam 20x3 on a block" % (nx, ny))
    for k in (1, 9, 30):
        Fg, tip = cg.step(k)
        for _ in range(k):
            Fo = co.step()
        u, v = gb.state()
        # Relative to the largest displacement (at least 1e-6 lattice units,
        # so the gate is 1e-15 while the beam has hardly moved).
        du = np.abs(u - ob.u).max() / max(np.abs(ob.u).max(), 1e-6)
        fl = d.solid() == 0
        fgp, fop = s.get_populations(), d.get_populations()
        df = np.abs(fgp[:, fl] - fop[:, fl]).max()
        say("  t=%d: tip %s, |du|/|u| %.2e, max |df| %.2e, beam force gpu %s oracle %s"
            % (d.time, tip[-1], du, df, Fg[-1][:2], Fo[:2]))
        assert du < 1e-9 and df < 1e-12
        assert np.allclose(Fg[-1][:2], Fo[:2], rtol=1e-9, atol=1e-14)
    assert np.abs(ob.u).max() > 1e-6   # the beam did move


def test_fsi3_setup_runs_stably():
    """The FSI3 configuration (1000x164 FP64 fluid, 20x2 beam, theta = 0.55)
    for 0.1 s of physical time during the inflow ramp: the coupled steps stay
    valid, the beam barely moves yet, and a step takes well under 2 ms."""
    import time

    import workloads as W
    from paper_1710_02375_amd import lbm

    c = W.fsi3()
    s = lbm.Solver([dict(Q=9, nx=c["nx"], ny=c["ny"], nz=1, nu=c["nu"], storage="f64",
                         faces=c["faces"], u_in=(c["u_mean"], 0, 0), inlet_profile=1,
                         ramp_steps=c["ramp_steps"])])
    N = c["nx"] * c["ny"]
    s.init_fields(np.ones(N), np.zeros((2, N)))
    b = lbm.Beam(*c["beam"])
    cp = lbm.Coupling(s, b, c["arc"])
    steps = c["steps_per_second"] // 10
    t0 = time.perf_counter()
    F, tip = cp.step(steps)
    ms = (time.perf_counter() - t0) * 1e3 / steps
    u, v = b.state()
    say("  FSI3 %d coupled steps: %.3f ms per step, tip %s lu, max |v| %.2e" %
        (steps, ms, tip[-1], np.abs(v).max()))
    assert np.all(np.isfinite(tip)) and np.abs(tip).max() < 0.1 and np.abs(v).max() < 1e-3
    assert ms < 2.0

"""CPU FP64 oracle for the KBC lattice Boltzmann step (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never imports, links or calls it, and shares no code with it.

The numerics live in ``kbc_oracle.cpp`` (plain C++17, double precision, built
with g++ and OpenMP).  This module builds that file into a shared library and
wraps its C functions with ctypes.  Each wrapped function states the passage of
the paper it follows; the C source carries the details.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kbc_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle_kbc.so")

FACE = {"periodic": 0, "inlet": 1, "outlet": 2, "wall": 3}
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile kbc_oracle.cpp with g++ (-O2, OpenMP, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_lattice.argtypes = [C.c_int, _ip, _dp]
        L.orc_equilibrium.argtypes = [C.c_int, C.c_double, _dp, _dp]
        L.orc_moment_inverse.argtypes = [C.c_int, _dp]
        L.orc_split.argtypes = [C.c_int, _dp, C.c_int, _dp, _dp, _dp]
        L.orc_collide.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int, _dp, _dp,
                                  C.POINTER(C.c_double)]
        L.orc_grad_fstar.argtypes = [C.c_int, C.c_double, _dp, _dp, _dp]
        L.orc_stress.argtypes = [C.c_int, C.c_double, _dp, _dp]
        L.orc_round_storage.argtypes = [C.c_int, C.c_long, _dp, _dp]
        L.orc_body_inside.argtypes = [C.c_int, _dp, C.c_int, _dp, C.c_double]
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                 C.c_int, _ip, _dp, C.c_int, C.c_int, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_void_p, C.c_int]
        L.orc_init_fields.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_set_populations.argtypes = [C.c_void_p, _dp]
        L.orc_get_populations.argtypes = [C.c_void_p, _dp]
        L.orc_get_precollision.argtypes = [C.c_void_p, _dp]
        L.orc_set_body.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_time.restype = C.c_long
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_solid.argtypes = [C.c_void_p, _u8p]
        L.orc_moments.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_wall_force.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_int, _dp, _dp]
        L.orc_stream_only.argtypes = [C.c_void_p]
        L.orc_grad_targets.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp]
        L.orc_set_time.argtypes = [C.c_void_p, C.c_long]
        L.orc_set_mesh.argtypes = [C.c_void_p, C.c_int, _dp, _dp, C.c_int, _ip]
        L.orc_body_velocity.argtypes = [C.c_void_p, _dp, C.c_double, _dp]
        L.orc_collide_forced.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int, _dp, _dp, _dp,
                                         C.POINTER(C.c_double)]
        L.orc_eos_pressure.restype = C.c_double
        L.orc_eos_pressure.argtypes = [C.c_double]
        L.orc_set_multiphase.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
        L.orc_mp_force.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_mp_last_force.argtypes = [C.c_void_p, _dp]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Per-node functions
# ---------------------------------------------------------------------------
def lattice(Q):
    """Velocities (Q,3) int and weights (Q,) of D2Q9 / D3Q27 (tensor D1Q3)."""
    c = np.zeros(3 * Q, np.int32)
    w = np.zeros(Q)
    assert lib().orc_lattice(Q, c, w) == 0
    return c.reshape(Q, 3), w


def equilibrium(Q, rho, u):
    """Entropic equilibrium, minimiser of H under mass/momentum (Sec. II.A, Eqs. 4-5)."""
    out = np.zeros(Q)
    uu = np.zeros(3)
    uu[: len(u)] = u
    assert lib().orc_equilibrium(Q, float(rho), uu, out) == 0
    return out


def moment_inverse(Q):
    out = np.zeros(Q * Q)
    lib().orc_moment_inverse(Q, out)
    return out.reshape(Q, Q)


def split(Q, f, trace_in_s=0):
    """(f^eq, Delta s, Delta h) of a node state (Sec. II.A, Eqs. 2-3)."""
    feq, ds, dh = np.zeros(Q), np.zeros(Q), np.zeros(Q)
    lib().orc_split(Q, _f64(f), int(trace_in_s), feq, ds, dh)
    return feq, ds, dh


def collide(Q, beta, f, collision=0, trace_in_s=0):
    """KBC (collision=0) or LBGK (collision=1) post-collision state and gamma (Eqs. 1, 3, 6)."""
    out = np.zeros(Q)
    g = C.c_double(0.0)
    st = lib().orc_collide(Q, float(beta), int(collision), int(trace_in_s), _f64(f), out,
                           C.byref(g))
    return out, g.value, st


def collide_forced(Q, beta, f, F, collision=0, trace_in_s=0):
    """Forced KBC collision of Sec. III.B (exact difference method, gamma from
    the scalar product shifted to f^eq(rho, u + F/rho)); returns (f', gamma,
    status)."""
    out = np.zeros(Q)
    FF = np.zeros(3)
    FF[: len(F)] = F
    g = C.c_double(0.0)
    st = lib().orc_collide_forced(Q, float(beta), int(collision), int(trace_in_s), _f64(f), FF,
                                  out, C.byref(g))
    return out, g.value, st


def eos_pressure(rho):
    """Non-ideal pressure p(rho) of Sec. III.B, Eq. eos."""
    return lib().orc_eos_pressure(float(rho))


def grad_fstar(Q, rho, v, Pi):
    """Grad's approximation f*(rho, v, Pi) (Sec. II.C.1)."""
    out = np.zeros(Q)
    vv = np.zeros(3)
    vv[: len(v)] = v
    P = np.zeros((3, 3))
    Pi = np.asarray(Pi, dtype=np.float64)
    P[: Pi.shape[0], : Pi.shape[1]] = Pi
    lib().orc_grad_fstar(Q, float(rho), vv, _f64(P.ravel()), out)
    return out


def stress(Q, beta, f):
    """Fluid stress sigma = -p I - (1-beta) Pi^(1) (Sec. II.C.2); 3x3."""
    out = np.zeros(9)
    lib().orc_stress(Q, float(beta), _f64(f), out)
    return out.reshape(3, 3)


def round_storage(mode, x):
    """Round-to-nearest-even of doubles to binary32/binary16/bfloat16 (mode 1/2/3)."""
    x = _f64(x).ravel()
    out = np.zeros_like(x)
    lib().orc_round_storage(STORAGE[mode] if isinstance(mode, str) else int(mode), x.size, x, out)
    return out


def body_inside(kind, params, D, x, t):
    p = np.zeros(16)
    p[: len(params)] = params
    xx = np.zeros(3)
    xx[: len(x)] = x
    return bool(lib().orc_body_inside(int(kind), p, int(D), xx, float(t)))


# ---------------------------------------------------------------------------
# Domain
# ---------------------------------------------------------------------------
class Domain:
    """One lattice instance stepped by the oracle (all FP64, AoS internally).

    faces: six of 'periodic' | 'inlet' (-x only) | 'outlet' (+x only) | 'wall',
    ordered -x, +x, -y, +y, -z, +z.  storage: 'f64' (exact) or 'f32' | 'f16' |
    'bf16' to round the shifted populations f_i - W_i after every step.
    """

    def __init__(self, Q, nx, ny, nz, nu, collision=0, trace_in_s=0, faces=None,
                 u_in=(0.0, 0.0, 0.0), inlet_profile=0, ramp_steps=0, storage="f64",
                 threads=None):
        self.Q, self.nx, self.ny, self.nz = Q, nx, ny, nz
        self.D = 2 if Q == 9 else 3
        self.N = nx * ny * nz
        self.beta = 1.0 / (6.0 * nu + 1.0)
        faces = faces or ["periodic"] * 6
        fa = np.array([FACE[f] if isinstance(f, str) else int(f) for f in faces], np.int32)
        uin = np.zeros(3)
        uin[: len(u_in)] = u_in
        self._h = lib().orc_create(Q, nx, ny, nz, float(nu), int(collision), int(trace_in_s), fa,
                                   uin, int(inlet_profile), int(ramp_steps),
                                   STORAGE[storage] if isinstance(storage, str) else int(storage))
        if not self._h:
            raise ValueError("oracle: invalid domain description")
        if threads:
            lib().orc_set_threads(self._h, int(threads))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def set_threads(self, n):
        lib().orc_set_threads(self._h, int(n))

    def init_fields(self, rho, u):
        """f := f^eq(rho, u); rho (N,), u (D, N) planar, x-fastest."""
        rho = _f64(np.asarray(rho).reshape(-1))
        u = _f64(np.asarray(u).reshape(self.D, -1))
        assert lib().orc_init_fields(self._h, rho, u.ravel()) == 0

    def set_populations(self, f):
        lib().orc_set_populations(self._h, _f64(np.asarray(f).reshape(-1)))

    def get_populations(self):
        out = np.zeros(self.Q * self.N)
        lib().orc_get_populations(self._h, out)
        return out.reshape(self.Q, self.N)

    def get_precollision(self):
        out = np.zeros(self.Q * self.N)
        lib().orc_get_precollision(self._h, out)
        return out.reshape(self.Q, self.N)

    def set_body(self, kind, params):
        p = np.zeros(16)
        p[: len(params)] = params
        if lib().orc_set_body(self._h, int(kind), p) != 0:
            raise ValueError("oracle: invalid body")

    def step(self, n=1):
        return lib().orc_step(self._h, int(n))

    @property
    def time(self):
        return lib().orc_time(self._h)

    def solid(self):
        out = np.zeros(self.N, np.uint8)
        lib().orc_solid(self._h, out)
        return out

    def moments(self):
        """(rho (N,), u (D,N), totals dict); solid nodes report zeros."""
        rho = np.zeros(self.N)
        u = np.zeros(self.D * self.N)
        tot = np.zeros(7)
        st = lib().orc_moments(self._h, rho, u, tot)
        totals = dict(mass=tot[0], momentum=tot[1:4].copy(), gamma_min=tot[4],
                      gamma_mean=tot[5], gamma_max=tot[6], invalid=bool(st))
        return rho, u.reshape(self.D, self.N), totals

    def wall_force(self, xq, nq, wq):
        """Force of the fluid on the body and per-point tractions (Sec. II.C.2)."""
        xq = _f64(np.asarray(xq).reshape(-1, self.D))
        nq = _f64(np.asarray(nq).reshape(-1, self.D))
        wq = _f64(np.asarray(wq).reshape(-1))
        n = wq.size
        tr = np.zeros(n * self.D)
        F = np.zeros(3)
        st = lib().orc_wall_force(self._h, xq.ravel(), nq.ravel(), wq, n, tr, F)
        return F[: self.D].copy(), tr.reshape(n, self.D), st

    def stream_only(self):
        assert lib().orc_stream_only(self._h) == 0

    def grad_targets(self, x, y, z=0):
        """Grad target values the next step would use at node (x, y, z)
        (Sec. II.C.1): dict(rho, u (3,), grad (3, 3) with grad[a, b] =
        d u_a / d x_b, missing = number of missing populations), or None for a
        node without missing populations, a solid node or an inflow / outflow
        node."""
        out = np.zeros(13)
        k = lib().orc_grad_targets(self._h, int(x), int(y), int(z), out)
        if k <= 0:
            return None
        return dict(rho=out[0], u=out[1:4].copy(), grad=out[4:13].reshape(3, 3).copy(), missing=k)

    def set_mesh(self, verts, vel, tris):
        """Surface-mesh body (Sec. II.C.1): verts (V, 3), vel (V, 3), tris
        (T, 3) vertex indices (2D: the first two of each row form a segment);
        sets the geometry at the current time."""
        V = _f64(np.asarray(verts).reshape(-1, 3))
        Vv = _f64(np.asarray(vel).reshape(-1, 3))
        T = np.ascontiguousarray(np.asarray(tris).reshape(-1, 3), dtype=np.int32)
        if lib().orc_set_mesh(self._h, V.shape[0], V.ravel(), Vv.ravel(), T.shape[0],
                              T.ravel()) != 0:
            raise ValueError("oracle: invalid mesh")

    def body_velocity(self, x, t=None):
        """Velocity of the body at point x (mesh: interpolated at the closest
        surface point)."""
        xx = np.zeros(3)
        xx[: len(x)] = x
        v = np.zeros(3)
        lib().orc_body_velocity(self._h, xx, float(self.time if t is None else t), v)
        return v

    def set_multiphase(self, kappa, kappa_w=0.0, on=True):
        """Multiphase forcing of Sec. III.B (faces periodic or walls only)."""
        if lib().orc_set_multiphase(self._h, int(bool(on)), float(kappa), float(kappa_w)) != 0:
            raise ValueError("oracle: multiphase needs periodic or wall faces")

    def mp_force(self, rho):
        """Body force of Sec. III.B for density field rho (N,) over the
        current geometry; (D, N)."""
        out = np.zeros(3 * self.N)
        lib().orc_mp_force(self._h, _f64(np.asarray(rho).reshape(-1)), out)
        return out.reshape(3, self.N)[: self.D]

    def mp_last_force(self):
        """Body force the last multiphase step used; (D, N)."""
        out = np.zeros(3 * self.N)
        assert lib().orc_mp_last_force(self._h, out) == 0
        return out.reshape(3, self.N)[: self.D]

    def set_time(self, t):
        """Sets the step count of the stored state (then call set_body)."""
        assert lib().orc_set_time(self._h, int(t)) == 0

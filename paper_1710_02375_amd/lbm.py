"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the lattice Boltzmann path runs in the HIP library
``libkbc_lbm.so``; this module only converts numpy arrays and Python values
to the C types and raises on error codes.  If the library is missing the
import of the functions raises: there is no CPU fallback.

The functions keep the C names (lbm_create, lbm_step, ...).  ``Solver`` is a
small convenience wrapper around one context.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkbc_lbm.so")

LBM_OK = 0
STATUS = {0: "LBM_OK", -1: "LBM_ERR_INVALID", -2: "LBM_ERR_OOM", -3: "LBM_ERR_DEVICE",
          -4: "LBM_ERR_NONFINITE", -5: "LBM_ERR_GEOMETRY", -6: "LBM_ERR_UNSUPPORTED"}
LBM_ERR_INVALID, LBM_ERR_OOM, LBM_ERR_DEVICE = -1, -2, -3
LBM_ERR_NONFINITE, LBM_ERR_GEOMETRY, LBM_ERR_UNSUPPORTED = -4, -5, -6
LBM_D2Q9, LBM_D3Q27 = 9, 27
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
STORAGE_BYTES = {0: 8, 1: 4, 2: 2, 3: 2}
FACE = {"periodic": 0, "inlet": 1, "outlet": 2, "wall": 3}
LBM_BODY_NONE, LBM_BODY_SPHERE, LBM_BODY_FLAP, LBM_BODY_MESH, LBM_BODY_PLATES = 0, 1, 2, 3, 4
COLLISION = {"kbc": 0, "lbgk": 1}


class lbm_instance_desc(C.Structure):
    _fields_ = [("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("nu", C.c_double), ("storage", C.c_int), ("collision", C.c_int),
                ("kbc_trace_in_s", C.c_int), ("face", C.c_int * 6), ("u_in", C.c_double * 3),
                ("inlet_profile", C.c_int), ("ramp_steps", C.c_int)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class lbm_device_opts(C.Structure):
    _fields_ = [("device", C.c_int), ("hip_stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_ctx", C.c_void_p), ("use_graph", C.c_int)]


class lbm_body(C.Structure):
    _fields_ = [("kind", C.c_int), ("params", C.c_double * 16), ("nverts", C.c_int),
                ("ntris", C.c_int), ("verts", C.c_void_p), ("vert_vel", C.c_void_p),
                ("tris", C.c_void_p)]


class lbm_fem_desc(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("length", C.c_double),
                ("height", C.c_double), ("nex", C.c_int), ("ney", C.c_int), ("rho", C.c_double),
                ("lambda_", C.c_double), ("mu", C.c_double), ("dt", C.c_double),
                ("theta", C.c_double)]


class lbm_totals(C.Structure):
    _fields_ = [("mass", C.c_double), ("momentum", C.c_double * 3), ("gamma_min", C.c_double),
                ("gamma_mean", C.c_double), ("gamma_max", C.c_double),
                ("fp64_gamma_fraction", C.c_double), ("step", C.c_int64)]


class LBMError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    """Loads libkbc_lbm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime with the same soname as the system
        # one; loading torch first makes the library bind to that runtime, so
        # one process never holds two HIP runtimes (torch would then see no
        # device).  Without torch the system runtime is used.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built (run __graft_entry__.build())" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.lbm_create.argtypes = [C.POINTER(lbm_instance_desc), C.c_int,
                                 C.POINTER(lbm_device_opts), C.POINTER(vp)]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_init_fields.argtypes = [vp, C.c_int, _dp, _dp]
        L.lbm_set_geometry.argtypes = [vp, C.c_int, C.POINTER(lbm_body)]
        L.lbm_step.argtypes = [vp, C.c_int]
        L.lbm_moments.argtypes = [vp, C.c_int, vp, vp, C.POINTER(lbm_totals)]
        L.lbm_wall_force.argtypes = [vp, C.c_int, _dp, _dp, _dp, C.c_int, vp,
                                     C.POINTER(C.c_double)]
        L.lbm_wall_force_noalloc.argtypes = [vp, C.c_int, _dp, _dp, _dp, C.c_int, vp,
                                             C.POINTER(C.c_double)]
        L.lbm_get_populations.argtypes = [vp, C.c_int, _dp]
        L.lbm_set_populations.argtypes = [vp, C.c_int, _dp]
        L.lbm_get_populations_box.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                              _dp]
        L.lbm_set_multiphase.argtypes = [vp, C.c_int, C.c_int, C.c_double, C.c_double]
        L.lbm_fem_create.argtypes = [C.POINTER(lbm_fem_desc), C.POINTER(C.c_void_p)]
        L.lbm_fem_destroy.argtypes = [vp]
        L.lbm_fem_info.argtypes = [vp, C.POINTER(C.c_int), vp]
        L.lbm_fem_body_force.argtypes = [vp, _dp, _dp]
        L.lbm_fem_step.argtypes = [vp, _dp, C.POINTER(C.c_int)]
        L.lbm_fem_get_state.argtypes = [vp, vp, vp]
        L.lbm_fem_set_state.argtypes = [vp, vp, vp]
        L.lbm_fsi_create.argtypes = [vp, C.c_int, vp, vp, C.c_int, C.POINTER(C.c_void_p)]
        L.lbm_fsi_destroy.argtypes = [vp]
        L.lbm_fsi_step.argtypes = [vp, C.c_int, vp, vp]
        L.lbm_set_stats.argtypes = [vp, C.c_int]
        L.lbm_set_launch_mode.argtypes = [vp, C.c_int]
        L.lbm_autotune.argtypes = [vp, C.c_char_p, C.POINTER(C.c_int)]
        L.lbm_set_variant.argtypes = [vp, C.c_int]
        L.lbm_variant_count.argtypes = []
        L.lbm_variant_name.restype = C.c_char_p
        L.lbm_variant_name.argtypes = [C.c_int]
        L.lbm_info.argtypes = [vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                               C.POINTER(C.c_int), C.POINTER(C.c_int64)]
        L.lbm_synchronize.argtypes = [vp]
        L.lbm_status_string.restype = C.c_char_p
        L.lbm_status_string.argtypes = [C.c_int]
        L.lbm_last_error.restype = C.c_char_p
        L.lbm_last_error.argtypes = [vp]
        _lib = L
    return _lib


EXPORTED = ["lbm_create", "lbm_destroy", "lbm_init_fields", "lbm_set_geometry", "lbm_step",
            "lbm_moments", "lbm_wall_force", "lbm_wall_force_noalloc", "lbm_get_populations",
            "lbm_set_populations", "lbm_get_populations_box", "lbm_set_multiphase",
            "lbm_fem_create", "lbm_fem_destroy", "lbm_fem_info", "lbm_fem_body_force",
            "lbm_fem_step", "lbm_fem_get_state", "lbm_fem_set_state", "lbm_fsi_create",
            "lbm_fsi_destroy", "lbm_fsi_step",
            "lbm_set_stats", "lbm_set_launch_mode", "lbm_autotune", "lbm_set_variant",
            "lbm_variant_count", "lbm_variant_name", "lbm_info", "lbm_synchronize",
            "lbm_status_string", "lbm_last_error"]


def _check(ctx, status):
    if status != LBM_OK:
        msg = lib().lbm_last_error(ctx)
        raise LBMError(status, msg.decode() if msg else "")
    return status


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64).ravel()


def make_desc(Q, nx, ny, nz, nu, storage="f32", collision="kbc", trace_in_s=0, faces=None,
              u_in=(0.0, 0.0, 0.0), inlet_profile=0, ramp_steps=0):
    d = lbm_instance_desc()
    d.lattice = int(Q)
    d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
    d.nu = float(nu)
    d.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    d.collision = COLLISION[collision] if isinstance(collision, str) else int(collision)
    d.kbc_trace_in_s = int(trace_in_s)
    faces = faces or ["periodic"] * 6
    for k, f in enumerate(faces):
        d.face[k] = FACE[f] if isinstance(f, str) else int(f)
    for a in range(3):
        d.u_in[a] = float(u_in[a]) if a < len(u_in) else 0.0
    d.inlet_profile = int(inlet_profile)
    d.ramp_steps = int(ramp_steps)
    return d


class TorchAllocator:
    """Device allocation callbacks backed by PyTorch tensors (torch owns the
    memory; the allocator object must outlive the context).

    stream: the torch.cuda.Stream the library launches on.  Blocks are then
    allocated with that stream current, so torch's caching allocator orders
    their reuse after the library's work on it.  Without a stream (the
    library then uses a stream of its own) each release first waits for the
    device, so that a released block cannot be handed out while the library
    may still write it."""

    def __init__(self, device=0, stream=None):
        import torch

        self._torch = torch
        self.device = device
        self.stream = stream
        self._live = {}
        self.n_alloc = 0   # allocation callbacks served
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, nbytes, _ctx):
        torch = self._torch
        self.n_alloc += 1
        dev = "cuda:%d" % self.device
        if self.stream is not None:
            with torch.cuda.stream(self.stream):
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
        else:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
            # Pending work of torch's current stream may still use a block
            # the caching allocator hands back; the library writes on its own
            # stream, so wait for it first.
            torch.cuda.current_stream(self.device).synchronize()
        p = t.data_ptr()
        self._live[p] = t
        return p

    def _free(self, ptr, _ctx):
        if self.stream is None and ptr in self._live:
            self._torch.cuda.synchronize(self.device)
        self._live.pop(ptr, None)


def lbm_create(descs, device=0, stream=None, use_graph=True, allocator=None):
    """Creates a context for a list of lbm_instance_desc.  stream: a HIP stream
    handle (int) or a torch.cuda.Stream; allocator: a TorchAllocator or None."""
    arr = (lbm_instance_desc * len(descs))(*descs)
    opts = lbm_device_opts()
    opts.device = int(device)
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    opts.hip_stream = C.c_void_p(int(stream)) if stream else None
    if allocator is not None:
        opts.alloc = allocator.alloc_fn
        opts.free = allocator.free_fn
    opts.use_graph = 1 if use_graph else 0
    ctx = C.c_void_p()
    st = lib().lbm_create(arr, len(descs), C.byref(opts), C.byref(ctx))
    if st != LBM_OK:
        msg = lib().lbm_last_error(None)
        raise LBMError(st, msg.decode() if msg else "")
    return ctx


def lbm_destroy(ctx):
    return lib().lbm_destroy(ctx)


def lbm_init_fields(ctx, inst, rho, u):
    return _check(ctx, lib().lbm_init_fields(ctx, int(inst), _f64(rho), _f64(u)))


def lbm_set_geometry(ctx, inst, kind, params=(), verts=None, vert_vel=None, tris=None):
    """kind: LBM_BODY_*; params for the analytic bodies; verts (V, 3),
    vert_vel (V, 3) and tris (T, 3) for a surface mesh (copied before the call
    returns)."""
    b = lbm_body()
    b.kind = int(kind)
    for k, v in enumerate(params):
        b.params[k] = float(v)
    keep = []
    if verts is not None:
        V = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 3)
        Vv = np.ascontiguousarray(vert_vel if vert_vel is not None else np.zeros_like(V),
                                  dtype=np.float64).reshape(-1, 3)
        T = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
        keep = [V, Vv, T]
        b.nverts, b.ntris = V.shape[0], T.shape[0]
        b.verts, b.vert_vel, b.tris = V.ctypes.data, Vv.ctypes.data, T.ctypes.data
    st = lib().lbm_set_geometry(ctx, int(inst), C.byref(b))
    del keep
    return _check(ctx, st)


def lbm_step(ctx, n_steps):
    return _check(ctx, lib().lbm_step(ctx, int(n_steps)))


def lbm_moments(ctx, inst, N, D, want_fields=True):
    rho = np.zeros(N) if want_fields else None
    u = np.zeros(D * N) if want_fields else None
    tot = lbm_totals()
    st = lib().lbm_moments(ctx, int(inst), rho.ctypes.data if want_fields else None,
                           u.ctypes.data if want_fields else None, C.byref(tot))
    totals = dict(mass=tot.mass, momentum=np.array(tot.momentum[:]), gamma_min=tot.gamma_min,
                  gamma_mean=tot.gamma_mean, gamma_max=tot.gamma_max,
                  fp64_gamma_fraction=tot.fp64_gamma_fraction, step=tot.step,
                  status=st)
    if st not in (LBM_OK, LBM_ERR_NONFINITE):
        _check(ctx, st)
    return rho, (u.reshape(D, N) if want_fields else None), totals


def lbm_wall_force(ctx, inst, xq, nq, wq, D, want_traction=True):
    xq, nq, wq = _f64(xq), _f64(nq), _f64(wq)
    n = wq.size
    tr = np.zeros(n * D) if want_traction else None
    F = (C.c_double * 3)()
    st = lib().lbm_wall_force(ctx, int(inst), xq, nq, wq, n,
                              tr.ctypes.data if want_traction else None, F)
    _check(ctx, st)
    return np.array(F[:D]), (tr.reshape(n, D) if want_traction else None)


def lbm_wall_force_noalloc(ctx, inst, xq, nq, wq, D, want_traction=True):
    """lbm_wall_force through the library's static workspace (no device
    allocation; at most 65536 points)."""
    xq, nq, wq = _f64(xq), _f64(nq), _f64(wq)
    n = wq.size
    tr = np.zeros(n * D) if want_traction else None
    F = (C.c_double * 3)()
    st = lib().lbm_wall_force_noalloc(ctx, int(inst), xq, nq, wq, n,
                                      tr.ctypes.data if want_traction else None, F)
    _check(ctx, st)
    return np.array(F[:D]), (tr.reshape(n, D) if want_traction else None)


def lbm_get_populations(ctx, inst, Q, N):
    f = np.zeros(Q * N)
    _check(ctx, lib().lbm_get_populations(ctx, int(inst), f))
    return f.reshape(Q, N)


def lbm_get_populations_box(ctx, inst, Q, lo, hi):
    """Populations of the box [lo, hi) (3 ints each; periodic axes may wrap
    once) as an array (Q, nz_b, ny_b, nx_b)."""
    lo3 = (C.c_int * 3)(*[int(v) for v in lo])
    hi3 = (C.c_int * 3)(*[int(v) for v in hi])
    ext = [int(h) - int(l) for l, h in zip(lo, hi)]
    f = np.zeros(Q * ext[0] * ext[1] * ext[2])
    _check(ctx, lib().lbm_get_populations_box(ctx, int(inst), lo3, hi3, f))
    return f.reshape(Q, ext[2], ext[1], ext[0])


def lbm_set_populations(ctx, inst, f):
    return _check(ctx, lib().lbm_set_populations(ctx, int(inst), _f64(f)))


def lbm_set_multiphase(ctx, inst, kappa, kappa_w=0.0, enable=True):
    """Multiphase forcing of Sec. III.B on instance inst (or off)."""
    return _check(ctx, lib().lbm_set_multiphase(ctx, int(inst), int(bool(enable)), float(kappa),
                                                float(kappa_w)))


class Beam:
    """Finite-element beam of the structure solver (lbm_fem_*): Sec. II.B."""

    def __init__(self, x0, y0, length, height, nex, ney, rho, lam, mu, dt, theta=0.5):
        d = lbm_fem_desc(float(x0), float(y0), float(length), float(height), int(nex), int(ney),
                         float(rho), float(lam), float(mu), float(dt), float(theta))
        h = C.c_void_p()
        _check(None, lib().lbm_fem_create(C.byref(d), C.byref(h)))
        self.h = h
        n = C.c_int(0)
        lib().lbm_fem_info(self.h, C.byref(n), None)
        self.nn = n.value
        self.X = np.zeros(2 * self.nn)
        lib().lbm_fem_info(self.h, None, self.X.ctypes.data_as(C.c_void_p))
        self.X = self.X.reshape(-1, 2)
        self.nex, self.ney = nex, ney

    def body_force(self, b):
        f = np.zeros(2 * self.nn)
        _check(None, lib().lbm_fem_body_force(self.h, _f64(b), f))
        return f

    def step(self, fext):
        it = C.c_int(0)
        _check(None, lib().lbm_fem_step(self.h, _f64(fext), C.byref(it)))
        return it.value

    def state(self):
        u, v = np.zeros(2 * self.nn), np.zeros(2 * self.nn)
        lib().lbm_fem_get_state(self.h, u.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p))
        return u, v

    def set_state(self, u, v):
        u, v = _f64(u), _f64(v)
        lib().lbm_fem_set_state(self.h, u.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p))

    def tip(self):
        u, _ = self.state()
        k = self.ney + (2 * self.ney + 1) * (2 * self.nex)
        return u[2 * k: 2 * k + 2]

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_fem_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Coupling:
    """Two-way coupling of a context instance with a Beam (lbm_fsi_*): Sec. II.C."""

    def __init__(self, solver, beam, arc=None, inst=0):
        a = _f64(arc) if arc is not None and len(arc) else np.zeros(0)
        h = C.c_void_p()
        _check(solver.ctx, lib().lbm_fsi_create(solver.ctx, int(inst), beam.h,
                                               a.ctypes.data_as(C.c_void_p) if a.size else None,
                                               a.size // 2, C.byref(h)))
        self.h, self.solver, self.beam = h, solver, beam

    def step(self, n=1):
        """n coupled steps; returns (beam force (n, 3), tip displacement (n, 2))."""
        F = np.zeros(3 * n)
        tip = np.zeros(2 * n)
        _check(self.solver.ctx, lib().lbm_fsi_step(self.h, int(n), F.ctypes.data_as(C.c_void_p),
                                                  tip.ctypes.data_as(C.c_void_p)))
        return F.reshape(n, 3), tip.reshape(n, 2)

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_fsi_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def lbm_set_stats(ctx, enabled):
    return _check(ctx, lib().lbm_set_stats(ctx, int(bool(enabled))))


def lbm_set_launch_mode(ctx, mode):
    return _check(ctx, lib().lbm_set_launch_mode(ctx, int(mode)))


def lbm_autotune(ctx, cache_path=None):
    v = C.c_int(-1)
    _check(ctx, lib().lbm_autotune(ctx, cache_path.encode() if cache_path else None, C.byref(v)))
    return v.value


def lbm_set_variant(ctx, v):
    return _check(ctx, lib().lbm_set_variant(ctx, int(v)))


def lbm_variant_count():
    return lib().lbm_variant_count()


def lbm_variant_name(v):
    return lib().lbm_variant_name(int(v)).decode()


def lbm_info(ctx, inst=0):
    n, tn, b, s = C.c_int64(), C.c_int64(), C.c_int(), C.c_int64()
    _check(ctx, lib().lbm_info(ctx, int(inst), C.byref(n), C.byref(tn), C.byref(b), C.byref(s)))
    return dict(nodes=n.value, total_nodes=tn.value, bytes_per_update=b.value, step=s.value)


def lbm_synchronize(ctx):
    return _check(ctx, lib().lbm_synchronize(ctx))


def lbm_status_string(status):
    return lib().lbm_status_string(int(status)).decode()


def lbm_last_error(ctx):
    m = lib().lbm_last_error(ctx)
    return m.decode() if m else ""


class Solver:
    """One context with numpy in/out.  descs: list of dicts for make_desc."""

    def __init__(self, descs, device=0, stream=None, use_graph=True, allocator=None):
        self.descs = [make_desc(**d) if isinstance(d, dict) else d for d in descs]
        if allocator is not None and allocator.stream is None and hasattr(stream, "cuda_stream"):
            allocator.stream = stream
        self.allocator = allocator
        self.ctx = lbm_create(self.descs, device, stream, use_graph, allocator)
        self.Q = self.descs[0].lattice
        self.D = 3 if self.Q == 27 else 2

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def nodes(self, inst=0):
        d = self.descs[inst]
        return d.nx * d.ny * d.nz

    def init_fields(self, rho, u, inst=0):
        lbm_init_fields(self.ctx, inst, rho, u)

    def set_body(self, kind, params=(), inst=0, verts=None, vert_vel=None, tris=None):
        lbm_set_geometry(self.ctx, inst, kind, params, verts, vert_vel, tris)

    def set_multiphase(self, kappa, kappa_w=0.0, inst=0, enable=True):
        lbm_set_multiphase(self.ctx, inst, kappa, kappa_w, enable)

    def step(self, n=1):
        lbm_step(self.ctx, n)

    def synchronize(self):
        lbm_synchronize(self.ctx)

    def moments(self, inst=0, fields=True):
        return lbm_moments(self.ctx, inst, self.nodes(inst), self.D, fields)

    def wall_force(self, xq, nq, wq, inst=0):
        return lbm_wall_force(self.ctx, inst, xq, nq, wq, self.D)

    def get_populations(self, inst=0):
        return lbm_get_populations(self.ctx, inst, self.Q, self.nodes(inst))

    def set_populations(self, f, inst=0):
        lbm_set_populations(self.ctx, inst, f)

    def set_stats(self, on):
        lbm_set_stats(self.ctx, on)

    def set_launch_mode(self, mode):
        lbm_set_launch_mode(self.ctx, mode)

    def info(self, inst=0):
        return lbm_info(self.ctx, inst)

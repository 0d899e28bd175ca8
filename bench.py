"""Throughput benchmark of the KBC lattice Boltzmann step on one MI355X.

Workload (headline): D3Q27 KBC Taylor-Green vortex, 256^3 periodic, FP32,
Re = 1600, Ma = 0.1, seeded 1e-4 velocity perturbation; inputs resident in HBM.
A step is one full pass of the hot path over the lattice (pull streaming,
moments, entropic equilibrium, per-node gamma, collision).

Prints one JSON line: MLUPS (value), the HBM roofline of the bulk kernel from
HIP events on the launch stream, the same workload with FP16- and BF16-shifted
storage, the velocity error of each form against the FP64 form of the same
kernel after a fixed number of steps, and the CPU oracle timed on a bounded
sample on the host cores.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--no-cpu]
  python bench.py --copy-calibration     # plain copy kernel for counter scaling
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FORM_TEXT = {"f32": "FP32 storage and arithmetic", "f64": "FP64 storage and arithmetic",
             "f16": "FP16 storage of f - W with FP32 arithmetic",
             "bf16": "BF16 storage of f - W with FP32 arithmetic"}
METRIC = "MLUPS and % HBM roofline, D3Q27 KBC, FP32 vs FP16-shifted at stated error"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_bulk_d3q27_tg256_f32.txt")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1710_02375_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(nodes, variant):
    """HBM bytes per launch of the bulk kernel variant from the committed
    rocprofv3 counter summary (lines "key: value", per variant
    "hbm_bytes_per_launch[<variant>]"), or None if it is missing, was taken on
    a different kernel source, a different lattice size or another variant."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(l.split(":", 1) for l in f if ":" in l and not l.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        if kv.get("kernel_source_hash") != kernel_source_hash() or int(kv.get("nodes", 0)) != nodes:
            return None
        return float(kv["hbm_bytes_per_launch[%s]" % variant])
    except (OSError, ValueError, KeyError):
        return None


def copy_ceiling(nbytes=1 << 31, reps=20):
    """Measured streaming ceiling over 2 GiB buffers (read + write): the faster
    of a plain device copy and a scale kernel b = 2a.  Returns (GB/s, name)."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    best = (0.0, "")
    for name, op in (("copy b = a", lambda: b.copy_(a)),
                     ("scale b = 2a", lambda: torch.mul(a, 2.0, out=b))):
        op()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            op()
        e.record()
        torch.cuda.synchronize()
        gbs = 2 * nbytes / (s.elapsed_time(e) / reps) / 1e6
        best = max(best, (gbs, name))
    del a, b
    torch.cuda.empty_cache()
    return best


def copy_calibration(nbytes=1 << 31, reps=20):
    """Plain device copy for scaling the HBM counters (run under rocprofv3)."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.copy_(a)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                      "ms_per_copy": ms, "copy_GBs": 2 * nbytes / ms / 1e6}))


def time_form(lbm, torch, n, storage, rho, u, nu, steps, warmup, variant=None):
    """MLUPS of one storage form; returns (mlups, ms_per_step, kernel_ms, info).
    variant: a bulk-kernel variant name, or None to autotune."""
    # A dedicated (default-priority) stream: the library launches on it and the
    # timing events are recorded on it.
    stream = torch.cuda.Stream()
    s = lbm.Solver([dict(Q=27, nx=n, ny=n, nz=n, nu=nu, storage=storage)], stream=stream)
    s.init_fields(rho, u)
    if variant:
        names = [lbm.lbm_variant_name(k) for k in range(lbm.lbm_variant_count())]
        v = names.index(variant)
        lbm.lbm_set_variant(s.ctx, v)
    else:
        v = lbm.lbm_autotune(s.ctx, os.environ.get("KBC_AUTOTUNE_CACHE"))
    s.step(warmup)
    stream.synchronize()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    s.step(steps)
    ev1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    kernel_ms = ev0.elapsed_time(ev1) / steps
    info = s.info()
    info["variant"] = lbm.lbm_variant_name(v)
    s.close()
    mlups = n ** 3 / (ms_step * 1e3)
    return mlups, ms_step, kernel_ms, info


def error_vs_f64(lbm, n, rho, u, nu, steps, variants=None):
    """Velocity rel L2 of each storage form against the FP64 form after
    `steps` steps from the same initial fields.  variants maps a storage form
    to the bulk-kernel variant name it was timed with, so that the error is
    that of the kernel that was timed."""
    ref = None
    out = {}
    names = [lbm.lbm_variant_name(k) for k in range(lbm.lbm_variant_count())]
    for storage in ("f64", "f32", "f16", "bf16"):
        s = lbm.Solver([dict(Q=27, nx=n, ny=n, nz=n, nu=nu, storage=storage)])
        s.init_fields(rho, u)
        if variants and storage in variants:
            lbm.lbm_set_variant(s.ctx, names.index(variants[storage]))
        s.step(steps)
        _, uu, _ = s.moments()
        s.close()
        if ref is None:
            ref = uu
            continue
        out[storage] = float(np.linalg.norm(uu - ref) / np.linalg.norm(ref))
    return out


def batched_form(lbm, torch, steps, warmup, count=64):
    """64 uneven D2Q9 flap channels (seed 2375), FP32: aggregate MLUPS with one
    launch per kernel per step for all instances, against one launch per
    instance; the two final states must be bitwise equal."""
    import workloads as W

    chans = W.flap_channels(count=count, seed=2375)
    descs = [dict(Q=9, nx=c["nx"], ny=c["ny"], nz=1, nu=c["nu"], storage="f32",
                  faces=c["faces"], u_in=c["u_in"], inlet_profile=1) for c in chans]
    total = sum(d["nx"] * d["ny"] for d in descs)
    out = {}
    finals = []
    for mode, name in ((0, "batched"), (1, "per_instance")):
        stream = torch.cuda.Stream()
        s = lbm.Solver(descs, stream=stream)
        for k, (c, d) in enumerate(zip(chans, descs)):
            N = d["nx"] * d["ny"]
            s.init_fields(np.ones(N), np.zeros((2, N)), inst=k)
            s.set_body(*c["body"], inst=k)
        s.set_launch_mode(mode)
        if mode == 0:
            v = lbm.lbm_autotune(s.ctx, os.environ.get("KBC_AUTOTUNE_CACHE"))
            out["variant"] = lbm.lbm_variant_name(v)
        else:
            lbm.lbm_set_variant(s.ctx, v)
        s.step(warmup)
        stream.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        s.step(steps)
        ev1.record(stream)
        stream.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"MLUPS": round(total * steps / el / 1e6, 1),
                     "ms_per_step": round(el * 1e3 / steps, 5),
                     "event_ms_per_step": round(ev0.elapsed_time(ev1) / steps, 5)}
        finals.append([s.get_populations(k) for k in (0, count // 2, count - 1)])
        s.close()
    out["nodes"] = total
    out["bytes_per_lattice_update"] = 72
    out["bitwise_equal"] = all(np.array_equal(a, b) for a, b in zip(*finals))
    return out


def sphere_form(lbm, torch, storage, steps, sample_every, variant=None, dims=(512, 128, 128),
                radius=16.0):
    """Channel with the oscillating sphere (Re 300, Grad boundary nodes): MLUPS
    over the stepping alone, then drag/lift coefficients every sample_every
    steps from the wall force on an icosphere quadrature (5120 facets)."""
    import math

    import workloads as W

    nx, ny, nz = dims
    cfg = W.sphere_channel(nx, ny, nz, radius)
    stream = torch.cuda.Stream()
    s = lbm.Solver([dict(Q=27, nx=nx, ny=ny, nz=nz, nu=cfg["nu"], storage=storage,
                         faces=cfg["faces"], u_in=cfg["u_in"], ramp_steps=cfg["ramp_steps"])],
                   stream=stream)
    N = nx * ny * nz
    s.init_fields(np.ones(N), np.zeros((3, N)))
    kind, p = cfg["body"]
    s.set_body(kind, p)
    if variant:
        names = [lbm.lbm_variant_name(k) for k in range(lbm.lbm_variant_count())]
        lbm.lbm_set_variant(s.ctx, names.index(variant))
    else:
        variant = lbm.lbm_variant_name(lbm.lbm_autotune(s.ctx, os.environ.get("KBC_AUTOTUNE_CACHE")))
    U, R = cfg["U"], cfg["radius"]
    norm = 0.5 * U * U * math.pi * R * R
    series = []
    t_force, t_force_na = [], []
    t_step = 0.0
    chunks = []   # (first step, steps, seconds) of each timed chunk
    done = 0
    while done < steps:
        k = min(sample_every, steps - done)
        stream.synchronize()
        t0 = time.perf_counter()
        s.step(k)
        stream.synchronize()
        el = time.perf_counter() - t0
        t_step += el
        chunks.append((done, k, el))
        done += k
        c = p[0:3] + p[4:7] * math.sin(p[7] * done + p[8])
        xq, nq, wq = W.sphere_quadrature(c, R, subdiv=4)
        t0 = time.perf_counter()
        F, _ = s.wall_force(xq, nq, wq)
        t_force.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        lbm.lbm_wall_force_noalloc(s.ctx, 0, xq, nq, wq, 3)
        t_force_na.append(time.perf_counter() - t0)
        series.append((done, F[0] / norm, F[1] / norm, F[2] / norm))
    _, uu, tot = s.moments()
    s.close()
    # The first call allocates the persistent workspace; report the median.
    # The rate once the inflow ramp is over (the chunks from its end on).
    after = [(k, el) for d0, k, el in chunks if d0 >= cfg["ramp_steps"]]
    after_ramp = (round(N * sum(k for k, _ in after) / sum(el for _, el in after) / 1e6, 1)
                  if after else None)
    return {"MLUPS": round(N * steps / t_step / 1e6, 1), "ms_per_step": round(t_step * 1e3 / steps, 5),
            "MLUPS_after_ramp": after_ramp, "ramp_steps": cfg["ramp_steps"],
            "variant": variant,
            "series": series, "u": uu, "mass": tot["mass"],
            "wall_force_ms_5120_points": round(1e3 * float(np.median(t_force)), 4),
            "wall_force_noalloc_ms_5120_points": round(1e3 * float(np.median(t_force_na)), 4)}


def sphere_workload(lbm, torch, args, forms=("f64", "f32", "f16")):
    """Config: D3Q27 channel 512x128x128, oscillating sphere R=16, Re=300;
    FP32 and FP16-shifted against the FP64 form of the same kernel (itself
    checked against the CPU oracle on a scaled copy in the test suite)."""
    out = {}
    ref = None
    for storage in forms:
        r = sphere_form(lbm, torch, storage, args.sphere_steps, args.sphere_sample)
        if ref is None:
            ref = r
        entry = {"MLUPS": r["MLUPS"], "ms_per_step": r["ms_per_step"],
                 "MLUPS_after_ramp": r["MLUPS_after_ramp"], "ramp_steps": r["ramp_steps"],
                 "variant": r["variant"],
                 "wall_force_ms_5120_points": r["wall_force_ms_5120_points"],
                 "wall_force_noalloc_ms_5120_points": r["wall_force_noalloc_ms_5120_points"],
                 "Cd_Cl_last": [round(v, 6) for v in r["series"][-1][1:3]]}
        if storage != "f64":
            a, b = np.array(r["series"])[:, 1:3], np.array(ref["series"])[:, 1:3]
            entry["force_coeff_max_abs_diff_vs_f64"] = float(np.max(np.abs(a - b)))
            entry["velocity_rel_l2_vs_f64"] = float(np.linalg.norm(r["u"] - ref["u"]) /
                                                    np.linalg.norm(ref["u"]))
        out[storage] = entry
    out["series_f64"] = [[int(t)] + [round(v, 6) for v in row] for t, *row in ref["series"]]
    return {"metric": "MLUPS, drag/lift vs FP64", "unit": "MLUPS",
            "config": {"workload": "D3Q27 KBC channel 512x128x128, oscillating sphere R=16 "
                                   "(amplitude 4, period 3200), Re=300, Grad boundary nodes, "
                                   "%d steps" % args.sphere_steps},
            "forms": out}


def channel3d_workload(lbm, torch, steps=200, warmup=300, dims=(512, 128, 128)):
    """D3Q27 FP32 channel without a body, three face sets: periodic, four
    walls (wall-row nodes on the y and z faces), four walls with inflow and
    outflow; MLUPS of each, to show the cost of the wall rows."""
    nx, ny, nz = dims
    N = nx * ny * nz
    cases = {"periodic": ["periodic"] * 6,
             "walls": ["periodic", "periodic", "wall", "wall", "wall", "wall"],
             "walls_inflow_outflow": ["inlet", "outlet", "wall", "wall", "wall", "wall"]}
    out = {}
    for name, faces in cases.items():
        stream = torch.cuda.Stream()
        s = lbm.Solver([dict(Q=27, nx=nx, ny=ny, nz=nz, nu=0.01, storage="f32", faces=faces,
                             u_in=(0.05, 0.0, 0.0), ramp_steps=0)], stream=stream)
        s.init_fields(np.ones(N), np.zeros((3, N)))
        v = lbm.lbm_autotune(s.ctx, os.environ.get("KBC_AUTOTUNE_CACHE"))
        s.step(warmup)
        stream.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        stream.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"MLUPS": round(N * steps / el / 1e6, 1), "ms_per_step": round(el * 1e3 / steps, 5),
                     "variant": lbm.lbm_variant_name(v)}
        s.close()
    return {"metric": "MLUPS by face set", "unit": "MLUPS",
            "config": {"workload": "D3Q27 KBC channel %dx%dx%d, FP32, no body, inflow 0.05" % dims},
            "forms": out}


def multiphase_form(lbm, torch, storage, steps, warmup, dims=(320, 250, 320), kappa=0.025,
                    kappa_w=-0.145, nu=0.05):
    """Droplet of diameter 80 hitting a non-wetting wall (Sec. III.B
    multiphase KBC, D3Q27): MLUPS and the step's achieved bandwidth over the
    bytes the three multiphase passes move per node."""
    import workloads as W

    nx, ny, nz = dims
    rho, u, info = W.droplet_impact(nx, ny, nz)
    stream = torch.cuda.Stream()
    s = lbm.Solver([dict(Q=27, nx=nx, ny=ny, nz=nz, nu=nu, storage=storage,
                         faces=info["faces"])], stream=stream)
    s.set_multiphase(kappa, kappa_w)
    s.init_fields(rho, u)
    s.step(warmup)
    stream.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    s.step(steps)
    ev1.record(stream)
    stream.synchronize()
    t1 = time.perf_counter()
    r, uu, tot = s.moments()
    s.close()
    N = nx * ny * nz
    ms = (t1 - t0) * 1e3 / steps
    kms = ev0.elapsed_time(ev1) / steps
    es = 8 if storage == "f64" else 4
    # Populations read and written twice (stream pass, collision pass), the
    # density and phi fields written once and read once, the Laplacian
    # field written and read once.
    moved = 4 * 27 * es + 6 * es
    return {"MLUPS": round(N / (ms * 1e3), 1), "ms_per_step": round(ms, 5),
            "event_ms_per_step": round(kms, 5), "bytes_per_lattice_update": moved,
            "achieved_GBs": round(moved * N / (kms * 1e-3) / 1e9, 1),
            "frac_of_hbm_peak": round(moved * N / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "rho_max": round(float(r.max()), 4), "rho_min": round(float(r[r > 0].min()), 5),
            "mass": tot["mass"], "gamma_mean": tot.get("gamma_mean")}


def multiphase_workload(lbm, torch, args):
    out = {storage: multiphase_form(lbm, torch, storage, args.mp_steps, 20)
           for storage in ("f32", "f64")}
    return {"metric": "MLUPS, multiphase KBC", "unit": "MLUPS",
            "config": {"workload": "D3Q27 multiphase KBC droplet impact, 320x250x320, droplet "
                                   "diameter 80, kappa 0.025, kappa_w -0.145 (non-wetting), "
                                   "walls at -y/+y, %d steps" % args.mp_steps},
            "forms": out}


def fsi3_workload(lbm, torch, args):
    """FSI3 (Sec. III.A.1) at uniform resolution D = 40: the D2Q9 KBC fluid
    in FP64 on the GPU coupled every step with the FEM beam (lbm_fsi_step).
    Reports the tip displacement of the flag (point A, mid-height of the free
    end) over the last window: mean and amplitude of u_x and u_y in metres and
    their frequencies in Hz, beside the values the paper prints."""
    import workloads as W

    cfg = W.fsi3()
    nx, ny = cfg["nx"], cfg["ny"]
    s = lbm.Solver([dict(Q=9, nx=nx, ny=ny, nz=1, nu=cfg["nu"], storage="f64",
                         faces=cfg["faces"], u_in=(cfg["u_mean"], 0.0, 0.0), inlet_profile=1,
                         ramp_steps=cfg["ramp_steps"])])
    N = nx * ny
    s.init_fields(np.ones(N), np.zeros((2, N)))
    beam = lbm.Beam(*cfg["beam"])
    cp = lbm.Coupling(s, beam, cfg["arc"])
    sps = cfg["steps_per_second"]
    total = int(round(args.fsi_seconds * sps))
    chunk = sps // 10
    tips, t0 = [], time.perf_counter()
    done = 0
    while done < total:
        k = min(chunk, total - done)
        _, tip = cp.step(k)
        tips.append(tip)
        done += k
        print("fsi3: t = %.2f s, tip (%.5f, %.5f) m, %.2f ms per coupled step"
              % (done / sps, tip[-1, 0] * cfg["dx"], tip[-1, 1] * cfg["dx"],
                 (time.perf_counter() - t0) * 1e3 / done), file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    tip = np.concatenate(tips) * cfg["dx"]
    out = {"metric": "FSI3 flag tip displacement (mean +- amplitude) and frequency",
           "config": {"workload": "FSI3, D2Q9 KBC FP64 1000x164 (D = 40) coupled every step "
                                  "with a 20 x 2 nine-node SVK beam, %.1f s simulated" % args.fsi_seconds},
           "ms_per_coupled_step": round(el * 1e3 / total, 4),
           "paper": {"ux": [-0.00268, 0.00257], "uy": [0.00145, 0.03380], "fx_Hz": 11, "fy_Hz": 5.5}}
    w = tip[-int(args.fsi_window * sps):] if args.fsi_window * sps < len(tip) else tip
    res = {}
    for a, name in ((0, "ux"), (1, "uy")):
        x = w[:, a]
        m, amp = (x.max() + x.min()) / 2, (x.max() - x.min()) / 2
        y = x - m
        up = np.where((y[:-1] < 0) & (y[1:] >= 0))[0]
        f = (len(up) - 1) / ((up[-1] - up[0]) / sps) if len(up) > 1 else None
        res[name] = [round(float(m), 6), round(float(amp), 6)]
        res["f" + name[-1] + "_Hz"] = round(f, 3) if f else None
    out["present"] = res
    out["tip_series_every_100_steps"] = [[round(float(v), 7) for v in r] for r in tip[::100]]
    return out


def tg512_workload(lbm, torch, args):
    """Config: D3Q27 TG 512^3, Re=1600: MLUPS and HBM fraction per storage form,
    velocity error of each against the FP64 form at steps 100 and 1000."""
    import workloads as W

    n = 512
    rho, u, nu = W.taylor_green_3d(n)
    forms = {}
    for storage in ("f32", "f16", "bf16"):
        m, ms, k, info = time_form(lbm, torch, n, storage, rho, u, nu, args.steps, args.warmup)
        a = info["bytes_per_update"] * n ** 3 / (k * 1e-3) / 1e9
        forms[storage] = {"MLUPS": round(m, 1), "ms_per_step": round(ms, 5),
                          "achieved_GBs": round(a, 1), "frac": round(a / HBM_PEAK_GBS, 4),
                          "variant": info["variant"]}
    marks = (100, 1000)
    fields = {}
    for storage in ("f64", "f32", "f16", "bf16"):
        s = lbm.Solver([dict(Q=27, nx=n, ny=n, nz=n, nu=nu, storage=storage)])
        s.init_fields(rho, u)
        done = 0
        for mk in marks:
            s.step(mk - done)
            done = mk
            _, uu, _ = s.moments()
            fields[(storage, mk)] = uu if storage == "f64" else \
                float(np.linalg.norm(uu - fields[("f64", mk)]) / np.linalg.norm(fields[("f64", mk)]))
        s.close()
    for storage in ("f32", "f16", "bf16"):
        forms[storage]["velocity_rel_l2_vs_f64"] = {str(mk): fields[(storage, mk)] for mk in marks}
    return {"metric": "MLUPS and % HBM roofline per storage form, error vs FP64", "unit": "MLUPS",
            "config": {"workload": "D3Q27 KBC Taylor-Green 512^3 periodic, Re=1600, Ma=0.1"},
            "forms": forms}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(seconds=12.0, one_thread_seconds=6.0, sphere_seconds=20.0, sphere_steps=None):
    """The oracle as it stands, on bounded samples of the workloads: the
    headline Taylor-Green case on 64^3 with all host threads (the reported
    value) and with one thread; the D2Q9 Taylor-Green 64^2 run of 500 steps in
    full; the sphere channel 512x128x128 for as many steps as fit in
    sphere_seconds (or exactly sphere_steps steps)."""
    import math

    import oracle
    import workloads as W

    n = 64
    rho, u, nu = W.taylor_green_3d(n)

    def run(threads, budget):
        d = oracle.Domain(27, n, n, n, nu)
        d.init_fields(rho, u)
        d.set_threads(threads)
        d.step(1)
        steps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget:
            d.step(1)
            steps += 1
        el = time.perf_counter() - t0
        return n ** 3 * steps / el / 1e6, steps, el

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    v, steps, el = run(threads, seconds)
    v1, steps1, el1 = run(1, one_thread_seconds)
    samples = {}
    # D2Q9 Taylor-Green 64^2, FP64, 500 steps, in full.
    r2, u2 = W.taylor_green_2d(64, 0.02)
    d = oracle.Domain(9, 64, 64, 1, 0.01)
    d.init_fields(r2, u2)
    t0 = time.perf_counter()
    d.step(500)
    el2 = time.perf_counter() - t0
    samples["d2q9_tg_64x64_500_steps"] = {"MLUPS": 64 * 64 * 500 / el2 / 1e6, "seconds": el2}
    # Sphere channel, bounded.
    cfg = W.sphere_channel()
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    N = nx * ny * nz
    d = oracle.Domain(27, nx, ny, nz, cfg["nu"], faces=cfg["faces"], u_in=cfg["u_in"],
                      ramp_steps=cfg["ramp_steps"])
    d.init_fields(np.ones(N), np.zeros((3, N)))
    d.set_body(*cfg["body"])
    d.step(1)
    k = 0
    t0 = time.perf_counter()
    while (sphere_steps is not None and k < sphere_steps) or \
            (sphere_steps is None and time.perf_counter() - t0 < sphere_seconds):
        d.step(1)
        k += 1
    el3 = time.perf_counter() - t0
    del d
    samples["sphere_channel_512x128x128"] = {"MLUPS": N * k / el3 / 1e6, "steps": k,
                                             "seconds": el3}
    return {"value": v, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "D3Q27 KBC Taylor-Green 64^3 periodic (same Re, Ma, perturbation), "
                      "FP64, %d steps in %.1f s" % (steps, el),
            "one_thread": {"value": v1, "sample": "%d steps in %.1f s" % (steps1, el1)},
            "other_samples_all_threads": samples,
            "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--error-steps", type=int, default=100)
    ap.add_argument("--batched-steps", type=int, default=1000)
    ap.add_argument("--batched-warmup", type=int, default=500)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--variant", default=None, help="bulk-kernel variant (default: autotune)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "f64"])
    ap.add_argument("--mp-steps", type=int, default=200)
    ap.add_argument("--fsi-seconds", type=float, default=8.0)
    ap.add_argument("--fsi-window", type=float, default=2.0)
    ap.add_argument("--workload", default="tg256",
                    choices=["tg256", "tg512", "sphere", "batched", "multiphase", "fsi3",
                             "channel3d"],
                    help="tg256 is the headline line; the others print their own line")
    ap.add_argument("--sphere-steps", type=int, default=1200)
    ap.add_argument("--sphere-sample", type=int, default=200)
    ap.add_argument("--cpu-sphere-steps", type=int, default=None,
                    help="oracle steps of the sphere channel in the CPU baseline "
                         "(default: as many as fit in 20 s)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); the "
              "multi-GPU decomposition is a design, not an implementation." % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch

    import workloads as W
    from paper_1710_02375_amd import lbm

    if args.workload == "sphere":
        print(json.dumps(sphere_workload(lbm, torch, args)), flush=True)
        return
    if args.workload == "batched":
        r = batched_form(lbm, torch, args.batched_steps, args.batched_warmup)
        print(json.dumps({"metric": "aggregate MLUPS, batched vs per-instance launches",
                          "unit": "MLUPS", "config": {"workload": "64 D2Q9 KBC flap channels "
                                                      "(seed 2375), FP32"}, "forms": r}),
              flush=True)
        return
    if args.workload == "fsi3":
        print(json.dumps(fsi3_workload(lbm, torch, args)), flush=True)
        return
    if args.workload == "channel3d":
        print(json.dumps(channel3d_workload(lbm, torch)), flush=True)
        return
    if args.workload == "multiphase":
        print(json.dumps(multiphase_workload(lbm, torch, args)), flush=True)
        return
    if args.workload == "tg512":
        print(json.dumps(tg512_workload(lbm, torch, args)), flush=True)
        return
    n = args.n
    rho, u, nu = W.taylor_green_3d(n)
    mlups, ms, kms, info = time_form(lbm, torch, n, args.storage, rho, u, nu, args.steps,
                                     args.warmup, args.variant)
    bytes_per_lup = info["bytes_per_update"]
    achieved = bytes_per_lup * n ** 3 / (kms * 1e-3) / 1e9
    traffic = read_traffic(n ** 3, info["variant"])
    result = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": "D3Q27 KBC Taylor-Green %d^3 periodic, Re=1600, Ma=0.1, "
                               "1e-4 seeded perturbation, %s" % (n, FORM_TEXT[args.storage]),
                   "nodes": n ** 3, "bytes_per_lattice_update": bytes_per_lup},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic if args.storage == "f32" else None,
                     "kernel": "kbc::k_bulk<27, %s> (%s)" % (args.storage.upper(), info["variant"]),
                     "kernel_ms": round(kms, 5)},
    }
    # Measured streaming ceiling beside the published peak.
    copy_gbs, copy_name = copy_ceiling()
    result["roofline"]["stream_ceiling_GBs"] = round(copy_gbs, 1)
    result["roofline"]["stream_ceiling_kernel"] = "torch " + copy_name + ", 2 GiB"
    result["roofline"]["frac_of_stream_ceiling"] = round(achieved / copy_gbs, 4)
    if not args.no_variants:
        var = {}
        for storage in ("f16", "bf16"):
            m2, ms2, k2, i2 = time_form(lbm, torch, n, storage, rho, u, nu, args.steps,
                                        args.warmup)
            a2 = i2["bytes_per_update"] * n ** 3 / (k2 * 1e-3) / 1e9
            var[storage + "_shifted"] = {"MLUPS": round(m2, 1), "ms_per_step": round(ms2, 5),
                                         "achieved_GBs": round(a2, 1),
                                         "frac": round(a2 / HBM_PEAK_GBS, 4),
                                         "bytes_per_lattice_update": i2["bytes_per_update"],
                                         "variant": i2["variant"]}
        var["batched_d2q9_flap_channels_f32"] = batched_form(lbm, torch, args.batched_steps,
                                                             args.batched_warmup)
        sph = sphere_workload(lbm, torch, args)
        var["sphere_channel"] = {"config": sph["config"], "forms": sph["forms"]}
        timed = {args.storage: info["variant"], "f16": var["f16_shifted"]["variant"],
                 "bf16": var["bf16_shifted"]["variant"]}
        err = error_vs_f64(lbm, n, rho, u, nu, args.error_steps, timed)
        var["velocity_rel_l2_vs_f64_at_step_%d" % args.error_steps] = err
        var["velocity_rel_l2_variants"] = timed
        result["variants"] = var
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(sphere_steps=args.cpu_sphere_steps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

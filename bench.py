"""Benchmark of the FSLBM hot path on one MI355X.

Default workload (the line's value, roofline and cpu_baseline): the HBM
roofline probe, a gas bubble of radius 64 in a liquid-filled periodic 512^3
lattice (99.2 % of the cells fluid), LSQR curvature, sigma 1e-3, tau 0.8,
FP32 storage and arithmetic. One step is one time step of the whole hot path
(stream-collide with mass exchange, conversions, interface-list update,
obstacle fill, curvature). Inputs are synthetic: exact sphere volume
fractions.

Extra keys of the same JSON line: the probe with F16 and BF16 storage of
f - w_q; the 512^3 oscillating droplet (ellipsoid 96/80/80, sigma 1e-3,
tau 0.55) over 10,000 steps per storage form; the static-droplet sweep of
eight 128^3 lattices; the 256 x 256 x 128 sessile droplets; the adjoint
window's cost; the FP64 CPU oracle on one core and on all cores.
"""
from __future__ import annotations

import argparse
import functools
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D3Q19 FSLBM MLUPS + %HBM roofline (FP32 vs FP16 store); adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
STREAM_SRCS = [os.path.join(ROOT, "paper_1509_07691_amd", "csrc", f) for f in ("fslbm_stream.hpp", "fslbm_device.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stream_collide_traffic.json")
FBYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
RBYTES = {"f64": 8, "f32": 4, "f16": 4, "bf16": 4}


SWEEP_RADIUS = 32.0  # droplet of the droplet sweep


@functools.lru_cache(maxsize=3)
def workload_runs(name):
    """List of (label, fill, obstacle, params) of one workload (cached: the
    512^3 inputs take seconds to build)."""
    from paper_1509_07691_amd import inputs as I

    if name == "droplet-sweep":
        fill, obst = I.droplet(128, SWEEP_RADIUS, noise=1e-6, seed=0)
        runs = []
        for model in ("fd", "lsqr"):
            for tau in (0.6, 1.0):
                for sigma in (1e-4, 1e-3):
                    runs.append((f"{model}-tau{tau}-sigma{sigma}", fill, obst,
                                 dict(curv_model=model, tau=tau, sigma=sigma)))
        desc = ("static droplet R=32 in periodic 128^3, 8 runs (tau 0.6/1.0 x sigma 1e-4/1e-3 x FD/LSQR) "
                "stepped together")
        return runs, desc
    if name == "ellipsoid":
        fill, obst = I.ellipsoid_droplet(512, (96, 80, 80), noise=1e-6, seed=0)
        return [("ellipsoid", fill, obst, dict(curv_model="lsqr", tau=0.55, sigma=1e-3))], \
            "oscillating droplet, ellipsoid 96/80/80 in periodic 512^3, LSQR"
    if name == "bubble-probe":
        fill, obst = I.bubble_probe(512, 64.0)
        return [("bubble", fill, obst, dict(curv_model="lsqr", tau=0.8, sigma=1e-3))], \
            ("roofline probe: gas bubble R=64 in a liquid-filled periodic 512^3 lattice (99.2 % fluid cells), "
             "LSQR, sigma 1e-3, tau 0.8")
    raise SystemExit(f"unknown workload {name}")


def fluid_box_cells(flags):
    """Cells of the bounding box of the fluid (liquid and interface) cells,
    the range the stream-collide kernel reads flags over."""
    fl = (flags == 1) | (flags == 2)
    if not fl.any():
        return 0
    ext = [np.flatnonzero(fl.any(axis=a)) for a in ((1, 2), (0, 2), (0, 1))]
    return int(np.prod([e[-1] - e[0] + 1 for e in ext]))


def sc_bytes(flags, prec):
    """Algorithmic bytes of one stream-collide launch: 19 reads + 19 writes
    of a distribution per fluid cell, one flag byte per cell of the fluid
    bounding box (the range the kernel covers), and at interface cells m
    (read, write), rho (write), K and phi (read) and one status byte.
    Returns (liquid part incl. flags, interface part, liquid cells,
    interface cells, box cells)."""
    nl = int((flags == 1).sum())
    ni = int((flags == 2).sum())
    nbox = fluid_box_cells(flags)
    return 38 * FBYTES[prec] * nl + nbox, ni * (38 * FBYTES[prec] + 5 * RBYTES[prec] + 1), nl, ni, nbox


def stored_traffic(workload, precision):
    """The counted traffic record if it was taken on this workload and
    storage precision with the current stream-collide sources, else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    same = (rec.get("source_sha256") == stream_source_hash() and rec.get("workload") == workload
            and rec.get("precision", "f32") == precision)
    return rec if same else None


def stream_source_hash():
    h = hashlib.sha256()
    for f in STREAM_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def traffic_from_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, workload_note, precision):
    """HBM bytes per stream-collide launch from rocprofv3 FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for a plain copy of 2^28 floats (1 GiB read, 1 GiB written)."""
    import csv

    def mean_kib(path, kernel_part):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if kernel_part in r["Kernel_Name"]]
        return sum(vals) / len(vals), len(vals)

    f_kib, nf = mean_kib(fetch_csv, "k_stream_collide<")
    w_kib, nw = mean_kib(write_csv, "k_stream_collide<")
    cf_kib, _ = mean_kib(copy_fetch_csv, "AUnaryFunctor")
    cw_kib, _ = mean_kib(copy_write_csv, "AUnaryFunctor")
    gib_kib = (4 << 28) / 1024.0
    f_scale, w_scale = gib_kib / cf_kib, gib_kib / cw_kib
    rec = {"source_sha256": stream_source_hash(), "workload": workload_note, "precision": precision,
           "fetch_kib_per_launch": f_kib, "write_kib_per_launch": w_kib, "dispatches": [nf, nw],
           "copy_fetch_kib": cf_kib, "copy_write_kib": cw_kib, "fetch_scale": f_scale, "write_scale": w_scale,
           "bytes_per_launch": int(1024 * (f_kib * f_scale + w_kib * w_scale))}
    return rec


PROBE_SAMPLE = (128, 16.0)  # the probe scaled to 128^3: bubble R = 16, the same cell mix


def _oracle_rate(budget_s):
    """One process: the FP64 oracle on the 128^3 downscale of the probe
    (LSQR, sigma 1e-3, tau 0.8), stepped until budget_s has elapsed.
    Returns (cells, steps, seconds)."""
    import oracle as O
    from paper_1509_07691_amd import inputs as I

    n, R = PROBE_SAMPLE
    fill, obst = I.bubble_probe(n, R)
    orc = O.Oracle(fill, obst, sigma=1e-3, tau=0.8, curv_model=O.CURV_LSQR)
    steps = 0
    t0 = time.perf_counter()
    while True:
        orc.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            return fill.size, steps, el


def cpu_baseline(budget_s):
    """The FP64 oracle as it stands (plain C, one thread per process) on a
    bounded sample of the probe: its 128^3 downscale, on one core and then
    as one process per core of this host, each stepping for budget_s. The
    rate is MLUPS over all cells of the sample."""
    import multiprocessing as mp

    cores = len(os.sched_getaffinity(0))
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ctx = mp.get_context("spawn")  # fresh interpreters: nothing of this process's GPU state
    with ctx.Pool(1) as pool:
        (c1, s1, e1), = pool.map(_oracle_rate, [budget_s])
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_rate, [budget_s] * cores)
    one = c1 * s1 / e1 / 1e6
    allc = sum(c * st / el for c, st, el in res) / 1e6
    n, R = PROBE_SAMPLE
    return {"value": round(allc, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"the probe scaled to {n}^3 (gas bubble R={R:g} in liquid, LSQR, FP64), one oracle process "
                      f"per core for {budget_s:g} s each ({sum(r[1] for r in res)} steps in all); MLUPS over all "
                      f"cells of the sample",
            "single_core": {"value": round(one, 3), "unit": "MLUPS", "steps": s1, "seconds": round(e1, 2)},
            "host": {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cores": cores}}


def adjoint_cost(dev, stream, steps, K, precision, fd_check=True):
    """Cost of the differentiation window (frozen cell types, checkpoints
    every K steps, hand-written adjoint) on a sessile drop: hemisphere R=24
    on the wall k=0 of a 128^3 lattice (walls k=0 and k=127, periodic x, y),
    LSQR curvature with the wetting condition, sigma 1e-3, tau 0.8, theta
    90 deg. Loss: squared distance of phi_T to the window's result at theta
    70 deg, sigma 8e-4. Times T plain steps, the checkpointed window and the
    reverse sweep (recompute + adjoint) on the same stream."""
    import torch
    from paper_1509_07691_amd import inputs as I
    from paper_1509_07691_amd.fslbm import Lattice

    fill, obst = I.sessile_droplet(128, 128, 128, 24.0, noise=1e-6, seed=1)
    prm = dict(curv_model="lsqr", sigma=1e-3, tau=0.8, theta=math.pi / 2)
    with torch.cuda.stream(stream):
        lat = Lattice(fill, obst, precision=precision, device=dev, stream=stream, **prm)
    start = lat.save_state()
    keep = torch.tensor((obst == 0).astype(np.float64), device=dev)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    lat.step(20)  # warm-up of the plain step
    lat.load_state(start)
    t_plain, _ = timed(lambda: lat.step(steps))
    lat.load_state(start)
    lat.set_params(sigma=8e-4, theta=math.radians(70.0))
    lat.adjoint_forward(steps, K)
    target = lat.fill_tensor()
    lat.load_state(start)
    lat.set_params(sigma=1e-3, theta=math.pi / 2)
    t_fwd, _ = timed(lambda: lat.adjoint_forward(steps, K))
    inside_steps, fill_events, unconverted_steps = lat.adjoint_status()
    phi = lat.fill_tensor()
    dphi = 2.0 * (phi - target) * keep
    loss = float((((phi - target) * keep) ** 2).sum())
    ifc = torch.tensor(lat.flags() == 2, device=dev)
    phi_range = [float(phi[ifc].min()), float(phi[ifc].max())]
    t_bwd, (d0, ds, dt) = timed(lambda: lat.adjoint_backward(dphi))
    ws_gb = lat._adj_ws.numel() / 1e9
    lat.close()
    del lat, start
    torch.cuda.empty_cache()
    valid = fill_events == 0
    return {"workload": "sessile drop R=24 on the wall of a 128^3 lattice, LSQR + wetting, frozen-topology "
                        f"window of {steps} steps, checkpoints every {K}",
            "precision": precision, "steps": steps, "K": K,
            "plain_ms_per_step": round(1e3 * t_plain / steps, 4),
            "window_forward_ms_per_step": round(1e3 * t_fwd / steps, 4),
            "backward_ms_per_step": round(1e3 * t_bwd / steps, 4),
            "backward_over_forward": round(t_bwd / t_plain, 3),
            "cost_ratio": round((t_fwd + t_bwd) / t_plain, 3),
            "window_inside_steps": inside_steps, "window_fill_events": fill_events,
            "window_unconverted_steps": unconverted_steps,
            "loss": loss if valid else None, "dL_dsigma": ds if valid else None, "dL_dtheta": dt if valid else None,
            "dL_dphi0_norm": float(torch.linalg.vector_norm(d0)) if valid else None,
            "interface_fill_range_T": phi_range,
            "workspace_GB": round(ws_gb, 2),
            "note": "the cost is measured on the whole window; its gradients are reported only when every interface "
                    "fill stays inside (0, 1) (window_fill_events == 0): otherwise the frozen step is not smooth "
                    "along the trajectory and they are null",
            "fd_check": adjoint_fd_check(dev, 64, 12.0, steps, K) if fd_check else None,
            "oracle_check": adjoint_oracle_check(dev) if fd_check else None}


def adjoint_fd_check(dev, n, R, steps, K):
    """The gradients of the differentiation workload on the n^3 downscale
    (sessile drop R on the wall, same parameters, window and loss) in FP64
    against central differences of the same forward window, extrapolated
    over the step h and 2h: dL/dsigma (h = 1e-4 sigma), dL/dtheta (1e-4 rad)
    and <dL/dphi_0, v> (1e-5, v seeded on interface cells)."""
    from paper_1509_07691_amd import inputs as I
    from paper_1509_07691_amd.fslbm import Lattice

    fill, obst = I.sessile_droplet(n, n, n, R, noise=1e-6, seed=1)
    sigma, theta = 1e-3, math.pi / 2
    keep = (obst == 0).astype(float)
    g = Lattice(fill, obst, precision="f64", device=dev, curv_model="lsqr", sigma=sigma, tau=0.8, theta=theta)
    start = g.save_state()
    phi0 = g.fill()
    ifc = g.flags() == 2
    v = np.random.default_rng(3).uniform(-1.0, 1.0, fill.shape) * (ifc & (phi0 > 1e-3) & (phi0 < 1 - 1e-3))
    g.set_params(sigma=8e-4, theta=math.radians(70.0))
    g.adjoint_forward(steps, K)
    target = g.fill()

    def L(s=sigma, t=theta, x=0.0):
        g.load_state(start)
        if x:
            g.set_interface_fill(phi0 + x * v)
        g.set_params(sigma=s, theta=t)
        g.adjoint_forward(steps, K)
        return float((((g.fill() - target) * keep) ** 2).sum())

    def rich(f, x, e):
        return (4 * (f(x + e) - f(x - e)) / (2 * e) - (f(x + 2 * e) - f(x - 2 * e)) / (4 * e)) / 3

    fd = {"sigma": rich(lambda x: L(s=x), sigma, 1e-4 * sigma), "theta": rich(lambda x: L(t=x), theta, 1e-4),
          "phi0_dir": rich(lambda x: L(x=x), 0.0, 1e-5)}
    L()
    phi = g.fill()
    rng = [float(phi[ifc].min()), float(phi[ifc].max())]
    d0, ds, dt = g.adjoint_backward(2.0 * (phi - target) * keep)
    adj = {"sigma": ds, "theta": dt, "phi0_dir": float((d0.cpu().numpy() * v).sum())}
    g.close()
    return {"workload": f"the same drop scaled to {n}^3 (R={R:g}), window of {steps} steps, checkpoints every {K}, FP64",
            "interface_fill_range_T": rng,
            **{k: {"adjoint": adj[k], "fd": fd[k], "rel": abs(adj[k] - fd[k]) / abs(fd[k])} for k in fd}}


GOLDEN_ADJ = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "adjoint_c4_oracle.json")


def adjoint_oracle_check(dev, precisions=("f64", "f32")):
    """The differentiation workload at its configured size against the FP64
    oracle's stored values (tests/golden/adjoint_c4_oracle.json, written by
    tests/golden/make_adjoint_c4_reference.py from the oracle alone): the
    window lengths T_inside (every interface fill inside (0, 1)) and
    T_unconverted (no cell that the free method would convert), and for the
    stored windows the relative errors of dL/dsigma, dL/dtheta and
    <dL/dphi_0, v> against the tangent-linear oracle (same loss as the cost
    measurement). Within T_inside the oracle's central differences agree
    with its tangent-linear values; beyond it the loss is only piecewise
    smooth along the trajectory."""
    from paper_1509_07691_amd import inputs as I
    from paper_1509_07691_amd.fslbm import Lattice

    if not os.path.exists(GOLDEN_ADJ):
        return None
    ref = json.load(open(GOLDEN_ADJ))
    fill, obst = I.sessile_droplet(128, 128, 128, 24.0, noise=1e-6, seed=1)
    keep = (obst == 0).astype(float)
    out = {"oracle_T_inside": ref["T_inside"], "oracle_T_unconverted": ref["T_unconverted"], "windows": []}
    for win in ref["windows"]:
        T = win["T"]
        row = {"T": T, "tangent_linear": win["tangent_linear"], "oracle_central_differences": win["central_differences"]}
        for prec in precisions:
            g = Lattice(fill, obst, precision=prec, device=dev, curv_model="lsqr", sigma=1e-3, tau=0.8,
                        theta=math.pi / 2)
            start = g.save_state()
            ifc = g.flags() == 2
            v = np.random.default_rng(3).uniform(-1.0, 1.0, fill.shape) * (ifc & (fill > 1e-3) & (fill < 1 - 1e-3))
            g.set_params(sigma=8e-4, theta=math.radians(70.0))
            g.adjoint_forward(T, 100)
            target = g.fill()
            g.load_state(start)
            g.set_params(sigma=1e-3, theta=math.pi / 2)
            g.adjoint_forward(T, 100)
            inside, events, unconverted = g.adjoint_status()
            d0, ds, dt = g.adjoint_backward(2.0 * (g.fill() - target) * keep)
            adj = {"sigma": ds, "theta": dt, "phi0_dir": float((d0.cpu().numpy() * v).sum())}
            g.close()
            row[prec] = {"window_inside_steps": inside, "window_unconverted_steps": unconverted,
                         "rel_err_vs_tangent_linear": {k: abs(adj[k] - t) / abs(t) for k, t in win["tangent_linear"].items()}}
        out["windows"].append(row)
    return out


def advection_table(dev, precision):
    """Pure advection test of Sec. III.A (sigma = 0, f = feq(1, u0)): a gas
    bubble of diameter d in a periodic 3d x 2d x 2d box translated by d along
    x, for d = 10, 20, 40, 80 under convective (u0 = 0.05) and diffusive
    (u0 = 0.05 * 10 / d) scaling; L1 and L2 errors of phi."""
    import torch
    from paper_1509_07691_amd import inputs as I
    from paper_1509_07691_amd.fslbm import Lattice

    rows = []
    for d in (10, 20, 40, 80):
        fill, obst = I.advected_bubble(d)
        for scaling, u0 in (("convective", 0.05), ("diffusive", 0.05 * 10 / d)):
            if scaling == "diffusive" and d == 10:
                rows.append(dict(rows[-1], scaling="diffusive"))
                continue
            lat = Lattice(fill, obst, precision=precision, curv_model="fd", sigma=0.0, tau=1.0, device=dev)
            u = np.zeros((3,) + fill.shape)
            u[0] = u0
            lat.set_equilibrium(1.0, u)
            T = int(round(d / u0))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat.step(T)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            l1, l2 = I.advection_errors(fill, lat.fill(), d)
            rows.append({"d": d, "scaling": scaling, "u0": u0, "steps": T, "L1": round(l1, 5), "L2": round(l2, 5),
                         "ms_per_step": round(1e3 * el / T, 4)})
            print(f"# advection d={d} {scaling}: L1 {l1:.4f} L2 {l2:.4f}", file=sys.stderr, flush=True)
            lat.close()
            torch.cuda.empty_cache()
    return rows


# Printed values of the equilibrium-bubble study (Sec. III.A.1, Figs.
# spuriousConvergence and curvatureError / curvatureStdev) after 500,000
# steps at dt = 1e-4, physical units: max and average spurious speed,
# L2(kappa) and STDEV(kappa).
PAPER_LAPLACE = {
    ("fd", 48): (2.8325e-2, 3.585375e-4, 0.0902448, 1.0521024),
    ("fd", 96): (2.1301458e-3, 4.27811458e-6, 0.0490684, 0.343152),
    ("fd", 144): (8.639653e-4, 7.64131944e-7, 0.016254, 0.127167408),
    ("fd", 192): (2.749667e-4, 4.334734375e-7, 0.0155673, 0.123288192),
    ("lsqr", 48): (2.3191875e-10, 1.63838542e-11, 0.0180768, 2.31408e-7),
    ("lsqr", 96): (1.51490625e-10, 9.93127083e-12, 0.00421798, 3.1994304e-7),
    ("lsqr", 144): (1.98145139e-11, 7.88409722e-13, 0.00177479, 8.449776e-8),
    ("lsqr", 192): (7.79395833e-12, 4.72019271e-13, 0.000991554, 8.448192e-8),
    ("tr", 48): (4.886375e-11, 4.29270833e-12, 0.00773397, 2.765856e-7),
    ("tr", 96): (1.03624583e-10, 5.86341667e-12, 0.00617829, 1.71e-7),
    ("tr", 144): (2.20902778e-11, 1.50839583e-12, 0.00519107, 1.19405232e-7),
    ("tr", 192): (1.5055625e-11, 1.87496875e-12, 0.00517137, 1.69e-7),
}


def bubble_measures(lat, n, dt, u0=0.0):
    """Spurious speed (max, average over fluid cells; deviation from the
    background velocity u0 along x) and the curvature error of the bubble
    surface, all in the physical units of the unit cube: speed u dx/dt,
    kappa = -K/(2 dx) with K the library's curvature (-2/R_L for a bubble),
    L2(kappa) = sqrt(sum (kappa - 1/R)^2 / sum (1/R)^2) and STDEV(kappa)
    over the interface cells."""
    from paper_1509_07691_amd.fslbm import FSLBM_LIQUID, FSLBM_INTERFACE

    dx = 1.0 / n
    fl = lat.flags()
    fluid = (fl == FSLBM_LIQUID) | (fl == FSLBM_INTERFACE)
    u = lat.velocity()
    u[0] -= u0
    speed = np.sqrt((u ** 2).sum(0))[fluid] * dx / dt
    kap = -lat.curvature()[fl == FSLBM_INTERFACE] / (2.0 * dx)
    k0 = 8.0  # 1/R with R = 0.125
    l2 = float(np.sqrt(((kap - k0) ** 2).sum() / (k0 * k0 * kap.size)))
    return float(speed.max()), float(speed.mean()), l2, float(kap.std())


def gas_link_kappa_stdev(lat, n):
    """STDEV(kappa) over the interface cells that have a gas neighbour along
    one of the D3Q19 directions, i.e. the cells whose curvature enters the
    pressure boundary condition."""
    from paper_1509_07691_amd.fslbm import FSLBM_GAS, FSLBM_INTERFACE

    fl = lat.flags()
    gas = fl == FSLBM_GAS
    near = np.zeros_like(gas)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx_ in (-1, 0, 1):
                if 0 < abs(dz) + abs(dy) + abs(dx_) <= 2:
                    near |= np.roll(gas, (dz, dy, dx_), axis=(0, 1, 2))
    sel = (fl == FSLBM_INTERFACE) & near
    kap = -lat.curvature()[sel] * n / 2.0
    return float(kap.std()), int(sel.sum()), int((fl == FSLBM_INTERFACE).sum())


def laplace_table(dev, resolutions, steps, models=("fd", "lsqr"), precision="f64", eps_c=None):
    """Equilibrium bubble of Sec. III.A.1 with the bubble model: dx = 1/n,
    dt = 1e-4, no-slip walls at z = 0 and 1; spurious speeds at log-spaced
    times and the curvature error at the end, beside the printed values."""
    import torch
    from paper_1509_07691_amd import inputs as I
    from paper_1509_07691_amd.fslbm import Lattice

    dt = 1e-4
    rows = []
    for n in resolutions:
        fill, obst = I.laplace_bubble(n)
        tau, sig = I.renardy_units(n, dt)
        for model in models:
            lat = Lattice(fill, obst, precision=precision, curv_model=model, sigma=sig, tau=tau, bubble=True,
                          eps_c=eps_c, device=dev)
            hist, t = [], 0
            # a progress line at least every 50k steps
            marks = sorted(set([m for m in (1000, 2000, 5000, 10000, 20000) if m < steps]
                               + list(range(50000, steps, 50000)) + [steps]))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for m in marks:
                lat.step(m - t)
                t = m
                umax, uavg, l2, sd = bubble_measures(lat, n, dt)
                hist.append([t, umax, uavg])
                print(f"# laplace n={n} {model} t={t}: max|u| {umax:.3e} avg {uavg:.3e} L2(k) {l2:.4g} "
                      f"std {sd:.3e} rho_g {lat.gas_density():.9f}", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            paper = PAPER_LAPLACE.get((model, n))
            sd_gl, n_gl, n_if = gas_link_kappa_stdev(lat, n)
            rows.append({"n": n, "model": model, "tau": round(tau, 4), "sigma_L": sig, "steps": steps, "eps_c": eps_c,
                         "max_u": umax, "avg_u": uavg, "L2_kappa": l2, "stdev_kappa": sd,
                         "stdev_kappa_gas_link_cells": sd_gl, "gas_link_cells": n_gl, "interface_cells": n_if,
                         "rho_gas_t": lat.gas_density(), "history": hist,
                         "paper_500k": None if paper is None else dict(zip(("max_u", "avg_u", "L2_kappa",
                                                                               "stdev_kappa"), paper)),
                         "ms_per_step_incl_readout": round(1e3 * el / steps, 4)})
            lat.close()
            torch.cuda.empty_cache()
    return rows


def moving_bubble_table(dev, resolutions, models=("fd", "lsqr"), precision="f64", samples=10, eps_c=None):
    """Moving frame of Sec. III.A.2: the equilibrium bubble with a uniform
    background velocity u0 = 1 along x, traversing the periodic unit cube
    once (T = n / u0_L steps, u0_L = dt/dx) under diffusive scaling
    dt = 1e-4 (48/n)^2; L2(kappa) and the spurious speed relative to u0
    over time. The box is periodic in z as well (walls at rest would not
    be a moving frame)."""
    import torch
    from paper_1509_07691_amd import inputs as I
    from paper_1509_07691_amd.fslbm import Lattice

    rows = []
    for n in resolutions:
        dt = 1e-4 * (48.0 / n) ** 2
        shape = (n, n, n)
        fill = np.clip(1.0 - I.sphere_fraction(shape, (n / 2, n / 2, n / 2), n / 8.0), 0.0, 1.0)
        obst = np.zeros(shape, np.uint8)
        tau, sig = I.renardy_units(n, dt)
        u0 = dt * n
        T = int(round(n / u0))
        for model in models:
            lat = Lattice(fill, obst, precision=precision, curv_model=model, sigma=sig, tau=tau, bubble=True,
                          eps_c=eps_c, device=dev)
            u = np.zeros((3,) + shape)
            u[0] = u0
            lat.set_equilibrium(1.0, u)
            hist, t = [], 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(1, samples + 1):
                m = (T * k) // samples
                lat.step(m - t)
                t = m
                umax, uavg, l2, sd = bubble_measures(lat, n, dt, u0)
                hist.append([t, round(t / T, 3), l2, umax, uavg])
                print(f"# moving n={n} {model} t={t}/{T}: L2(k) {l2:.4g} max|u-u0| {umax:.3e}",
                      file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            l1, l2phi = I.advection_errors(fill, lat.fill(), 0)
            rows.append({"n": n, "model": model, "tau": round(tau, 4), "sigma_L": sig, "u0_lattice": u0, "eps_c": eps_c,
                         "steps": T, "history_t_frac_L2kappa_maxu_avgu": hist, "phi_L1_after_one_pass": l1,
                         "phi_L2_after_one_pass": l2phi, "ms_per_step_incl_readout": round(1e3 * el / T, 4)})
            lat.close()
            torch.cuda.empty_cache()
    return rows


# L2(r) of the contact-line radius printed for the grid study of Sec. III.B.1
# (Fig. DropletConvergence) at dx = 1/48, 1/96, 1/144.
PAPER_SESSILE_L2R = {
    ("fd", 60): (0.0610761, 0.0256658, 0.0207583),
    ("fd", 90): (0.0426878, 0.0190497, 0.0134927),
    ("fd", 120): (0.0973444, 0.0389345, 0.0387821),
    ("lsqr", 60): (0.0594971, 0.0211923, 0.0134882),
    ("lsqr", 90): (0.00559683, 0.00508519, 0.0029987),
    ("lsqr", 120): (0.0597827, 0.0322758, 0.0248789),
}


def sessile_measures(lat, n, h, r):
    """h*/h - 1, L2(r) and STDEV of r~ over the contact-line cells, and the
    apparent angle 2 atan(h*/r*) (Sec. III.B.1): h* = max over interface
    cells of z + phi - 0.5 (z the cell centre above the wall), r~ = |x - x_o|
    + phi - 0.5 over the contact-line cells (interface cells with an
    obstacle D3Q19 neighbour, here the first fluid layer), r* their mean."""
    from paper_1509_07691_amd.fslbm import FSLBM_INTERFACE

    fl = lat.flags()
    ph = lat.fill()
    k, j, i = np.nonzero(fl == FSLBM_INTERFACE)
    hs = float(np.max((k + 0.5 - 1.0) + ph[k, j, i] - 0.5))
    c = k == 1
    kc, jc, ic = k[c], j[c], i[c]
    rt = np.hypot(ic + 0.5 - n / 2, jc + 0.5 - n / 2) + ph[kc, jc, ic] - 0.5
    l2 = float(np.sqrt(((r - rt) ** 2).sum() / (r * r * rt.size)))
    rs = float(rt.mean())
    return hs / h - 1.0, l2, float(rt.std()) / r, float(np.degrees(2 * np.arctan(hs / rs)))


def sessile_contact_angles(dev, steps, thetas=(60.0, 90.0, 120.0)):
    """Sessile droplet on a no-slip wall: hemisphere R = 48 on the wall of a
    256 x 256 x 128 lattice (walls k = 0 and 127), LSQR with the wetting
    condition, sigma 5e-4, tau 0.8, FP32, per prescribed angle theta:
    the apparent angle 2 atan(h*/r*) after `steps` steps, and the height
    against the spherical cap of angle theta with the hemisphere's volume;
    then the same from that ideal cap as the start."""
    from paper_1509_07691_amd import inputs as I
    from paper_1509_07691_amd.fslbm import Lattice

    R = 48.0
    fill, obst = I.sessile_droplet(256, 256, 128, R, noise=1e-6, seed=2)
    rows = []
    for th in thetas:
        c = math.cos(math.radians(th))
        rc = R * (2.0 / (2.0 - 3.0 * c + c ** 3)) ** (1.0 / 3.0)  # equal-volume cap
        h, r = rc * (1.0 - c), rc * math.sin(math.radians(th))
        lat = Lattice(fill, obst, precision="f32", device=dev, curv_model="lsqr", sigma=5e-4, tau=0.8,
                      theta=math.radians(th))
        lat.step(steps)
        dh, l2r, _, ang = sessile_measures(lat, 256, h, r)
        lat.close()
        # the same run started from the equal-volume cap of angle theta: the
        # hemisphere start is still moving after `steps` steps at 60 and 120
        # degrees, the cap start shows whether that angle is held
        cap = np.zeros_like(fill)
        cap[1:-1] = I.sphere_fraction(fill.shape, (128.0, 128.0, 1.0 + h - rc), rc)[1:-1]
        cap = I.perturb_interface(cap, 1e-6, 2)
        lat = Lattice(cap, obst, precision="f32", device=dev, curv_model="lsqr", sigma=5e-4, tau=0.8,
                      theta=math.radians(th))
        lat.step(steps)
        cdh, cl2r, _, cang = sessile_measures(lat, 256, h, r)
        lat.close()
        rows.append({"theta": th, "steps": steps, "measured_deg": round(ang, 2),
                     "error_deg": round(ang - th, 2), "h_rel_err": round(dh, 4), "L2_r": round(l2r, 4),
                     "ideal_cap_start": {"measured_deg": round(cang, 2), "error_deg": round(cang - th, 2),
                                         "h_rel_err": round(cdh, 4), "L2_r": round(cl2r, 4)}})
    return rows


def sessile_table(dev, resolutions, models, thetas, eps_c=None, t_phys=2.0):
    """Equilibrium sessile droplets of Sec. III.B.1: the ideal spherical cap
    of each contact angle (hemisphere volume, R = 0.125) on the wall of the
    unit cube, dx = 1/n with diffusive scaling dt = 1e-4 (96/n)^2 (tau = 1.1912,
    the paper's dt = 1e-4 at dx = 1/96), run for t_phys in the units of the
    problem; height error, L2(r), STDEV(r~)/r and the apparent angle."""
    import torch
    from paper_1509_07691_amd import inputs as I
    from paper_1509_07691_amd.fslbm import Lattice

    rows = []
    for n in resolutions:
        dt = 1e-4 * (96.0 / n) ** 2
        tau, sig = I.renardy_units(n, dt)
        steps = int(round(t_phys / dt))
        for th in thetas:
            fill, obst, h, r = I.sessile_cap(n, th)
            for model in models:
                lat = Lattice(fill, obst, precision="f64", curv_model=model, sigma=sig, tau=tau,
                              theta=np.radians(th), eps_c=eps_c, device=dev)
                t, hist = 0, []
                for m in sorted(set(list(range(steps // 4, steps, steps // 4)) + [steps])):
                    lat.step(m - t)
                    t = m
                    he, l2, sd, ang = sessile_measures(lat, n, h, r)
                    hist.append([t, he, l2])
                    print(f"# sessile n={n} theta={th} {model} t={t}/{steps}: h*/h-1 {he:+.4f} L2(r) {l2:.4f} "
                          f"angle {ang:.1f}", file=sys.stderr, flush=True)
                paper = PAPER_SESSILE_L2R.get((model, int(th)))
                idx = {48: 0, 96: 1, 144: 2}.get(n)
                rows.append({"n": n, "theta": th, "model": model, "tau": round(tau, 4), "sigma_L": sig,
                             "steps": steps, "h_err": he, "L2_r": l2, "stdev_r_rel": sd, "apparent_angle": ang,
                             "paper_L2_r": None if paper is None or idx is None else paper[idx],
                             "history": hist})
                lat.close()
                torch.cuda.empty_cache()
    return rows


def oscillation_table(dev, precisions, steps, every=500):
    """Oscillating droplet (the precision form's workload): the ellipsoid
    96/80/80 in a periodic 512^3, LSQR, sigma = 1e-3, tau = 0.55, per storage
    form. The x semi-axis a(t) = sqrt(5 <(x - <x>)^2>) (phi-weighted, exact
    for a solid ellipsoid) is sampled every `every` steps; the period is
    twice the mean spacing of its successive extrema (parabolic refinement),
    compared with Lamb's l = 2 mode, omega^2 = 8 sigma / (rho R^3), R the
    equal-volume radius, and its viscous decay rate 5 nu / R^2."""
    import torch
    from paper_1509_07691_amd.fslbm import Lattice

    (label, fill, obst, p), = workload_runs("ellipsoid")[0]
    nz, ny, nx = fill.shape
    x = torch.arange(nx, dtype=torch.float64, device=dev) + 0.5
    R = (96.0 * 80.0 * 80.0) ** (1.0 / 3.0)
    nu = (p["tau"] - 0.5) / 3.0
    w0 = math.sqrt(8.0 * p["sigma"] / R ** 3)
    out = {"lamb_period_steps": round(2 * math.pi / w0, 1), "lamb_decay_per_step": 5.0 * nu / R ** 2}
    for prec in precisions:
        lat = Lattice(fill, obst, precision=prec, device=dev, **p)
        m0 = lat.mass()
        ts, a = [], []
        t = 0
        while True:
            ph = lat.fill_tensor()
            wsum = ph.sum()
            px = ph.sum(dim=(0, 1))
            mx = (px * x).sum() / wsum
            a.append(math.sqrt(5.0 * float((px * (x - mx) ** 2).sum() / wsum)))
            ts.append(t)
            del ph, px
            if t >= steps:
                break
            lat.step(every)
            t += every
            if t % (10 * every) == 0:
                print(f"# oscillation {prec} t={t}: a={a[-1]:.3f}", file=sys.stderr, flush=True)
        a = np.array(a)
        ext = []
        for k in range(1, len(a) - 1):
            if (a[k] - a[k - 1]) * (a[k + 1] - a[k]) < 0:
                den = a[k - 1] - 2 * a[k] + a[k + 1]
                off = 0.5 * (a[k - 1] - a[k + 1]) / den if den != 0 else 0.0
                ext.append(ts[k] + off * every)
        period = 2.0 * float(np.mean(np.diff(ext))) if len(ext) >= 2 else None
        out[prec] = {"period_steps": None if period is None else round(period, 1),
                     "period_vs_lamb": None if period is None else round(period * w0 / (2 * math.pi), 4),
                     "extrema_steps": [round(e, 1) for e in ext], "a_first_last": [round(a[0], 3), round(a[-1], 3)],
                     "a_series": [round(v, 3) for v in a], "sample_every": every,
                     "mass_drift": (lat.mass() - m0) / m0, "steps": steps}
        lat.close()
        del lat
        torch.cuda.empty_cache()
    return out


def pull_copy_rate(dev, stream, shape, prec, launches=10):
    """The stream-collide's memory bound on this device: the library's
    pull-only copy (19 planes in the lattice layout, D3Q19 upstream offsets,
    the stream-collide's grid; no arithmetic) on an nx x ny x nz lattice,
    timed by the library with HIP events on `stream`. Returns (us per
    launch, GB/s over the 38 s N bytes it moves)."""
    import torch
    from paper_1509_07691_amd import fslbm as F

    code = F.PRECISIONS[prec]
    nx, ny, nz = shape
    nbytes = F.fslbm_pull_copy_bytes(nx, ny, nz, code)
    src = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    us = F.fslbm_pull_copy_time(nx, ny, nz, code, src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream,
                                launches)
    del src, dst
    torch.cuda.empty_cache()
    moved = 38 * {"f64": 8, "f32": 4}.get(prec, 2) * nx * ny * nz
    return us, moved / (us * 1e-6) / 1e9


def run_workload(dev, stream, name, prec, steps, warmup, split=None, graph=False, keep=False):
    """Times `steps` steps of a workload (after `warmup`) with per-phase HIP
    events on the lattices' stream; returns the record and, with keep, the
    lattices and their batch (else they are released)."""
    import torch
    from paper_1509_07691_amd.fslbm import Batch, Lattice

    runs, desc = workload_runs(name)
    lats = []
    with torch.cuda.stream(stream):
        for label, fill, obst, p in runs:
            lats.append(Lattice(fill, obst, precision=prec, device=dev, stream=stream, **p))
    batch = Batch(lats)
    batch.set_split_interface(split)
    torch.cuda.synchronize()
    print(f"# {len(lats)} lattice(s) created: {desc}, {prec}", file=sys.stderr, flush=True)
    batch.step(warmup)
    torch.cuda.synchronize()
    batch.set_timing(True)
    batch.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phase, st = batch.timing()
    assert st == steps
    batch.set_timing(False)
    bl = bi = nl = ni = nbox = ncell = 0
    for lat in lats:
        a, b, c, d, e = sc_bytes(lat.flags(), prec)
        bl, bi, nl, ni, nbox = bl + a, bi + b, nl + c, ni + d, nbox + e
        ncell += lat.n
        lat.check_numeric()
    split = batch.split_active()
    sc_ms = phase[0]
    launch = bl if split else bl + bi  # the merged kernel also moves the interface cells' bytes
    achieved = launch * steps / (sc_ms * 1e-3) / 1e9
    rec = {"workload": desc, "lattice": list(runs[0][1].shape[::-1]), "lattices": len(lats), "storage": prec,
           "steps": steps, "warmup": warmup, "ms_per_step": round(1e3 * el / steps, 4),
           "mlups": round(ncell * steps / el / 1e6, 1), "mflups": round((nl + ni) * steps / el / 1e6, 1),
           "fluid_cells": nl + ni, "interface_cells": ni, "fluid_box_cells": nbox,
           "split_passes": split,
           "stream_collide_us": round(1e3 * sc_ms / steps, 3), "algorithmic_bytes_per_launch": int(launch),
           "stream_collide_GBs": round(achieved, 1), "roofline_frac": round(achieved / HBM_PEAK_GBS, 4),
           "phases_ms_per_step": {k: round(v / steps, 4) for k, v in
                                  zip(("stream_collide", "stream_collide_interface_list", "conversion",
                                       "list_update", "obstacle_fill_and_curvature"), phase)}}
    if graph:
        batch.set_graph(True)
        batch.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.step(steps)
        torch.cuda.synchronize()
        gms = 1e3 * (time.perf_counter() - t0) / steps
        batch.set_graph(False)
        rec["graph_replay"] = {"ms_per_step": round(gms, 4), "mlups": round(ncell / gms / 1e3, 1)}
    if keep:
        return rec, runs, lats, batch
    batch.close()
    for lat in lats:
        lat.close()
    del batch, lats
    torch.cuda.empty_cache()
    return rec


def c3_record(dev, precisions, steps, every=500):
    """The oscillating droplet (precision form's workload): ellipsoid
    96/80/80 in a periodic 512^3, LSQR, sigma 1e-3, tau 0.55, per storage
    form: ms per step (stepping only, synchronised every `every` steps),
    relative mass drift after `steps`, the x semi-axis a(t) =
    sqrt(5 <(x - <x>)^2>) of the fill level every `every` steps and its
    extrema. The l = 2 period of Lamb's formula is printed beside it."""
    import torch
    from paper_1509_07691_amd.fslbm import Lattice

    (label, fill, obst, p), = workload_runs("ellipsoid")[0]
    nz, ny, nx = fill.shape
    x = torch.arange(nx, dtype=torch.float64, device=dev) + 0.5
    R = (96.0 * 80.0 * 80.0) ** (1.0 / 3.0)
    w0 = math.sqrt(8.0 * p["sigma"] / R ** 3)
    out = {"workload": "oscillating droplet: ellipsoid 96/80/80 in periodic 512^3, LSQR, sigma 1e-3, tau 0.55",
           "steps": steps, "lamb_period_steps": round(2 * math.pi / w0, 1),
           "note": "the l = 2 period (~55k steps) exceeds the run; the 128^3 downscale's period is measured "
                   "against the FP64 oracle in the tests"}
    for prec in precisions:
        lat = Lattice(fill, obst, precision=prec, device=dev, **p)
        m0 = lat.mass()
        ts, a, t, tstep = [], [], 0, 0.0
        while True:
            ph = lat.fill_tensor()
            px = ph.sum(dim=(0, 1))
            wsum = px.sum()
            mx = (px * x).sum() / wsum
            a.append(math.sqrt(5.0 * float((px * (x - mx) ** 2).sum() / wsum)))
            ts.append(t)
            del ph, px
            if t >= steps:
                break
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat.step(every)
            torch.cuda.synchronize()
            tstep += time.perf_counter() - t0
            t += every
        ext = [ts[k] for k in range(1, len(a) - 1) if (a[k] - a[k - 1]) * (a[k + 1] - a[k]) < 0]
        out[prec] = {"ms_per_step": round(1e3 * tstep / steps, 4), "mlups": round(fill.size * steps / tstep / 1e6, 1),
                     "mass_drift": (lat.mass() - m0) / m0, "a_every": every, "a": [round(v, 3) for v in a],
                     "a_extrema_steps": ext}
        print(f"# C3 {prec}: {out[prec]['ms_per_step']} ms/step, drift {out[prec]['mass_drift']:.2e}",
              file=sys.stderr, flush=True)
        lat.close()
        del lat
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="bubble-probe", choices=["bubble-probe", "droplet-sweep", "ellipsoid"])
    ap.add_argument("--precision", default="f32", choices=["f64", "f32", "f16", "bf16"])
    ap.add_argument("--graph", type=int, default=1,
                    help="also time a graph-replay pass after the timed region")
    ap.add_argument("--split", type=int, default=-1,
                    help="1: interface cells in their own list kernel, 0: one pass, -1: the library's choice")
    ap.add_argument("--compare", default="f16,bf16",
                    help="comma list of storage precisions also timed on the same workload ('' for none)")
    ap.add_argument("--sweep-steps", type=int, default=200,
                    help="timed steps of the 8 x 128^3 droplet sweep reported beside the headline (0: skip)")
    ap.add_argument("--c3-steps", type=int, default=10000,
                    help="steps of the 512^3 oscillating droplet per storage form (0: skip)")
    ap.add_argument("--c3-precisions", default="f32,f16,bf16")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain copy of 2^28 floats (for scaling rocprofv3 byte counters)")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-bandwidth reference")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write profiles/stream_collide_traffic.json from rocprofv3 --pmc counter CSVs and exit")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="steps of the differentiation window timed for the adjoint cost (0: skip)")
    ap.add_argument("--adjoint-k", type=int, default=100, help="checkpoint interval of that window")
    ap.add_argument("--sessile-steps", type=int, default=20000,
                    help="sessile droplet 256x256x128 at 60/90/120 deg: apparent angle after this many steps (0: skip)")
    ap.add_argument("--diag-steps", type=int, default=5000,
                    help="droplet sweep: spurious currents and Laplace law of each run after this many steps (0: skip)")
    ap.add_argument("--adjoint-fd-check", type=int, default=1,
                    help="0: skip the difference check of the adjoint on the 64^3 downscale")
    ap.add_argument("--advection", action="store_true",
                    help="only run the pure advection test table (d = 10..80) and print it")
    ap.add_argument("--laplace", type=int, nargs="*", metavar="N",
                    help="equilibrium-bubble study at dx = 1/N (default 48 96) instead of the bench")
    ap.add_argument("--laplace-steps", type=int, default=500000)
    ap.add_argument("--moving", type=int, nargs="*", metavar="N",
                    help="moving-frame bubble at dx = 1/N (default 48 96) instead of the bench")
    ap.add_argument("--models", default="fd,lsqr")
    ap.add_argument("--oscillation", type=int, default=0, metavar="STEPS",
                    help="oscillating 512^3 droplet for STEPS steps per storage form instead of the bench")
    ap.add_argument("--osc-precisions", default="f64,f32,f16,bf16")
    ap.add_argument("--sessile", type=int, nargs="*", metavar="N",
                    help="equilibrium sessile droplets at dx = 1/N (default 48 96 144) instead of the bench")
    ap.add_argument("--eps-c", type=float, default=None,
                    help="conversion offset for the bubble studies (library default 1e-3)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.traffic_from:
        rec = traffic_from_counters(*args.traffic_from, workload_note=args.workload, precision=args.precision)
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    if args.advection:
        print(json.dumps({"advection": advection_table(dev, "f64")}))
        return
    models = tuple(args.models.split(","))
    if args.laplace is not None:
        res = args.laplace or [48, 96]
        print(json.dumps({"laplace": laplace_table(dev, res, args.laplace_steps, models, eps_c=args.eps_c)}))
        return
    if args.oscillation > 0:
        print(json.dumps({"oscillation": oscillation_table(dev, args.osc_precisions.split(","), args.oscillation)}))
        return
    if args.sessile is not None:
        res = args.sessile or [48, 96, 144]
        print(json.dumps({"sessile": sessile_table(dev, res, models, (60.0, 90.0, 120.0), eps_c=args.eps_c)}))
        return
    if args.moving is not None:
        res = args.moving or [48, 96]
        print(json.dumps({"moving_bubble": moving_bubble_table(dev, res, models, eps_c=args.eps_c)}))
        return
    if args.copy_calibration:
        # a plain elementwise copy: 1 GiB read and 1 GiB written per launch
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 << 28, "bytes_written": 4 << 28, "launches": 5}))
        return
    # achievable HBM bandwidth on this device: a plain elementwise copy of
    # 2 x 1 GiB (read + write), timed with events
    copy_gbs = None
    if not args.no_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(10):
            torch.mul(src, 1.0, out=dst)
        ev1.record()
        torch.cuda.synchronize()
        copy_gbs = 10 * 2 * (4 << 28) / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
        del src, dst
        torch.cuda.empty_cache()

    stream = torch.cuda.Stream(dev)
    head = run_workload(dev, stream, args.workload, args.precision, args.steps, args.warmup,
                        split=None if args.split < 0 else bool(args.split), graph=bool(args.graph))
    traffic = stored_traffic(args.workload, args.precision)
    nunits = head["fluid_cells"]
    pull = None
    if not args.no_copy and head["lattices"] == 1:
        pus, pgbs = pull_copy_rate(dev, stream, head["lattice"], args.precision)
        pull = {"us": round(pus, 3), "GBs": round(pgbs, 1),
                "kernel_frac_of_pull_copy": round(head["stream_collide_GBs"] / pgbs, 4),
                "what": "the library's pull-only copy (fslbm_pull_copy_time) on the same lattice shape and "
                        "layout: the 38 distribution streams with no arithmetic, the memory bound of the pass"}
    res = {
        "metric": METRIC,
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{head['workload']}, {args.precision} storage and arithmetic",
                   "lattice": head["lattice"], "lattices": head["lattices"], "storage": args.precision,
                   "split_passes": head["split_passes"], "fluid_cells": head["fluid_cells"],
                   "interface_cells": head["interface_cells"], "fluid_box_cells": head["fluid_box_cells"]},
        "roofline": {"bound": "hbm", "achieved": head["stream_collide_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["roofline_frac"],
                     "traffic": traffic.get("bytes_per_launch") if traffic else None,
                     "copy_kernel_GBs": round(copy_gbs, 1) if copy_gbs else None,
                     "pull_copy": pull,
                     "kernel": "k_stream_collide" + (" (lean liquid pass)" if head["split_passes"] else ""),
                     "avg_launch_us": head["stream_collide_us"],
                     "algorithmic_bytes_per_launch": head["algorithmic_bytes_per_launch"],
                     "units_per_launch": nunits,
                     "bytes_per_unit": round(head["algorithmic_bytes_per_launch"] / max(nunits, 1), 3),
                     "unit_definition": "fluid cell: 38 distribution values, plus one flag byte per fluid-box cell "
                                        "and m, rho, K, phi and a status byte per interface cell"},
        "mflups": head["mflups"],
        "phases_ms_per_step": head["phases_ms_per_step"],
    }
    if "graph_replay" in head:
        res["graph_replay"] = head["graph_replay"]
    print(f"# headline: {res['value']} MLUPS, roofline {res['roofline']['frac']}", file=sys.stderr, flush=True)

    compare = {}
    for prec in [p for p in args.compare.split(",") if p and p != args.precision]:
        rec = run_workload(dev, stream, args.workload, prec, args.steps, args.warmup)
        rec["speedup_vs_" + args.precision] = round(head["ms_per_step"] / rec["ms_per_step"], 3)
        rec["stream_collide_speedup_vs_" + args.precision] = round(head["stream_collide_us"] / rec["stream_collide_us"], 3)
        if not args.no_copy and rec["lattices"] == 1:
            pus, pgbs = pull_copy_rate(dev, stream, rec["lattice"], prec)
            rec["pull_copy"] = {"us": round(pus, 3), "GBs": round(pgbs, 1),
                                "kernel_frac_of_pull_copy": round(rec["stream_collide_GBs"] / pgbs, 4)}
        compare[prec] = rec
        print(f"# storage {prec}: {rec['mlups']} MLUPS", file=sys.stderr, flush=True)
    if compare:
        res["storage_comparison"] = compare

    if args.sweep_steps > 0 and args.workload != "droplet-sweep":
        rec, runs, lats, batch = run_workload(dev, stream, "droplet-sweep", "f32", args.sweep_steps, args.warmup,
                                              graph=bool(args.graph), keep=True)
        if args.diag_steps > 0:
            more = args.diag_steps - lats[0].steps_taken()
            if more > 0:
                batch.step(more)
            torch.cuda.synchronize()
            diag = []
            for (label, _, _, p), lat in zip(runs, lats):
                d = lat.diagnostics()
                dpl = 2.0 * p["sigma"] / SWEEP_RADIUS
                diag.append({"run": label, "steps": lat.steps_taken(), "max_u": d["max_u"], "mean_u": d["mean_u"],
                             "dp": d["dp"], "dp_laplace": dpl, "dp_rel_err": round((d["dp"] - dpl) / dpl, 5),
                             "n_inner": d["n_inner"]})
            rec["diagnostics"] = diag
        batch.close()
        for lat in lats:
            lat.close()
        del batch, lats
        torch.cuda.empty_cache()
        res["droplet_sweep"] = rec
        print("# droplet sweep done", file=sys.stderr, flush=True)

    if args.c3_steps > 0:
        res["c3_oscillating_droplet"] = c3_record(dev, [p for p in args.c3_precisions.split(",") if p],
                                                  args.c3_steps)
    if args.sessile_steps > 0:
        res["sessile_contact_angles"] = sessile_contact_angles(dev, args.sessile_steps)
        print("# sessile contact angles done", file=sys.stderr, flush=True)
    if args.adjoint_steps > 0:
        res["adjoint"] = adjoint_cost(dev, stream, args.adjoint_steps, args.adjoint_k, "f32",
                                      fd_check=bool(args.adjoint_fd_check))
        print(f"# adjoint window done: {res['adjoint']['cost_ratio']}x forward", file=sys.stderr, flush=True)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

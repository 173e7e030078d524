"""Parity at the benchmark sizes, in the launch configuration bench.py
times (batched lattices, one stream, merged stream-collide).

- Droplet sweep: the eight 128^3 lattices (radius 32; tau 0.6 / 1.0 x
  sigma 1e-4 / 1e-3 x FD / LSQR) advanced as one batch in FP32 for 3 steps,
  each compared cell by cell with the FP64 oracle run on the whole lattice:
  identical cell types, fill level and pressure within the FP32 bar (1e-5
  relative), velocity within 1e-6 absolute and 1e-5 of max(|u|, sigma/mu)
  (the plain relative error is printed).
- Sessile droplet (hemisphere R = 48 on the wall of 256 x 256 x 128,
  theta 60 / 90 / 120 deg): sampled cells, contact-line cells among them,
  each against the oracle on the full-height 28 x 28 column around it.
- 512^3 workloads (the ellipsoid of radii 96/80/80 and the gas bubble of
  radius 64): the state after 2 steps at sampled cells, each against the
  oracle run on the 28^3 block of the initial fill centred on the cell. One
  step reaches at most 5 cells (1 for streaming, 2 for the LSQR block of
  PLIC points, 2 more for the normals and the obstacle reflection), so
  after 2 steps the block's centre does not see the block's own periodic
  wrap. Sampled: 16 interface cells and 8 liquid cells.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1509_07691_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def test_droplet_sweep_batch_fp32_vs_oracle(torch_dev):
    torch = torch_dev
    import bench
    from paper_1509_07691_amd.fslbm import Batch, Lattice

    runs, _ = bench.workload_runs("droplet-sweep")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        lats = [Lattice(fill, obst, precision="f32", stream=stream, **p) for _, fill, obst, p in runs]
    b = Batch(lats)
    b.step(3)
    torch.cuda.synchronize()
    for (label, fill, obst, p), g in zip(runs, lats):
        o = O.Oracle(fill, obst, sigma=p["sigma"], tau=p["tau"],
                     curv_model=O.CURV_FD if p["curv_model"] == "fd" else O.CURV_LSQR)
        o.step(3)
        fl = o.flags()
        assert np.array_equal(g.flags(), fl), label
        fluid = (fl == O.LIQUID) | (fl == O.INTERFACE)
        for name, a, r in (("fill", g.fill(), o.fill()), ("pressure", g.pressure(), o.pressure())):
            e = np.linalg.norm((a - r)[fluid]) / np.linalg.norm(r[fluid])
            assert e < 1e-5, f"{label} {name} {e:.2e}"
        # velocity: largest absolute difference, the relative L2 error, and
        # the L2 error normalised by max(|u_ref|, (sigma / mu) sqrt(n)) with
        # mu = rho nu, the parity measure of the droplet tests
        dv = (g.velocity() - o.velocity())[:, fluid]
        ur = o.velocity()[:, fluid]
        du = np.abs(dv).max()
        mu = (p["tau"] - 0.5) / 3.0
        e_rel = np.linalg.norm(dv) / np.linalg.norm(ur)
        e_norm = np.linalg.norm(dv) / max(np.linalg.norm(ur), p["sigma"] / mu * math.sqrt(fluid.sum()))
        print(f"{label}: velocity max |du| {du:.2e}, relative {e_rel:.2e}, normalised {e_norm:.2e}")
        assert du < 1e-6 and e_norm < 1e-5, f"{label} velocity {du:.2e} {e_norm:.2e}"
        del o
    b.close()
    for g in lats:
        g.close()


BLOCK = 28


def sampled_parity(torch, fill, obst, prm, steps=2, n_if=16, n_liq=8, seed=0, full_z=False, n_wall=0):
    """Worst differences at sampled cells between the HIP path (FP32, whole
    lattice) and the oracle on the block of the initial state around each
    cell: BLOCK^3 with periodic wrap, or BLOCK x BLOCK columns over the
    whole height when full_z (walls at k = 0 and k = nz - 1 then enter the
    oracle as they are). n_wall of the interface picks touch a wall."""
    from paper_1509_07691_amd.fslbm import Lattice

    g = Lattice(fill, obst, precision="f32", **prm)
    flags0 = g.flags()
    g.step(steps)
    phi, rho, u = g.fill(), g.density(), g.velocity()
    g.close()
    torch.cuda.empty_cache()
    rng = np.random.default_rng(seed)
    ifc = flags0 == O.INTERFACE
    picks = []
    if n_wall:
        wall_ifc = ifc & (np.roll(flags0, 1, axis=0) == O.OBSTACLE)
        picks += list(rng.choice(np.flatnonzero(wall_ifc), n_wall, replace=False))
        ifc &= ~wall_ifc
    picks += list(rng.choice(np.flatnonzero(ifc), n_if, replace=False))
    picks += list(rng.choice(np.flatnonzero(flags0 == O.LIQUID), n_liq, replace=False))
    nz, ny, nx = fill.shape
    h = BLOCK // 2
    model = O.CURV_FD if prm["curv_model"] == "fd" else O.CURV_LSQR
    kw = {k: prm[k] for k in ("sigma", "tau", "theta") if k in prm}
    mu = (prm["tau"] - 0.5) / 3.0
    worst = {"fill": 0.0, "rho": 0.0, "u": 0.0, "u_rel": 0.0, "u_norm": 0.0}
    for c in picks:
        z, y, x = np.unravel_index(c, fill.shape)
        zz = (np.arange(nz) if full_z else np.arange(z - h, z + h) % nz)[:, None, None]
        yy = (np.arange(y - h, y + h) % ny)[None, :, None]
        xx = (np.arange(x - h, x + h) % nx)[None, None, :]
        sub = np.ascontiguousarray(fill[zz, yy, xx])
        sob = None if obst is None else np.ascontiguousarray(obst[zz, yy, xx])
        o = O.Oracle(sub, sob, curv_model=model, **kw)
        o.step(steps)
        zc = z if full_z else h
        worst["fill"] = max(worst["fill"], abs(o.fill()[zc, h, h] - phi[z, y, x]))
        worst["rho"] = max(worst["rho"], abs(o.density()[zc, h, h] - rho[z, y, x]))
        ur = o.velocity()[:, zc, h, h]
        du = np.abs(ur - u[:, z, y, x])
        worst["u"] = max(worst["u"], du.max())
        # relative to |u_ref| and to max(|u_ref|, sigma / mu)
        un = np.linalg.norm(ur)
        worst["u_rel"] = max(worst["u_rel"], np.linalg.norm(du) / un if un > 0 else 0.0)
        worst["u_norm"] = max(worst["u_norm"], np.linalg.norm(du) / max(un, prm["sigma"] / mu))
        del o
    return worst


@pytest.mark.parametrize("name", ["ellipsoid", "bubble"])
def test_512_sampled_cells_vs_oracle_blocks(torch_dev, name):
    if name == "ellipsoid":
        fill, obst = I.ellipsoid_droplet(512, (96, 80, 80), noise=1e-6, seed=0)
        prm = dict(curv_model="lsqr", tau=0.55, sigma=1e-3)
    else:
        fill, obst = I.bubble_probe(512, 64.0)
        prm = dict(curv_model="lsqr", tau=0.8, sigma=1e-3)
    worst = sampled_parity(torch_dev, fill, obst, prm)
    print(name, worst)
    assert worst["fill"] < 2e-6 and worst["rho"] < 2e-6 and worst["u"] < 1e-6 and worst["u_norm"] < 1e-5, worst


@pytest.mark.parametrize("theta_deg", [60.0, 90.0, 120.0])
def test_sessile_256_sampled_columns_vs_oracle(torch_dev, theta_deg):
    """Sessile droplet at its benchmark size: hemisphere R = 48 on the wall
    of a 256 x 256 x 128 lattice, LSQR with the wetting condition, sigma
    5e-4, tau 0.8. Sampled: 12 contact-line cells (interface cells on the
    wall), 8 other interface cells and 4 liquid cells, each against the
    oracle on its full-height 28 x 28 column."""
    fill, obst = I.sessile_droplet(256, 256, 128, 48.0, noise=1e-6, seed=2)
    prm = dict(curv_model="lsqr", tau=0.8, sigma=5e-4, theta=math.radians(theta_deg))
    worst = sampled_parity(torch_dev, fill, obst, prm, n_if=8, n_liq=4, n_wall=12, full_z=True, seed=1)
    print("sessile", theta_deg, worst)
    assert worst["fill"] < 2e-6 and worst["rho"] < 2e-6 and worst["u"] < 1e-6 and worst["u_norm"] < 1e-5, worst

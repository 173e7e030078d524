"""Parity at the benchmark sizes, in the launch configuration bench.py
times (batched lattices, one stream, merged stream-collide).

- Droplet sweep: the eight 128^3 lattices (radius 32; tau 0.6 / 1.0 x
  sigma 1e-4 / 1e-3 x FD / LSQR) advanced as one batch in FP32 for 3 steps,
  each compared cell by cell with the FP64 oracle run on the whole lattice:
  identical cell types, fill level, pressure and velocity within the FP32
  bar (1e-5 relative).
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

    runs, _ = bench.workload_runs("c1")
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
        du = np.abs(g.velocity() - o.velocity())[:, fluid].max()
        assert du < 1e-6, f"{label} velocity {du:.2e}"
        del o
    b.close()
    for g in lats:
        g.close()


BLOCK = 28


def sampled_parity(torch, fill, obst, prm, steps=2, n_if=16, n_liq=8, seed=0):
    from paper_1509_07691_amd.fslbm import Lattice

    g = Lattice(fill, obst, precision="f32", **prm)
    flags0 = g.flags()
    g.step(steps)
    phi, rho, u = g.fill(), g.density(), g.velocity()
    g.close()
    torch.cuda.empty_cache()
    rng = np.random.default_rng(seed)
    ifc = np.flatnonzero(flags0 == O.INTERFACE)
    liq = np.flatnonzero(flags0 == O.LIQUID)
    picks = list(rng.choice(ifc, n_if, replace=False)) + list(rng.choice(liq, n_liq, replace=False))
    nz, ny, nx = fill.shape
    h = BLOCK // 2
    worst = {"fill": 0.0, "rho": 0.0, "u": 0.0}
    for c in picks:
        z, y, x = np.unravel_index(c, fill.shape)
        zz = (np.arange(z - h, z + h) % nz)[:, None, None]
        yy = (np.arange(y - h, y + h) % ny)[None, :, None]
        xx = (np.arange(x - h, x + h) % nx)[None, None, :]
        sub = np.ascontiguousarray(fill[zz, yy, xx])
        o = O.Oracle(sub, None, sigma=prm["sigma"], tau=prm["tau"],
                     curv_model=O.CURV_FD if prm["curv_model"] == "fd" else O.CURV_LSQR)
        o.step(steps)
        worst["fill"] = max(worst["fill"], abs(o.fill()[h, h, h] - phi[z, y, x]))
        worst["rho"] = max(worst["rho"], abs(o.density()[h, h, h] - rho[z, y, x]))
        worst["u"] = max(worst["u"], np.abs(o.velocity()[:, h, h, h] - u[:, z, y, x]).max())
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
    assert worst["fill"] < 2e-6 and worst["rho"] < 2e-6 and worst["u"] < 1e-6, worst

"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: FP64 mode: bit-exact cell types and interface lists, fill level,
pressure and velocity within 1e-10 relative. FP32: 1e-5 relative; 16-bit
storage of f - w_q: 2e-3 relative. Relative means
||x - x_ref||_2 / ||x_ref||_2 over the fluid cells of the oracle; for the
velocity the denominator is at least the capillary velocity scale
sigma/mu (mu = rho nu, nu = (tau - 1/2)/3) per cell, because the spurious
currents of a static droplet are far below it and their FP32 round-off is
not small relative to themselves.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1509_07691_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Lattice():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1509_07691_amd.fslbm import Lattice as L

    return L


def rel(a, b, mask):
    num = np.linalg.norm((a - b)[..., mask])
    den = np.linalg.norm(b[..., mask])
    return num / den if den > 0 else num


def vel_err(u, uref, mask, vscale=0.0):
    """Relative velocity error, denominator at least vscale per fluid cell."""
    d = np.sqrt(((u - uref) ** 2).sum(0))[mask]
    scale = np.sqrt((uref ** 2).sum(0))[mask]
    return np.linalg.norm(d) / max(np.linalg.norm(scale), vscale * np.sqrt(mask.sum()), 1e-300)


MODELS = {"fd": O.CURV_FD, "lsqr": O.CURV_LSQR, "tr": O.CURV_TR}


def pair(Lattice, fill, obst, model, precision="f64", **kw):
    g = Lattice(fill, obst, precision=precision, curv_model=model, **kw)
    o = O.Oracle(fill, obst, curv_model=MODELS[model], **kw)
    return g, o


def compare(g, o, tol, exact_flags=True, what="", vscale=0.0):
    fl_g, fl_o = g.flags(), o.flags()
    if exact_flags:
        assert np.array_equal(fl_g, fl_o), f"{what}: {int((fl_g != fl_o).sum())} cell types differ"
        assert np.array_equal(g.interface_list(), o.interface_list()), f"{what}: interface lists differ"
    fluid = (fl_o == O.LIQUID) | (fl_o == O.INTERFACE)
    e_phi = rel(g.fill(), o.fill(), fluid)
    e_u = vel_err(g.velocity(), o.velocity(), fluid, vscale)
    e_p = rel(g.pressure(), o.pressure(), fluid)
    assert e_phi < tol, f"{what}: fill rel err {e_phi:.3e}"
    assert e_u < tol, f"{what}: velocity rel err {e_u:.3e}"
    assert e_p < tol, f"{what}: pressure rel err {e_p:.3e}"
    return e_phi, e_u


@pytest.mark.parametrize("model", ["fd", "lsqr", "tr"])
def test_initial_geometry_fp64(Lattice, model):
    fill, obst = I.droplet(32, 8.0, noise=1e-6, seed=0)
    g, o = pair(Lattice, fill, obst, model, sigma=1e-3, tau=1.0)
    assert np.array_equal(g.flags(), o.flags())
    assert np.array_equal(g.interface_list(), o.interface_list())
    ifc = o.flags() == O.INTERFACE
    np.testing.assert_allclose(g.normal()[:, ifc], o.normal()[:, ifc], rtol=0, atol=1e-13)
    np.testing.assert_allclose(g.plic()[ifc], o.plic()[ifc], rtol=0, atol=1e-12)
    np.testing.assert_allclose(g.curvature()[ifc], o.curvature()[ifc], rtol=0, atol=1e-11)
    np.testing.assert_array_equal(g.fill(), o.fill())


@pytest.mark.parametrize("model", ["fd", "lsqr", "tr"])
def test_static_droplet_fp64_500_steps(Lattice, model):
    """Static droplet R = 8 in 32^3, tau = 1, sigma = 1e-3, 500 steps (FP64)."""
    fill, obst = I.droplet(32, 8.0, noise=1e-6, seed=0)
    g, o = pair(Lattice, fill, obst, model, sigma=1e-3, tau=1.0)
    for n in (1, 9, 90, 400):
        g.step(n)
        o.step(n)
        # the spurious currents decay towards round-off: velocity relative
        # to the capillary scale sigma / mu
        compare(g, o, 1e-10, what=f"{model} after +{n}", vscale=1e-3 / (0.5 / 3.0))
    assert abs(g.mass() - o.mass()) / o.mass() < 1e-13


@pytest.mark.parametrize("model", ["fd", "lsqr", "tr"])
def test_moving_droplet_conversions_fp64(Lattice, model):
    """A droplet advected through the lattice: cells fill and empty every step."""
    fill, obst = I.droplet(20, 4.5, noise=1e-6, seed=1)
    g, o = pair(Lattice, fill, obst, model, sigma=2e-3, tau=0.8)
    u = np.zeros((3,) + fill.shape)
    u[0] = 0.04
    u[2] = -0.02
    g.set_equilibrium(1.0, u)
    o.set_equilibrium(np.ones(fill.shape), u)
    fl0 = o.flags()
    M0 = g.mass()
    for n in (1, 5, 20, 34):
        g.step(n)
        o.step(n)
        compare(g, o, 1e-10, what=f"{model} moving after +{n}")
    assert (o.flags() != fl0).sum() > 20
    assert abs(g.mass() - M0) / M0 < 1e-13


@pytest.mark.parametrize("model", ["lsqr", "fd"])
@pytest.mark.parametrize("theta", [60.0, 120.0])
def test_sessile_wetting_fp64(Lattice, theta, model):
    """Hemisphere on a no-slip wall with the wetting condition: the LSQR
    gradient condition, or the FD contact normal at obstacle nodes."""
    fill, obst = I.sessile_droplet(28, 28, 14, 7.0, noise=1e-6)
    g, o = pair(Lattice, fill, obst, model, sigma=2e-3, tau=0.8, theta=math.radians(theta))
    ifc = o.flags() == O.INTERFACE
    np.testing.assert_allclose(g.curvature()[ifc], o.curvature()[ifc], rtol=0, atol=1e-11)
    for n in (1, 30, 120):
        g.step(n)
        o.step(n)
        compare(g, o, 1e-10, what=f"sessile {theta} after +{n}")


@pytest.mark.parametrize("collision", ["trt"])
def test_trt_fp64(Lattice, collision):
    fill, obst = I.sessile_droplet(24, 24, 12, 6.0, noise=1e-6)
    g = Lattice(fill, obst, precision="f64", curv_model="fd", sigma=1e-3, tau=0.7, collision=collision)
    o = O.Oracle(fill, obst, curv_model=O.CURV_FD, sigma=1e-3, tau=0.7, collision=O.TRT)
    g.step(60)
    o.step(60)
    compare(g, o, 1e-10, what="trt")


@pytest.mark.parametrize("model", ["fd", "lsqr"])
def test_static_droplet_fp32(Lattice, model):
    fill, obst = I.droplet(32, 8.0, noise=1e-6, seed=0)
    g, o = pair(Lattice, fill, obst, model, precision="f32", sigma=1e-3, tau=1.0)
    g.step(50)
    o.step(50)
    compare(g, o, 1e-5, exact_flags=False, what=f"fp32 {model}", vscale=1e-3 / (0.5 / 3.0))


@pytest.mark.parametrize("precision,tol", [("f32", 1e-5), ("f16", 2e-3), ("bf16", 2e-3)])
def test_moving_droplet_reduced_precision(Lattice, precision, tol):
    """Velocities of O(0.04): plain relative errors, over a window in which
    the cell types still agree with the FP64 reference."""
    fill, obst = I.droplet(20, 4.5, noise=1e-6, seed=1)
    g, o = pair(Lattice, fill, obst, "lsqr", precision=precision, sigma=2e-3, tau=0.8)
    u = np.zeros((3,) + fill.shape)
    u[0] = 0.04
    u[2] = -0.02
    g.set_equilibrium(1.0, u)
    o.set_equilibrium(np.ones(fill.shape), u)
    g.step(3)
    o.step(3)
    compare(g, o, tol, exact_flags=False, what=f"moving {precision}")


@pytest.mark.parametrize("precision", ["f16", "bf16"])
def test_static_droplet_16bit_storage(Lattice, precision):
    fill, obst = I.droplet(32, 8.0, noise=1e-6, seed=0)
    g, o = pair(Lattice, fill, obst, "lsqr", precision=precision, sigma=1e-3, tau=1.0)
    g.step(50)
    o.step(50)
    compare(g, o, 2e-3, exact_flags=False, what=f"{precision}", vscale=1e-3 / (0.5 / 3.0))


def _fields(lat):
    return lat.flags(), lat.fill(), lat.velocity(), lat.pressure(), lat.curvature()


def test_batch_and_graph_replay_match_eager_steps(Lattice):
    """Four lattices (FD/LSQR, SRT/TRT, different sigma and tau) stepped one
    by one, as one batch, and as one batch replayed from HIP graphs: all three
    give bit-identical states, checked after every graph replay with eager
    work and synchronisation in between."""
    import torch

    from paper_1509_07691_amd.fslbm import Batch

    fill, obst = I.droplet(24, 6.0, noise=1e-6, seed=3)
    sfill, sobst = I.sessile_droplet(24, 24, 12, 6.0, noise=1e-6)
    specs = [(fill, obst, dict(curv_model="fd", sigma=1e-3, tau=1.0)),
             (fill, obst, dict(curv_model="lsqr", sigma=1e-4, tau=0.6)),
             (sfill, sobst, dict(curv_model="lsqr", sigma=2e-3, tau=0.8, theta=math.radians(60))),
             (sfill, sobst, dict(curv_model="fd", sigma=1e-3, tau=0.7, collision="trt"))]
    s = torch.cuda.Stream()
    mk = lambda: [Lattice(f, o, precision="f64", stream=s, **kw) for f, o, kw in specs]
    eager, batched, graphed, split = mk(), mk(), mk(), mk()
    b1 = Batch(batched)
    b2 = Batch(graphed)
    b2.set_graph(True)
    b3 = Batch(split)
    b3.set_split_interface(True)
    for rep in range(6):
        for lat in eager:
            lat.step(3)
        b1.step(3)
        b2.step(3)
        b3.step(3)
        torch.cuda.synchronize()
        for e, x, g, sp in zip(eager, batched, graphed, split):
            fe = _fields(e)
            for a, b_, c, d in zip(fe, _fields(x), _fields(g), _fields(sp)):
                np.testing.assert_array_equal(a, b_)
                np.testing.assert_array_equal(a, c)
                np.testing.assert_array_equal(a, d)
    for bb in (b1, b2, b3):
        bb.close()


def test_advection_test_fp64(Lattice):
    """Pure advection (Sec. III.A): sigma = 0, f = feq(1, u0), gas bubble of
    diameter 10 translated by its diameter; cell types, interface lists and
    fill levels against the oracle."""
    d, u0 = 10, 0.05
    fill, obst = I.advected_bubble(d)
    g, o = pair(Lattice, fill, obst, "fd", sigma=0.0, tau=1.0)
    u = np.zeros((3,) + fill.shape)
    u[0] = u0
    g.set_equilibrium(1.0, u)
    o.set_equilibrium(np.ones(fill.shape), u)
    for n in (50, 150):
        g.step(n)
        o.step(n)
        compare(g, o, 1e-10, what=f"advection after +{n}")
    l1g = I.advection_errors(fill, g.fill(), d)
    l1o = I.advection_errors(fill, o.fill(), d)
    assert abs(l1g[0] - l1o[0]) < 1e-12 and abs(l1g[1] - l1o[1]) < 1e-12


@pytest.mark.parametrize("model", ["fd", "lsqr", "tr"])
def test_bubble_model_fp64(Lattice, model):
    """Equilibrium-bubble setup (walls at z = 0, 1) with the bubble model:
    the gas density follows the gas volume every step."""
    fill, obst = I.laplace_bubble(32)
    g, o = pair(Lattice, fill, obst, model, sigma=1e-3, tau=0.8, bubble=True)
    assert g.gas_density() == o.gas_density() == 1.0
    g.step(200)
    o.step(200)
    compare(g, o, 1e-10, what=f"bubble {model}", vscale=1e-3 / (0.3 / 3.0))
    assert g.gas_density() != 1.0
    assert abs(g.gas_density() - o.gas_density()) < 1e-13


def test_moving_bubble_fp64(Lattice):
    """Moving frame of reference: a uniform background velocity along x,
    the bubble model and LSQR curvature."""
    fill, obst = I.laplace_bubble(32)
    g, o = pair(Lattice, fill, obst, "lsqr", sigma=1e-3, tau=0.8, bubble=True)
    u = np.zeros((3,) + fill.shape)
    u[0] = 0.02
    g.set_equilibrium(1.0, u)
    o.set_equilibrium(1.0, u)
    g.step(150)
    o.step(150)
    compare(g, o, 1e-10, what="moving bubble", vscale=0.02)
    assert abs(g.gas_density() - o.gas_density()) < 1e-13


def test_bubble_model_fp32(Lattice):
    fill, obst = I.laplace_bubble(32)
    g, o = pair(Lattice, fill, obst, "lsqr", precision="f32", sigma=1e-3, tau=0.8, bubble=True)
    g.step(100)
    o.step(100)
    compare(g, o, 1e-5, exact_flags=False, what="bubble f32", vscale=1e-3 / (0.3 / 3.0))
    assert abs(g.gas_density() - o.gas_density()) / o.gas_density() < 1e-5


def test_tr_at_walls_fp64(Lattice):
    """TR has no wetting model: at a wall its fans are open on the wall side."""
    fill, obst = I.sessile_droplet(32, 32, 20, 9.0, noise=1e-6, seed=2)
    g, o = pair(Lattice, fill, obst, "tr", sigma=1e-3, tau=0.8)
    ifc = o.flags() == O.INTERFACE
    np.testing.assert_allclose(g.curvature()[ifc], o.curvature()[ifc], rtol=0, atol=1e-11)
    g.step(60)
    o.step(60)
    compare(g, o, 1e-10, what="tr walls", vscale=1e-3 / (0.3 / 3.0))


def test_tr_curvature_fp32(Lattice):
    fill, obst = I.droplet(32, 8.0, noise=1e-6, seed=0)
    g, o = pair(Lattice, fill, obst, "tr", precision="f32", sigma=1e-3, tau=1.0)
    g.step(50)
    o.step(50)
    compare(g, o, 1e-5, exact_flags=False, what="tr f32", vscale=1e-3 / (0.5 / 3.0))


def _diagnostics_reference(o, rho_gas):
    """The diagnostics written out on the oracle's fields: |u| over the fluid
    cells, and the pressure jump over the liquid cells with no gas or
    interface cell within a Euclidean distance of 2.5 cells (periodic)."""
    fl, u, rho = o.flags(), o.velocity(), o.density()
    fluid = (fl == O.LIQUID) | (fl == O.INTERFACE)
    speed = np.sqrt((u ** 2).sum(0))[fluid]
    surface = (fl == O.GAS) | (fl == O.INTERFACE)
    near = np.zeros_like(surface)
    for dz in range(-2, 3):
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                if dx * dx + dy * dy + dz * dz <= 6:
                    near |= np.roll(surface, (dz, dy, dx), axis=(0, 1, 2))
    inner = (fl == O.LIQUID) & ~near
    dp = (rho[inner].mean() - rho_gas) / 3.0 if inner.any() else 0.0
    return speed.max(), speed.mean(), dp, int(inner.sum())


@pytest.mark.parametrize("case", ["droplet_fd_f64", "bubble_lsqr_f64", "droplet_lsqr_f32"])
def test_diagnostics_vs_oracle(Lattice, case):
    """fslbm_diagnostics (device FP64 reductions) against the same measures
    taken on the oracle's fields: the static droplet of the Laplace test
    (a positive jump near 2 sigma / R), and the wall-bounded bubble with the
    bubble model (a negative jump against the current gas density)."""
    if case.startswith("bubble"):
        fill, obst = I.laplace_bubble(32)
        kw = dict(sigma=1e-3, tau=0.8, bubble=True)
        steps, uscale = 150, 1e-3 / (0.3 / 3.0)
    else:
        fill, obst = I.droplet(32, 8.0, noise=1e-6, seed=0)
        kw = dict(sigma=1e-3, tau=1.0)
        steps, uscale = 150, 1e-3 / (0.5 / 3.0)
    model = case.split("_")[1]
    precision = case.split("_")[2]
    tol = 1e-10 if precision == "f64" else 1e-5
    g, o = pair(Lattice, fill, obst, model, precision=precision, **kw)
    g.step(steps)
    o.step(steps)
    d = g.diagnostics()
    u_max, u_mean, dp, n_inner = _diagnostics_reference(o, o.gas_density())
    print(case, d, (u_max, u_mean, dp, n_inner))
    assert d["n_inner"] == n_inner > 0
    assert abs(d["max_u"] - u_max) <= tol * max(u_max, uscale)
    assert abs(d["mean_u"] - u_mean) <= tol * max(u_mean, uscale)
    # the jump is a difference of two pressures near 1/3: its bar is the
    # pressure bar
    assert abs(d["dp"] - dp) <= tol * max(abs(dp), o.gas_density() / 3.0)
    assert (dp > 0) == case.startswith("droplet")
    if precision == "f64":
        # the reduction's max is the max over the library's own read-out
        ug = g.velocity()
        fl = g.flags()
        fluid = (fl == O.LIQUID) | (fl == O.INTERFACE)
        assert d["max_u"] == np.sqrt((ug ** 2).sum(0))[fluid].max()


@pytest.mark.parametrize("precision", ["f32", "f16", "bf16"])
def test_split_passes_equal_the_merged_pass(Lattice, precision):
    """The shifted storage forms: the two-pass step (lean pass over the
    plain liquid cells, which works in the units of the store, and the
    interface and wall cells from their lists; one launch in FP32, two in
    the 16-bit forms) equals the one-pass step bit for bit, stochastic
    rounding included (its bits depend on cell and step only). Cases: a
    moving gas bubble in liquid with even and odd nx, and a sessile drop
    with walls. The automatic choice takes the two passes for a 16-bit
    lattice that is nearly all liquid and one pass for the small boxes."""
    cases = []
    for nx in (24, 25):
        fill = np.clip(1.0 - I.sphere_fraction((24, 24, nx), (nx / 2, 12.0, 12.0), 5.0), 0.0, 1.0)
        cases.append((fill, None, dict(curv_model="lsqr", sigma=1e-3, tau=0.8), True))
    sfill, sobst = I.sessile_droplet(24, 24, 12, 6.0, noise=1e-6)
    cases.append((sfill, sobst, dict(curv_model="lsqr", sigma=2e-3, tau=0.8, theta=math.radians(70)), False))
    for fill, obst, kw, moving in cases:
        lats = [Lattice(fill, obst, precision=precision, **kw) for _ in range(2)]
        lats[0].set_split_interface(False)
        lats[1].set_split_interface(True)
        if moving:
            u = np.zeros((3,) + fill.shape)
            u[0], u[1] = 0.03, -0.02
            for lat in lats:
                lat.set_equilibrium(1.0, u)
        for lat in lats:
            lat.step(25)
        assert not lats[0].split_active() and lats[1].split_active()
        for a, b in zip(_fields(lats[0]), _fields(lats[1])):
            np.testing.assert_array_equal(a, b)
        for lat in lats:
            lat.close()
    # the automatic choice (FP32 always takes the merged pass, measured the
    # faster on every workload)
    fill = np.clip(1.0 - I.sphere_fraction((64, 64, 64), (32.0, 32.0, 32.0), 4.0), 0.0, 1.0)
    big = Lattice(fill, None, precision=precision, curv_model="lsqr", sigma=1e-3, tau=0.8)
    big.step(2)
    assert big.split_active() == (precision != "f32")
    big.close()
    fill, obst = I.droplet(24, 6.0, noise=1e-6, seed=3)
    small = Lattice(fill, obst, precision=precision, curv_model="lsqr", sigma=1e-3, tau=0.8)
    small.step(2)
    assert not small.split_active()
    small.close()

"""Pins of the tangent-linear oracle (the reference source built with dual
numbers, frozen cell types): its values are the plain oracle's bit for bit,
and its directional derivatives of a linear functional of phi_T agree with
central differences of the plain oracle, Richardson-extrapolated over the
step and twice the step, for sigma (droplets, SRT and TRT, moving or at
rest), theta (sessile drops: the FD contact normal, the LSQR contact
condition) and the initial fill level (a seeded direction on the interface
cells), with the FD, LSQR and TR curvature models. The LSQR and TR cases
also pin the implicit derivative of the PLIC offset that replaces the
bisection's."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1509_07691_amd import inputs as I

T = 24


def _case(name):
    model = {"lsqr": O.CURV_LSQR, "tr": O.CURV_TR}.get(name.split("_")[0], O.CURV_FD)
    fill, obst, prm, u = _case_fd(name.split("_", 1)[1] if model != O.CURV_FD else name)
    prm["curv_model"] = model
    return fill, obst, prm, u


def _case_fd(name):
    if name == "droplet":
        fill, obst = I.droplet(20, 5.0, noise=1e-6, seed=6)
        return fill, obst, dict(sigma=5e-3, tau=0.8, theta=math.pi / 2), None
    if name == "droplet_moving":
        fill, obst = I.droplet(20, 5.0, noise=1e-6, seed=3)
        u = np.zeros((3,) + fill.shape)
        u[0], u[1] = 0.02, -0.01
        return fill, obst, dict(sigma=5e-3, tau=0.8, theta=math.pi / 2), u
    if name == "droplet_trt":
        fill, obst = I.droplet(20, 5.0, noise=1e-6, seed=4)
        return fill, obst, dict(sigma=5e-3, tau=0.7, theta=math.pi / 2, collision=O.TRT), None
    fill, obst = I.sessile_droplet(22, 22, 12, 6.0, noise=1e-6, seed=7)
    return fill, obst, dict(sigma=5e-3, tau=0.8, theta=math.radians(70.0)), None


def _plain(fill, obst, prm, u):
    o = O.Oracle(fill, obst, frozen=True, **prm)
    if u is not None:
        o.set_equilibrium(np.ones(fill.shape), u)
    o.step(T)
    return o.fill()


def _tl(fill, obst, prm, u, **seed):
    t = O.TangentLinear(fill, obst, **prm, **seed)
    if u is not None:
        t.set_equilibrium(1.0, u)
    t.step(T)
    return t.fill_and_derivative()


def _richardson(f, x, e):
    d1 = (f(x + e) - f(x - e)) / (2 * e)
    d2 = (f(x + 2 * e) - f(x - 2 * e)) / (4 * e)
    return (4 * d1 - d2) / 3


# The PLIC models are pinned at rest: in a moving droplet some cells pass
# close to phi = 0 within the window, where the offset goes like phi^(1/3)
# and a difference step of 1e-5 is no longer in the smooth regime.
@pytest.mark.parametrize("name", ["droplet_moving", "droplet_trt", "sessile", "lsqr_droplet", "lsqr_sessile",
                                  "tr_droplet"])
def test_tangent_linear_values_and_derivatives(name):
    fill, obst, prm, u = _case(name)
    ifc = O.Oracle(fill, obst, frozen=True).flags() == O.INTERFACE
    rng = np.random.default_rng(5)
    w = rng.uniform(-1.0, 1.0, fill.shape)
    v = rng.uniform(-1.0, 1.0, fill.shape) * ifc * (fill > 1e-3) * (fill < 1 - 1e-3)

    phi = _plain(fill, obst, prm, u)
    val, dsig = _tl(fill, obst, prm, u, dsigma=1.0)
    assert np.array_equal(val, phi)

    def L(**over):
        p = dict(prm)
        fl = over.pop("fill", fill)
        p.update(over)
        return float((w * _plain(fl, obst, p, u)).sum())

    checks = {"sigma": ((w * dsig).sum(), _richardson(lambda x: L(sigma=x), prm["sigma"], 1e-4 * prm["sigma"]))}
    _, ddir = _tl(fill, obst, prm, u, fill_dot=v)
    checks["fill"] = ((w * ddir).sum(), _richardson(lambda x: L(fill=fill + x * v), 0.0, 1e-5))
    if obst.any():
        _, dth = _tl(fill, obst, prm, u, dtheta=1.0)
        checks["theta"] = ((w * dth).sum(), _richardson(lambda x: L(theta=x), prm["theta"], 1e-4))
    for k, (tl, fd) in checks.items():
        print(name, k, tl, fd)
        assert abs(tl - fd) <= 1e-6 * abs(fd), (k, tl, fd)


def test_stored_benchmark_window_tangent_linear_matches_differences():
    """The stored oracle values of the differentiation workload
    (tests/golden/make_adjoint_c4_reference.py): over the window in which
    every interface fill stays inside (0, 1) the tangent-linear derivatives
    agree with the oracle's extrapolated central differences; over the
    longer window, where fills cross 0, the loss is only piecewise smooth
    and the two may differ by percents."""
    ref = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_c4_oracle.json")))
    assert 1 <= ref["T_inside"] <= ref["T_unconverted"] <= ref["TMAX"]
    inside = [w for w in ref["windows"] if w["T"] <= ref["T_inside"]]
    assert inside
    for w in inside:
        lo, hi = w["interface_fill_range_T"]
        assert 0.0 < lo and hi < 1.0
        for k, tl in w["tangent_linear"].items():
            cd = w["central_differences"][k]
            assert abs(tl - cd) <= 1e-7 * abs(tl), (w["T"], k, tl, cd)

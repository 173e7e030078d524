"""Writes adjoint_c4_oracle.json, the reference of the differentiation
workload at its configured size: a sessile drop (hemisphere R = 24 centred
on the wall z = 1 of a 128^3 lattice, obstacle layers k = 0 and 127,
periodic x, y, exact volume fractions plus 1e-6 noise on interface cells,
seed 1), LSQR curvature with the contact condition, sigma 1e-3, tau 0.8,
theta 90 deg, cell types frozen.

1. Window lengths of the FP64 oracle from the start (searched up to TMAX
   steps): T_inside, the steps before an interface fill first leaves
   (0, 1); T_unconverted, the steps before a fill first leaves
   [-eps, 1 + eps] (eps = 1e-3, the conversion offset), i.e. before the
   method with free cell types would first fill or empty a cell. Up to
   T_unconverted the frozen window is the method's own trajectory.
2. For each window T in (T_inside, min(T_unconverted, TWIN)): the loss
   L = sum over non-obstacle cells of (phi_T - phi*)^2, phi* the same
   window's result at theta 70 deg and sigma 8e-4, and its derivatives along
   sigma, theta (radians) and a seeded direction v of phi_0 (uniform in
   [-1, 1] on the interface cells with 1e-3 < phi_0 < 1 - 1e-3, numpy
   default_rng(3)), each from the oracle's tangent-linear build and from
   central differences of the oracle (Richardson over the step h and 2h:
   h = 1e-4 sigma, 1e-4 rad, 1e-5).

Calls only the oracle and the seeded input generator. Run from the
repository root:  python tests/golden/make_adjoint_c4_reference.py
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1509_07691_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_c4_oracle.json")
TMAX = 2000
TWIN = 600
EPS_C = 1e-3
SIGMA, THETA, TAU = 1e-3, math.pi / 2, 0.8
SIGMA_T, THETA_T = 8e-4, math.radians(70.0)


def inputs():
    return I.sessile_droplet(128, 128, 128, 24.0, noise=1e-6, seed=1)


def frozen(fill, obst, sigma, theta):
    return O.Oracle(fill, obst, sigma=sigma, tau=TAU, theta=theta, curv_model=O.CURV_LSQR, frozen=True)


def window(fill, obst, ifc, T):
    """Loss and its derivatives (tangent-linear and differences) over T steps."""
    t0 = time.time()
    keep = (obst == 0).astype(float)
    target = frozen(fill, obst, SIGMA_T, THETA_T)
    target.step(T)
    phis = target.fill()
    v = np.random.default_rng(3).uniform(-1.0, 1.0, fill.shape) * (ifc & (fill > 1e-3) & (fill < 1 - 1e-3))

    def L(sigma=SIGMA, theta=THETA, x=0.0):
        o = frozen(fill + x * v, obst, sigma, theta)
        o.step(T)
        return float((((o.fill() - phis) * keep) ** 2).sum())

    def rich(f, x, e):
        return (4 * (f(x + e) - f(x - e)) / (2 * e) - (f(x + 2 * e) - f(x - 2 * e)) / (4 * e)) / 3

    o = frozen(fill, obst, SIGMA, THETA)
    o.step(T)
    phiT = o.fill()
    g = 2.0 * (phiT - phis) * keep

    def tl(**seed):
        t = O.TangentLinear(fill, obst, sigma=SIGMA, tau=TAU, theta=THETA, curv_model=O.CURV_LSQR, **seed)
        t.step(T)
        val, dot = t.fill_and_derivative()
        assert np.array_equal(val, phiT)
        return float((g * dot).sum())

    res = {"T": T, "loss": float((((phiT - phis) * keep) ** 2).sum()),
           "interface_fill_range_T": [float(phiT[ifc].min()), float(phiT[ifc].max())],
           "tangent_linear": {"sigma": tl(dsigma=1.0), "theta": tl(dtheta=1.0), "phi0_dir": tl(fill_dot=v)}}
    print(T, "tangent-linear", res["tangent_linear"], f"({time.time() - t0:.0f} s)", flush=True)
    res["central_differences"] = {"sigma": rich(lambda s: L(sigma=s), SIGMA, 1e-4 * SIGMA),
                                  "theta": rich(lambda th: L(theta=th), THETA, 1e-4),
                                  "phi0_dir": rich(lambda x: L(x=x), 0.0, 1e-5)}
    print(T, "differences", res["central_differences"], f"({time.time() - t0:.0f} s)", flush=True)
    return res


def main():
    t0 = time.time()
    fill, obst = inputs()
    o = frozen(fill, obst, SIGMA, THETA)
    ifc = o.flags() == O.INTERFACE
    t_in = t_unconv = None
    for t in range(1, TMAX + 1):
        o.step(1)
        ph = o.fill()[ifc]
        if t_in is None and not (np.all(ph > 0.0) and np.all(ph < 1.0)):
            t_in = t - 1
        if not (np.all(ph >= -EPS_C) and np.all(ph <= 1.0 + EPS_C)):
            t_unconv = t - 1
            break
    t_in = TMAX if t_in is None else t_in
    t_unconv = TMAX if t_unconv is None else t_unconv
    print(f"T_inside = {t_in}, T_unconverted = {t_unconv} (searched to {TMAX}; {time.time() - t0:.0f} s)", flush=True)
    res = {"TMAX": TMAX, "eps_c": EPS_C, "T_inside": t_in, "T_unconverted": t_unconv, "windows": []}
    for T in sorted({t_in, min(t_unconv, TWIN)}):
        if T > 0:
            res["windows"].append(window(fill, obst, ifc, T))
    with open(OUT, "w") as fh:
        json.dump(res, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()

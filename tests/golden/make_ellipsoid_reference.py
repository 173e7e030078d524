"""Writes ellipsoid128_oracle.npz: the FP64 oracle's state of the oscillating
droplet's 128^3 downscale (ellipsoid 24/20/20 centred in a periodic 128^3
lattice, sigma = 1e-3, tau = 0.55, LSQR curvature, exact volume fractions
plus 1e-6 noise on interface cells, seed 0) after 10,000 steps, and the x
semi-axis a(t) = sqrt(5 <(x - <x>)^2>) of the fill level every 250 steps.

Calls only the oracle and the seeded input generator. Run from the
repository root:  python tests/golden/make_ellipsoid_reference.py
(about 25 minutes on one core).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1509_07691_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ellipsoid128_oracle.npz")
STEPS, EVERY = 10000, 250


def semi_axis_x(phi):
    x = np.arange(phi.shape[2]) + 0.5
    px = phi.sum(axis=(0, 1))
    w = px.sum()
    mx = (px * x).sum() / w
    return float(np.sqrt(5.0 * (px * (x - mx) ** 2).sum() / w))


def main():
    fill, obst = I.ellipsoid_droplet(128, (24, 20, 20), noise=1e-6, seed=0)
    orc = O.Oracle(fill, obst, sigma=1e-3, tau=0.55, curv_model=O.CURV_LSQR)
    m0 = orc.mass()
    ts, a = [0], [semi_axis_x(orc.fill())]
    t0 = time.time()
    for t in range(EVERY, STEPS + 1, EVERY):
        orc.step(EVERY)
        ts.append(t)
        a.append(semi_axis_x(orc.fill()))
        print(f"t={t} a={a[-1]:.4f} ({time.time() - t0:.0f} s)", flush=True)
    fl = orc.flags()
    fluid = np.flatnonzero((fl.reshape(-1) == O.LIQUID) | (fl.reshape(-1) == O.INTERFACE)).astype(np.int32)
    phi = orc.fill().reshape(-1)[fluid]
    rho = orc.density().reshape(-1)[fluid]
    u = orc.velocity().reshape(3, -1)[:, fluid]
    np.savez_compressed(OUT, steps=STEPS, flags=fl.astype(np.uint8), fluid_index=fluid, phi=phi, rho=rho, u=u,
                        mass0=m0, mass=orc.mass(), a_t=np.array(ts), a=np.array(a))
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()

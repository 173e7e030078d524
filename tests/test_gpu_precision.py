"""Error of the reduced-precision forms (FP32 arithmetic and storage; FP32
arithmetic with f - w_q stored in FP16 (scale 2^12) or BF16) against the
FP64 oracle on the oscillating-droplet workload scaled down to 128^3:
ellipsoid semi-axes 24/20/20 (x, y, z) at the centre, sigma 1e-3,
tau 0.55, LSQR curvature, 100 steps with cell conversions.

Reported per precision: relative L2 error of the fill level and of the
pressure over the oracle's fluid cells, velocity error normalised by
max(|u_ref|, sigma/mu) (mu = rho nu), the fraction of cells whose type
differs from the oracle's, and the mass drift |M(t) - M(0)| / M(0).
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_1509_07691_amd import inputs as I

pytestmark = pytest.mark.gpu

STEPS = 100
PRM = dict(sigma=1e-3, tau=0.55)
# about ten times the errors measured on MI355X (FP32 fill 7.9e-6, velocity
# 7.7e-6, mass drift 2.8e-6; F16 2.2e-5, 1.0e-5, 9.3e-6; BF16 5.4e-5,
# 2.3e-5, 2.3e-5; up to 5e-7 of the cells typed differently in BF16)
BARS = {"f32": dict(fill=1e-4, vel=1e-4, flags=1e-5, mass=3e-5),
        "f16": dict(fill=3e-4, vel=2e-4, flags=1e-5, mass=1e-4),
        "bf16": dict(fill=6e-4, vel=3e-4, flags=1e-5, mass=3e-4)}


@pytest.fixture(scope="module")
def reference():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    fill, obst = I.ellipsoid_droplet(128, (24, 20, 20), noise=1e-6, seed=0)
    o = O.Oracle(fill, obst, curv_model=O.CURV_LSQR, **PRM)
    M0 = o.mass()
    o.step(STEPS)
    return fill, obst, dict(fill=o.fill(), p=o.pressure(), u=o.velocity(), flags=o.flags(), mass=o.mass(), M0=M0)


@pytest.mark.parametrize("precision", ["f32", "f16", "bf16"])
def test_ellipsoid_downscale_errors(reference, precision):
    from paper_1509_07691_amd.fslbm import Lattice

    fill, obst, ref = reference
    g = Lattice(fill, obst, precision=precision, curv_model="lsqr", **PRM)
    M0 = g.mass()
    g.step(STEPS)
    fl = ref["flags"]
    fluid = (fl == O.LIQUID) | (fl == O.INTERFACE)
    e_fill = np.linalg.norm((g.fill() - ref["fill"])[fluid]) / np.linalg.norm(ref["fill"][fluid])
    e_p = np.linalg.norm((g.pressure() - ref["p"])[fluid]) / np.linalg.norm(ref["p"][fluid])
    mu = (PRM["tau"] - 0.5) / 3.0
    du = np.sqrt(((g.velocity() - ref["u"]) ** 2).sum(0))[fluid]
    uref = np.sqrt((ref["u"] ** 2).sum(0))[fluid]
    e_u = np.linalg.norm(du) / max(np.linalg.norm(uref), PRM["sigma"] / mu * np.sqrt(fluid.sum()))
    e_flags = float((g.flags() != fl).mean())
    drift = abs(g.mass() - M0) / M0
    print(f"{precision}: fill {e_fill:.3e} pressure {e_p:.3e} velocity {e_u:.3e} "
          f"flags {e_flags:.2e} mass drift {drift:.2e} (oracle drift {abs(ref['mass'] - ref['M0']) / ref['M0']:.1e})")
    b = BARS[precision]
    assert e_fill < b["fill"] and e_u < b["vel"] and e_flags < b["flags"] and drift < b["mass"]


GOLDEN_C3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ellipsoid128_oracle.npz")
LONG_STEPS = 10000
# errors after 10,000 steps: the oscillation accumulates phase, and the
# FP32 arithmetic converts some interface cells a step earlier or later than
# the oracle, so the fill error is carried by a few hundred cells typed
# differently; the semi-axis a(t) and the mass are the smooth measures. The
# bars are about three times the values measured on MI355X (FP32: fill
# 1.9e-2 to 2.7e-2, velocity 1.5e-3 to 2.1e-3, cells 2.1e-4 to 2.7e-4, mass
# drift 8.1e-8, semi-axis 1.6e-3 to 2.0e-3; F16 3.6e-2 to 5.6e-2, 2.0e-3,
# 3.0e-4 to 5.0e-4, 7.6e-8, 1.2e-3; BF16 1.8e-2, 1.7e-3 to 2.0e-3, 1.6e-4 to
# 2.3e-4, 1.5e-8 to 3.2e-7, 5.9e-4 to 9.6e-4; other runs of the 16-bit forms
# up to 6.5e-2 and 6.2e-4 for fill and cells), printed by the test; the
# spread between builds that differ only in rounding is the conversion
# timing of single cells, not a trend. The stochastic 16-bit
# stores make the mass a random walk (zero mean, spread growing like the
# square root of the steps; 0.8e-7 to 3.6e-7 seen), so their mass bar is
# 1e-6.
LONG_BARS = {"f32": dict(fill=6e-2, vel=7e-3, flags=7e-4, mass=3e-7, axis=5e-3),
             "f16": dict(fill=0.15, vel=7e-3, flags=1.5e-3, mass=1e-6, axis=5e-3),
             "bf16": dict(fill=0.2, vel=7e-3, flags=2e-3, mass=1e-6, axis=5e-3)}


def _refined_min(a, every):
    """Step of the smallest sample of a series, refined by a parabola through
    it and its two neighbours; and its index."""
    k = int(np.argmin(a))
    if 0 < k < len(a) - 1:
        den = a[k - 1] - 2 * a[k] + a[k + 1]
        if den:
            return (k + 0.5 * (a[k - 1] - a[k + 1]) / den) * every, k
    return float(k * every), k


def _rising_crossing(a, every, k0, level):
    """Step at which the series first rises through `level` after sample k0
    (linear interpolation between samples), or None."""
    for k in range(k0, len(a) - 1):
        if a[k] < level <= a[k + 1]:
            return (k + (level - a[k]) / (a[k + 1] - a[k])) * every
    return None


def _semi_axis_x(phi):
    x = np.arange(phi.shape[2]) + 0.5
    px = phi.sum(axis=(0, 1))
    w = px.sum()
    mx = (px * x).sum() / w
    return float(np.sqrt(5.0 * (px * (x - mx) ** 2).sum() / w))


@pytest.mark.parametrize("precision", ["f32", "f16", "bf16"])
def test_ellipsoid_downscale_errors_after_10000_steps(precision):
    """The same workload over the oscillating droplet's configured length,
    10,000 steps, against the FP64 oracle's state stored by
    tests/golden/make_ellipsoid_reference.py (oracle and seeded inputs only):
    fill level, pressure and velocity errors over the oracle's fluid cells,
    cells typed differently, mass drift, the x semi-axis a(t) of the
    oscillation sampled every 250 steps against the oracle's (largest
    difference relative to a(0)), and the timing of the oscillation (the step
    of its first minimum and of the rise after it)."""
    import torch

    from paper_1509_07691_amd.fslbm import Lattice

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ref = np.load(GOLDEN_C3)
    assert int(ref["steps"]) == LONG_STEPS
    fill, obst = I.ellipsoid_droplet(128, (24, 20, 20), noise=1e-6, seed=0)
    g = Lattice(fill, obst, precision=precision, curv_model="lsqr", **PRM)
    M0 = g.mass()
    a = [_semi_axis_x(g.fill())]
    for _ in range(LONG_STEPS // 250):
        g.step(250)
        a.append(_semi_axis_x(g.fill()))
    idx = ref["fluid_index"]
    fl = g.flags().reshape(-1)
    e_flags = float((fl != ref["flags"].reshape(-1)).mean())
    phi = g.fill().reshape(-1)[idx]
    p = g.pressure().reshape(-1)[idx]
    u = g.velocity().reshape(3, -1)[:, idx]
    e_fill = np.linalg.norm(phi - ref["phi"]) / np.linalg.norm(ref["phi"])
    e_p = np.linalg.norm(p - ref["rho"] / 3.0) / np.linalg.norm(ref["rho"] / 3.0)
    mu = (PRM["tau"] - 0.5) / 3.0
    du = np.sqrt(((u - ref["u"]) ** 2).sum(0))
    uref = np.sqrt((ref["u"] ** 2).sum(0))
    e_u = np.linalg.norm(du) / max(np.linalg.norm(uref), PRM["sigma"] / mu * np.sqrt(idx.size))
    drift = abs(g.mass() - M0) / M0
    e_axis = np.abs(np.array(a) - ref["a"]).max() / ref["a"][0]
    # the oscillation's timing: the step of its first minimum (sharp: the
    # oracle's near 3030) and the step at which a(t) rises back through the
    # level halfway between the oracle's minimum and its following maximum
    # (about 4190), both within one sample spacing of the oracle's. The
    # maximum itself is too flat to time: between 8000 and 10000 steps the
    # oracle's a(t) varies by 0.04 cells, as much as the GPU's a(t) error.
    ra = np.asarray(ref["a"])
    t_min_ref, k_ref = _refined_min(ra, 250)
    level = 0.5 * (ra[k_ref] + ra[k_ref:].max())
    t_up_ref = _rising_crossing(ra, 250, k_ref, level)
    t_min, k_g = _refined_min(np.asarray(a), 250)
    t_up = _rising_crossing(np.asarray(a), 250, k_g, level)
    print(f"{precision}: a(t) minimum at {t_min:.0f} steps (oracle {t_min_ref:.0f}), rises through {level:.3f} "
          f"at {t_up if t_up is None else round(t_up)} (oracle {t_up_ref:.0f})")
    assert abs(t_min - t_min_ref) < 250 and t_up is not None and abs(t_up - t_up_ref) < 250
    print(f"{precision} after {LONG_STEPS} steps: fill {e_fill:.3e} pressure {e_p:.3e} velocity {e_u:.3e} "
          f"flags {e_flags:.2e} mass drift {drift:.2e} semi-axis {e_axis:.2e} "
          f"(oracle drift {abs(float(ref['mass']) - float(ref['mass0'])) / float(ref['mass0']):.1e})", flush=True)
    g.close()
    b = LONG_BARS[precision]
    assert e_fill < b["fill"] and e_u < b["vel"] and e_flags < b["flags"]
    assert drift < b["mass"] and e_axis < b["axis"]

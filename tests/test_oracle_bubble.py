"""Pins of the oracle's bubble model (Sec. III.A.1): the gas of the lattice
is one bubble with isothermal pressure, p_g(t) V(t) = p_g(0) V(0).

- The Laplace jump across the bubble surface at equilibrium.
- The equilibrium gas density predicted without simulation from the two
  weakly compressible volumes: the gas obeys rho_g V = rho_0 V0, the liquid
  keeps its mass M = rho_l (N_free - V), and rho_g - rho_l = 3 (2 sigma/R).
  Dropping the model (constant rho_gas) or a wrong volume fails it.
- The isothermal invariant rho_g V = rho_0 V0 with V summed from the fill
  levels that the oracle reports.
- The parameters of the paper's resolution study (tau and sigma_L printed in
  Sec. III.A.1) from the physical units of the problem.
"""
import numpy as np
import pytest

import oracle as O
from paper_1509_07691_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

N, R, SIGMA = 32, 8.0, 1e-3


def _bubble_box():
    fill = 1.0 - I.sphere_fraction((N, N, N), (N / 2, N / 2, N / 2), R)
    fill = np.clip(fill, 0.0, 1.0)
    obst = np.zeros(fill.shape, np.uint8)
    obst[0] = obst[-1] = 1
    fill[0] = fill[-1] = 0.0
    return fill, obst


def _liquid_pressure(o):
    from scipy import ndimage

    fl = o.flags()
    near = (fl == O.GAS) | (fl == O.INTERFACE)
    far = (fl == O.LIQUID) & (ndimage.distance_transform_edt(~near) > 3)
    return o.density()[far].mean() / 3.0


@pytest.fixture(scope="module")
def bubble_run():
    fill, obst = _bubble_box()
    o = O.Oracle(fill, obst, sigma=SIGMA, tau=1.0, curv_model=O.CURV_FD, bubble=True)
    free = obst == 0
    # V0 from the fill levels after the interface layer's closure at creation
    v0 = float((1.0 - o.fill())[free].sum())
    m0 = o.mass()
    o.step(300)
    return o, fill, obst, v0, m0


def test_laplace_jump_with_bubble_model(bubble_run):
    o, *_ = bubble_run
    dp = o.gas_density() / 3.0 - _liquid_pressure(o)
    assert abs(dp - 2 * SIGMA / R) / (2 * SIGMA / R) < 0.1, dp


def test_equilibrium_gas_density_prediction(bubble_run):
    o, fill, obst, v0, _ = bubble_run
    n_free = float((obst == 0).sum())
    vl0 = n_free - v0  # liquid at unit density fills the rest
    eps = 3 * (2 * SIGMA / R) / (1.0 + v0 / vl0)
    got = o.gas_density() - 1.0
    assert abs(got - eps) / eps < 0.1, (got, eps)


def test_isothermal_invariant_and_mass(bubble_run):
    o, fill, obst, v0, m0 = bubble_run
    free = obst == 0
    v = float((1.0 - o.fill())[free].sum())
    assert abs(o.gas_density() * v - v0) / v0 < 1e-12
    assert abs(o.mass() - m0) / m0 < 1e-12


def test_constant_gas_density_without_bubble_model():
    fill, obst = _bubble_box()
    o = O.Oracle(fill, obst, sigma=SIGMA, tau=1.0, curv_model=O.CURV_FD, bubble=False)
    o.step(20)
    assert o.gas_density() == 1.0


def test_resolution_study_parameters():
    # tau and sigma_L / 1e-3 printed for dx = 1/48 ... 1/192 at dt = 1e-4
    printed = {48: (0.6728, 0.0987), 96: (1.191, 0.7896), 144: (2.055, 2.665), 192: (3.264, 6.317)}
    for n, (tau_p, sig_p) in printed.items():
        tau, sig = I.renardy_units(n)
        assert 0 <= tau - tau_p < 1e-3, (n, tau)  # printed truncated to 3 decimals
        assert abs(sig / 1e-3 - sig_p) / sig_p < 1e-3, (n, sig)
    # moving frame: dx = 1/96, dt = 2.5e-5 gives tau = 0.6728
    assert abs(I.renardy_units(96, 2.5e-5)[0] - 0.6728) < 1e-4

"""Pins of the oracle's frozen-topology mode, the setting in which the
adjoint window is differentiated (cell types held fixed, Sec. II without
the fill / empty conversion).

- Types never change and the mass M = sum_L rho + sum_I m stays constant
  (the mass-form exchange is antisymmetric per link, eqs. advection1/2).
- One step from equilibrium f' = feq(1, 0): the exchange uses only f'(0),
  so m_1 does not depend on sigma, while each gas link q of an interface
  cell receives f_in,q = feq_q(rho_b, 0) + feq_qbar(rho_b, 0) - f'_qbar =
  2 w_q rho_b - w_q with rho_b = rho_gas + 3 sigma K_0 (eq. reconstruct).
  Hence d phi_1/d sigma = -(m_1 / rho_1^2) * 6 K_0 * sum_{gas links} w_q
  in closed form; central differences of the oracle and its tangent-linear
  build must reproduce it.
"""
import numpy as np

import oracle as O
from paper_1509_07691_amd import inputs as I

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
# D3Q19 directions in the oracle's order (rest, 6 faces, 12 edges)
C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
              [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])


def test_frozen_types_and_mass_conserved():
    fill, obst = I.droplet(16, 4.5, noise=1e-6, seed=1)
    u = np.zeros((3,) + fill.shape)
    u[0] = 0.05
    u[2] = -0.03
    ref = O.Oracle(fill, obst, sigma=2e-3, tau=0.8)
    frz = O.Oracle(fill, obst, sigma=2e-3, tau=0.8, frozen=True)
    for o in (ref, frz):
        o.set_equilibrium(np.ones(fill.shape), u)
    fl0 = frz.flags().copy()
    M0 = frz.mass()
    ref.step(25)
    frz.step(25)
    assert (ref.flags() != fl0).sum() > 10, "the unfrozen run should convert cells"
    assert np.array_equal(frz.flags(), fl0)
    assert abs(frz.mass() - M0) <= 1e-13 * M0
    assert frz.reservoir() == 0.0


def test_one_step_sigma_derivative_closed_form():
    fill, obst = I.droplet(16, 4.5, noise=1e-6, seed=2)
    sigma, eps = 1e-2, 1e-4
    base = O.Oracle(fill, obst, sigma=sigma, tau=0.8, frozen=True)
    K0 = base.curvature()
    flags = base.flags()
    base.step(1)
    m1, rho1 = base.mass_field(), base.density()
    phis = []
    for s in (sigma * (1 + eps), sigma * (1 - eps)):
        o = O.Oracle(fill, obst, sigma=s, tau=0.8, frozen=True)
        o.step(1)
        phis.append(o.fill())
    fd = (phis[0] - phis[1]) / (2 * eps * sigma)
    # sum of w_q over the gas links: upstream node x - c_q is a gas cell
    gas = flags == O.GAS
    wsum = np.zeros(fill.shape)
    for q in range(1, 19):
        cx, cy, cz = C[q]
        up = np.roll(gas, shift=(cz, cy, cx), axis=(0, 1, 2))  # gas at x - c_q
        wsum += W[q] * up
    ifc = flags == O.INTERFACE
    closed = -(m1 / rho1 ** 2) * 6.0 * K0 * wsum
    assert np.abs(closed[ifc]).max() > 1e-4
    np.testing.assert_allclose(fd[ifc], closed[ifc], rtol=1e-6, atol=1e-12)
    assert np.abs(fd[~ifc]).max() == 0.0
    # the tangent-linear oracle gives the same derivative to rounding
    tl = O.TangentLinear(fill, obst, dsigma=1.0, sigma=sigma, tau=0.8)
    tl.step(1)
    _, dphi = tl.fill_and_derivative()
    np.testing.assert_allclose(dphi[ifc], closed[ifc], rtol=1e-10, atol=1e-15)
    assert np.abs(dphi[~ifc]).max() == 0.0

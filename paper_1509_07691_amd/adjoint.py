"""Differentiation form of the FSLBM step: a frozen-topology window as a
torch.autograd.Function.

phi_T = W(phi_0, sigma, theta) runs T steps of the method (Sec. II) on a
`Lattice` with the cell types held fixed, checkpointing every K steps; the
backward pass is the hand-written discrete adjoint of libfslbm
(fslbm_adjoint_backward): transposed stream-collide, mass exchange and
boundary rules, and the reverse of the FD (Sec. II.A) or LSQR (Sec. II.C)
curvature, including the PLIC offsets and the wetting condition. This module
only marshals arguments; every step runs in the HIP kernels.
"""
from __future__ import annotations

import torch


class FrozenWindow(torch.autograd.Function):
    """phi_T = FrozenWindow.apply(fill0, sigma, theta, lattice, nsteps, K, start_state).

    fill0: (nz, ny, nx) float64 tensor, the fill level of the interface cells
    at the window start (other entries ignored); sigma, theta: 0-d float64
    tensors (theta in radians). start_state (optional): a buffer from
    lattice.save_state() loaded before the window, so that repeated calls
    start from the same distributions. The lattice ends at step T.
    Gradients: dL/dfill0 at interface cells (0 elsewhere), dL/dsigma and
    dL/dtheta.
    """

    @staticmethod
    def forward(ctx, fill0, sigma, theta, lattice, nsteps, K, start_state=None):
        if start_state is not None:
            lattice.load_state(start_state)
        lattice.set_params(sigma=float(sigma), theta=float(theta))
        lattice.set_interface_fill(fill0)
        lattice.adjoint_forward(int(nsteps), int(K))
        ctx.lattice = lattice
        ctx.meta = (sigma.dtype, sigma.device, theta.dtype, theta.device)
        return lattice.fill_tensor()

    @staticmethod
    def backward(ctx, grad_phi):
        lat = ctx.lattice
        dfill0, ds, dt = lat.adjoint_backward(grad_phi.detach())
        sd, sdev, td, tdev = ctx.meta
        g_fill = dfill0.to(grad_phi.device) if ctx.needs_input_grad[0] else None
        g_sigma = torch.tensor(ds, dtype=sd, device=sdev) if ctx.needs_input_grad[1] else None
        g_theta = torch.tensor(dt, dtype=td, device=tdev) if ctx.needs_input_grad[2] else None
        return g_fill, g_sigma, g_theta, None, None, None, None


def frozen_window(lattice, fill0, sigma, theta, nsteps, K, start_state=None):
    """Functional form of FrozenWindow.apply."""
    return FrozenWindow.apply(fill0, sigma, theta, lattice, nsteps, K, start_state)

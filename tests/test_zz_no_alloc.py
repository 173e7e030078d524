"""The allocation-free read-out of the interface list
(fslbm_read_interface_list_noalloc, scratch in a static device array)
against the workspace read-out (fslbm_read_interface_list), both through
the C ABI, on two calls in a row: a 48^3 lattice, then a smaller 24^3 one,
so the second call finds the first call's longer list in the shared
scratch. Index lists must agree exactly and equal the ascending interface
cells of the read-back cell types."""
import numpy as np
import pytest
import torch

from paper_1509_07691_amd import inputs as I
from paper_1509_07691_amd.fslbm import (FSLBM_INTERFACE, Lattice, fslbm_read_interface_list,
                                        fslbm_read_interface_list_noalloc)

pytestmark = pytest.mark.gpu


def _moving_droplet(n, R, seed):
    fill, obst = I.droplet(n, R, noise=1e-6, seed=seed)
    lat = Lattice(fill, obst, precision="f32", curv_model="lsqr", sigma=1e-3, tau=0.8, device=torch.device("cuda:0"))
    u = np.zeros((3,) + fill.shape)
    u[0], u[1] = 0.03, -0.02
    lat.set_equilibrium(1.0, u)
    lat.step(25)  # conversions: the lattice's own list is no longer ascending
    return lat


def _both(lat):
    ws = fslbm_read_interface_list(lat.handle)
    na = fslbm_read_interface_list_noalloc(lat.handle)
    print(f"interface cells: workspace {ws.size}, no-alloc {na.size}", flush=True)
    np.testing.assert_array_equal(na, ws)
    ref = np.flatnonzero(lat.flags().reshape(-1) == FSLBM_INTERFACE)
    np.testing.assert_array_equal(na, ref)
    return na


def test_noalloc_interface_list_equals_workspace_read_out():
    big = _moving_droplet(48, 12.0, 0)
    n_big = _both(big).size
    small = _moving_droplet(24, 5.0, 1)
    n_small = _both(small).size
    assert 0 < n_small < n_big
    # and once more on the larger lattice after the smaller one
    assert _both(big).size == n_big
    big.close()
    small.close()

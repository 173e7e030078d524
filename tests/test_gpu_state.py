"""Failure detection and checkpoint/resume through the C ABI.

- fslbm_check_numeric: a clean state passes; a non-positive or non-finite
  density planted from the host (fslbm_set_equilibrium at one liquid cell)
  is reported as FSLBM_E_NUMERIC. No step runs on the planted state.
- fslbm_save_state / fslbm_load_state: resuming from a checkpoint, in the
  same lattice or in another lattice of the same shape, precision and
  curvature model, reproduces the continued run bit for bit (a sessile drop
  with walls, wetting and cell conversions); a checkpoint of another shape
  is rejected with FSLBM_E_ARG.
"""
import math

import numpy as np
import pytest

from paper_1509_07691_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1509_07691_amd import fslbm

    return fslbm


@pytest.mark.parametrize("bad", [-1.0, float("nan")])
def test_check_numeric_reports_bad_density(fs, bad):
    fill, obst = I.droplet(16, 4.0, noise=1e-6, seed=0)
    lat = fs.Lattice(fill, obst, precision="f32", curv_model="fd", sigma=1e-3, tau=1.0)
    lat.step(3)
    lat.check_numeric()
    rho = np.ones(fill.shape)
    z, y, x = np.argwhere(lat.flags() == fs.FSLBM_LIQUID)[0]
    rho[z, y, x] = bad
    lat.set_equilibrium(rho, np.zeros((3,) + fill.shape))
    with pytest.raises(fs.FslbmError) as err:
        lat.check_numeric()
    assert err.value.code == fs.FSLBM_E_NUMERIC
    lat.close()


def _snapshot(lat):
    return {"flags": lat.flags(), "fill": lat.fill(), "pressure": lat.pressure(), "velocity": lat.velocity(),
            "curvature": lat.curvature(), "ilist": lat.interface_list(), "mass": lat.mass(),
            "steps": lat.steps_taken()}


def _assert_same(a, b):
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


@pytest.mark.parametrize("precision,model", [("f64", "lsqr"), ("f32", "fd")])
def test_checkpoint_resume_bit_identical(fs, precision, model):
    fill, obst = I.sessile_droplet(24, 24, 14, 6.0, noise=1e-6, seed=1)
    kw = dict(precision=precision, curv_model=model, sigma=2e-3, tau=0.8, theta=math.radians(60.0))
    a = fs.Lattice(fill, obst, **kw)
    a.step(10)
    ck = a.save_state()
    a.step(25)
    ref = _snapshot(a)
    assert ref["steps"] == 35
    a.load_state(ck)
    assert a.steps_taken() == 10
    a.step(25)
    _assert_same(_snapshot(a), ref)
    # another lattice of the same shape, created from another drop
    fill_b, obst_b = I.sessile_droplet(24, 24, 14, 5.0, noise=1e-6, seed=3)
    b = fs.Lattice(fill_b, obst_b, **kw)
    b.load_state(ck)
    b.step(25)
    _assert_same(_snapshot(b), ref)
    fill_c, obst_c = I.sessile_droplet(20, 24, 14, 5.0, noise=1e-6, seed=3)
    c = fs.Lattice(fill_c, obst_c, **kw)
    with pytest.raises(fs.FslbmError) as err:
        c.load_state(ck)
    assert err.value.code == fs.FSLBM_E_ARG
    for lat in (a, b, c):
        lat.close()

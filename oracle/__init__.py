"""FP64 CPU oracle of the FSLBM time step (plain C, loaded with ctypes).

TEST INFRASTRUCTURE ONLY: the checker of the GPU library. Only the test
suite, the smoke check and the benchmark's CPU-baseline leg import this
package; the product path never does. It shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_fslbm.so")
_SRC = os.path.join(_HERE, "fslbm_oracle.c")
TL_LIB_PATH = os.path.join(_HERE, "liboracle_fslbm_tl.so")
_TL_SRCS = [os.path.join(_HERE, f) for f in ("fslbm_oracle_tl.cpp", "fslbm_dual.hpp", "fslbm_oracle.c")]

GAS, LIQUID, INTERFACE, OBSTACLE = 0, 1, 2, 3
CURV_FD, CURV_LSQR, CURV_TR = 0, 1, 2
SRT, TRT = 0, 1


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (no fused multiply-add contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wno-unused-function", _SRC, "-o", LIB_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    build_tl(verbose)
    return LIB_PATH


def build_tl(verbose: bool = False) -> str:
    """Compile the tangent-linear build (the same source with dual numbers)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
           "-I", _HERE, _TL_SRCS[0], "-o", TL_LIB_PATH]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return TL_LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("tau", ctypes.c_double),
                ("theta", ctypes.c_double), ("rho_gas", ctypes.c_double),
                ("eps_c", ctypes.c_double), ("trt_magic", ctypes.c_double),
                ("curv_model", ctypes.c_int), ("collision", ctypes.c_int), ("frozen", ctypes.c_int),
                ("bubble", ctypes.c_int)]


_lib = None


def load(path):
    """A ctypes handle of an oracle build at `path` with the signatures set."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    up = ctypes.POINTER(ctypes.c_ubyte)
    ip = ctypes.POINTER(ctypes.c_int)
    vp = ctypes.c_void_p
    L.orc_create.restype = vp
    L.orc_create.argtypes = [ctypes.c_int] * 3 + [dp, up, ctypes.POINTER(_Params)]
    L.orc_destroy.argtypes = [vp]
    L.orc_step.argtypes = [vp, ctypes.c_long]
    for name in ("orc_get_fill", "orc_get_density", "orc_get_velocity", "orc_get_curvature",
                 "orc_get_normal", "orc_get_plic", "orc_get_mass_field", "orc_get_pdf"):
        getattr(L, name).argtypes = [vp, dp]
    L.orc_set_pdf.argtypes = [vp, dp]
    L.orc_set_equilibrium.argtypes = [vp, dp, dp]
    L.orc_get_flags.argtypes = [vp, up]
    L.orc_get_mass.restype = ctypes.c_double
    L.orc_get_mass.argtypes = [vp]
    L.orc_get_reservoir.restype = ctypes.c_double
    L.orc_get_reservoir.argtypes = [vp]
    L.orc_get_gas_density.restype = ctypes.c_double
    L.orc_get_gas_density.argtypes = [vp]
    L.orc_interface_list.restype = ctypes.c_long
    L.orc_interface_list.argtypes = [vp, ip]
    L.orc_cut_volume.restype = ctypes.c_double
    L.orc_cut_volume.argtypes = [dp, ctypes.c_double]
    L.orc_plic_offset.restype = ctypes.c_double
    L.orc_plic_offset.argtypes = [dp, ctypes.c_double]
    L.orc_lsq_solve.restype = ctypes.c_int
    L.orc_lsq_solve.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
    L.orc_quadric_curvature.restype = ctypes.c_double
    L.orc_quadric_curvature.argtypes = [ctypes.c_double] * 5
    L.orc_lsqr_fit_points.restype = ctypes.c_int
    L.orc_lsqr_fit_points.argtypes = [ctypes.c_int, dp, dp, dp]
    L.orc_tr_curvature_points.restype = ctypes.c_double
    L.orc_tr_curvature_points.argtypes = [ctypes.c_int, dp, dp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = load(LIB_PATH)
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def cut_volume(nhat, a):
    n = np.ascontiguousarray(nhat, dtype=np.float64)
    return lib().orc_cut_volume(_dptr(n), float(a))


def plic_offset(nhat, phi):
    n = np.ascontiguousarray(nhat, dtype=np.float64)
    return lib().orc_plic_offset(_dptr(n), float(phi))


def lsq_solve(M, b):
    M = np.ascontiguousarray(M, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(M.shape[1])
    ok = lib().orc_lsq_solve(M.shape[0], M.shape[1], _dptr(M), _dptr(b), _dptr(x))
    return (x if ok else None)


def quadric_curvature(A, B, C, H, I):
    return lib().orc_quadric_curvature(A, B, C, H, I)


def lsqr_fit_points(pts, nhat):
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n = np.ascontiguousarray(nhat, dtype=np.float64)
    c = np.zeros(5)
    ok = lib().orc_lsqr_fit_points(pts.shape[0], _dptr(pts), _dptr(n), _dptr(c))
    return c if ok else None


def tr_curvature_points(d, nhat):
    """TR curvature K (2 x mean curvature) from neighbour offsets d (m x 3)."""
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
    n = np.ascontiguousarray(nhat, dtype=np.float64)
    return lib().orc_tr_curvature_points(d.shape[0], _dptr(d), _dptr(n))


class Oracle:
    """One lattice of the FP64 reference. Arrays are (nz, ny, nx), x fastest."""

    def __init__(self, fill, obstacle=None, *, sigma=0.0, tau=1.0, theta=np.pi / 2,
                 rho_gas=1.0, eps_c=1e-3, curv_model=CURV_FD, collision=SRT,
                 trt_magic=3.0 / 16.0, frozen=False, bubble=False):
        fill = np.ascontiguousarray(fill, dtype=np.float64)
        self.shape = fill.shape
        nz, ny, nx = fill.shape
        self.n = fill.size
        if obstacle is None:
            obstacle = np.zeros(fill.shape, dtype=np.uint8)
        obstacle = np.ascontiguousarray(obstacle, dtype=np.uint8)
        p = _Params(sigma, tau, theta, rho_gas, eps_c, trt_magic, curv_model, collision, 1 if frozen else 0,
                    1 if bubble else 0)
        self._L = lib()  # the build this lattice was created with
        h = self._L.orc_create(nx, ny, nz, _dptr(fill),
                             obstacle.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), ctypes.byref(p))
        if not h:
            raise ValueError("oracle rejected the lattice arguments")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            self._L.orc_destroy(self._h)
            self._h = None

    def step(self, nsteps=1):
        self._L.orc_step(self._h, int(nsteps))

    def _get(self, name, comps=1):
        out = np.zeros((comps * self.n,), dtype=np.float64)
        getattr(self._L, name)(self._h, _dptr(out))
        return out.reshape((comps,) + self.shape) if comps > 1 else out.reshape(self.shape)

    def fill(self):
        return self._get("orc_get_fill")

    def density(self):
        return self._get("orc_get_density")

    def pressure(self):
        return self.density() / 3.0

    def velocity(self):
        return self._get("orc_get_velocity", 3)

    def curvature(self):
        return self._get("orc_get_curvature")

    def normal(self):
        return self._get("orc_get_normal", 3)

    def plic(self):
        return self._get("orc_get_plic")

    def mass_field(self):
        return self._get("orc_get_mass_field")

    def pdf(self):
        return self._get("orc_get_pdf", 19)

    def set_pdf(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        assert f.size == 19 * self.n
        self._L.orc_set_pdf(self._h, _dptr(f))

    def set_equilibrium(self, rho, u):
        """f' = feq(rho, u) at fluid cells; rho shape (nz,ny,nx), u (3,nz,ny,nx)."""
        rho = np.ascontiguousarray(np.broadcast_to(rho, self.shape), dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        assert u.size == 3 * self.n
        self._L.orc_set_equilibrium(self._h, _dptr(rho), _dptr(u))

    def flags(self):
        out = np.zeros(self.n, dtype=np.uint8)
        self._L.orc_get_flags(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
        return out.reshape(self.shape)

    def mass(self):
        return self._L.orc_get_mass(self._h)

    def reservoir(self):
        return self._L.orc_get_reservoir(self._h)

    def gas_density(self):
        return self._L.orc_get_gas_density(self._h)

    def interface_list(self):
        c = self._L.orc_interface_list(self._h, None)
        out = np.zeros(max(c, 1), dtype=np.int32)
        self._L.orc_interface_list(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        return out[:c]


_tl = None


def tl_lib():
    global _tl
    if _tl is None:
        if not os.path.exists(TL_LIB_PATH) or os.path.getmtime(TL_LIB_PATH) < max(map(os.path.getmtime, _TL_SRCS)):
            build_tl()
        L = ctypes.CDLL(TL_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        d, i = ctypes.c_double, ctypes.c_int
        L.orc_tl_create.restype = vp
        L.orc_tl_create.argtypes = [i, i, i, dp, dp, ctypes.POINTER(ctypes.c_ubyte), d, d, d, d, d, d, d, i, i, d]
        L.orc_tl_set_equilibrium.argtypes = [vp, dp, dp]
        L.orc_tl_step.argtypes = [vp, ctypes.c_long]
        L.orc_tl_get_fill.argtypes = [vp, dp, dp]
        L.orc_tl_destroy.argtypes = [vp]
        _tl = L
    return _tl


class TangentLinear:
    """The frozen-type oracle in tangent-linear mode: the value of phi and
    its derivative along one direction of (sigma, theta, phi_0), given by the
    seeds dsigma, dtheta and fill_dot (the last on the initial fill levels).
    Arrays are (nz, ny, nx), x fastest."""

    def __init__(self, fill, obstacle=None, *, fill_dot=None, dsigma=0.0, dtheta=0.0, sigma=0.0, tau=1.0,
                 theta=np.pi / 2, rho_gas=1.0, eps_c=1e-3, curv_model=CURV_FD, collision=SRT,
                 trt_magic=3.0 / 16.0):
        fill = np.ascontiguousarray(fill, dtype=np.float64)
        self.shape = fill.shape
        nz, ny, nx = fill.shape
        self.n = fill.size
        if obstacle is None:
            obstacle = np.zeros(fill.shape, dtype=np.uint8)
        obstacle = np.ascontiguousarray(obstacle, dtype=np.uint8)
        dot = None if fill_dot is None else np.ascontiguousarray(fill_dot, dtype=np.float64)
        h = tl_lib().orc_tl_create(nx, ny, nz, _dptr(fill), None if dot is None else _dptr(dot),
                                   obstacle.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), sigma, dsigma, tau,
                                   theta, dtheta, rho_gas, eps_c, curv_model, collision, trt_magic)
        if not h:
            raise ValueError("tangent-linear oracle rejected the lattice arguments")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            tl_lib().orc_tl_destroy(self._h)
            self._h = None

    def set_equilibrium(self, rho, u):
        rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dtype=np.float64), self.shape))
        u = np.ascontiguousarray(u, dtype=np.float64)
        tl_lib().orc_tl_set_equilibrium(self._h, _dptr(rho), _dptr(u))

    def step(self, nsteps=1):
        tl_lib().orc_tl_step(self._h, int(nsteps))

    def fill_and_derivative(self):
        v = np.zeros(self.n)
        d = np.zeros(self.n)
        tl_lib().orc_tl_get_fill(self._h, _dptr(v), _dptr(d))
        return v.reshape(self.shape), d.reshape(self.shape)

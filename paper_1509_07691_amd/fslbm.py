"""Python binding of libfslbm (C ABI in include/fslbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libfslbm.so. PyTorch provides the device workspace and the stream. The
module raises ImportError-style errors when the library is missing; there is
no CPU fallback.

Module-level functions carry the names of the C entry points; `Lattice`
bundles one handle with its workspace.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfslbm.so")

FSLBM_F64, FSLBM_F32, FSLBM_F16_STORE, FSLBM_BF16_STORE = 0, 1, 2, 3
FSLBM_CURV_FD, FSLBM_CURV_LSQR, FSLBM_CURV_TR = 0, 1, 2
FSLBM_SRT, FSLBM_TRT = 0, 1
FSLBM_GAS, FSLBM_LIQUID, FSLBM_INTERFACE, FSLBM_OBSTACLE = 0, 1, 2, 3
FSLBM_OPT_EPS_C, FSLBM_OPT_COLLISION, FSLBM_OPT_TRT_MAGIC, FSLBM_OPT_TIMING, FSLBM_OPT_GRAPH = 0, 1, 2, 3, 4
FSLBM_OPT_SPLIT_INTERFACE = 5
FSLBM_OPT_BUBBLE = 6
FSLBM_OPT_STRONG_WETTING = 7
FSLBM_OK, FSLBM_E_ARG, FSLBM_E_SHAPE, FSLBM_E_HIP, FSLBM_E_STATE, FSLBM_E_NUMERIC = 0, -1, -2, -3, -4, -5
FSLBM_E_TOPOLOGY = -6

PRECISIONS = {"f64": FSLBM_F64, "f32": FSLBM_F32, "f16": FSLBM_F16_STORE, "bf16": FSLBM_BF16_STORE}
MODELS = {"fd": FSLBM_CURV_FD, "lsqr": FSLBM_CURV_LSQR, "tr": FSLBM_CURV_TR}


class FslbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libfslbm error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfslbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with paper_1509_07691_amd/build_lib.py (no CPU fallback exists)")
    L = ctypes.CDLL(path)
    vp, dp, i32, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int64
    u8p = ctypes.POINTER(ctypes.c_uint8)
    sig = {
        "fslbm_required_bytes": [i32, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)],
        "fslbm_create": [i32, i32, i32, i32, i32, dp, u8p, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)],
        "fslbm_set_params": [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double],
        "fslbm_layer_closure": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), dp, dp],
        "fslbm_set_option": [vp, i32, ctypes.c_double],
        "fslbm_set_stream": [vp, vp],
        "fslbm_set_equilibrium": [vp, dp, dp],
        "fslbm_step": [vp, i64],
        "fslbm_read_fill": [vp, vp, i32],
        "fslbm_read_pressure": [vp, vp, i32],
        "fslbm_read_curvature": [vp, vp, i32],
        "fslbm_read_velocity": [vp, vp, i32],
        "fslbm_read_normal": [vp, vp, i32],
        "fslbm_read_plic": [vp, vp, i32],
        "fslbm_read_mass_field": [vp, vp, i32],
        "fslbm_read_flags": [vp, vp, i32],
        "fslbm_read_interface_list": [vp, ctypes.POINTER(ctypes.c_int32), i64, ctypes.POINTER(i64)],
        "fslbm_read_interface_list_noalloc": [vp, ctypes.POINTER(ctypes.c_int32), i64, ctypes.POINTER(i64)],
        "fslbm_mass": [vp, dp],
        "fslbm_gas_density": [vp, dp],
        "fslbm_check_numeric": [vp],
        "fslbm_diagnostics": [vp, dp],
        "fslbm_steps_taken": [vp, ctypes.POINTER(i64)],
        "fslbm_read_timing": [vp, dp, ctypes.POINTER(i64)],
        "fslbm_reset_timing": [vp],
        "fslbm_batch_create": [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)],
        "fslbm_batch_step": [vp, i64],
        "fslbm_batch_set_option": [vp, i32, ctypes.c_double],
        "fslbm_batch_read_timing": [vp, dp, ctypes.POINTER(i64)],
        "fslbm_batch_reset_timing": [vp],
        "fslbm_batch_split_active": [vp, ctypes.POINTER(i32)],
        "fslbm_split_active": [vp, ctypes.POINTER(i32)],
        "fslbm_set_interface_fill": [vp, vp, i32],
        "fslbm_state_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "fslbm_save_state": [vp, vp, ctypes.c_size_t],
        "fslbm_load_state": [vp, vp, ctypes.c_size_t],
        "fslbm_adjoint_required_bytes": [vp, i64, i32, ctypes.POINTER(ctypes.c_size_t)],
        "fslbm_adjoint_forward": [vp, i64, i32, vp, ctypes.c_size_t],
        "fslbm_adjoint_backward": [vp, vp, i32, dp, dp, vp, i32],
        "fslbm_adjoint_status": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "fslbm_pull_copy_bytes": [i32, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)],
        "fslbm_pull_copy_time": [i32, i32, i32, i32, vp, vp, ctypes.c_size_t, vp, i32, dp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.fslbm_destroy.argtypes = [vp]
    L.fslbm_destroy.restype = None
    L.fslbm_batch_destroy.argtypes = [vp]
    L.fslbm_batch_destroy.restype = None
    L.fslbm_last_error.argtypes = []
    L.fslbm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise FslbmError(rc, load_library().fslbm_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------- C entry points, same names
def fslbm_required_bytes(nx, ny, nz, precision):
    out = ctypes.c_size_t(0)
    _check(load_library().fslbm_required_bytes(nx, ny, nz, precision, ctypes.byref(out)))
    return out.value


def fslbm_create(nx, ny, nz, precision, curv_model, fill, obstacle, workspace_ptr, workspace_bytes, stream_ptr):
    fill = np.ascontiguousarray(fill, dtype=np.float64).reshape(-1)
    if fill.size != nx * ny * nz:
        raise ValueError("fill has the wrong size")
    obs = None
    if obstacle is not None:
        obs = np.ascontiguousarray(obstacle, dtype=np.uint8).reshape(-1)
        if obs.size != fill.size:
            raise ValueError("obstacle has the wrong size")
    h = ctypes.c_void_p()
    _check(load_library().fslbm_create(
        nx, ny, nz, precision, curv_model, _dptr(fill),
        obs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if obs is not None else None,
        ctypes.c_void_p(workspace_ptr), workspace_bytes, ctypes.c_void_p(stream_ptr), ctypes.byref(h)))
    return h


def fslbm_set_params(h, sigma, tau, theta_rad, rho_gas):
    _check(load_library().fslbm_set_params(h, sigma, tau, theta_rad, rho_gas))


def fslbm_set_option(h, key, value):
    _check(load_library().fslbm_set_option(h, key, float(value)))


def fslbm_set_stream(h, stream_ptr):
    _check(load_library().fslbm_set_stream(h, ctypes.c_void_p(stream_ptr)))


def fslbm_set_equilibrium(h, rho, u3):
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    u3 = np.ascontiguousarray(u3, dtype=np.float64).reshape(-1)
    _check(load_library().fslbm_set_equilibrium(h, _dptr(rho), _dptr(u3)))


def fslbm_step(h, nsteps):
    _check(load_library().fslbm_step(h, int(nsteps)))


def _read(name, h, out, device):
    ptr = out.data_ptr() if device else out.ctypes.data
    _check(getattr(load_library(), name)(h, ctypes.c_void_p(ptr), 1 if device else 0))
    return out


def fslbm_read_fill(h, out, device=False):
    return _read("fslbm_read_fill", h, out, device)


def fslbm_read_pressure(h, out, device=False):
    return _read("fslbm_read_pressure", h, out, device)


def fslbm_read_curvature(h, out, device=False):
    return _read("fslbm_read_curvature", h, out, device)


def fslbm_read_velocity(h, out3, device=False):
    return _read("fslbm_read_velocity", h, out3, device)


def fslbm_read_normal(h, out3, device=False):
    return _read("fslbm_read_normal", h, out3, device)


def fslbm_read_plic(h, out, device=False):
    return _read("fslbm_read_plic", h, out, device)


def fslbm_read_mass_field(h, out, device=False):
    return _read("fslbm_read_mass_field", h, out, device)


def fslbm_read_flags(h, out, device=False):
    return _read("fslbm_read_flags", h, out, device)


def fslbm_read_interface_list(h):
    L = load_library()
    cnt = ctypes.c_int64(0)
    _check(L.fslbm_read_interface_list(h, None, 0, ctypes.byref(cnt)))
    out = np.zeros(max(cnt.value, 1), dtype=np.int32)
    _check(L.fslbm_read_interface_list(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       out.size, ctypes.byref(cnt)))
    return out[:cnt.value]


def fslbm_read_interface_list_noalloc(h):
    L = load_library()
    cnt = ctypes.c_int64(0)
    _check(L.fslbm_read_interface_list_noalloc(h, None, 0, ctypes.byref(cnt)))
    out = np.zeros(max(cnt.value, 1), dtype=np.int32)
    _check(L.fslbm_read_interface_list_noalloc(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                               out.size, ctypes.byref(cnt)))
    return out[:cnt.value]


def fslbm_layer_closure(h):
    """(cells closed to liquid, cells closed to gas, fill added, fill removed)
    by the closure of the interface layer at creation."""
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    c, d = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(load_library().fslbm_layer_closure(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
    return a.value, b.value, c.value, d.value


def fslbm_gas_density(h):
    out = ctypes.c_double(0.0)
    _check(load_library().fslbm_gas_density(h, ctypes.byref(out)))
    return out.value


def fslbm_mass(h):
    out = ctypes.c_double(0.0)
    _check(load_library().fslbm_mass(h, ctypes.byref(out)))
    return out.value


def fslbm_check_numeric(h):
    _check(load_library().fslbm_check_numeric(h))


def fslbm_diagnostics(h):
    """(max |u|, mean |u| over fluid cells, pressure jump, inner liquid cells)."""
    out = (ctypes.c_double * 4)()
    _check(load_library().fslbm_diagnostics(h, out))
    return out[0], out[1], out[2], int(out[3])


def fslbm_steps_taken(h):
    out = ctypes.c_int64(0)
    _check(load_library().fslbm_steps_taken(h, ctypes.byref(out)))
    return out.value


def fslbm_read_timing(h):
    """(phase milliseconds [liquid stream-collide, interface stream-collide,
    conversion, compaction, geometry], steps)."""
    out = np.zeros(5)
    steps = ctypes.c_int64(0)
    _check(load_library().fslbm_read_timing(h, _dptr(out), ctypes.byref(steps)))
    return out, steps.value


def fslbm_reset_timing(h):
    _check(load_library().fslbm_reset_timing(h))


def fslbm_destroy(h):
    load_library().fslbm_destroy(h)


def _ptr_dev(a):
    """(pointer, is_device) of a contiguous float64 numpy array or torch tensor."""
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data), 0
    return ctypes.c_void_p(a.data_ptr()), 1 if a.is_cuda else 0


def fslbm_set_interface_fill(h, fill):
    ptr, dev = _ptr_dev(fill)
    _check(load_library().fslbm_set_interface_fill(h, ptr, dev))


def fslbm_state_bytes(h):
    out = ctypes.c_size_t(0)
    _check(load_library().fslbm_state_bytes(h, ctypes.byref(out)))
    return out.value


def fslbm_save_state(h, dst_ptr, nbytes):
    _check(load_library().fslbm_save_state(h, ctypes.c_void_p(dst_ptr), nbytes))


def fslbm_load_state(h, src_ptr, nbytes):
    _check(load_library().fslbm_load_state(h, ctypes.c_void_p(src_ptr), nbytes))


def fslbm_adjoint_required_bytes(h, nsteps, K):
    out = ctypes.c_size_t(0)
    _check(load_library().fslbm_adjoint_required_bytes(h, int(nsteps), int(K), ctypes.byref(out)))
    return out.value


def fslbm_adjoint_forward(h, nsteps, K, workspace_ptr, workspace_bytes):
    _check(load_library().fslbm_adjoint_forward(h, int(nsteps), int(K), ctypes.c_void_p(workspace_ptr),
                                                workspace_bytes))


def fslbm_adjoint_status(h):
    """(inside_steps, fill_events, unconverted_steps) of the recorded window."""
    a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load_library().fslbm_adjoint_status(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def fslbm_adjoint_backward(h, dfill_T, dfill_0):
    """dfill_T, dfill_0: float64 arrays of n entries (numpy or torch, host or
    device, each on its own). Returns (dL/dsigma, dL/dtheta)."""
    gp, gd = _ptr_dev(dfill_T)
    op, od = _ptr_dev(dfill_0)
    ds, dt = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(load_library().fslbm_adjoint_backward(h, gp, gd, ctypes.byref(ds), ctypes.byref(dt), op, od))
    return ds.value, dt.value


def fslbm_pull_copy_bytes(nx, ny, nz, precision):
    out = ctypes.c_size_t(0)
    _check(load_library().fslbm_pull_copy_bytes(nx, ny, nz, precision, ctypes.byref(out)))
    return out.value


def fslbm_pull_copy_time(nx, ny, nz, precision, src_ptr, dst_ptr, buffer_bytes, stream_ptr, launches):
    """Average duration (us) of the pull-only copy over `launches` launches."""
    us = ctypes.c_double(0.0)
    _check(load_library().fslbm_pull_copy_time(nx, ny, nz, precision, ctypes.c_void_p(src_ptr),
                                               ctypes.c_void_p(dst_ptr), buffer_bytes, ctypes.c_void_p(stream_ptr),
                                               int(launches), ctypes.byref(us)))
    return us.value


def fslbm_batch_create(handles):
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    b = ctypes.c_void_p()
    _check(load_library().fslbm_batch_create(arr, len(handles), ctypes.byref(b)))
    return b


def fslbm_batch_step(b, nsteps):
    _check(load_library().fslbm_batch_step(b, int(nsteps)))


def fslbm_batch_set_option(b, key, value):
    _check(load_library().fslbm_batch_set_option(b, key, float(value)))


def fslbm_batch_read_timing(b):
    out = np.zeros(5)
    steps = ctypes.c_int64(0)
    _check(load_library().fslbm_batch_read_timing(b, _dptr(out), ctypes.byref(steps)))
    return out, steps.value


def fslbm_batch_reset_timing(b):
    _check(load_library().fslbm_batch_reset_timing(b))


def fslbm_batch_split_active(b):
    out = ctypes.c_int(0)
    _check(load_library().fslbm_batch_split_active(b, ctypes.byref(out)))
    return bool(out.value)


def fslbm_split_active(h):
    out = ctypes.c_int(0)
    _check(load_library().fslbm_split_active(h, ctypes.byref(out)))
    return bool(out.value)


def fslbm_batch_destroy(b):
    load_library().fslbm_batch_destroy(b)


# ---------------------------------------------------------------- wrapper
class Lattice:
    """One FSLBM lattice on a HIP device; arrays are (nz, ny, nx), x fastest.

    The device workspace is a torch uint8 tensor owned by this object; work
    runs on the torch stream that is current at construction unless a
    stream is given.
    """

    def __init__(self, fill, obstacle=None, *, precision="f64", curv_model="fd", sigma=0.0, tau=1.0,
                 theta=math.pi / 2, rho_gas=1.0, eps_c=None, collision="srt", trt_magic=None,
                 bubble=False, strong_wetting=False, device="cuda:0", stream=None):
        import torch

        fill = np.ascontiguousarray(fill, dtype=np.float64)
        if fill.ndim != 3:
            raise ValueError("fill must be 3-d (nz, ny, nx)")
        self.shape = fill.shape
        nz, ny, nx = fill.shape
        self.n = fill.size
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.curv_model = MODELS[curv_model] if isinstance(curv_model, str) else int(curv_model)
        self.device = torch.device(device)
        nbytes = fslbm_required_bytes(nx, ny, nz, self.precision)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = None
        self._h = fslbm_create(nx, ny, nz, self.precision, self.curv_model, fill, obstacle,
                               self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        if eps_c is not None:
            fslbm_set_option(self._h, FSLBM_OPT_EPS_C, eps_c)
        if trt_magic is not None:
            fslbm_set_option(self._h, FSLBM_OPT_TRT_MAGIC, trt_magic)
        fslbm_set_option(self._h, FSLBM_OPT_COLLISION, FSLBM_TRT if collision == "trt" else FSLBM_SRT)
        if strong_wetting:
            fslbm_set_option(self._h, FSLBM_OPT_STRONG_WETTING, 1)
        self.sigma, self.tau, self.theta, self.rho_gas = sigma, tau, theta, rho_gas
        fslbm_set_params(self._h, sigma, tau, theta, rho_gas)
        if bubble:
            fslbm_set_option(self._h, FSLBM_OPT_BUBBLE, 1)
        self._adj_ws = None

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None:
            fslbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, sigma=None, tau=None, theta=None, rho_gas=None):
        new = (self.sigma if sigma is None else float(sigma), self.tau if tau is None else float(tau),
               self.theta if theta is None else float(theta), self.rho_gas if rho_gas is None else float(rho_gas))
        fslbm_set_params(self._h, *new)  # raises, leaving the parameters unchanged, on a rejected value
        self.sigma, self.tau, self.theta, self.rho_gas = new

    def set_equilibrium(self, rho, u):
        rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), self.shape)
        fslbm_set_equilibrium(self._h, rho, u)

    def step(self, nsteps=1):
        fslbm_step(self._h, nsteps)

    def _host(self, fn, comps=1):
        out = np.zeros(comps * self.n, dtype=np.float64)
        fn(self._h, out)
        return out.reshape((comps,) + self.shape) if comps > 1 else out.reshape(self.shape)

    def fill(self):
        return self._host(fslbm_read_fill)

    def pressure(self):
        return self._host(fslbm_read_pressure)

    def density(self):
        return 3.0 * self.pressure()

    def curvature(self):
        return self._host(fslbm_read_curvature)

    def velocity(self):
        return self._host(fslbm_read_velocity, 3)

    def normal(self):
        return self._host(fslbm_read_normal, 3)

    def plic(self):
        return self._host(fslbm_read_plic)

    def mass_field(self):
        return self._host(fslbm_read_mass_field)

    def flags(self):
        out = np.zeros(self.n, dtype=np.uint8)
        fslbm_read_flags(self._h, out)
        return out.reshape(self.shape)

    def interface_list(self):
        return fslbm_read_interface_list(self._h)

    def mass(self):
        return fslbm_mass(self._h)

    def check_numeric(self):
        fslbm_check_numeric(self._h)

    def diagnostics(self):
        """max_u, mean_u (fluid cells), dp (inner liquid minus gas pressure)
        and n_inner, from device reductions."""
        u_max, u_mean, dp, n_inner = fslbm_diagnostics(self._h)
        return {"max_u": u_max, "mean_u": u_mean, "dp": dp, "n_inner": n_inner}

    def steps_taken(self):
        return fslbm_steps_taken(self._h)

    def set_timing(self, on=True):
        fslbm_set_option(self._h, FSLBM_OPT_TIMING, 1 if on else 0)

    def set_graph(self, on=True):
        fslbm_set_option(self._h, FSLBM_OPT_GRAPH, 1 if on else 0)

    def set_split_interface(self, on=True):
        """True: two passes, False: one pass, None: automatic (default)."""
        fslbm_set_option(self._h, FSLBM_OPT_SPLIT_INTERFACE, -1 if on is None else (1 if on else 0))

    def split_active(self):
        return fslbm_split_active(self._h)

    def set_bubble(self, on=True):
        fslbm_set_option(self._h, FSLBM_OPT_BUBBLE, 1 if on else 0)

    def gas_density(self):
        return fslbm_gas_density(self._h)

    def timing(self):
        return fslbm_read_timing(self._h)

    def reset_timing(self):
        fslbm_reset_timing(self._h)

    # ------------------------------------------ checkpoints, adjoint window
    def set_interface_fill(self, fill):
        """phi (and m = phi rho) of the interface cells from an (nz, ny, nx)
        float64 numpy array or torch tensor."""
        if isinstance(fill, np.ndarray):
            fill = np.ascontiguousarray(fill, dtype=np.float64)
        else:
            fill = fill.detach().to(dtype=self._torch.float64).contiguous()
        size = fill.size if isinstance(fill, np.ndarray) else fill.numel()
        if size != self.n:
            raise ValueError("fill has the wrong size")
        fslbm_set_interface_fill(self._h, fill)

    @property
    def _torch(self):
        import torch
        return torch

    def save_state(self):
        """The whole state as a device uint8 tensor (for load_state)."""
        nbytes = fslbm_state_bytes(self._h)
        buf = self._torch.empty(nbytes, dtype=self._torch.uint8, device=self.device)
        fslbm_save_state(self._h, buf.data_ptr(), nbytes)
        return buf

    def load_state(self, buf):
        fslbm_load_state(self._h, buf.data_ptr(), buf.numel())

    def adjoint_forward(self, nsteps, K):
        """Advance nsteps steps with frozen cell types, checkpointing every K
        steps into a device workspace held by this object."""
        nbytes = fslbm_adjoint_required_bytes(self._h, nsteps, K)
        if self._adj_ws is None or self._adj_ws.numel() < nbytes:
            self._adj_ws = None
            self._adj_ws = self._torch.empty(nbytes, dtype=self._torch.uint8, device=self.device)
        fslbm_adjoint_forward(self._h, nsteps, K, self._adj_ws.data_ptr(), self._adj_ws.numel())

    def adjoint_status(self):
        """(inside_steps, fill_events, unconverted_steps) of the recorded
        window: the steps before an interface fill first left (0, 1), how
        many (step, cell) pairs did, and the steps before the method with
        free cell types would first have converted a cell."""
        return fslbm_adjoint_status(self._h)

    def adjoint_backward(self, dfill_T):
        """(dL/dphi_0 as a device float64 tensor (nz, ny, nx), dL/dsigma,
        dL/dtheta) for dL/dphi_T given as an array of the lattice shape."""
        torch = self._torch
        g = torch.as_tensor(dfill_T, dtype=torch.float64, device=self.device).contiguous()
        if g.numel() != self.n:
            raise ValueError("dL/dphi_T has the wrong size")
        out = torch.zeros(self.shape, dtype=torch.float64, device=self.device)
        ds, dt = fslbm_adjoint_backward(self._h, g, out)
        return out, ds, dt

    def fill_tensor(self):
        """phi as a device float64 tensor (nz, ny, nx)."""
        out = self._torch.empty(self.shape, dtype=self._torch.float64, device=self.device)
        fslbm_read_fill(self._h, out, device=True)
        return out


class Batch:
    """Lattices on one stream advanced by one launch per kernel and step."""

    def __init__(self, lattices):
        self.lattices = list(lattices)
        self._b = None
        self._b = fslbm_batch_create([lat.handle for lat in self.lattices])

    def step(self, nsteps=1):
        fslbm_batch_step(self._b, nsteps)

    def set_timing(self, on=True):
        fslbm_batch_set_option(self._b, FSLBM_OPT_TIMING, 1 if on else 0)

    def set_graph(self, on=True):
        fslbm_batch_set_option(self._b, FSLBM_OPT_GRAPH, 1 if on else 0)

    def set_split_interface(self, on=True):
        """True: two passes, False: one pass, None: automatic (default)."""
        fslbm_batch_set_option(self._b, FSLBM_OPT_SPLIT_INTERFACE, -1 if on is None else (1 if on else 0))

    def split_active(self):
        return fslbm_batch_split_active(self._b)

    def timing(self):
        return fslbm_batch_read_timing(self._b)

    def reset_timing(self):
        fslbm_batch_reset_timing(self._b)

    def close(self):
        if self._b is not None:
            fslbm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Python binding of libppmb (ctypes): argument marshalling only.

Every step of the PPM + PPB pass, the base-state integration, the CFL and
total reductions and the state conversions run in the HIP library; PyTorch
only provides device memory and the stream.  There is no CPU fallback: if
the library or a GPU is missing, constructing a `Sim` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PPMB_LIB names another build of the same sources (for comparing builds)
LIB_PATH = os.environ.get("PPMB_LIB") or os.path.join(HERE, "libppmb.so")

FP64, FP32 = 0, 1
NFIELDS = 15

# every entry point declared in include/ppmb.h
EXPORTS = ("ppmb_create", "ppmb_destroy", "ppmb_state_bytes", "ppmb_state_layout", "ppmb_bind_state",
           "ppmb_current_state", "ppmb_set_base_state", "ppmb_get_base", "ppmb_set_state",
           "ppmb_set_state_device", "ppmb_get_state", "ppmb_get_conserved",
           "ppmb_set_conserved", "ppmb_compute_dt", "ppmb_step", "ppmb_step_auto",
           "ppmb_last_dt", "ppmb_pass", "ppmb_get_nstep", "ppmb_set_nstep",
           "ppmb_reduce_totals", "ppmb_counters", "ppmb_profile_enable", "ppmb_profile_read",
           "ppmb_synchronize", "ppmb_status_string", "ppmb_last_error", "ppmb_batch_create",
           "ppmb_brick_count", "ppmb_brick_set_base_state", "ppmb_brick_get_base",
           "ppmb_brick_set_state", "ppmb_brick_get_state", "ppmb_brick_get_conserved",
           "ppmb_brick_totals", "ppmb_brick_last_dt", "ppmb_batch_step", "ppmb_set_pass_shape",
           "ppmb_get_pass_shape", "ppmb_autotune", "ppmb_ppb2d_create", "ppmb_ppb2d_destroy",
           "ppmb_ppb2d_set", "ppmb_ppb2d_get", "ppmb_ppb2d_steps", "ppmb_ppb2d_get_nstep",
           "ppmb_ppb2d_set_nstep", "ppmb_set_spinup", "ppmb_spin_add", "ppmb_shell_profile",
           "ppmb_set_shock_dissipation", "ppmb_set_flattening", "ppmb_set_gravity",
           "ppmb_set_heating", "ppmb_set_cfl_check", "ppmb_shell_profile_noalloc",
           "ppmb_set_solid_skip", "ppmb_set_pass_tiling", "ppmb_get_pass_tiling",
           "ppmb_set_rotating_frame", "ppmb_set_state_planes", "ppmb_get_state_planes")


class PPMBError(RuntimeError):
    pass


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("dx", ctypes.c_double), ("origin", ctypes.c_double * 3),
                ("bc", ctypes.c_int * 3), ("gamma", ctypes.c_double), ("sphere", ctypes.c_int),
                ("sphere_r", ctypes.c_double), ("grav_kind", ctypes.c_int),
                ("grav", ctypes.c_double * 4), ("heat_kind", ctypes.c_int),
                ("heat", ctypes.c_double * 3), ("smooth_detect", ctypes.c_int)]


class Grid2D(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 2), ("dx", ctypes.c_double), ("origin", ctypes.c_double * 2),
                ("centre", ctypes.c_double * 2), ("omega", ctypes.c_double)]


_D = ctypes.POINTER(ctypes.c_double)
_DD = ctypes.POINTER(_D)
_V = ctypes.c_void_p
_lib = None


def load():
    """Load libppmb.so (built by paper_1810_13416_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PPMBError(f"{LIB_PATH} is not built; run `python -m paper_1810_13416_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i, d, p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    sig = {
        "ppmb_create": [ctypes.POINTER(Grid), i, p, ctypes.POINTER(p)],
        "ppmb_destroy": [p],
        "ppmb_state_bytes": [p, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
        "ppmb_bind_state": [p, p, p],
        "ppmb_current_state": [p, ctypes.POINTER(p)],
        "ppmb_state_layout": [p, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)],
        "ppmb_set_base_state": [p, i, _D],
        "ppmb_get_base": [p, _D, _D],
        "ppmb_set_state": [p, _DD],
        "ppmb_set_state_device": [p, _DD],
        "ppmb_get_state": [p, _DD],
        "ppmb_get_conserved": [p, _DD],
        "ppmb_set_conserved": [p, _DD],
        "ppmb_compute_dt": [p, d, _D],
        "ppmb_step": [p, d],
        "ppmb_step_auto": [p, d, i],
        "ppmb_last_dt": [p, _D],
        "ppmb_pass": [p, i, d, i],
        "ppmb_get_nstep": [p, ctypes.POINTER(ctypes.c_long)],
        "ppmb_set_nstep": [p, ctypes.c_long],
        "ppmb_reduce_totals": [p, _D],
        "ppmb_counters": [p, ctypes.POINTER(ctypes.c_ulonglong)],
        "ppmb_profile_enable": [p, i],
        "ppmb_profile_read": [p, _D, ctypes.POINTER(ctypes.c_long)],
        "ppmb_synchronize": [p],
        "ppmb_batch_create": [i, ctypes.POINTER(Grid), i, p, ctypes.POINTER(p)],
        "ppmb_brick_count": [p, ctypes.POINTER(i)],
        "ppmb_brick_set_base_state": [p, i, i, _D],
        "ppmb_brick_get_base": [p, i, _D, _D],
        "ppmb_brick_set_state": [p, i, _DD],
        "ppmb_brick_get_state": [p, i, _DD],
        "ppmb_brick_get_conserved": [p, i, _DD],
        "ppmb_brick_totals": [p, i, _D],
        "ppmb_brick_last_dt": [p, i, _D],
        "ppmb_batch_step": [p, d, i, i],
        "ppmb_set_pass_shape": [p, i, i],
        "ppmb_get_pass_shape": [p, ctypes.POINTER(i), ctypes.POINTER(i)],
        "ppmb_autotune": [p, d, i, ctypes.c_char_p, ctypes.POINTER(i)],
        "ppmb_ppb2d_create": [ctypes.POINTER(Grid2D), i, p, ctypes.POINTER(p)],
        "ppmb_ppb2d_destroy": [p],
        "ppmb_ppb2d_set": [p, _DD],
        "ppmb_ppb2d_get": [p, _DD],
        "ppmb_ppb2d_steps": [p, d, i],
        "ppmb_ppb2d_get_nstep": [p, ctypes.POINTER(ctypes.c_long)],
        "ppmb_ppb2d_set_nstep": [p, ctypes.c_long],
        "ppmb_set_spinup": [p, d, ctypes.c_long],
        "ppmb_spin_add": [p, d],
        "ppmb_shell_profile": [p, i, i, d, _D],
        "ppmb_set_shock_dissipation": [p, d],
        "ppmb_set_flattening": [p, ctypes.c_int],
        "ppmb_set_gravity": [p, i, _D, i],
        "ppmb_set_heating": [p, i, _D, i],
        "ppmb_set_cfl_check": [p, d],
        "ppmb_shell_profile_noalloc": [p, i, i, d, p],
        "ppmb_set_solid_skip": [p, i],
        "ppmb_set_pass_tiling": [p, i, i],
        "ppmb_get_pass_tiling": [p, ctypes.POINTER(i), ctypes.POINTER(i)],
        "ppmb_set_rotating_frame": [p, d, i],
        "ppmb_set_state_planes": [p, i, i, _DD],
        "ppmb_get_state_planes": [p, i, i, _DD],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.ppmb_status_string.argtypes = [i]
    L.ppmb_status_string.restype = ctypes.c_char_p
    L.ppmb_last_error.argtypes = [p]
    L.ppmb_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def grid_of(params) -> Grid:
    g = Grid()
    g.n[:] = [int(v) for v in params.n]
    g.dx = float(params.dx)
    g.origin[:] = [float(v) for v in params.origin]
    g.bc[:] = [int(v) for v in params.bc]
    g.gamma = float(params.gamma)
    g.sphere = int(params.sphere)
    g.sphere_r = float(params.sphere_r)
    g.grav_kind = int(params.grav_kind)
    g.grav[:] = [float(v) for v in params.grav]
    g.heat_kind = int(params.heat_kind)
    g.heat[:] = [float(v) for v in params.heat]
    g.smooth_detect = int(params.smooth_detect)
    return g


def _ptrs(arrs):
    return (_D * len(arrs))(*[a.ctypes.data_as(_D) for a in arrs])


class Sim:
    """One grid on one GPU stream.

    params: a GridParams-like object (n, dx, origin, bc, gamma, sphere,
    sphere_r, grav_kind, grav, heat_kind, heat, smooth_detect, base_kind,
    base).  precision: FP64 or FP32.  The two state buffers are torch
    tensors on `device`; the library ping-pongs between them."""

    def __init__(self, params, precision=FP64, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise PPMBError("no GPU: the PPM+PPB path runs only in the HIP library")
        self.torch = torch
        self.L = load()
        self.params = params
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._grid = grid_of(params)
        h = ctypes.c_void_p()
        self._check(self.L.ppmb_create(ctypes.byref(self._grid), precision,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                    None)
        self.h = h
        nbytes = ctypes.c_size_t()
        esz = ctypes.c_size_t()
        self._check(self.L.ppmb_state_bytes(self.h, ctypes.byref(nbytes), ctypes.byref(esz)))
        dtype = torch.float64 if precision == FP64 else torch.float32
        count = nbytes.value // esz.value
        self.buffers = [torch.empty(count, dtype=dtype, device=self.device) for _ in range(2)]
        self._check(self.L.ppmb_bind_state(self.h, ctypes.c_void_p(self.buffers[0].data_ptr()),
                                           ctypes.c_void_p(self.buffers[1].data_ptr())))
        self.set_base_state(int(getattr(params, "base_kind", 0)), getattr(params, "base", (0.0,) * 6))

    # -- plumbing --------------------------------------------------------
    def _check(self, status, h="self"):
        if status != 0:
            hh = self.h if h == "self" else None
            msg = self.L.ppmb_status_string(status).decode()
            if hh:
                msg += ": " + self.L.ppmb_last_error(hh).decode()
            raise PPMBError(f"ppmb error {status}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            self.L.ppmb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.params.n[2], self.params.n[1], self.params.n[0])

    # -- API -------------------------------------------------------------
    def set_base_state(self, kind, params6):
        arr = np.ascontiguousarray(params6, dtype=np.float64)
        self._check(self.L.ppmb_set_base_state(self.h, int(kind), arr.ctypes.data_as(_D)))

    def base(self):
        r = np.empty(self.shape)
        p = np.empty(self.shape)
        self._check(self.L.ppmb_get_base(self.h, r.ctypes.data_as(_D), p.ctypes.data_as(_D)))
        return r, p

    def set_state(self, state):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in state]
        self._check(self.L.ppmb_set_state(self.h, _ptrs(arrs)))

    def set_state_device(self, tensors):
        ptrs = (_D * NFIELDS)(*[ctypes.cast(t.data_ptr(), _D) for t in tensors])
        self._check(self.L.ppmb_set_state_device(self.h, ptrs))

    def get_state(self):
        out = [np.empty(self.shape) for _ in range(NFIELDS)]
        self._check(self.L.ppmb_get_state(self.h, _ptrs(out)))
        return out

    def set_state_planes(self, k0, state):
        """z-planes k0 .. k0 + nk - 1 from 15 arrays of shape (nk, ny, nx)."""
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in state]
        self._check(self.L.ppmb_set_state_planes(self.h, int(k0), int(arrs[0].shape[0]), _ptrs(arrs)))

    def get_state_planes(self, k0, nk):
        out = [np.empty((int(nk), self.shape[1], self.shape[2])) for _ in range(NFIELDS)]
        self._check(self.L.ppmb_get_state_planes(self.h, int(k0), int(nk), _ptrs(out)))
        return out

    def get_conserved(self):
        out = [np.empty(self.shape) for _ in range(NFIELDS)]
        self._check(self.L.ppmb_get_conserved(self.h, _ptrs(out)))
        return out

    def set_conserved(self, cons):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in cons]
        self._check(self.L.ppmb_set_conserved(self.h, _ptrs(arrs)))

    def dt(self, cfl):
        v = ctypes.c_double()
        self._check(self.L.ppmb_compute_dt(self.h, float(cfl), ctypes.byref(v)))
        return v.value

    def step(self, dt):
        self._check(self.L.ppmb_step(self.h, float(dt)))

    def step_auto(self, cfl, nsteps):
        self._check(self.L.ppmb_step_auto(self.h, float(cfl), int(nsteps)))

    def last_dt(self):
        v = ctypes.c_double()
        self._check(self.L.ppmb_last_dt(self.h, ctypes.byref(v)))
        return v.value

    def run(self, nsteps, cfl):
        for _ in range(nsteps):
            self.step(self.dt(cfl))

    def pass_(self, axis, dt, heat=0):
        self._check(self.L.ppmb_pass(self.h, int(axis), float(dt), int(heat)))

    @property
    def nstep(self):
        v = ctypes.c_long()
        self._check(self.L.ppmb_get_nstep(self.h, ctypes.byref(v)))
        return v.value

    @nstep.setter
    def nstep(self, v):
        self._check(self.L.ppmb_set_nstep(self.h, int(v)))

    def totals(self):
        out = np.zeros(8)
        self._check(self.L.ppmb_reduce_totals(self.h, out.ctypes.data_as(_D)))
        return out

    def counters(self):
        out = (ctypes.c_ulonglong * 4)()
        self._check(self.L.ppmb_counters(self.h, out))
        return [int(v) for v in out]

    def set_shock_dissipation(self, k: float):
        """Dissipation coefficient of the 3-D shock dissipation (0: off)."""
        self._check(self.L.ppmb_set_shock_dissipation(self.h, float(k)))

    def set_flattening(self, on: bool):
        """Flattening of the parabolas near strong shocks (CW84 Sec. 4)."""
        self._check(self.L.ppmb_set_flattening(self.h, 1 if on else 0))

    def set_gravity(self, kind: int, params=()):
        """Gravity of every brick (kind NONE 0, CONST 1 with 3 values,
        RADIAL 2 with 4 values); the base state is kept."""
        arr = np.ascontiguousarray(params, dtype=np.float64).reshape(-1)
        self._check(self.L.ppmb_set_gravity(self.h, int(kind), arr.ctypes.data_as(_D) if arr.size else None,
                                            int(arr.size)))

    def set_heating(self, kind: int, params=()):
        """Heating of every brick (kind NONE 0, LAYER_Z 1 with 3 values,
        BALL 2 with 2 or 3 values)."""
        arr = np.ascontiguousarray(params, dtype=np.float64).reshape(-1)
        self._check(self.L.ppmb_set_heating(self.h, int(kind), arr.ctypes.data_as(_D) if arr.size else None,
                                            int(arr.size)))

    def set_cfl_check(self, courant_max: float):
        """Courant check of the dt given to step / pass_ (0: off)."""
        self._check(self.L.ppmb_set_cfl_check(self.h, float(courant_max)))

    def set_solid_skip(self, on: bool):
        """Passes leave out solid cells beyond the stencil reach (default on)."""
        self._check(self.L.ppmb_set_solid_skip(self.h, 1 if on else 0))

    def set_tiling(self, march_chunk: int, x_rows: int):
        """Cells per wave along a pencil (0: whole) and rows per wave of the x pass."""
        self._check(self.L.ppmb_set_pass_tiling(self.h, int(march_chunk), int(x_rows)))

    def tiling(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        self._check(self.L.ppmb_get_pass_tiling(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_spinup(self, omega: float, nramp: int):
        """Steps 0 .. nramp-1 each end with a solid-body rotation increment
        omega / nramp about the z axis."""
        self._check(self.L.ppmb_set_spinup(self.h, float(omega), int(nramp)))

    def spin_add(self, domega: float):
        self._check(self.L.ppmb_spin_add(self.h, float(domega)))

    def set_rotating_frame(self, omega: float, centrifugal: bool = True):
        """Coriolis (and centrifugal) sources of axes turning at omega about z."""
        self._check(self.L.ppmb_set_rotating_frame(self.h, float(omega), 1 if centrifugal else 0))

    def shell_profile(self, nbins: int, dr: float, brick: int = 0):
        """(nbins, 8) FP64 shell sums: volume, mass, f0, rho u_r, rho u_r^2,
        rho |u|^2, angular momentum about z, f0^2 (each times dV)."""
        out = np.zeros((int(nbins), 8))
        self._check(self.L.ppmb_shell_profile(self.h, int(brick), int(nbins), float(dr),
                                              out.ctypes.data_as(_D)))
        return out

    def shell_profile_noalloc(self, out, nbins: int, dr: float, brick: int = 0):
        """Shell sums into `out`, a device tensor of nbins * 8 float64, with no
        allocation by the library (static workspace); asynchronous."""
        self._check(self.L.ppmb_shell_profile_noalloc(self.h, int(brick), int(nbins), float(dr),
                                                      ctypes.c_void_p(out.data_ptr())))

    def profile(self, enable=True):
        self._check(self.L.ppmb_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self):
        """Per axis: (number of timed pass kernels, summed milliseconds)."""
        ms = (ctypes.c_double * 3)()
        cnt = (ctypes.c_long * 3)()
        self._check(self.L.ppmb_profile_read(self.h, ms, cnt))
        return [int(v) for v in cnt], [float(v) for v in ms]

    def synchronize(self):
        self._check(self.L.ppmb_synchronize(self.h))

    def layout(self):
        """(offset, field stride, plane stride, row pitch) of the device state,
        in elements."""
        out = (ctypes.c_longlong * 4)()
        self._check(self.L.ppmb_state_layout(self.h, 0, out))
        return tuple(int(v) for v in out)

    def current_state_tensor(self):
        p = ctypes.c_void_p()
        self._check(self.L.ppmb_current_state(self.h, ctypes.byref(p)))
        for b in self.buffers:
            if b.data_ptr() == p.value:
                return b
        raise PPMBError("current state is not one of the bound buffers")


class Batch:
    """Many independent bricks advanced together (each with its own grid,
    boundaries, base state and CFL dt).  The library owns both state arenas;
    `stream` must be a non-default torch stream for graph replay (mode 1)."""

    def __init__(self, params_list, precision=FP32, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise PPMBError("no GPU: the PPM+PPB path runs only in the HIP library")
        self.L = load()
        self.params = list(params_list)
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        grids = (Grid * len(self.params))(*[grid_of(p) for p in self.params])
        h = ctypes.c_void_p()
        st = self.L.ppmb_batch_create(len(self.params), grids, precision,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise PPMBError(f"ppmb_batch_create failed: {st}")
        self.h = h
        for b, p in enumerate(self.params):
            arr = np.ascontiguousarray(getattr(p, "base", (0.0,) * 6), dtype=np.float64)
            self._check(self.L.ppmb_brick_set_base_state(self.h, b, int(getattr(p, "base_kind", 0)),
                                                         arr.ctypes.data_as(_D)))

    _check = Sim._check
    close = Sim.close
    __del__ = Sim.__del__

    def _shape(self, b):
        n = self.params[b].n
        return (n[2], n[1], n[0])

    def set_state(self, b, state):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in state]
        self._check(self.L.ppmb_brick_set_state(self.h, int(b), _ptrs(arrs)))

    def get_state(self, b):
        out = [np.empty(self._shape(b)) for _ in range(NFIELDS)]
        self._check(self.L.ppmb_brick_get_state(self.h, int(b), _ptrs(out)))
        return out

    def get_conserved(self, b):
        out = [np.empty(self._shape(b)) for _ in range(NFIELDS)]
        self._check(self.L.ppmb_brick_get_conserved(self.h, int(b), _ptrs(out)))
        return out

    def totals(self, b):
        out = np.zeros(8)
        self._check(self.L.ppmb_brick_totals(self.h, int(b), out.ctypes.data_as(_D)))
        return out

    def last_dt(self, b):
        v = ctypes.c_double()
        self._check(self.L.ppmb_brick_last_dt(self.h, int(b), ctypes.byref(v)))
        return v.value

    def step_dt(self, dt):
        """One step of every brick with the same given dt (asynchronous)."""
        self._check(self.L.ppmb_step(self.h, float(dt)))

    def step(self, cfl, nsteps, mode=0):
        """mode 0: one launch per stage for all bricks; 1: replayed hipGraph;
        2: one launch per stage and brick; 3: one launch of the persistent
        step kernel per step; 4: mode 3 replayed from a hipGraph."""
        self._check(self.L.ppmb_batch_step(self.h, float(cfl), int(nsteps), int(mode)))

    def set_shape(self, march_waves, x_waves):
        self._check(self.L.ppmb_set_pass_shape(self.h, int(march_waves), int(x_waves)))

    def shape(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        self._check(self.L.ppmb_get_pass_shape(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def autotune(self, cfl, reps=3, cache_path=None):
        out = (ctypes.c_int * 2)()
        cp = cache_path.encode() if cache_path else None
        self._check(self.L.ppmb_autotune(self.h, float(cfl), int(reps), cp, out))
        return out[0], out[1]

    def counters(self):
        out = (ctypes.c_ulonglong * 4)()
        self._check(self.L.ppmb_counters(self.h, out))
        return [int(v) for v in out]

    def set_shock_dissipation(self, k: float):
        """Dissipation coefficient of the 3-D shock dissipation (0: off)."""
        self._check(self.L.ppmb_set_shock_dissipation(self.h, float(k)))

    def set_flattening(self, on: bool):
        """Flattening of the parabolas near strong shocks (CW84 Sec. 4)."""
        self._check(self.L.ppmb_set_flattening(self.h, 1 if on else 0))

    set_gravity = Sim.set_gravity
    set_heating = Sim.set_heating
    set_cfl_check = Sim.set_cfl_check
    set_solid_skip = Sim.set_solid_skip
    set_tiling = Sim.set_tiling
    tiling = Sim.tiling
    set_rotating_frame = Sim.set_rotating_frame

    def set_spinup(self, omega: float, nramp: int):
        """Steps 0 .. nramp-1 each end with a solid-body rotation increment
        omega / nramp about the z axis."""
        self._check(self.L.ppmb_set_spinup(self.h, float(omega), int(nramp)))

    def spin_add(self, domega: float):
        self._check(self.L.ppmb_spin_add(self.h, float(domega)))

    def shell_profile(self, nbins: int, dr: float, brick: int = 0):
        """(nbins, 8) FP64 shell sums: volume, mass, f0, rho u_r, rho u_r^2,
        rho |u|^2, angular momentum about z, f0^2 (each times dV)."""
        out = np.zeros((int(nbins), 8))
        self._check(self.L.ppmb_shell_profile(self.h, int(brick), int(nbins), float(dr),
                                              out.ctypes.data_as(_D)))
        return out

    def synchronize(self):
        self._check(self.L.ppmb_synchronize(self.h))


class PPB2D:
    """2-D PPB advection of the 6 fv moments (f0, fx, fy, fxx, fyy, fxy)
    under a rigid rotation (the slotted-disk test); the HIP library does all
    the work, this class only marshals arguments."""

    def __init__(self, n, dx, origin, centre, omega, precision=FP64, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise PPMBError("no GPU: the PPB path runs only in the HIP library")
        self.L = load()
        self.n = (int(n[0]), int(n[1]))
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        g = Grid2D()
        g.n[:] = list(self.n)
        g.dx = float(dx)
        g.origin[:] = [float(v) for v in origin]
        g.centre[:] = [float(v) for v in centre]
        g.omega = float(omega)
        h = ctypes.c_void_p()
        st = self.L.ppmb_ppb2d_create(ctypes.byref(g), precision, ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h))
        if st != 0:
            raise PPMBError(f"ppmb_ppb2d_create failed: {st}")
        self.h = h

    def _check(self, st):
        if st != 0:
            raise PPMBError(self.L.ppmb_status_string(st).decode())

    def set(self, coef):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in coef]
        self._check(self.L.ppmb_ppb2d_set(self.h, _ptrs(arrs)))

    def get(self):
        out = [np.empty((self.n[1], self.n[0])) for _ in range(6)]
        self._check(self.L.ppmb_ppb2d_get(self.h, _ptrs(out)))
        return out

    def steps(self, dt, nsteps):
        self._check(self.L.ppmb_ppb2d_steps(self.h, float(dt), int(nsteps)))

    def close(self):
        if getattr(self, "h", None):
            self.L.ppmb_ppb2d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

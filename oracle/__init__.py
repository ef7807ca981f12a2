"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  It loads `liboracle.so`, built from `ppmb_oracle.c`
with gcc; it never touches the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ppmb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BUILD_CMD = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
             "-fPIC", "-Wall", "-o", _LIB, _SRC, "-lm"]


def build() -> str:
    """Compile the oracle shared library (always rebuilds)."""
    subprocess.check_call(BUILD_CMD)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("dx", ctypes.c_double), ("origin", ctypes.c_double * 3),
                ("bc", ctypes.c_int * 3), ("gamma", ctypes.c_double), ("sphere", ctypes.c_int),
                ("sphere_r", ctypes.c_double), ("grav_kind", ctypes.c_int),
                ("grav", ctypes.c_double * 4), ("base_kind", ctypes.c_int),
                ("base", ctypes.c_double * 6), ("heat_kind", ctypes.c_int),
                ("heat", ctypes.c_double * 3), ("smooth_detect", ctypes.c_int)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_DD = ctypes.POINTER(_D)


def lib():
    """The loaded oracle library.  PPMB_ORACLE_LIB names another build of the
    same source to load instead (the planted-mistake tests build altered
    copies of the oracle and check that its pins reject them)."""
    global _lib
    if _lib is None:
        path = os.environ.get("PPMB_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        L = ctypes.CDLL(path)
        L.or_create.restype = ctypes.c_void_p
        L.or_create.argtypes = [ctypes.POINTER(_Params), ctypes.c_int]
        L.or_destroy.argtypes = [ctypes.c_void_p]
        L.or_set_threads.argtypes = [ctypes.c_void_p, ctypes.c_int]
        for f in ("or_set_state", "or_get_state", "or_get_conserved", "or_set_conserved"):
            getattr(L, f).argtypes = [ctypes.c_void_p, _DD]
        L.or_get_base.argtypes = [ctypes.c_void_p, _D, _D]
        L.or_base_profile.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _D, _D, _D]
        L.or_compute_dt.restype = ctypes.c_double
        L.or_compute_dt.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.or_pass.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
        L.or_step.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.or_nstep.restype = ctypes.c_long
        L.or_nstep.argtypes = [ctypes.c_void_p]
        L.or_set_nstep.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.or_totals.argtypes = [ctypes.c_void_p, _D]
        L.or_spin_add.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.or_set_dissipation.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.or_divergence.argtypes = [ctypes.c_void_p, _D]
        L.or_set_flattening.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.or_set_gravity.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.or_set_heating.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.or_flattening.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.or_set_spinup.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_long]
        L.or_set_rotating_frame.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
        L.or_shell_profile.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _D]
        L.or_counters.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_ulonglong)]
        L.or_face4.restype = ctypes.c_double
        L.or_face4.argtypes = [ctypes.c_double] * 4
        L.or_smooth_weight.restype = ctypes.c_double
        L.or_smooth_weight.argtypes = [_D]
        L.or_riemann.restype = ctypes.c_int
        L.or_riemann.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
        L.or_ppb_pencil.restype = ctypes.c_int
        L.or_ppb_pencil.argtypes = [ctypes.c_int, _DD, _D, _DD]
        L.or_ppb2d_steps.restype = None
        L.or_ppb2d_steps.argtypes = [ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 7 + \
            [ctypes.c_int, ctypes.c_long, _DD]
        L.or_sizeof_params.restype = ctypes.c_int
        assert L.or_sizeof_params() == ctypes.sizeof(_Params)
        _lib = L
    return _lib


def to_params(gp) -> _Params:
    P = _Params()
    P.n[:] = [int(v) for v in gp.n]
    P.dx = float(gp.dx)
    P.origin[:] = [float(v) for v in gp.origin]
    P.bc[:] = [int(v) for v in gp.bc]
    P.gamma = float(gp.gamma)
    P.sphere = int(gp.sphere)
    P.sphere_r = float(gp.sphere_r)
    P.grav_kind = int(gp.grav_kind)
    P.grav[:] = [float(v) for v in gp.grav]
    P.base_kind = int(gp.base_kind)
    P.base[:] = [float(v) for v in gp.base]
    P.heat_kind = int(gp.heat_kind)
    P.heat[:] = [float(v) for v in gp.heat]
    P.smooth_detect = int(gp.smooth_detect)
    return P


def _ptrs(arrs):
    arr_t = _D * len(arrs)
    return arr_t(*[a.ctypes.data_as(_D) for a in arrs])


class Oracle:
    """One simulation held by the C oracle."""

    def __init__(self, params, threads: int | None = None):
        self.params = params
        self._P = to_params(params)
        self.threads = threads or int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        self.h = lib().or_create(ctypes.byref(self._P), self.threads)
        if not self.h:
            raise MemoryError("oracle allocation failed")

    def close(self):
        if self.h:
            lib().or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _alloc(self, k=15):
        return [np.empty(self.params.shape, dtype=np.float64) for _ in range(k)]

    def set_state(self, state):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in state]
        lib().or_set_state(self.h, _ptrs(arrs))

    def get_state(self):
        out = self._alloc()
        lib().or_get_state(self.h, _ptrs(out))
        return out

    def get_conserved(self):
        out = self._alloc()
        lib().or_get_conserved(self.h, _ptrs(out))
        return out

    def set_conserved(self, cons):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in cons]
        lib().or_set_conserved(self.h, _ptrs(arrs))

    def base(self):
        r, p = self._alloc(2)
        lib().or_get_base(self.h, r.ctypes.data_as(_D), p.ctypes.data_as(_D))
        return r, p

    def dt(self, cfl: float) -> float:
        return lib().or_compute_dt(self.h, cfl)

    def step(self, dt: float):
        lib().or_step(self.h, dt)

    def run(self, nsteps: int, cfl: float):
        for _ in range(nsteps):
            self.step(self.dt(cfl))

    def pass_(self, axis: int, dt: float):
        lib().or_pass(self.h, axis, dt)

    @property
    def nstep(self) -> int:
        return lib().or_nstep(self.h)

    @nstep.setter
    def nstep(self, v: int):
        lib().or_set_nstep(self.h, v)

    def totals(self):
        out = np.zeros(8)
        lib().or_totals(self.h, out.ctypes.data_as(_D))
        return out

    def set_dissipation(self, k: float):
        lib().or_set_dissipation(self.h, k)

    def divergence(self):
        out = np.empty(self.params.shape)
        lib().or_divergence(self.h, out.ctypes.data_as(_D))
        return out

    def set_flattening(self, on: bool):
        lib().or_set_flattening(self.h, 1 if on else 0)

    def flattening(self, axis: int):
        """Flattening coefficients of the current state for a pass along axis."""
        out = np.empty(self.params.shape)
        lib().or_flattening(self.h, int(axis), out.ctypes.data_as(_D))
        return out

    def set_gravity(self, kind: int, params=()):
        g = np.zeros(4)
        g[:len(params)] = params
        lib().or_set_gravity(self.h, int(kind), g.ctypes.data_as(_D))

    def set_heating(self, kind: int, params=()):
        q = np.zeros(3)
        q[:len(params)] = params
        lib().or_set_heating(self.h, int(kind), q.ctypes.data_as(_D))

    def spin_add(self, domega: float):
        lib().or_spin_add(self.h, domega)

    def set_spinup(self, omega: float, nramp: int):
        lib().or_set_spinup(self.h, omega, nramp)

    def set_rotating_frame(self, omega: float, centrifugal: bool = True):
        lib().or_set_rotating_frame(self.h, float(omega), 1 if centrifugal else 0)

    def shell_profile(self, nbins: int, dr: float):
        out = np.zeros((nbins, 8))
        lib().or_shell_profile(self.h, nbins, dr, out.ctypes.data_as(_D))
        return out

    def counters(self):
        out = (ctypes.c_ulonglong * 4)()
        lib().or_counters(self.h, out)
        return [int(v) for v in out]


def base_profile(params, s):
    s = np.ascontiguousarray(s, dtype=np.float64)
    rho = np.empty_like(s)
    p = np.empty_like(s)
    P = to_params(params)
    lib().or_base_profile(ctypes.byref(P), s.size, s.ctypes.data_as(_D),
                          rho.ctypes.data_as(_D), p.ctypes.data_as(_D))
    return rho, p


def face4(am, a, b, bp) -> float:
    return lib().or_face4(am, a, b, bp)


def smooth_weight(q) -> float:
    """Weight of the unconstrained parabola for a 5-cell window."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    return lib().or_smooth_weight(q.ctypes.data_as(_D))


def riemann(L, R, rho0f=0.0, p0f=0.0, gamma=1.4):
    """Face state (rho', u, v, w, p') and the signed iteration count."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    out = np.zeros(5)
    it = lib().or_riemann(L.ctypes.data_as(_D), R.ctypes.data_as(_D), rho0f, p0f, gamma,
                          out.ctypes.data_as(_D))
    return out, it


NG = 4


def ppb2d_steps(coef6, n, dx, origin, centre, omega, dt, nsteps, step0=0):
    """nsteps steps of 2-D PPB under a rigid rotation (see the C source):
    coef6 = 6 arrays (ny, nx): f0, fx, fy, fxx, fyy, fxy.  Returns new arrays."""
    nx, ny = n
    arrs = [np.array(a, dtype=np.float64, copy=True, order="C") for a in coef6]
    lib().or_ppb2d_steps(int(nx), int(ny), float(dx), float(origin[0]), float(origin[1]),
                         float(centre[0]), float(centre[1]), float(omega), float(dt),
                         int(nsteps), int(step0), _ptrs(arrs))
    return arrs


def ppb_pencil(coef, sigma):
    """One PPB pass over a pencil.  coef: (10, n + 8) pass-local coefficients
    (quadratic along the pass, two linear transverse slopes, three constants);
    sigma: (n + 8,) face Courant numbers, entry J being face J - 4 + 1/2.
    Returns the updated coefficients (interior entries) and the limiter count."""
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    n = coef.shape[1] - 2 * NG
    out = np.array(coef, copy=True)
    rows_in = [coef[q] for q in range(10)]
    rows_out = [np.ascontiguousarray(out[q]) for q in range(10)]
    hits = lib().or_ppb_pencil(n, _ptrs(rows_in), sigma.ctypes.data_as(_D), _ptrs(rows_out))
    return np.stack(rows_out), hits

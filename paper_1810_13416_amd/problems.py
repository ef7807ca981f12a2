"""Seeded synthetic inputs for the PPM + PPB step.

This module only builds initial conditions and run parameters.  It holds
none of the method's arithmetic: the HIP library and the CPU oracle both
consume what it returns, and each integrates its own hydrostatic base state
from the parameters given here.

State handed to either side is a list of 15 float64 arrays of shape
(nz, ny, nx), x fastest:

    rho', u_x, u_y, u_z, p'     perturbations from the base state (plain
                                 runs have no base, so these are the full
                                 density and pressure)
    f0, fx, fy, fz, fxx, fyy, fzz, fxy, fyz, fzx
                                 the fluid fraction fv as coefficients of the
                                 orthogonal basis 1, x, y, z, P2(x), P2(y),
                                 P2(z), xy, yz, zx on the unit cell
                                 (P2(s) = s^2 - 1/12), i.e. its cell average
                                 and 9 lowest moments (paper Sec. 4)

The five workloads stand in for the paper's low-Mach stellar convection runs
(Sec. 2, Sec. 3); the paper's stellar models are not available, so every
field is synthetic, drawn from numpy's PCG64 with seed 1810 + config number.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FIELD_NAMES = ("rho", "ux", "uy", "uz", "p",
               "f0", "fx", "fy", "fz", "fxx", "fyy", "fzz", "fxy", "fyz", "fzx")

BC_PERIODIC, BC_REFLECT = 0, 1
GRAV_NONE, GRAV_CONST, GRAV_RADIAL = 0, 1, 2
BASE_NONE, BASE_CONST, BASE_POLY_Z, BASE_POLY_R = 0, 1, 2, 3
HEAT_NONE, HEAT_LAYER_Z, HEAT_BALL = 0, 1, 2


@dataclasses.dataclass
class GridParams:
    """Grid and physics parameters, mirrored field by field by both the
    library's grid descriptor and the oracle's parameter block."""
    n: tuple = (32, 32, 32)
    dx: float = 1.0 / 32
    origin: tuple = (0.0, 0.0, 0.0)
    bc: tuple = (BC_PERIODIC,) * 3
    gamma: float = 5.0 / 3.0
    sphere: int = 0
    sphere_r: float = 0.0
    grav_kind: int = GRAV_NONE
    grav: tuple = (0.0, 0.0, 0.0, 0.0)
    base_kind: int = BASE_NONE
    base: tuple = (0.0,) * 6
    heat_kind: int = HEAT_NONE
    heat: tuple = (0.0, 0.0, 0.0)
    smooth_detect: int = 1

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def ncell(self):
        return self.n[0] * self.n[1] * self.n[2]


@dataclasses.dataclass
class Problem:
    params: GridParams
    state: list          # 15 float64 arrays, shape (nz, ny, nx)
    cfl: float
    nsteps: int
    name: str


# ----------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------

def _centres(params: GridParams, axis: int) -> np.ndarray:
    return params.origin[axis] + (np.arange(params.n[axis]) + 0.5) * params.dx


def _mesh(params: GridParams):
    x = _centres(params, 0)
    y = _centres(params, 1)
    z = _centres(params, 2)
    return z[:, None, None], y[None, :, None], x[None, None, :]


def _zeros(params: GridParams) -> np.ndarray:
    return np.zeros(params.shape, dtype=np.float64)


def _sinc(z):
    return np.sinc(np.asarray(z) / np.pi)


def _lattice_dirs(rng, d: int, count: int):
    """Random nonzero integer vectors in {-1,0,1}^3 with component d = 0, so
    that a sine wave along them carries a divergence-free d-velocity."""
    out = []
    while len(out) < count:
        v = rng.integers(-1, 2, size=3)
        v[d] = 0
        if np.any(v != 0):
            out.append(v.astype(np.float64))
    return out


def fv_moments_quadrature(params: GridParams, func, mask=None, order: int = 4,
                          chunk: int = 1 << 16, k0: int = 0):
    """Cell average and 9 moments of fv = func(x, y, z) by order^3-point
    Gauss-Legendre quadrature per cell.  Only cells where `mask` is True are
    integrated (default: all).  k0: the grid's first z index, for a slab of
    planes of a larger grid with the same origin."""
    g, w = np.polynomial.legendre.leggauss(order)
    s = 0.5 * g                       # nodes on [-1/2, 1/2]
    wt = 0.5 * w                      # weights summing to 1
    S3 = np.stack(np.meshgrid(s, s, s, indexing="ij"), -1).reshape(-1, 3)   # (xi, eta, zeta)
    W3 = np.einsum("i,j,k->ijk", wt, wt, wt).reshape(-1)
    p2 = lambda t: t * t - 1.0 / 12.0
    xi, eta, zeta = S3[:, 0], S3[:, 1], S3[:, 2]
    basis = np.stack([np.ones_like(xi), xi, eta, zeta, p2(xi), p2(eta), p2(zeta),
                      xi * eta, eta * zeta, zeta * xi], 0)
    norm = np.array([1.0, 12.0, 12.0, 12.0, 180.0, 180.0, 180.0, 144.0, 144.0, 144.0])
    proj = (basis * W3[None, :]) * norm[:, None]          # (10, P)
    out = [_zeros(params) for _ in range(10)]
    if mask is None:
        idx = np.arange(params.ncell)
    else:
        idx = np.flatnonzero(mask.reshape(-1))
    nx, ny = params.n[0], params.n[1]
    for a in range(0, idx.size, chunk):
        ii = idx[a:a + chunk]
        i = ii % nx
        j = (ii // nx) % ny
        k = ii // (nx * ny)
        xc = params.origin[0] + (i + 0.5) * params.dx
        yc = params.origin[1] + (j + 0.5) * params.dx
        zc = params.origin[2] + (k + k0 + 0.5) * params.dx
        X = xc[:, None] + params.dx * xi[None, :]
        Y = yc[:, None] + params.dx * eta[None, :]
        Z = zc[:, None] + params.dx * zeta[None, :]
        F = func(X, Y, Z)                                  # (cells, P)
        # row by row, in a fixed order (a matrix product's rounding could
        # depend on how many cells a chunk holds)
        M = np.stack([(F * proj[q][None, :]).sum(axis=1) for q in range(10)], axis=1)
        for q in range(10):
            out[q].reshape(-1)[ii] = M[:, q]
    return out


def fv_step_z(params: GridParams, z_i: float):
    """Exact moments of fv = 1 for z >= z_i (only z-structure is nonzero)."""
    out = [_zeros(params) for _ in range(10)]
    z = _centres(params, 2)
    lo = z - 0.5 * params.dx
    # fraction of the cell above z_i, in cell coordinates zeta in [-1/2, 1/2]
    a = np.clip((z_i - z) / params.dx, -0.5, 0.5)          # lower limit of the fv = 1 part
    f0 = 0.5 - a
    fz = 12.0 * (0.125 - 0.5 * a * a)                      # 12 * int_a^{1/2} zeta
    fzz = 180.0 * ((0.125 - a ** 3) / 3.0 - (0.5 - a) / 12.0)
    del lo
    out[0][:] = f0[:, None, None]
    out[3][:] = fz[:, None, None]
    out[6][:] = fzz[:, None, None]
    return out


def polytrope_closed_form(z, rho_b, p_b, gamma, g_along, z_b, z_i, f_jump):
    """Closed-form hydrostatic piecewise polytrope for constant gravity
    (used only to choose parameters and noise amplitudes of the inputs)."""
    z = np.asarray(z, dtype=np.float64)
    K1 = p_b / rho_b ** gamma
    gm1 = gamma - 1.0

    def seg(zz, rb, zb, K):
        with np.errstate(invalid="ignore"):
            return (rb ** gm1 + gm1 * g_along * (zz - zb) / (gamma * K)) ** (1.0 / gm1)

    rho_i = seg(z_i, rho_b, z_b, K1)
    K2 = K1 * f_jump ** (-gamma)
    rho = np.where(z < z_i, seg(z, rho_b, z_b, K1), seg(z, f_jump * rho_i, z_i, K2))
    K = np.where(z < z_i, K1, K2)
    return rho, K * rho ** gamma


# ----------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------

def config1(n: int = 32, seed: int = 1811, base: str = "none", nsteps: int = 20) -> Problem:
    """Periodic cube [0,1)^3, gamma = 5/3, rho = p = 1, velocity 0.1 x sum of
    4 random-phase sines (wavenumbers 1..4, divergence-free), fv a smoothed
    ball of radius 0.25.  base = 'none' (plain FP64) or 'const' (rho0 = p0 = 1
    subtracted)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = GridParams(n=(n, n, n), dx=1.0 / n, origin=(0.0, 0.0, 0.0),
                   bc=(BC_PERIODIC,) * 3, gamma=5.0 / 3.0)
    if base == "const":
        P.base_kind, P.base = BASE_CONST, (1.0, 1.0, 0.0, 0.0, 0.0, 0.0)
    Z, Y, X = _mesh(P)
    h = P.dx
    vel = []
    for d in range(3):
        dirs = _lattice_dirs(rng, d, 4)
        phases = rng.uniform(0.0, 2.0 * math.pi, size=4)
        u = _zeros(P)
        for k in range(4):
            a = 2.0 * math.pi * (k + 1) * dirs[k]
            # exact cell average of sin(a.x + phi) over the cube of side h
            fac = _sinc(a[0] * h / 2) * _sinc(a[1] * h / 2) * _sinc(a[2] * h / 2)
            u += fac * np.sin(a[0] * X + a[1] * Y + a[2] * Z + phases[k])
        vel.append(0.1 * u)
    rho = _zeros(P) + (0.0 if base == "const" else 1.0)
    p = _zeros(P) + (0.0 if base == "const" else 1.0)
    dxw = P.dx

    def ball(x, y, z):
        r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2)
        return 0.5 * (1.0 - np.tanh((r - 0.25) / dxw))

    fv = fv_moments_quadrature(P, ball)
    return Problem(P, [rho, *vel, p, *fv], cfl=0.8, nsteps=nsteps, name=f"config1_{n}")


def config2_gravity(gamma=5.0 / 3.0, ratio=0.1, z_i=0.8, f_jump=0.5):
    """g0 such that the hydrostatic base falls by `ratio` in density over the
    unit height, including the density jump f_jump at z_i (bisection on the
    closed form)."""
    lo, hi = 1e-6, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        rho, _ = polytrope_closed_form([1.0 - 1e-12], 1.0, 1.0, gamma, -mid, 0.0, z_i, f_jump)
        if not np.isfinite(rho[0]) or rho[0] < ratio:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def config2(n: int = 128, seed: int = 1812, base: str = "poly", nsteps: int = 200,
            mach: float = 0.03, noise: float = 1e-3) -> Problem:
    """Stratified box: x, y periodic on [0,1), z in [0,1] between reflecting
    walls, constant gravity -g0 z-hat, hydrostatic piecewise-polytrope base
    (density falls 10x over the box; a 0.5 density jump at z = 0.8 marks the
    light, entrainable fluid), heating in z < 0.1, fv = 1 for z >= 0.8,
    seeded 1e-3 pressure noise below z = 0.8, plus a seeded divergence-free
    horizontal flow confined to z < 0.75 at rms Mach `mach`.
    base = 'poly' (perturbation form) or 'none' (plain: full fields).
    The flow's modes are drawn before the per-cell noise, so that with
    noise = 0 the data at two resolutions sample one continuous field."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gamma = 5.0 / 3.0
    g0 = config2_gravity(gamma)
    P = GridParams(n=(n, n, n), dx=1.0 / n, origin=(0.0, 0.0, 0.0),
                   bc=(BC_PERIODIC, BC_PERIODIC, BC_REFLECT), gamma=gamma,
                   grav_kind=GRAV_CONST, grav=(0.0, 0.0, -g0, 0.0),
                   heat_kind=HEAT_LAYER_Z, heat=(0.1, 0.1, 0.0))
    P.base_kind = BASE_POLY_Z
    P.base = (1.0, 1.0, 0.0, 0.8, 0.5, 1.0)
    Z, Y, X = _mesh(P)
    rho_cf, p_cf = polytrope_closed_form(Z[:, 0, 0], 1.0, 1.0, gamma, -g0, 0.0, 0.8, 0.5)
    modes = []
    for d in range(2):
        dirs = _lattice_dirs(rng, d, 4)
        phases = rng.uniform(0.0, 2.0 * math.pi, size=4)
        modes.append((dirs, phases))
    cell_noise = rng.uniform(-1.0, 1.0, size=P.shape)
    pp = np.where(Z < 0.8, noise * p_cf[:, None, None] * cell_noise, 0.0)
    env = np.where(Z < 0.75, np.sin(math.pi * Z / 0.75) ** 2, 0.0)
    c_ref = math.sqrt(gamma)
    vel = [_zeros(P), _zeros(P), _zeros(P)]
    for d in range(2):
        dirs, phases = modes[d]
        u = _zeros(P)
        for k in range(4):
            a = 2.0 * math.pi * (k + 1) * dirs[k]
            u += np.sin(a[0] * X + a[1] * Y + a[2] * Z + phases[k])
        vel[d] = u * env
    rms = math.sqrt(float(np.mean(vel[0] ** 2 + vel[1] ** 2)) /
                    max(float(np.mean(env ** 2)), 1e-30))
    scale = mach * c_ref / rms
    vel = [v * scale for v in vel]
    rho = _zeros(P) + np.zeros_like(Z)
    p = pp + 0.0 * X
    if base == "none":
        P.base_kind = BASE_NONE
        P.base = (0.0,) * 6
        rho = rho + rho_cf[:, None, None] + 0.0 * X
        p = p + p_cf[:, None, None]
    fv = fv_step_z(P, 0.8)
    return Problem(P, [rho, *vel, p, *fv], cfl=0.8, nsteps=nsteps, name=f"config2_{n}")


def config3(n: int = 512, seed: int = 1813, nsteps: int = 50, g0: float = 6.0,
            quad_order: int = 6) -> Problem:
    """Spherical convection shell in the cube [-1,1]^3 (n^3 cells), solid
    outside the inscribed sphere r = 1 (Sec. 3), reflecting cube walls,
    radial gravity -g0 r-hat (r/rc inside rc = 0.1, (rc/r)^2 outside) tapered
    to zero between 5 and 1 cell widths inside the sphere, hydrostatic radial
    piecewise-polytrope base (density jump 0.5 at r = 0.5 above the
    convection zone), heating in r < 0.2, fv = 1 for r >= 0.5, seeded velocity
    noise 1e-4 c0 U(-1,1) per component."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gamma = 5.0 / 3.0
    dx = 2.0 / n
    P = GridParams(n=(n, n, n), dx=dx, origin=(-1.0, -1.0, -1.0),
                   bc=(BC_REFLECT,) * 3, gamma=gamma, sphere=1, sphere_r=1.0,
                   grav_kind=GRAV_RADIAL, grav=(g0, 0.1, 1.0 - 5 * dx, 1.0 - dx),
                   base_kind=BASE_POLY_R,
                   base=(1.0, 1.0, 0.0, 0.5, 0.5, math.sqrt(3.0) + dx),
                   heat_kind=HEAT_BALL, heat=(0.1, 0.2, 0.0))
    shape = P.shape
    c_ref = math.sqrt(gamma)
    z = _centres(P, 2)
    y = _centres(P, 1)
    x = _centres(P, 0)
    r2 = (z * z)[:, None, None] + (y * y)[None, :, None] + (x * x)[None, None, :]
    solid = r2 >= 1.0
    vel = []
    for d in range(3):
        u = rng.uniform(-1.0, 1.0, size=shape)
        u *= 1e-4 * c_ref
        u[solid] = 0.0
        vel.append(u)
    rho = np.zeros(shape)
    p = np.zeros(shape)
    # fv = 1 outside r = 0.5: exact 0/1 away from the surface, quadrature on cut cells
    half = 0.5 * math.sqrt(3.0) * dx
    r = np.sqrt(r2)
    cut = np.abs(r - 0.5) < half
    fv = [np.zeros(shape) for _ in range(10)]
    fv[0][r >= 0.5 + half] = 1.0
    if np.any(cut):
        def shell(X, Y, Z):
            return (X * X + Y * Y + Z * Z >= 0.25).astype(np.float64)
        mom = fv_moments_quadrature(P, shell, mask=cut, order=quad_order)
        for q in range(10):
            fv[q][cut] = mom[q][cut]
    del r, r2, cut
    return Problem(P, [rho, *vel, p, *fv], cfl=0.8, nsteps=nsteps, name=f"config3_{n}")


def config5(n: int = 1024, seed: int = 1815, nsteps: int = 20) -> Problem:
    """Config 3 at 1024^3 (dx = 1/512)."""
    prob = config3(n=n, seed=seed, nsteps=nsteps)
    prob.name = f"config5_{n}"
    return prob


def uniform(n=(16, 16, 16), rho=1.3, vel=(0.3, -0.2, 0.1), p=0.7, fv=0.4,
            base: str = "none") -> Problem:
    """Uniform state in a periodic box."""
    P = GridParams(n=tuple(n), dx=1.0 / n[0], bc=(BC_PERIODIC,) * 3, gamma=5.0 / 3.0)
    if base == "const":
        P.base_kind, P.base = BASE_CONST, (rho, p, 0.0, 0.0, 0.0, 0.0)
    st = [np.full(P.shape, 0.0 if base == "const" else rho),
          np.full(P.shape, vel[0]), np.full(P.shape, vel[1]), np.full(P.shape, vel[2]),
          np.full(P.shape, 0.0 if base == "const" else p)]
    f = [np.zeros(P.shape) for _ in range(10)]
    f[0][:] = fv
    return Problem(P, st + f, cfl=0.8, nsteps=10, name="uniform")


def ball(n: int = 32, rho: float = 1.3, p: float = 0.7, fv: float = 0.4) -> Problem:
    """Uniform gas at rest inside the confining sphere r = 1 inscribed in
    the cube [-1,1]^3 (Sec. 3), no gravity, no base state (the solid cells
    outside hold the same values and are never updated)."""
    P = GridParams(n=(n, n, n), dx=2.0 / n, origin=(-1.0, -1.0, -1.0), bc=(BC_REFLECT,) * 3,
                   gamma=5.0 / 3.0, sphere=1, sphere_r=1.0)
    st = [np.full(P.shape, rho), _zeros(P), _zeros(P), _zeros(P), np.full(P.shape, p)]
    f = [np.zeros(P.shape) for _ in range(10)]
    f[0][:] = fv
    return Problem(P, st + f, cfl=0.8, nsteps=10, name=f"ball_{n}")


def bricks(count: int = 256, seed: int = 1814, nmin: int = 16, nmax: int = 64):
    """Batched-brick workload: `count` independent bricks with per-axis sizes
    drawn uniformly from [nmin, nmax]; each is, by a fair coin, a periodic
    sine-flow cube (config-1 construction) or a stratified box (config-2
    construction), each from its own seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(count):
        nn = tuple(int(v) for v in rng.integers(nmin, nmax + 1, size=3))
        kind = int(rng.integers(0, 2))
        bseed = int(rng.integers(0, 2 ** 31))
        out.append(brick(nn, kind, bseed))
    return out


def brick(nn, kind: int, seed: int) -> Problem:
    """One brick of the batched workload (see `bricks`)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = nn
    h = 1.0 / max(nn)
    gamma = 5.0 / 3.0
    if kind == 0:
        P = GridParams(n=(nx, ny, nz), dx=h, bc=(BC_PERIODIC,) * 3, gamma=gamma,
                       base_kind=BASE_CONST, base=(1.0, 1.0, 0.0, 0.0, 0.0, 0.0))
        Z, Y, X = _mesh(P)
        L = (nx * h, ny * h, nz * h)
        vel = []
        for d in range(3):
            u = np.zeros(P.shape)
            for k in range(3):
                kv = rng.integers(-1, 2, size=3).astype(np.float64)
                kv[d] = 0.0
                if not np.any(kv):
                    kv[(d + 1) % 3] = 1.0
                ph = rng.uniform(0, 2 * math.pi)
                u += np.sin(2 * math.pi * (k + 1) * (kv[0] * X / L[0] + kv[1] * Y / L[1]
                                                     + kv[2] * Z / L[2]) + ph)
            vel.append(0.05 * u)
        cx = 0.5 * np.array(L)
        rad = 0.25 * min(L)

        def ball(x, y, z):
            r = np.sqrt((x - cx[0]) ** 2 + (y - cx[1]) ** 2 + (z - cx[2]) ** 2)
            return 0.5 * (1.0 - np.tanh((r - rad) / h))

        fv = fv_moments_quadrature(P, ball, order=3)
        st = [np.zeros(P.shape), *vel, np.zeros(P.shape)]
        return Problem(P, st + fv, cfl=0.8, nsteps=1, name="brick_sine")
    Lz = nz * h
    g0 = config2_gravity(gamma) / Lz
    P = GridParams(n=(nx, ny, nz), dx=h, bc=(BC_PERIODIC, BC_PERIODIC, BC_REFLECT), gamma=gamma,
                   grav_kind=GRAV_CONST, grav=(0.0, 0.0, -g0, 0.0),
                   base_kind=BASE_POLY_Z, base=(1.0, 1.0, 0.0, 0.8 * Lz, 0.5, Lz),
                   heat_kind=HEAT_LAYER_Z, heat=(0.1, 0.1 * Lz, 0.0))
    Z, Y, X = _mesh(P)
    _, p_cf = polytrope_closed_form(Z[:, 0, 0], 1.0, 1.0, gamma, -g0, 0.0, 0.8 * Lz, 0.5)
    noise = rng.uniform(-1.0, 1.0, size=P.shape)
    pp = np.where(Z < 0.8 * Lz, 1e-3 * p_cf[:, None, None] * noise, 0.0)
    vel = [rng.uniform(-1, 1, size=P.shape) * 1e-3 for _ in range(2)] + [np.zeros(P.shape)]
    st = [np.zeros(P.shape), *vel, pp]
    return Problem(P, st + fv_step_z(P, 0.8 * Lz), cfl=0.8, nsteps=1, name="brick_strat")


def sod(n: int = 200) -> Problem:
    """Sod shock tube along x on [0,1], diaphragm at 0.5, gamma = 1.4,
    (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1); fv marks the left gas."""
    P = GridParams(n=(n, 1, 1), dx=1.0 / n, bc=(BC_REFLECT, BC_PERIODIC, BC_PERIODIC),
                   gamma=1.4)
    x = _centres(P, 0)[None, None, :]
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125) + np.zeros(P.shape)
    p = np.where(left, 1.0, 0.1) + np.zeros(P.shape)
    f = [np.zeros(P.shape) for _ in range(10)]
    f[0][:] = np.where(left, 1.0, 0.0)
    return Problem(P, [rho, np.zeros(P.shape), np.zeros(P.shape), np.zeros(P.shape), p] + f,
                   cfl=0.8, nsteps=0, name=f"sod_{n}")


def blast(n=24, p_in: float = 10.0, radius: float = 0.2, bc=None, centre=(0.5, 0.5, 0.5)) -> Problem:
    """Spherical blast: gas at rest, rho = 1, p = p_in inside r < radius
    about `centre` and 1 outside (cell-centre values), gamma = 1.4; fv marks
    the hot gas.  A strong outgoing shock.  n: cells per axis, or (nx, ny,
    nz) with dx = 1 / nx; bc: per-axis boundary kinds (default periodic)."""
    nn = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    P = GridParams(n=nn, dx=1.0 / nn[0], bc=tuple(bc) if bc else (BC_PERIODIC,) * 3, gamma=1.4)
    z, y, x = _mesh(P)
    inside = ((x - centre[0]) ** 2 + (y - centre[1]) ** 2) + (z - centre[2]) ** 2 < radius * radius
    p = np.where(inside, p_in, 1.0)
    f = [np.zeros(P.shape) for _ in range(10)]
    f[0][:] = np.where(inside, 1.0, 0.0)
    return Problem(P, [np.ones(P.shape), _zeros(P), _zeros(P), _zeros(P), p] + f,
                   cfl=0.8, nsteps=10, name=f"blast_{'x'.join(str(v) for v in nn)}")


# ---------------------------------------------------------------------
# The advection test of Fig. 3: a slotted disk in a rigid rotation (2-D)
# ---------------------------------------------------------------------

@dataclasses.dataclass
class Zalesak:
    """2-D PPB advection problem: grid, rotation and the 6 fv moments
    (f0, fx, fy, fxx, fyy, fxy; arrays (ny, nx), x fastest)."""
    n: tuple
    dx: float
    origin: tuple
    centre: tuple
    omega: float
    coef: list
    disk: tuple          # (xc, yc, radius, slot half-width, slot top)

    def dt(self, courant: float = 0.5) -> float:
        """dt for the largest face Courant number `courant` on the grid."""
        nx, ny = self.n
        ext = max(abs(self.origin[0] - self.centre[0]), abs(self.origin[0] + nx * self.dx - self.centre[0]),
                  abs(self.origin[1] - self.centre[1]), abs(self.origin[1] + ny * self.dx - self.centre[1]))
        return courant * self.dx / (abs(self.omega) * ext)


def _square_moments(a, b, c, d):
    """Integrals of 1, s, t, P2(s), P2(t), s t over [a,b] x [c,d] (cell
    coordinates, P2(s) = s^2 - 1/12)."""
    w, h = b - a, d - c
    m1s = (b * b - a * a) / 2.0
    m1t = (d * d - c * c) / 2.0
    p2s = (b ** 3 - a ** 3) / 3.0 - w / 12.0
    p2t = (d ** 3 - c ** 3) / 3.0 - h / 12.0
    return np.stack([w * h, m1s * h, w * m1t, p2s * h, w * p2t, m1s * m1t])


def slotted_disk_moments(n: int = 100, xc: float = 0.5, yc: float = 0.75, radius: float = 0.15,
                         slot_half: float = 0.025, slot_top: float = 0.85, depth: int = 12):
    """Exact-to-quadrature-depth moments of the indicator of a disk (centre
    (xc, yc), radius) minus the vertical slot |x - xc| < slot_half below
    y = slot_top, on the unit square with n x n cells.  Cut cells are
    subdivided into quarters down to `depth` levels; a sub-square entirely
    inside or outside the shape contributes its exact polynomial moments,
    the last level is decided by its centre."""
    dx = 1.0 / n
    acc = np.zeros((6, n, n))
    # squares: (cell i, cell j, s0, t0, size) in cell coordinates, s0 <= s <= s0 + size
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ii.ravel().astype(np.int64)
    cj = jj.ravel().astype(np.int64)
    s0 = np.full(ci.shape, -0.5)
    t0 = np.full(ci.shape, -0.5)
    size = 1.0
    for level in range(depth + 1):
        x_lo = (ci + 0.5 + s0) * dx
        y_lo = (cj + 0.5 + t0) * dx
        x_hi, y_hi = x_lo + size * dx, y_lo + size * dx
        # disk: nearest and farthest point of the square from the centre
        nx_ = np.clip(xc, x_lo, x_hi) - xc
        ny_ = np.clip(yc, y_lo, y_hi) - yc
        near2 = nx_ * nx_ + ny_ * ny_
        fx_ = np.maximum(np.abs(x_lo - xc), np.abs(x_hi - xc))
        fy_ = np.maximum(np.abs(y_lo - yc), np.abs(y_hi - yc))
        far2 = fx_ * fx_ + fy_ * fy_
        disk_in = far2 <= radius * radius
        disk_out = near2 >= radius * radius
        # slot: x in (xc - h, xc + h), y < slot_top
        slot_in = (x_lo >= xc - slot_half) & (x_hi <= xc + slot_half) & (y_hi <= slot_top)
        slot_out = (x_hi <= xc - slot_half) | (x_lo >= xc + slot_half) | (y_lo >= slot_top)
        inside = disk_in & slot_out
        outside = disk_out | slot_in
        if level == depth:
            xm, ym = 0.5 * (x_lo + x_hi), 0.5 * (y_lo + y_hi)
            cen = ((xm - xc) ** 2 + (ym - yc) ** 2 < radius * radius) & \
                ~((np.abs(xm - xc) < slot_half) & (ym < slot_top))
            inside = cen
            outside = ~cen
        sel = inside
        if np.any(sel):
            mom = _square_moments(s0[sel], s0[sel] + size, t0[sel], t0[sel] + size)
            for q in range(6):
                np.add.at(acc[q], (cj[sel], ci[sel]), mom[q])
        cut = ~(inside | outside)
        if not np.any(cut):
            break
        ci, cj, s0, t0 = ci[cut], cj[cut], s0[cut], t0[cut]
        half = 0.5 * size
        ci = np.concatenate([ci] * 4)
        cj = np.concatenate([cj] * 4)
        s0 = np.concatenate([s0, s0 + half, s0, s0 + half])
        t0 = np.concatenate([t0, t0, t0 + half, t0 + half])
        size = half
    norm = np.array([1.0, 12.0, 12.0, 180.0, 180.0, 144.0])
    return [acc[q] * norm[q] for q in range(6)]


def zalesak(n: int = 100) -> Zalesak:
    """The slotted disk of the classic Zalesak test on the unit square
    (n x n cells): disk of radius 0.15 centred at (0.5, 0.75), slot 0.05 wide
    reaching up to y = 0.85, rotating rigidly about (0.5, 0.5) once per unit
    time."""
    coef = slotted_disk_moments(n)
    return Zalesak(n=(n, n), dx=1.0 / n, origin=(0.0, 0.0), centre=(0.5, 0.5),
                   omega=2.0 * math.pi, coef=coef, disk=(0.5, 0.75, 0.15, 0.025, 0.85))


def render_subcells(coef, sub: int = 4) -> np.ndarray:
    """fv averaged over sub x sub squares of every cell from its 6 moments
    (Fig. 3's rendering): array (ny * sub, nx * sub)."""
    f0, fx, fy, fxx, fyy, fxy = [np.asarray(a, dtype=np.float64) for a in coef]
    ny, nx = f0.shape
    edges = np.linspace(-0.5, 0.5, sub + 1)
    out = np.zeros((ny * sub, nx * sub))
    area = (1.0 / sub) ** 2
    for b in range(sub):
        for a in range(sub):
            m = _square_moments(edges[a], edges[a + 1], edges[b], edges[b + 1])
            val = (f0 * m[0] + fx * m[1] + fy * m[2] + fxx * m[3] + fyy * m[4] + fxy * m[5]) / area
            out[b::sub, a::sub] = val
    return out


def config3_params(n: int = 512, g0: float = 6.0) -> GridParams:
    """The grid and physics of the spherical convection shell (config3) at
    n^3 cells, without its state."""
    dx = 2.0 / n
    return GridParams(n=(n, n, n), dx=dx, origin=(-1.0, -1.0, -1.0),
                      bc=(BC_REFLECT,) * 3, gamma=5.0 / 3.0, sphere=1, sphere_r=1.0,
                      grav_kind=GRAV_RADIAL, grav=(g0, 0.1, 1.0 - 5 * dx, 1.0 - dx),
                      base_kind=BASE_POLY_R,
                      base=(1.0, 1.0, 0.0, 0.5, 0.5, math.sqrt(3.0) + dx),
                      heat_kind=HEAT_BALL, heat=(0.1, 0.2, 0.0))


def config3_planes(n: int, k0: int, nk: int, seed: int = 1813, g0: float = 6.0,
                   quad_order: int = 6) -> list:
    """Planes k0 .. k0 + nk - 1 of config3(n, seed)'s state, the same values
    (15 arrays of shape (nk, n, n)): the velocity noise is drawn from the
    same PCG64 stream advanced to the slab's first cell (component d of cell
    c is draw d n^3 + c), the fv moments come from the same exact values
    and quadrature of the cut cells.  For grids too large to hold whole."""
    P = config3_params(n, g0)
    S = GridParams(n=(n, n, nk), dx=P.dx, origin=P.origin, bc=P.bc, gamma=P.gamma, sphere=1, sphere_r=1.0)
    shape = S.shape
    c_ref = math.sqrt(P.gamma)
    z = _centres(P, 2)[k0:k0 + nk]
    y = _centres(P, 1)
    x = _centres(P, 0)
    r2 = (z * z)[:, None, None] + (y * y)[None, :, None] + (x * x)[None, None, :]
    solid = r2 >= 1.0
    vel = []
    for d in range(3):
        bg = np.random.PCG64(seed)
        bg.advance(d * n ** 3 + k0 * n * n)
        u = np.random.Generator(bg).uniform(-1.0, 1.0, size=shape)
        u *= 1e-4 * c_ref
        u[solid] = 0.0
        vel.append(u)
    half = 0.5 * math.sqrt(3.0) * P.dx
    r = np.sqrt(r2)
    cut = np.abs(r - 0.5) < half
    fv = [np.zeros(shape) for _ in range(10)]
    fv[0][r >= 0.5 + half] = 1.0
    if np.any(cut):
        def shell(X, Y, Z):
            return (X * X + Y * Y + Z * Z >= 0.25).astype(np.float64)
        mom = fv_moments_quadrature(S, shell, mask=cut, order=quad_order, k0=k0)
        for q in range(10):
            fv[q][cut] = mom[q][cut]
    return [np.zeros(shape), *vel, np.zeros(shape), *fv]

"""Pins of the oracle's source terms and of its characteristic tracing,
each against a closed form or an exact solution of the Euler equations:

  free fall          a uniform gas in constant gravity (periodic, plain form)
                     accelerates as u = u0 + g t, and its pressure stays
                     fixed: the momentum source, the work of gravity in the
                     energy equation and the half-step gravity source of the
                     traced face states together give exactly the kinetic
                     energy gain (Sec. 1 gravity on the perturbation form; the
                     energy work is g times the mass flux);
  heating            the total energy rises by dt Q0 times the closed-form
                     volume integral of the heating profile (Sec. 2: the
                     heated core that drives the convection);
  moving column      a hydrostatic polytrope translating at a uniform speed
                     along constant gravity is an exact solution; in the
                     perturbation form its density and pressure changes come
                     entirely from the base-advection sources (Sec. 1: the
                     base state is subtracted and advanced analytically), so
                     second-order convergence to it pins their signs and
                     their half-step timing;
  transverse shear   a transverse velocity profile is carried at the normal
                     speed u (the entropy/shear family of the tracing);
  acoustic waves     small-amplitude simple waves of either family, in gas at
                     rest, in subsonic flow and in supersonic flow both ways,
                     travel at u -/+ c unchanged (linear theory): these reach
                     every projection of the characteristic tracing, the
                     supersonic ones included;
  Sod                plateau values at N = 400 against the exact solution.

A planted mistake in any of these terms (a flipped sign, a dropped term, the
wrong wave's domain of dependence) fails at least one pin below; the
planted-mistake tests build such altered copies of the oracle and check it.
"""
import math

import numpy as np
import pytest

import exact_riemann as er
import oracle
from paper_1810_13416_amd import problems as pr

GAMMA = 5.0 / 3.0


def _run_to(O, tend, cfl=0.8):
    t = 0.0
    while t < tend - 1e-13:
        dt = min(O.dt(cfl), tend - t)
        O.step(dt)
        t += dt
    return t


def _orders(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


# ----------------------------------------------------------------------
# free fall
# ----------------------------------------------------------------------

@pytest.mark.parametrize("g", [(0.0, 0.0, -0.7), (0.45, 0.0, 0.0), (0.3, -0.5, 0.7)])
def test_free_fall_closed_form(g):
    P = pr.GridParams(n=(8, 6, 10), dx=0.1, bc=(0, 0, 0), gamma=GAMMA, grav_kind=pr.GRAV_CONST,
                      grav=(g[0], g[1], g[2], 0.0))
    rho, u0, p = 1.3, np.array([0.1, -0.2, 0.05]), 0.9
    st = [np.full(P.shape, rho), np.full(P.shape, u0[0]), np.full(P.shape, u0[1]),
          np.full(P.shape, u0[2]), np.full(P.shape, p), np.full(P.shape, 0.4)] + \
         [np.zeros(P.shape) for _ in range(9)]
    O = oracle.Oracle(P, threads=2)
    O.set_state(st)
    dt, k = 0.01, 12
    for _ in range(k):
        O.step(dt)
    out = O.get_state()
    assert np.array_equal(out[0], st[0])                 # no mass moves
    for d in range(3):
        want = u0[d] + g[d] * k * dt
        assert np.max(np.abs(out[1 + d] - want)) <= 1e-13, (d, np.max(np.abs(out[1 + d] - want)))
    # pressure unchanged: the energy gain is exactly the kinetic energy gain
    assert np.max(np.abs(out[4] - p)) <= 1e-12 * p, np.max(np.abs(out[4] - p))
    assert np.array_equal(out[5], st[5])


# ----------------------------------------------------------------------
# heating
# ----------------------------------------------------------------------

def test_heating_layer_total_energy_closed_form():
    # h = Q0 below half the extent, smoothstep to 0 at the extent: its
    # integral over z from the layer's base is 0.75 * extent
    q0, ext = 0.2, 0.5
    P = pr.GridParams(n=(4, 4, 64), dx=1.0 / 64, bc=(0, 0, 1), gamma=GAMMA,
                      heat_kind=pr.HEAT_LAYER_Z, heat=(q0, ext, 0.0))
    st = [np.ones(P.shape), np.zeros(P.shape), np.zeros(P.shape), np.zeros(P.shape),
          np.ones(P.shape), np.full(P.shape, 0.5)] + [np.zeros(P.shape) for _ in range(9)]
    O = oracle.Oracle(P, threads=2)
    O.set_state(st)
    e0 = O.totals()[4]
    dt, k = 0.002, 4
    for _ in range(k):
        O.step(dt)
    gain = O.totals()[4] - e0
    area = (4 / 64) * (4 / 64)
    want = k * dt * q0 * area * 0.75 * ext
    assert abs(gain / want - 1.0) <= 2e-4, gain / want


def test_heating_ball_total_energy_closed_form():
    # integral of h(r / ext) over space: 4 pi ext^3 (1/24 + 13/120) = 0.6 pi ext^3
    q0, ext = 0.2, 0.6
    n = 40
    P = pr.GridParams(n=(n, n, n), dx=2.0 / n, origin=(-1.0, -1.0, -1.0), bc=(1, 1, 1), gamma=GAMMA,
                      sphere=1, sphere_r=0.95, heat_kind=pr.HEAT_BALL, heat=(q0, ext, 0.0))
    st = [np.ones(P.shape), np.zeros(P.shape), np.zeros(P.shape), np.zeros(P.shape),
          np.ones(P.shape), np.full(P.shape, 0.5)] + [np.zeros(P.shape) for _ in range(9)]
    O = oracle.Oracle(P, threads=8)
    O.set_state(st)
    e0 = O.totals()[4]
    dt, k = 0.002, 2
    for _ in range(k):
        O.step(dt)
    gain = O.totals()[4] - e0
    want = k * dt * q0 * 0.6 * math.pi * ext ** 3
    assert abs(gain / want - 1.0) <= 3e-3, gain / want


# ----------------------------------------------------------------------
# a hydrostatic column translating along constant gravity
# ----------------------------------------------------------------------

G0, U0, TEND = 1.3, 0.2, 0.15


def _moving_column(n):
    P = pr.GridParams(n=(1, 1, n), dx=1.0 / n, bc=(0, 0, 1), gamma=GAMMA, grav_kind=pr.GRAV_CONST,
                      grav=(0.0, 0.0, -G0, 0.0), base_kind=pr.BASE_POLY_Z,
                      base=(1.0, 1.0, 0.0, 2.0, 1.0, 1.0))
    z = (np.arange(n) + 0.5) / n
    st = [np.zeros(P.shape) for _ in range(15)]
    st[3][:] = U0
    st[5][:] = 0.5
    O = oracle.Oracle(P, threads=1)
    O.set_state(st)
    t = _run_to(O, TEND)
    out = O.get_state()
    r0, p0 = O.base()
    # exact: the base profile shifted by U0 t (closed-form polytrope, K = 1)
    rho_ex, p_ex = pr.polytrope_closed_form(z - U0 * t, 1.0, 1.0, GAMMA, -G0, 0.0, 2.0, 1.0)
    win = (z > 0.3) & (z < 0.7)        # not reached by the walls' signals by TEND
    rho = (r0 + out[0])[:, 0, 0]
    p = (p0 + out[4])[:, 0, 0]
    return (np.mean(np.abs(rho - rho_ex)[win]), np.mean(np.abs(p - p_ex)[win]),
            np.mean(np.abs(out[3][:, 0, 0] - U0)[win]))


def test_moving_hydrostatic_column_converges():
    e = np.array([_moving_column(n) for n in (64, 128, 256)])
    for q, name in enumerate(("rho", "p", "u")):
        o = _orders(e[:, q])
        assert min(o) >= 1.8, (name, o, e[:, q])
    assert e[-1, 0] <= 1e-6 and e[-1, 1] <= 1e-6, e[-1]


# ----------------------------------------------------------------------
# transverse shear carried at the flow speed
# ----------------------------------------------------------------------

def _shear(n, u=0.5):
    P = pr.GridParams(n=(n, 1, 1), dx=1.0 / n, bc=(0, 0, 0), gamma=GAMMA)
    x = (np.arange(n) + 0.5) / n
    sn = np.sinc(1.0 / n)               # cell average of sin / cos over one cell
    st = [np.zeros(P.shape) for _ in range(15)]
    st[0][:] = 1.0
    st[1][:] = u
    st[2][0, 0] = 0.1 * sn * np.sin(2 * math.pi * x)
    st[3][0, 0] = 0.05 * sn * np.cos(2 * math.pi * x)
    st[4][:] = 1.0
    st[5][:] = 0.5
    O = oracle.Oracle(P, threads=1)
    O.set_state(st)
    _run_to(O, 1.0 / u)                  # one period
    out = O.get_state()
    return (np.mean(np.abs(out[2] - st[2])) / 0.1, np.mean(np.abs(out[3] - st[3])) / 0.05)


def test_transverse_shear_order():
    e = np.array([_shear(n) for n in (32, 64, 128)])
    for q in range(2):
        o = _orders(e[:, q])
        assert min(o) >= 2.5, (q, o, e[:, q])


# ----------------------------------------------------------------------
# small-amplitude simple waves
# ----------------------------------------------------------------------

EPS = 1e-5
C0 = math.sqrt(GAMMA)


def _simple_wave_run(n, U, fam, eps):
    P = pr.GridParams(n=(n, 1, 1), dx=1.0 / n, bc=(0, 0, 0), gamma=GAMMA, base_kind=pr.BASE_CONST,
                      base=(1.0, 1.0, 0.0, 0.0, 0.0, 0.0))
    x = (np.arange(n) + 0.5) / n
    dp = eps * np.sinc(1.0 / n) * np.sin(2 * math.pi * x)
    st = [np.zeros(P.shape) for _ in range(15)]
    st[0][0, 0] = dp / C0 ** 2
    st[1][0, 0] = U + fam * dp / C0
    st[4][0, 0] = dp
    st[5][:] = 0.5
    O = oracle.Oracle(P, threads=1)
    O.set_state(st)
    _run_to(O, 1.0 / abs(U + fam * C0))
    return st, O.get_state()


def _simple_wave(n, U, fam):
    """Linear simple wave of family fam (+1: u + c, -1: u - c) on a constant
    base rho0 = p0 = 1 moving at U, after one period of the wave.  The runs
    with amplitudes +EPS and -EPS are differenced: the half difference keeps
    the linear response and cancels the quadratic (nonlinear) one, which
    would otherwise put a floor of order EPS under the truncation error."""
    st, a = _simple_wave_run(n, U, fam, EPS)
    _, b = _simple_wave_run(n, U, fam, -EPS)
    lin = [0.5 * (a[q] - b[q]) for q in (0, 1, 4)]
    want = [st[0], st[1] - U, st[4]]
    scale = (EPS / C0 ** 2, EPS / C0, EPS)
    return tuple(np.mean(np.abs(lin[q] - want[q])) / scale[q] for q in range(3))


@pytest.mark.parametrize("U,fam", [(0.0, 1), (0.0, -1), (0.5, 1), (-0.5, -1),
                                   (2 * C0, -1), (2 * C0, 1), (-2 * C0, 1), (-2 * C0, -1)],
                         ids=["rest+", "rest-", "sub+", "sub-", "super_u-c", "super_u+c",
                              "super_neg_u+c", "super_neg_u-c"])
def test_acoustic_simple_wave_order(U, fam):
    e = np.array([_simple_wave(n, U, fam) for n in (32, 64, 128)])
    for q, name in enumerate(("rho", "u", "p")):
        o = _orders(e[:, q])
        assert min(o) >= 2.5, (name, o, e[:, q])
    assert np.max(e[-1]) <= 2e-3, e[-1]


# ----------------------------------------------------------------------
# Sod at N = 400: plateaus
# ----------------------------------------------------------------------

def test_sod_plateaus_n400():
    n = 400
    prob = pr.sod(n)
    O = oracle.Oracle(prob.params, threads=2)
    O.set_state(prob.state)
    _run_to(O, 0.2)
    st = O.get_state()
    x = (np.arange(n) + 0.5) / n
    pstar, ustar = er.star_state(1, 0, 1, 0.125, 0, 0.1, 1.4)
    g = 1.4
    rho_l = (pstar / 1.0) ** (1 / g)                                     # behind the rarefaction
    rho_r = 0.125 * ((pstar / 0.1 + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * pstar / 0.1 + 1))
    w_s = ustar * rho_r / (rho_r - 0.125)                               # shock speed
    x_c, x_s = 0.5 + ustar * 0.2, 0.5 + w_s * 0.2
    rho, u, p = st[0][0, 0], st[1][0, 0], st[4][0, 0]
    # plateaus, a dozen cells clear of the smeared contact and of the shock
    # (measured: 2.8e-4, 1.2e-4, 1.8e-4, 5.2e-4)
    left = (x > x_c - 0.07) & (x < x_c - 0.03)
    right = (x > x_c + 0.03) & (x < x_s - 0.02)
    assert np.max(np.abs(rho[left] - rho_l)) <= 4e-4, np.max(np.abs(rho[left] - rho_l))
    assert np.max(np.abs(rho[right] - rho_r)) <= 2e-4, np.max(np.abs(rho[right] - rho_r))
    both = left | right
    assert np.max(np.abs(p[both] - pstar)) <= 3e-4, np.max(np.abs(p[both] - pstar))
    assert np.max(np.abs(u[both] - ustar)) <= 7e-4, np.max(np.abs(u[both] - ustar))
    # the shock: half-way density between rho_r and 0.125 within one cell of x_s
    mid = 0.5 * (rho_r + 0.125)
    k = np.flatnonzero((rho[:-1] >= mid) & (rho[1:] < mid) & (x[:-1] > x_c))[0]
    xs_num = x[k] + (rho[k] - mid) / (rho[k] - rho[k + 1]) / n
    assert abs(xs_num - x_s) <= 1.0 / n, (xs_num, x_s)

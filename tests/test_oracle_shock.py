"""Pins of the shock dissipation in the oracle (Sec. 1: a fully 3-D
dissipation inside shocks; the form here is a reading after the artificial
dissipation of Colella & Woodward 1984, Sec. 4, driven by the full 3-D
velocity divergence).  Expected values: the exact divergence of a linear
velocity field, exact preservation of a uniform state, round-off
conservation, mirror symmetry, and against the exact Sod solution (shock
position from the closed-form shock speed) the smoothing of the post-shock
state."""
import math

import numpy as np

import oracle
from paper_1810_13416_amd import problems as pr
import exact_riemann as er

ODD_X = {1, 6, 12, 14}


def test_divergence_of_a_linear_velocity_field_is_exact():
    n = 8
    P = pr.GridParams(n=(n, n, n), dx=1.0 / n, bc=(pr.BC_REFLECT,) * 3, gamma=1.4)
    z, y, x = np.meshgrid(*(pr._centres(P, a) for a in (2, 1, 0)), indexing="ij")
    a, b, c = 0.3, -0.2, 0.05
    st = [np.full(P.shape, 1.0), a * (x - 0.5), b * (y - 0.5), c * (z - 0.5),
          np.full(P.shape, 1.0)] + [np.zeros(P.shape) for _ in range(10)]
    O = oracle.Oracle(P, threads=2)
    O.set_state(st)
    D = O.divergence()
    inner = (slice(1, n - 1),) * 3
    # undivided central differences of a linear field: (a + b + c) dx
    assert np.allclose(D[inner], (a + b + c) / n, rtol=0, atol=1e-15)
    O.close()


def test_divergence_at_the_confining_sphere_sees_a_wall():
    # uniform flow (U, 0, 0) in the sphere: the wall's mirror image moves
    # at -U, so a fluid cell whose +x neighbour is solid has D = -U (the
    # flow runs into the wall), one whose -x neighbour is solid D = +U, and
    # every other fluid cell D = 0
    prob = pr.ball(16)
    U = 0.2
    st = [a.copy() for a in prob.state]
    st[1][:] = U
    O = oracle.Oracle(prob.params, threads=2)
    O.set_state(st)
    D = O.divergence()
    z, y, x = np.meshgrid(*(pr._centres(prob.params, a) for a in (2, 1, 0)), indexing="ij")
    dx = prob.params.dx
    fluid = lambda X: (X * X + y * y) + z * z < 1.0
    f0, fp, fm = fluid(x), fluid(x + dx), fluid(x - dx)
    want = np.where(f0 & ~fp, -U, 0.0) + np.where(f0 & ~fm, U, 0.0)
    assert np.allclose(D, want, rtol=0, atol=1e-16)
    assert np.any(f0 & ~fp) and np.any(f0 & ~fm)
    O.close()


def test_no_dissipative_flux_through_the_sphere_wall():
    # flow into the confining sphere's wall compresses the cells next to
    # it; the solid cells take no update, so any flux across the wall would
    # change the fluid's mass
    prob = pr.ball(16)
    st = [a.copy() for a in prob.state]
    st[1][:] = 0.3
    O = oracle.Oracle(prob.params, threads=2)
    O.set_state(st)
    O.set_dissipation(0.1)
    m0 = O.totals()[0]
    O.run(5, 0.8)
    assert abs(O.totals()[0] / m0 - 1.0) <= 1e-14
    O.close()


def test_uniform_state_is_unchanged_with_dissipation():
    prob = pr.uniform()
    O = oracle.Oracle(prob.params, threads=4)
    O.set_state(prob.state)
    O.set_dissipation(0.1)
    start = O.get_conserved()
    O.run(10, 0.8)
    end = O.get_conserved()
    for q in range(15):
        assert np.array_equal(start[q], end[q]), q
    O.close()


def test_conservation_with_dissipation():
    prob = pr.blast(16)
    O = oracle.Oracle(prob.params, threads=4)
    O.set_state(prob.state)
    O.set_dissipation(0.1)
    t0 = O.totals()
    O.run(10, 0.8)
    t1 = O.totals()
    # mass and total energy (fv volume is conserved only by divergence-free flow)
    for q in (0, 4):
        assert abs(t1[q] - t0[q]) <= 1e-13 * abs(t0[q]), q
    for q in (1, 2, 3):
        assert abs(t1[q] - t0[q]) <= 1e-13, q
    O.close()


def test_mirror_symmetry_with_dissipation():
    prob = pr.blast(16)
    O = oracle.Oracle(prob.params, threads=4)
    O.set_state(prob.state)
    O.set_dissipation(0.1)
    O.run(6, 0.8)
    c = O.get_conserved()
    for q in range(15):
        m = (-1.0 if q in ODD_X else 1.0) * c[q][:, :, ::-1]
        # the blast is centred between cells n/2-1 and n/2: x -> 1 - x maps cell i to n-1-i
        assert np.array_equal(c[q], m), q
    O.close()


def sod(n, k):
    prob = pr.sod(n)
    O = oracle.Oracle(prob.params, threads=2)
    O.set_state(prob.state)
    O.set_dissipation(k)
    t = 0.0
    while t < 0.2 - 1e-14:
        dt = min(O.dt(0.8), 0.2 - t)
        O.step(dt)
        t += dt
    st = O.get_state()
    O.close()
    return st


def test_sod_dissipation_smooths_the_post_shock_state_and_keeps_the_shock():
    n = 200
    g = 1.4
    plain, diss = sod(n, 0.0), sod(n, 0.1)
    x = (np.arange(n) + 0.5) / n
    ps, us = er.star_state(1, 0, 1, 0.125, 0, 0.1, g)
    # right shock speed (closed form for a shock into gas at rest)
    cr = math.sqrt(g * 0.1 / 0.125)
    S = cr * math.sqrt((g + 1) / (2 * g) * ps / 0.1 + (g - 1) / (2 * g))
    xs = 0.5 + S * 0.2
    rho_post = 0.125 * ((ps / 0.1 + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / 0.1 + 1))
    for st in (plain, diss):
        r = st[0][0, 0]
        # the shock: where rho crosses halfway between its two sides
        mid = 0.5 * (rho_post + 0.125)
        i = np.where((r[:-1] >= mid) & (r[1:] < mid))[0]
        assert i.size >= 1 and abs(x[i[-1]] + 0.5 / n - xs) <= 2.0 / n
    # total variation of the pressure on the star plateau (exactly constant)
    plateau = (x > 0.72) & (x < 0.82)
    tv = [np.sum(np.abs(np.diff(st[4][0, 0][plateau]))) for st in (plain, diss)]
    assert tv[1] < tv[0]
    # the rarefaction fan diverges: the dissipation leaves it alone (only
    # information from the shocked region reaches it, at round-off-like size)
    fan = (x > 0.28) & (x < 0.47)
    assert np.max(np.abs(plain[0][0, 0][fan] - diss[0][0, 0][fan])) <= 4e-4
    # overall accuracy stays that of the scheme
    ex = er.cell_averages(n, 0.2)
    e = [np.mean(np.abs(st[0][0, 0] - ex[0])) for st in (plain, diss)]
    assert e[1] <= 1.3 * e[0]


def test_dissipative_fluxes_closed_form_under_uniform_compression():
    # uniform compression u = -a (x - 1/2) (with a uniform transverse flow)
    # across a density step at uniform pressure: the undivided divergence is
    # -a dx in every interior cell, so every face between interior cells has
    # the coefficient K a dx and the dissipation is a discrete diffusion.
    # One x pass with K, minus the same pass without, is therefore
    # dt K a (U[j+1] - 2 U[j] + U[j-1]) for each of the five conserved hydro
    # fields U, and zero for the fv moments
    n, a, K = 32, 0.1, 0.1
    P = pr.GridParams(n=(n, 1, 1), dx=1.0 / n, bc=(pr.BC_REFLECT, pr.BC_PERIODIC, pr.BC_PERIODIC),
                      gamma=1.4)
    x = (np.arange(n) + 0.5) / n
    rho = np.where(x < 0.5, 1.0, 2.0)
    sh = P.shape
    fv = np.where(x < 0.5, 0.0, 1.0)
    st = [rho.reshape(sh), (-a * (x - 0.5)).reshape(sh), np.full(sh, 0.2), np.full(sh, -0.1), np.ones(sh),
          fv.reshape(sh)] + [np.zeros(sh) for _ in range(9)]
    res = []
    for k in (K, 0.0):
        O = oracle.Oracle(P, threads=1)
        O.set_state(st)
        O.set_dissipation(k)
        if k > 0.0:
            D = O.divergence()[0, 0]
            assert np.allclose(D[1:n - 1], -a / n, rtol=0, atol=1e-16)
            dt = 0.5 * O.dt(0.8)
            U = [c[0, 0].copy() for c in O.get_conserved()]
        O.pass_(0, dt)
        res.append([c[0, 0] for c in O.get_conserved()])
        O.close()
    j = slice(2, n - 2)
    for q in range(5):
        want = dt * K * a * (U[q][3:n - 1] - 2.0 * U[q][2:n - 2] + U[q][1:n - 3])
        assert np.allclose(res[0][q][j] - res[1][q][j], want, rtol=0, atol=2e-15), q
    # the step itself moved: the check is not vacuous
    assert abs(res[0][0][n // 2] - res[1][0][n // 2]) > 1e-6
    for q in range(5, 15):
        assert np.array_equal(res[0][q], res[1][q]), q

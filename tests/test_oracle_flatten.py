"""Pins of the flattening near strong shocks in the oracle (after Colella &
Woodward 1984, Sec. 4; the paper names only the 3-D shock dissipation, and
flattening is its customary companion).  Expected values come from
hand-worked pressure profiles (a smooth ramp, a one-cell and a two-cell
compressive step, an expanding step, a weak jump, a step at a chosen ratio
of the narrow to the wide pressure difference), from exact invariances
(mirror symmetry, a uniform state, a run in which no cell is flagged is the
run without flattening, bit for bit), round-off conservation, and the exact
Sod solution (shock position from the closed-form shock speed)."""
import math

import numpy as np

import oracle
from paper_1810_13416_amd import problems as pr
import exact_riemann as er

ODD_X = {1, 6, 12, 14}


def row(p, u, rho=1.0):
    """A 1-D state along x (reflecting ends) with the given p and u."""
    n = len(p)
    P = pr.GridParams(n=(n, 1, 1), dx=1.0 / n, bc=(pr.BC_REFLECT, pr.BC_PERIODIC, pr.BC_PERIODIC),
                      gamma=1.4)
    sh = P.shape
    st = [np.full(sh, rho), np.asarray(u, float).reshape(sh), np.zeros(sh), np.zeros(sh),
          np.asarray(p, float).reshape(sh)] + [np.zeros(sh) for _ in range(10)]
    O = oracle.Oracle(P, threads=1)
    O.set_state(st)
    f = O.flattening(0)[0, 0]
    O.close()
    return f


def test_smooth_steep_ramp_is_not_flattened():
    # p rises by 1 per cell, compressing: the narrow difference is half the
    # wide one, below the 3/4 that starts flattening
    n = 16
    f = row(1.0 + np.arange(n), -0.1 * np.arange(n))
    assert np.all(f[3:n - 3] == 0.0)


def test_one_cell_compressive_step_is_flattened():
    n = 16
    p = np.where(np.arange(n) < 8, 1.0, 10.0)
    u = np.where(np.arange(n) < 8, 0.5, 0.0)          # flow into the step
    f = row(p, u)
    assert f[7] == 1.0 and f[8] == 1.0
    assert np.all(f[:6] == 0.0) and np.all(f[11:] == 0.0)
    assert np.all((f >= 0.0) & (f <= 1.0))


def test_two_cell_step_flattens_the_middle_cell_and_the_one_behind():
    # p = 1 | 5.5 | 10: the middle cell's narrow and wide differences are
    # equal (fully flagged); its neighbours' are half (not flagged); the cell
    # on the high-pressure side takes the middle cell's value
    n = 16
    p = np.where(np.arange(n) < 7, 1.0, 10.0)
    p[7] = 5.5
    u = np.where(np.arange(n) < 8, 0.5, 0.0)
    f = row(p, u)
    assert f[7] == 1.0 and f[8] == 1.0 and f[6] == 0.0


def test_ratio_between_the_thresholds_gives_a_partial_coefficient():
    # narrow / wide difference 0.8 -> 10 (0.8 - 0.75) = 0.5
    n = 16
    p = np.ones(n)
    p[6], p[7], p[8], p[9] = 1.1, 1.9, 2.7, 3.0
    p[10:] = 3.0
    u = np.linspace(0.5, -0.5, n)
    f = row(p, u)
    assert abs(f[7] - 0.5) <= 1e-12


def test_expanding_step_is_not_flattened():
    n = 16
    p = np.where(np.arange(n) < 8, 1.0, 10.0)
    u = np.where(np.arange(n) < 8, -0.5, 0.5)         # flow away from the step
    assert np.all(row(p, u) == 0.0)


def test_weak_jump_is_not_flattened():
    n = 16
    p = np.where(np.arange(n) < 8, 1.0, 1.3)          # 30 % < 33 %
    u = np.where(np.arange(n) < 8, 0.5, 0.0)
    assert np.all(row(p, u) == 0.0)


def test_pressure_tie_keeps_the_coefficient_mirror_equivariant():
    # a 3-cell pressure plateau with compression only on its right edge:
    # the middle cell has equal pressures on both sides, so no side is the
    # low-pressure one; the coefficient of the mirrored profile must be the
    # mirror of the coefficient (a one-sided tie rule would break this)
    n = 16
    p = np.ones(n)
    p[7:10] = 10.0
    u = np.zeros(n)
    u[8:] = 0.3
    u[10:] = -0.4                                    # converges across cell 9 only
    f = row(p, u)
    g = row(p[::-1], -u[::-1])
    assert np.array_equal(f, g[::-1])
    assert f[9] == 1.0 and f[8] == 1.0


def test_coefficient_is_mirror_symmetric():
    prob = pr.blast(16)
    O = oracle.Oracle(prob.params, threads=4)
    O.set_state(prob.state)
    O.run(3, 0.8)
    f = O.flattening(0)
    assert np.any(f > 0.0)
    # x -> 1 - x maps cell i to n - 1 - i (the blast is centred between cells)
    assert np.array_equal(f, f[:, :, ::-1])
    O.close()


def test_run_with_no_flagged_cell_is_the_plain_run():
    prob = pr.config1(n=16)
    A = oracle.Oracle(prob.params, threads=4)
    A.set_state(prob.state)
    for d in range(3):
        assert np.all(A.flattening(d) == 0.0)
    B = oracle.Oracle(prob.params, threads=4)
    B.set_state(prob.state)
    B.set_flattening(True)
    A.run(3, 0.8)
    B.run(3, 0.8)
    for a, b in zip(A.get_conserved(), B.get_conserved()):
        assert np.array_equal(a, b)
    A.close()
    B.close()


def test_uniform_state_is_unchanged_with_flattening():
    prob = pr.uniform()
    O = oracle.Oracle(prob.params, threads=4)
    O.set_state(prob.state)
    O.set_flattening(True)
    start = O.get_conserved()
    O.run(10, 0.8)
    for a, b in zip(start, O.get_conserved()):
        assert np.array_equal(a, b)
    O.close()


def test_conservation_and_symmetry_with_flattening():
    prob = pr.blast(16)
    O = oracle.Oracle(prob.params, threads=4)
    O.set_state(prob.state)
    O.set_flattening(True)
    t0 = O.totals()
    O.run(8, 0.8)
    t1 = O.totals()
    for q in (0, 4):
        assert abs(t1[q] - t0[q]) <= 1e-13 * abs(t0[q]), q
    for q in (1, 2, 3):
        assert abs(t1[q] - t0[q]) <= 1e-13, q
    c = O.get_conserved()
    for q in range(15):
        m = (-1.0 if q in ODD_X else 1.0) * c[q][:, :, ::-1]
        assert np.array_equal(c[q], m), q
    O.close()


def sod(n, flat):
    prob = pr.sod(n)
    O = oracle.Oracle(prob.params, threads=2)
    O.set_state(prob.state)
    O.set_flattening(flat)
    t = 0.0
    while t < 0.2 - 1e-14:
        dt = min(O.dt(0.8), 0.2 - t)
        O.step(dt)
        t += dt
    st = O.get_state()
    O.close()
    return st


def test_sod_with_flattening_keeps_the_shock_and_the_accuracy():
    n = 200
    g = 1.4
    plain, flat = sod(n, False), sod(n, True)
    x = (np.arange(n) + 0.5) / n
    ps, us = er.star_state(1, 0, 1, 0.125, 0, 0.1, g)
    cr = math.sqrt(g * 0.1 / 0.125)
    S = cr * math.sqrt((g + 1) / (2 * g) * ps / 0.1 + (g - 1) / (2 * g))
    xs = 0.5 + S * 0.2
    rho_post = 0.125 * ((ps / 0.1 + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / 0.1 + 1))
    for st in (plain, flat):
        r = st[0][0, 0]
        mid = 0.5 * (rho_post + 0.125)
        i = np.where((r[:-1] >= mid) & (r[1:] < mid))[0]
        assert i.size >= 1 and abs(x[i[-1]] + 0.5 / n - xs) <= 2.0 / n
    # the flattening acted
    assert not np.array_equal(plain[0], flat[0])
    ex = er.cell_averages(n, 0.2)
    e = [np.mean(np.abs(st[0][0, 0] - ex[0])) for st in (plain, flat)]
    assert e[1] <= 1.3 * e[0]
    # post-shock pressure plateau (exactly constant): flattening damps the
    # oscillations the shock leaves behind (total variation about halved)
    plateau = (x > 0.72) & (x < 0.82)
    tv = [np.sum(np.abs(np.diff(st[4][0, 0][plateau]))) for st in (plain, flat)]
    assert tv[1] < 0.75 * tv[0]


def test_convergence_margin_ignores_rounding_and_keeps_real_compression():
    # A cell is a shock candidate only if u(i-1) - u(i+1) > 1e-10 (|u(i-1)|
    # + |u(i+1)|).  Under a compressive pressure step, a uniform flow whose
    # velocities differ in the last bits only is not a shock: no flattening
    # whichever way the last bits lean (a strict test, > 0, would flatten
    # fully when they lean one way and not at all the other way).
    n = 16
    p = np.where(np.arange(n) < 8, 1.0, 10.0)
    for lean in (+1, -1):
        u = np.full(n, 0.3)
        for k in range(n):                 # one ulp per cell, falling (+1) or rising (-1)
            for _ in range(n - k if lean > 0 else k):
                u[k] = np.nextafter(u[k], 1.0)
        assert (u[6] - u[8] > 0) == (lean > 0)
        f = row(p, u)
        assert np.all(f == 0.0), (lean, f)
    # a real compression, 1e-8 of the flow speed across the step (far below
    # any shock's, far above rounding): full flattening at the step
    u = np.where(np.arange(n) < 8, 0.3 * (1 + 1e-8), 0.3)
    f = row(p, u)
    assert f[7] == 1.0 and f[8] == 1.0, f

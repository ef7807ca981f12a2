"""Pins of the oracle's building blocks against closed forms and exact
integrals that are written out here independently (no oracle formula is
re-typed: each check uses a different route to the same number)."""
import math

import numpy as np
import pytest

import exact_riemann as er
import oracle


def cubic_avg(c, a, b):
    """Exact average of c0 + c1 x + c2 x^2 + c3 x^3 over [a, b]."""
    F = lambda x: c[0] * x + c[1] * x ** 2 / 2 + c[2] * x ** 3 / 3 + c[3] * x ** 4 / 4
    return (F(b) - F(a)) / (b - a)


def test_interface_value_exact_on_cubics():
    # Sec. 1: interface values one order higher than the parabola -> exact for cubics
    rng = np.random.default_rng(1)
    for _ in range(50):
        c = rng.normal(size=4)
        h = rng.uniform(0.01, 0.5)
        x0 = rng.uniform(-1, 1)
        avgs = [cubic_avg(c, x0 + k * h, x0 + (k + 1) * h) for k in range(4)]
        xf = x0 + 2 * h
        exact = c[0] + c[1] * xf + c[2] * xf ** 2 + c[3] * xf ** 3
        got = oracle.face4(*avgs)
        assert abs(got - exact) <= 1e-13 * max(1.0, abs(exact))


def test_interface_value_not_exact_on_quartic():
    # a 4th-degree term must leave an error: the formula is 4th order, not more
    h = 0.1
    q = [((k + 1) * h) ** 5 / (5 * h) - (k * h) ** 5 / (5 * h) for k in range(4)]
    assert abs(oracle.face4(*q) - (2 * h) ** 4) > 1e-8


@pytest.mark.parametrize("q,expect", [
    ([1.0, 1.0, 1.0, 1.0, 1.0], 1.0),               # constant
    ([0.0, 1.0, 2.0, 3.0, 4.0], 1.0),               # linear: all second differences 0
    ([4.0, 1.0, 0.0, 1.0, 4.0], 1.0),               # parabola: equal second differences
    ([0.0, 0.0, 0.0, 1.0, 1.0], 0.0),               # jump inside the window
    ([0.0, 1.0, 0.0, 1.0, 0.0], 0.0),               # odd-even oscillation
    ([0.0, 0.0, 1.0, 0.0, 0.0], 0.0),               # spike: second differences change sign
    ([0.0, 1.0, 3.0, 6.0, 10.0], 1.0),              # D = 1, 1, 1
    ([0.0, 1.0, 3.0, 7.0, 13.0], 1.0),              # D = 1, 2, 2: ratio 2 is smooth
    ([0.0, 1.0, 3.0, 7.5, 14.0], 0.5),              # D = 1, 2.5, 2: ratio 2.5, halfway
    ([0.0, 1.0, 3.0, 8.0, 15.0], 0.0),              # D = 1, 3, 2: ratio 3 is not smooth
])
def test_smoothness_weight_cases(q, expect):
    assert oracle.smooth_weight(np.array(q)) == expect


def test_smoothness_weight_is_continuous_and_symmetric():
    # the weight varies continuously through the graded band, and is the same
    # for the mirrored and the negated window
    xs = np.linspace(7.0, 8.0, 201)
    w = [oracle.smooth_weight(np.array([0.0, 1.0, 3.0, x, 2 * x - 1.0])) for x in xs]
    assert max(abs(a - b) for a, b in zip(w[1:], w[:-1])) <= 0.011
    rng = np.random.default_rng(2)
    for _ in range(200):
        q = np.cumsum(np.cumsum(rng.uniform(0.5, 1.5, 5)))
        a = oracle.smooth_weight(q)
        assert oracle.smooth_weight(q[::-1]) == a and oracle.smooth_weight(-q) == a


def test_smoothness_sinusoid_extremum_is_smooth():
    # a sampled sinusoid with >= 6 cells per wavelength is smooth at its crest
    for ppw in (6, 8, 16, 64):
        x = np.arange(-2, 3) * (2 * math.pi / ppw)
        assert oracle.smooth_weight(np.cos(x)) == 1.0


def test_smoothness_kink_not_smooth():
    x = np.arange(-2, 3) * 0.1
    assert oracle.smooth_weight(np.abs(x)) == 0.0


def collision_pstar(rho, p, U, g):
    """Exact symmetric collision (u_L = -u_R = U > 0): two shocks, closed form."""
    C = math.sqrt(g * p * rho)
    b = U * U * C * C * (g + 1.0) / (2.0 * g * p)
    return p + 0.5 * (b + math.sqrt(b * b + 4.0 * U * U * C * C))


@pytest.mark.parametrize("U", [1e-4, 0.01, 0.3, 2.0, 10.0])
@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0])
def test_two_shock_collision_closed_form(U, g):
    rho, p = 1.3, 0.7
    out, it = oracle.riemann([rho, U, 0.2, -0.1, p], [rho, -U, 0.2, -0.1, p], gamma=g)
    assert it > 0
    pst = collision_pstar(rho, p, U, g)
    assert abs(out[4] - pst) <= 1e-13 * pst
    assert out[1] == 0.0
    # and the independent exact solver agrees (both are exact for shocks)
    pe, ue = er.star_state(rho, U, p, rho, -U, p, g)
    assert abs(pe - pst) <= 1e-12 * pst


def test_two_shock_matches_exact_for_shock_tube_with_shocks():
    # both waves shocks: the two-shock solver is exact
    g = 1.4
    L = (1.0, 2.0, 1.0)
    R = (0.5, -1.0, 0.8)
    out, _ = oracle.riemann([L[0], L[1], 0, 0, L[2]], [R[0], R[1], 0, 0, R[2]], gamma=g)
    pe, ue = er.star_state(*L, *R, g)
    assert abs(out[4] - pe) <= 1e-12 * pe
    assert abs(out[1] - ue) <= 1e-12


def test_acoustic_limit_equals_linear_guess():
    g, rho, p = 5.0 / 3.0, 1.0, 1.0
    C = math.sqrt(g * p * rho)
    eps = 1e-7
    L = np.array([rho, eps, 0, 0, p + 2 * eps])
    R = np.array([rho, -eps, 0, 0, p - eps])
    out, _ = oracle.riemann(L, R, gamma=g)
    guess = (C * L[4] + C * R[4] + C * C * (L[1] - R[1])) / (2 * C)
    assert abs(out[4] - guess) <= 10 * eps * eps


def test_riemann_base_state_cancels():
    # splitting p = p0f + p' and rho = rho0f + rho' must give the same face state
    g = 5.0 / 3.0
    L = np.array([1.1, 0.05, 0.1, 0.2, 2.0])
    R = np.array([0.9, -0.03, 0.3, -0.2, 1.9])
    full, _ = oracle.riemann(L, R, gamma=g)
    r0, p0 = 0.8, 1.7
    Lp = L - np.array([r0, 0, 0, 0, p0])
    Rp = R - np.array([r0, 0, 0, 0, p0])
    pert, _ = oracle.riemann(Lp, Rp, rho0f=r0, p0f=p0, gamma=g)
    assert abs(pert[4] + p0 - full[4]) <= 1e-14 * full[4]
    assert abs(pert[1] - full[1]) <= 1e-14
    assert abs(pert[0] + r0 - full[0]) <= 1e-14


def test_riemann_mirror_equivariant():
    g = 1.4
    L = np.array([1.0, 0.3, 0.1, 0.2, 1.0])
    R = np.array([0.2, -0.5, -0.3, 0.4, 0.3])
    a, _ = oracle.riemann(L, R, gamma=g)
    mL = R * np.array([1, -1, 1, 1, 1])
    mR = L * np.array([1, -1, 1, 1, 1])
    b, _ = oracle.riemann(mL, mR, gamma=g)
    assert b[4] == a[4] and b[1] == -a[1] and b[0] == a[0]


def test_strong_double_rarefaction_bounded():
    # equal states moving apart at 1.5 sound speeds each: p* must stay positive
    g = 1.4
    c = math.sqrt(g)
    out, _ = oracle.riemann([1.0, -1.5 * c, 0, 0, 1.0], [1.0, 1.5 * c, 0, 0, 1.0], gamma=g)
    assert np.all(np.isfinite(out))
    assert out[4] > 0.0 and out[0] > 0.0


def test_exact_solver_two_rarefaction_closed_form():
    # pins the test-only exact solver itself
    g = 1.4
    for (rl, ul, pl, rr, ur, pr) in [(1, -0.5, 1, 1, 0.5, 1), (1, -1, 0.4, 0.5, 0.8, 0.2)]:
        cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
        z = (g - 1) / (2 * g)
        p2r = ((cl + cr - 0.5 * (g - 1) * (ur - ul)) / (cl * pl ** (-z) + cr * pr ** (-z))) ** (1 / z)
        pe, _ = er.star_state(rl, ul, pl, rr, ur, pr, g)
        assert abs(pe - p2r) <= 1e-13 * p2r


# ---------------------------------------------------------------- PPB

NG = 4


def quad_cells(coef, xc, h):
    """(a0, a_s, a_ss) of f(x) = c0 + c1 x + c2 x^2 on cells centred at xc."""
    c0, c1, c2 = coef
    f = c0 + c1 * xc + c2 * xc * xc
    fp = c1 + 2 * c2 * xc
    a2 = c2 * h * h + 0.0 * xc
    return f + a2 / 12.0, fp * h, a2


@pytest.mark.parametrize("sigma", [0.37, -0.61, 1.0, -1.0, 0.0, 1e-3])
def test_ppb_translates_global_quadratic_exactly(sigma):
    n, h = 16, 1.0 / 16
    xc = (np.arange(-NG, n + NG) + 0.5) * h
    q = (0.5, 0.2, -0.3)            # stays inside [0, 1] on the pencil
    lin1 = (0.05, 0.1)              # transverse slope b(x) = 0.05 + 0.1 x
    lin2 = (-0.02, 0.03)
    coef = np.zeros((10, n + 2 * NG))
    coef[0], coef[1], coef[2] = quad_cells(q, xc, h)
    coef[3] = lin1[0] + lin1[1] * xc
    coef[4] = lin1[1] * h
    coef[5] = lin2[0] + lin2[1] * xc
    coef[6] = lin2[1] * h
    coef[7], coef[8], coef[9] = 0.01, -0.02, 0.03
    sig = np.full(n + 2 * NG, sigma)
    out, hits = oracle.ppb_pencil(coef, sig)
    assert hits == 0
    # translated by sigma cells: f(x - sigma h)
    sh = sigma * h
    q2 = (q[0] - q[1] * sh + q[2] * sh * sh, q[1] - 2 * q[2] * sh, q[2])
    e0, e1, e2 = quad_cells(q2, xc, h)
    I = slice(NG, NG + n)
    assert np.max(np.abs(out[0, I] - e0[I])) <= 1e-14
    assert np.max(np.abs(out[1, I] - e1[I])) <= 1e-13
    assert np.max(np.abs(out[2, I] - e2[I])) <= 1e-12
    assert np.max(np.abs(out[3, I] - (lin1[0] + lin1[1] * (xc[I] - sh)))) <= 1e-14
    assert np.max(np.abs(out[4, I] - lin1[1] * h)) <= 1e-13
    assert np.max(np.abs(out[5, I] - (lin2[0] + lin2[1] * (xc[I] - sh)))) <= 1e-14
    assert np.max(np.abs(out[7:, I] - coef[7:, I])) <= 1e-15


def test_ppb_unit_shift_is_exact():
    rng = np.random.default_rng(3)
    n = 12
    coef = np.zeros((10, n + 2 * NG))
    coef[0] = rng.uniform(0.2, 0.8, size=n + 2 * NG)
    coef[1] = rng.uniform(-0.1, 0.1, size=n + 2 * NG)
    coef[2] = rng.uniform(-0.1, 0.1, size=n + 2 * NG)
    coef[3:] = rng.uniform(-0.1, 0.1, size=(7, n + 2 * NG))
    out, _ = oracle.ppb_pencil(coef, np.ones(n + 2 * NG))
    I = slice(NG, NG + n)
    Im = slice(NG - 1, NG + n - 1)
    # the P2 coefficient carries the 180x basis normalisation of its round-off
    assert np.max(np.abs(out[:, I] - coef[:, Im])) <= 1e-13


def _piecewise_moments(coef, sig, j):
    """Moments of cell j after the pass by direct integration: the new cell
    [-1/2, 1/2] (relative to x_j) is split where the Lagrangian images of the
    donors j-1, j, j+1 meet, and each piece is integrated with a 6-point
    Gauss rule (exact for the polynomial degrees involved)."""
    g, w = np.polynomial.legendre.leggauss(6)
    J = j + NG
    acc = np.zeros(6)
    for D in (J - 1, J, J + 1):
        off = D - J
        lo = off - 0.5 + sig[D - 1]
        hi = off + 0.5 + sig[D]
        a, b = max(lo, -0.5), min(hi, 0.5)
        if b <= a:
            continue
        x = 0.5 * (a + b) + 0.5 * (b - a) * g
        wt = 0.5 * (b - a) * w
        s = (x - lo) / (hi - lo) - 0.5
        A = coef[0, D] + coef[1, D] * s + coef[2, D] * (s * s - 1 / 12)
        B = coef[3, D] + coef[4, D] * s
        acc += np.array([np.sum(wt * A), 12 * np.sum(wt * A * x),
                         180 * np.sum(wt * A * (x * x - 1 / 12)),
                         np.sum(wt * B), 12 * np.sum(wt * B * x), np.sum(wt) * coef[7, D]])
    return acc


def test_ppb_divergent_flow_matches_quadrature():
    # random face Courant numbers (compressing and expanding cells); the new
    # moments equal brute-force integrals of the stretched donor profiles
    rng = np.random.default_rng(7)
    n = 10
    coef = np.zeros((10, n + 2 * NG))
    coef[0] = rng.uniform(0.3, 0.7, size=n + 2 * NG)
    coef[1] = rng.uniform(-0.2, 0.2, size=n + 2 * NG)
    coef[2] = rng.uniform(-0.1, 0.1, size=n + 2 * NG)
    coef[3:] = rng.uniform(-0.1, 0.1, size=(7, n + 2 * NG))
    sig = rng.uniform(-0.4, 0.4, size=n + 2 * NG)
    out, hits = oracle.ppb_pencil(coef, sig)
    assert hits == 0
    for j in range(n):
        ref = _piecewise_moments(coef, sig, j)
        got = np.array([out[0, j + NG], out[1, j + NG], out[2, j + NG], out[3, j + NG],
                        out[4, j + NG], out[7, j + NG]])
        assert np.max(np.abs(got - ref)) <= 1e-13, (j, got, ref)


def test_ppb_uniform_fraction_stays_uniform_in_divergent_flow():
    # fv is carried with the material: a uniform fraction stays uniform
    rng = np.random.default_rng(11)
    n = 20
    coef = np.zeros((10, n + 2 * NG))
    coef[0] = 0.37
    sig = rng.uniform(-0.45, 0.45, size=n + 2 * NG)
    out, _ = oracle.ppb_pencil(coef, sig)
    I = slice(NG, NG + n)
    assert np.max(np.abs(out[0, I] - 0.37)) <= 1e-15
    assert np.max(np.abs(out[1:, I])) <= 1e-14


def test_ppb_bounds_on_sharp_data():
    # fv stays in [0, 1] for 0/1 data with steep sub-cell structure
    rng = np.random.default_rng(5)
    n = 64
    for _ in range(20):
        coef = np.zeros((10, n + 2 * NG))
        coef[0] = rng.integers(0, 2, size=n + 2 * NG).astype(float)
        coef[1] = rng.uniform(-3, 3, size=n + 2 * NG) * (coef[0] * (1 - coef[0]) + 0.2)
        coef[2] = rng.uniform(-3, 3, size=n + 2 * NG) * 0.3
        # adjacent faces may converge by less than one cell width per pass
        # (Lagrangian lengths 1 + sigma_R - sigma_L stay positive)
        sig = rng.uniform(-0.45, 0.45, size=n + 2 * NG)
        out, hits = oracle.ppb_pencil(coef, sig)
        I = slice(NG, NG + n)
        assert np.min(out[0, I]) >= -1e-14
        assert np.max(out[0, I]) <= 1 + 1e-14

"""Pins of the spin-up increment and of the spherical-shell averages in the
oracle (Sec. 1: averages on spherical surfaces; Sec. 3: a solid-body
rotation added gradually, the star inside an inscribed confining sphere).
The expected values come from library routines (numpy's cross product),
closed forms (the volume and the moment of inertia of the unit ball),
exact invariants of rigid rotation and of radial flow, a second oracle
reduction that shares no code with the shell sums (the totals), and brute
force on a three-cell grid."""
import math

import numpy as np

import oracle
from paper_1810_13416_amd import problems as pr


def _ball_oracle(n=24, **kw):
    prob = pr.ball(n, **kw)
    O = oracle.Oracle(prob.params, threads=4)
    O.set_state(prob.state)
    z, y, x = np.meshgrid(*(pr._centres(prob.params, a) for a in (2, 1, 0)), indexing="ij")
    fluid = (x * x + y * y) + z * z < 1.0
    return prob, O, (x, y, z), fluid


def test_spin_add_is_the_rigid_rotation_velocity():
    prob, O, (x, y, z), fluid = _ball_oracle(24)
    om = 0.37
    O.spin_add(om)
    st = O.get_state()
    pos = np.stack([x, y, z], axis=-1)
    want = np.cross(np.array([0.0, 0.0, om]), pos)          # Omega z-hat x r
    for d in range(3):
        got = st[1 + d]
        assert np.allclose(got[fluid], want[..., d][fluid], rtol=0, atol=1e-15)
        assert np.all(got[~fluid] == 0.0)
    # density and pressure perturbation unchanged, fv untouched
    assert np.array_equal(st[0], prob.state[0])
    assert np.allclose(st[4][fluid], 0.7, rtol=1e-14, atol=0)
    assert np.array_equal(st[5], prob.state[5])
    # energy grows by the kinetic energy of the rotation
    E = O.get_conserved()[4]
    ke = 0.5 * 1.3 * om * om * (x * x + y * y)
    assert np.allclose(E[fluid], (0.7 / (5.0 / 3.0 - 1.0) + ke)[fluid], rtol=1e-14, atol=0)
    O.close()


def test_spin_increments_add_and_give_the_ball_moment_of_inertia():
    n = 32
    prob, O, (x, y, z), fluid = _ball_oracle(n)
    O2 = oracle.Oracle(prob.params, threads=4)
    O2.set_state(prob.state)
    om = 0.5
    O.spin_add(om)
    O2.spin_add(0.5 * om)
    O2.spin_add(0.5 * om)
    a, b = O.get_conserved(), O2.get_conserved()
    for q in range(15):
        assert np.allclose(a[q], b[q], rtol=1e-14, atol=1e-15)
    # angular momentum about z: rho Omega sum (x^2 + y^2) dV -> (8 pi / 15) rho Omega R^5
    dv = prob.params.dx ** 3
    lz = np.sum((x * a[2] - y * a[1])[fluid]) * dv
    assert abs(lz / (8 * math.pi / 15 * 1.3 * om) - 1.0) < 0.03
    O.close()
    O2.close()


def test_spin_ramp_schedule():
    # time steps so short that the passes leave the state as it was (to
    # O(dt)): the ramp adds omega / nramp after each of the first nramp
    # steps and nothing after
    prob, O, (x, y, z), fluid = _ball_oracle(16)
    om, nramp = 0.3, 3
    O.set_spinup(om, nramp)
    for k in range(5):
        O.step(1e-12)
        st = O.get_state()
        frac = min(k + 1, nramp) / nramp
        assert np.allclose(st[1][fluid], (-om * frac * y)[fluid], rtol=0, atol=1e-9)
        assert np.allclose(st[2][fluid], (om * frac * x)[fluid], rtol=0, atol=1e-9)
    O.close()


def test_shell_profile_volume_mass_and_fv_of_a_uniform_ball():
    n = 32
    prob, O, (x, y, z), fluid = _ball_oracle(n, rho=1.3, fv=0.4)
    dx = prob.params.dx
    nb = 24
    dr = 1.0 / nb
    prof = O.shell_profile(nb, dr)
    vol, mass, fvv, f2 = prof[:, 0], prof[:, 1], prof[:, 2], prof[:, 7]
    # every fluid cell falls in exactly one shell
    assert abs(vol.sum() - fluid.sum() * dx ** 3) < 1e-12
    # ball volume, and shells of width 6 dr against 4 pi r^2 dr integrated
    assert abs(vol.sum() / (4.0 / 3.0 * math.pi) - 1.0) < 0.02
    for a in range(6, nb, 6):
        want = 4.0 / 3.0 * math.pi * ((a + 6) ** 3 - a ** 3) * dr ** 3
        assert abs(vol[a:a + 6].sum() / want - 1.0) < 0.05
    # uniform fields: shell sums are the value times the volume
    assert np.allclose(mass, 1.3 * vol, rtol=1e-13, atol=0)
    assert np.allclose(fvv, 0.4 * vol, rtol=1e-13, atol=0)
    assert np.allclose(f2, 0.16 * vol, rtol=1e-13, atol=0)
    assert np.all(prof[:, 3:7] == 0.0)
    # the total mass of a second, independent reduction
    assert abs(mass.sum() / O.totals()[0] - 1.0) < 1e-13
    O.close()


def test_shell_profile_rigid_rotation_invariants():
    prob, O, (x, y, z), fluid = _ball_oracle(24)
    om = 0.8
    O.spin_add(om)
    prof = O.shell_profile(12, 1.0 / 12)
    # rigid rotation is tangential: no radial flux; rho |u|^2 = Omega * rho (x v - y u)
    assert np.all(np.abs(prof[:, 3]) < 1e-15)
    assert np.all(np.abs(prof[:, 4]) < 1e-15)
    assert np.allclose(prof[:, 5], om * prof[:, 6], rtol=1e-13, atol=0)
    # angular momentum of the ball, summed over shells
    lz = prof[:, 6].sum()
    assert abs(lz / (8 * math.pi / 15 * 1.3 * om) - 1.0) < 0.03
    O.close()


def test_shell_profile_radial_flow():
    prob = pr.ball(20)
    z, y, x = np.meshgrid(*(pr._centres(prob.params, a) for a in (2, 1, 0)), indexing="ij")
    r = np.sqrt((x * x + y * y) + z * z)
    fluid = r < 1.0
    U = 0.05
    st = [a.copy() for a in prob.state]
    for d, c in enumerate((x, y, z)):
        st[1 + d] = np.where(fluid, U * c / r, 0.0)
    O = oracle.Oracle(prob.params, threads=4)
    O.set_state(st)
    prof = O.shell_profile(10, 0.1)
    vol = prof[:, 0]
    assert np.allclose(prof[:, 3], 1.3 * U * vol, rtol=1e-13, atol=0)
    assert np.allclose(prof[:, 4], 1.3 * U * U * vol, rtol=1e-13, atol=0)
    assert np.allclose(prof[:, 5], 1.3 * U * U * vol, rtol=1e-13, atol=0)
    assert np.all(np.abs(prof[:, 6]) < 1e-17)
    O.close()


def test_shell_membership_at_exact_radii():
    # three cells with centres at x = 0, 1, 2 (y = z = 0): radii 0, 1, 2
    P = pr.GridParams(n=(3, 1, 1), dx=1.0, origin=(-0.5, -0.5, -0.5))
    st = [np.full(P.shape, 1.0), np.zeros(P.shape), np.zeros(P.shape), np.zeros(P.shape),
          np.full(P.shape, 1.0)] + [np.zeros(P.shape) for _ in range(10)]
    st[1][0, 0, :] = [0.3, 0.2, 0.1]
    O = oracle.Oracle(P, threads=1)
    O.set_state(st)
    prof = O.shell_profile(3, 1.0)
    # a radius on a shell boundary belongs to the outer shell
    assert np.array_equal(prof[:, 0], [1.0, 1.0, 1.0])
    # the cell at the origin has no radial direction: u_r = 0
    assert np.array_equal(prof[:, 3], [0.0, 0.2, 0.1])
    # radius 2 is the outer edge of 2 shells of width 1: excluded
    prof2 = O.shell_profile(2, 1.0)
    assert np.array_equal(prof2[:, 0], [1.0, 1.0])
    O.close()


# ---------------------------------------------------------------------
# Rotating frame (Coriolis and centrifugal source terms)
# ---------------------------------------------------------------------

def test_inertial_oscillation_turns_velocity_at_twice_omega():
    # a uniform flow in a periodic box feels only the Coriolis term (the
    # passes keep a uniform state exactly): du/dt = 2 omega (v, -u), so the
    # horizontal velocity turns clockwise at the rate 2 omega, keeping its
    # length, while u_z, the density, the pressure and the total energy stay
    om, u0 = 0.8, np.array([0.3, -0.2, 0.1])
    prob = pr.uniform(n=(8, 8, 8), rho=1.2, vel=tuple(u0), p=0.9)
    O = oracle.Oracle(prob.params, threads=2)
    O.set_state(prob.state)
    O.set_rotating_frame(om, centrifugal=False)
    e0 = O.totals()[4]
    dt, nsteps = 0.01, 37
    for _ in range(nsteps):
        O.step(dt)
    st = O.get_state()
    th = -2.0 * om * dt * nsteps
    want = (math.cos(th) * u0[0] - math.sin(th) * u0[1], math.sin(th) * u0[0] + math.cos(th) * u0[1])
    assert np.allclose(st[1], want[0], rtol=0, atol=1e-13)
    assert np.allclose(st[2], want[1], rtol=0, atol=1e-13)
    assert np.allclose(st[3], u0[2], rtol=0, atol=1e-15)
    assert np.allclose(st[0], 1.2, rtol=1e-15, atol=0) and np.allclose(st[4], 0.9, rtol=1e-13, atol=0)
    assert abs(O.totals()[4] - e0) <= 1e-13 * e0
    # half a period of the oscillation, pi / (2 omega): the flow reversed
    O2 = oracle.Oracle(prob.params, threads=2)
    O2.set_state(prob.state)
    O2.set_rotating_frame(om, centrifugal=False)
    for _ in range(40):
        O2.step(math.pi / (2.0 * om) / 40)
    st = O2.get_state()
    assert np.allclose(st[1], -u0[0], atol=1e-13) and np.allclose(st[2], -u0[1], atol=1e-13)
    O.close()
    O2.close()


def _rigid_rotation_deviation(n, om=0.5, T=0.2, centrifugal=True):
    """Gas at rest in the inertial frame, seen from axes turning at omega:
    a rigid rotation u = -omega z-hat x x = omega (y, -x, 0) of a uniform gas
    in the sphere.  In the rotating frame its advection (centripetal
    -omega^2 r) is balanced exactly by the Coriolis (-2 omega^2 r) and
    centrifugal (+omega^2 r) terms, so it is steady.  Returns the largest
    velocity change over time T inside r < 0.6 (away from the staircase
    wall, whose disturbance has not arrived there yet)."""
    prob = pr.ball(n, rho=1.0, p=1.0, fv=0.0)
    z, y, x = np.meshgrid(*(pr._centres(prob.params, a) for a in (2, 1, 0)), indexing="ij")
    fluid = (x * x + y * y) + z * z < 1.0
    st = list(prob.state)
    st[1] = np.where(fluid, om * y, 0.0)
    st[2] = np.where(fluid, -om * x, 0.0)
    O = oracle.Oracle(prob.params, threads=8)
    O.set_state(st)
    O.set_rotating_frame(om, centrifugal)
    t = 0.0
    while t < T - 1e-12:
        dt = min(O.dt(0.8), T - t)
        O.step(dt)
        t += dt
    g = O.get_state()
    O.close()
    inner = (x * x + y * y) + z * z < 0.36
    return max(float(np.max(np.abs(g[1] - st[1])[inner])), float(np.max(np.abs(g[2] - st[2])[inner])))


def test_rotating_frame_keeps_the_inertial_rest_state_steady():
    # a missing or misweighted source term leaves an acceleration of order
    # omega^2 r, a velocity change ~ 0.03 by T = 0.2 at r = 0.6 on every grid
    e32, e64 = _rigid_rotation_deviation(32), _rigid_rotation_deviation(64)
    print("rigid rotation in the rotating frame, max |du| inside r < 0.6:", e32, e64)
    assert e64 <= 1e-4
    assert e32 / e64 >= 8.0          # the deviation is truncation error
    # the same flow with the centrifugal term left out is not steady
    assert _rigid_rotation_deviation(32, centrifugal=False) >= 0.02

"""Planted mistakes: each case builds a copy of the oracle with one plausible
error (a flipped sign, a dropped term, the wrong wave's domain of
dependence), then runs the pins named beside it against that copy and
requires them to fail.  A control case builds the unaltered source the same
way and requires the same pins to pass.  This shows that the oracle's pins,
not its parity with the GPU path (which implements the same reading), are
what fixes each of these terms.

Every edit names an exact fragment of the oracle source and how many times
it occurs there, so an edit of the oracle that moves the fragment fails the
case loudly instead of planting nothing.
"""
import os
import subprocess
import sys

import pytest

import oracle

SRC = oracle._SRC
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SOURCES = "test_oracle_sources.py"
PHYSICS = "test_oracle_physics.py"
FLATTEN = "test_oracle_flatten.py"
ROTATION = "test_oracle_rotation.py"

# (name, [(fragment, replacement, occurrences)], pins that must fail)
MUTATIONS = [
    ("control", [], [f"{SOURCES}::test_free_fall_closed_form",
                     f"{SOURCES}::test_heating_layer_total_energy_closed_form",
                     f"{SOURCES}::test_moving_hydrostatic_column_converges",
                     f"{SOURCES}::test_transverse_shear_order",
                     f"{SOURCES}::test_acoustic_simple_wave_order",
                     f"{PHYSICS}::test_hydrostatic_base_is_exactly_static",
                     f"{PHYSICS}::test_convergence_order_1d",
                     f"{FLATTEN}::test_convergence_margin_ignores_rounding_and_keeps_real_compression",
                     f"{ROTATION}::test_inertial_oscillation_turns_velocity_at_twice_omega",
                     f"{ROTATION}::test_rotating_frame_keeps_the_inertial_rest_state_steady"]),
    ("momentum_gravity_sign",
     [("+ dt * pc->g[J] * (0.5 * (pc->rhop[J] + rn))", "- dt * pc->g[J] * (0.5 * (pc->rhop[J] + rn))", 1)],
     [f"{SOURCES}::test_free_fall_closed_form"]),
    ("energy_gravity_work_sign",
     [("+ dt * pc->g[J] * (0.5 * (Fl[0] + Fr[0]))", "- dt * pc->g[J] * (0.5 * (Fl[0] + Fr[0]))", 1)],
     [f"{SOURCES}::test_free_fall_closed_form"]),
    ("energy_gravity_work_dropped",
     [("+ dt * pc->g[J] * (0.5 * (Fl[0] + Fr[0]))", "+ 0.0 * (Fl[0] + Fr[0])", 1)],
     [f"{SOURCES}::test_free_fall_closed_form"]),
    ("half_step_gravity_sign",
     [("pc->TL[J][1] += su; pc->TR[J][1] += su;", "pc->TL[J][1] -= su; pc->TR[J][1] -= su;", 1)],
     [f"{SOURCES}::test_free_fall_closed_form"]),
    ("half_step_gravity_dropped",
     [("pc->TL[J][1] += su; pc->TR[J][1] += su;", "(void)su;", 1)],
     [f"{SOURCES}::test_free_fall_closed_form"]),
    ("base_advection_rho_sign",
     [("pc->TL[J][0] -= sr; pc->TR[J][0] -= sr;", "pc->TL[J][0] += sr; pc->TR[J][0] += sr;", 1)],
     [f"{SOURCES}::test_moving_hydrostatic_column_converges"]),
    ("base_advection_rho_dropped",
     [("pc->TL[J][0] -= sr; pc->TR[J][0] -= sr;", "(void)sr;", 1)],
     [f"{SOURCES}::test_moving_hydrostatic_column_converges"]),
    ("base_advection_p_sign",
     [("pc->TL[J][4] -= sp; pc->TR[J][4] -= sp;", "pc->TL[J][4] += sp; pc->TR[J][4] += sp;", 1)],
     [f"{SOURCES}::test_moving_hydrostatic_column_converges"]),
    ("base_advection_p_dropped",
     [("pc->TL[J][4] -= sp; pc->TR[J][4] -= sp;", "(void)sp;", 1)],
     [f"{SOURCES}::test_moving_hydrostatic_column_converges"]),
    ("heating_doubled",
     [("+= heating_at(P, x) * dt;", "+= 2.0 * heating_at(P, x) * dt;", 1)],
     [f"{SOURCES}::test_heating_layer_total_energy_closed_form"]),
    ("transverse_over_fast_wave_domain",
     [("double yv = fmax(lam[1], 0.0) * nu;", "double yv = fmax(lam[2], 0.0) * nu;", 1),
      ("double yv = fmax(-lam[1], 0.0) * nu;", "double yv = fmax(-lam[0], 0.0) * nu;", 1)],
     [f"{SOURCES}::test_transverse_shear_order"]),
    ("supersonic_projection_dropped",
     [("if (lam[0] > 0.0) {", "if (0) {", 1), ("if (lam[2] < 0.0) {", "if (0) {", 1)],
     [f"{SOURCES}::test_acoustic_simple_wave_order"]),
    ("supersonic_projection_sign",
     [("bm = dp / (2.0 * c2) - (rj / (2.0 * cj)) * du;", "bm = -(dp / (2.0 * c2) - (rj / (2.0 * cj)) * du);", 1),
      ("bp = dp / (2.0 * c2) + (rj / (2.0 * cj)) * du;", "bp = -(dp / (2.0 * c2) + (rj / (2.0 * cj)) * du);", 1)],
     [f"{SOURCES}::test_acoustic_simple_wave_order"]),
    ("acoustic_velocity_projection_sign",
     [("pc->TL[J][1] = ref[1] + bm * (cj / rj);", "pc->TL[J][1] = ref[1] - bm * (cj / rj);", 1),
      ("pc->TR[J][1] = ref[1] - bp * (cj / rj);", "pc->TR[J][1] = ref[1] + bp * (cj / rj);", 1)],
     [f"{SOURCES}::test_acoustic_simple_wave_order"]),
    ("entropy_projection_pressure_term_sign",
     [("b0 = dr - dp / c2;", "b0 = dr + dp / c2;", 2)],
     [f"{SOURCES}::test_acoustic_simple_wave_order"]),
    ("entropy_projection_sign",
     [("b0 = dr - dp / c2;", "b0 = -(dr - dp / c2);", 2)],
     [f"{PHYSICS}::test_convergence_order_1d"]),
    ("energy_flux_base_enthalpy_dropped",
     [("gamma / gm1 * (p0f[J] + f[4])", "gamma / gm1 * f[4]", 1)],
     [f"{SOURCES}::test_moving_hydrostatic_column_converges"]),
    ("flattening_convergence_test_strict",
     [("u[o + 2] - u[o + 4] > FLAT_TIE * (fabs(u[o + 2]) + fabs(u[o + 4]))", "u[o + 2] - u[o + 4] > 0.0", 1)],
     [f"{FLATTEN}::test_convergence_margin_ignores_rounding_and_keeps_real_compression"]),
    ("flattening_convergence_margin_too_wide",
     [("u[o + 2] - u[o + 4] > FLAT_TIE * (fabs(u[o + 2]) + fabs(u[o + 4]))",
       "u[o + 2] - u[o + 4] > 1e-6 * (fabs(u[o + 2]) + fabs(u[o + 4]))", 1)],
     [f"{FLATTEN}::test_convergence_margin_ignores_rounding_and_keeps_real_compression"]),
    ("coriolis_rate_omega_not_twice",
     [("const double th = -2.0 * om * dt", "const double th = -1.0 * om * dt", 1)],
     [f"{ROTATION}::test_inertial_oscillation_turns_velocity_at_twice_omega"]),
    ("coriolis_sense_reversed",
     [("const double th = -2.0 * om * dt", "const double th = 2.0 * om * dt", 1)],
     [f"{ROTATION}::test_inertial_oscillation_turns_velocity_at_twice_omega"]),
    ("coriolis_as_a_kick_not_a_rotation",
     [("double ur = cth * u - sth * v, vr = sth * u + cth * v;",
       "double ur = u - sth * v, vr = sth * u + v;", 1)],
     [f"{ROTATION}::test_inertial_oscillation_turns_velocity_at_twice_omega"]),
    ("centrifugal_sign",
     [("kick = S->rot_centrifugal ? 0.5 * om * om * dt", "kick = S->rot_centrifugal ? -0.5 * om * om * dt", 1)],
     [f"{ROTATION}::test_rotating_frame_keeps_the_inertial_rest_state_steady"]),
    ("centrifugal_half_dropped",
     [("u = ur + kick * x[0];", "u = ur;", 1), ("v = vr + kick * x[1];", "v = vr;", 1)],
     [f"{ROTATION}::test_rotating_frame_keeps_the_inertial_rest_state_steady"]),
    ("mass_flux_base_density_dropped",
     [("double rf = r0f[J] + f[0];", "double rf = f[0];", 1)],
     [f"{SOURCES}::test_moving_hydrostatic_column_converges"]),
]


def build_mutant(edits, outdir):
    """Compile the oracle source with `edits` applied into outdir; returns
    the library path."""
    src = open(SRC).read()
    for frag, repl, count in edits:
        found = src.count(frag)
        if found != count:
            raise AssertionError(f"fragment {frag!r} occurs {found} times, expected {count}")
        src = src.replace(frag, repl)
    c = os.path.join(outdir, "mutant.c")
    lib = os.path.join(outdir, "libmutant.so")
    with open(c, "w") as f:
        f.write(src)
    cmd = [lib if a == oracle._LIB else (c if a == SRC else a) for a in oracle.BUILD_CMD]
    subprocess.check_call(cmd)
    return lib


@pytest.mark.parametrize("name,edits,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(name, edits, pins, tmp_path):
    lib = build_mutant(edits, str(tmp_path))
    env = dict(os.environ, PPMB_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *[os.path.join(HERE, p) for p in pins]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-1500:]
    if name == "control":
        assert r.returncode == 0, tail
    else:
        # exit status 1: tests ran and at least one failed (not a collection
        # or usage error)
        assert r.returncode == 1, tail
        assert " failed" in r.stdout, tail

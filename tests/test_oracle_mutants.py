"""The structure-update pins reject plausible mistakes.  Each case compiles a copy of the oracle
with one planted mistake (a dropped factor, a swapped operand, a wrong sign or weight) and
checks that the pins of tests/test_oracle_structure.py named for it fail on that copy.  CPU only;
the oracle itself is untouched."""
import importlib.util
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _pins():
    spec = importlib.util.spec_from_file_location("structure_pins", os.path.join(HERE, "test_oracle_structure.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


# name: (replacements in lbib_oracle.c, pins that must fail)
MUTANTS = {
    # Eq. verletPos: the 1/2 of the acceleration term dropped
    "verlet_half_dropped": (
        [("double xt = b->x[i] + u0[i] + 0.5 * acc;", "double xt = b->x[i] + u0[i] + acc;")],
        ["membrane_displacement", "membrane_printed"]),
    # printed update: the second pass of Eq. verletPos without its acceleration term
    "printed_second_pass_without_acc": (
        [("xn = b->x[i] + un + 0.5 * acc;", "xn = b->x[i] + un;")],
        ["membrane_printed"]),
    # Eq. linearVelRig: wrong weight on the acceleration
    "bdf2_force_weight": (
        [("- 0.5 * b->ur1[a] + F[a] / b->mass);", "- 0.5 * b->ur1[a] + 1.5 * F[a] / b->mass);")],
        ["constant_force", "settling"]),
    # Eq. linearVelRig: the overall 2/3 dropped
    "bdf2_two_thirds_dropped": (
        [("un[a] = 2.0 / 3.0 * (2.0 * b->ur[a]", "un[a] = 1.0 * (2.0 * b->ur[a]")],
        ["constant_force", "settling"]),
    # weight without buoyancy
    "buoyancy_dropped": (
        [("(b->mass - b->V0) * b->d.gravity[a]", "b->mass * b->d.gravity[a]")],
        ["settling"]),
    # Eq. angularVelRig: wrong weight on the angular acceleration
    "bdf2_torque_weight": (
        [("- 0.5 * b->om1[a] + wd[a]);", "- 0.5 * b->om1[a] + 2.0 * wd[a]);")],
        ["torque"]),
    # inertia turned as R^T I R instead of R I R^T
    "inertia_transposed": (
        [("mat3_mul(b->R, b->Ib, tmp);\n    mat3_mul(tmp, Rt, Iw);",
          "mat3_mul(Rt, b->Ib, tmp);\n    mat3_mul(tmp, b->R, Iw);")],
        ["torque"]),
    # Rodrigues rotation with the wrong sense
    "rotation_sign": (
        [("Rm[i] += sin(th) * K[i] + (1.0 - cos(th)) * K2[i];",
          "Rm[i] += -sin(th) * K[i] + (1.0 - cos(th)) * K2[i];")],
        ["spin"]),
    # the increment applied in the body frame instead of the world frame
    "rotation_order": (
        [("mat3_mul(Rw, b->R, Rn);", "mat3_mul(b->R, Rw, Rn);")],
        ["torque"]),
    # centre moved with the previous velocity
    "centre_lags": (
        [("for (int a = 0; a < 3; ++a) b->X[a] += un[a];", "for (int a = 0; a < 3; ++a) b->X[a] += b->ur1[a];")],
        ["constant_force", "settling"]),
    # rigid desired velocity r x omega instead of omega x r
    "marker_velocity_cross_swapped": (
        [("for (int a = 0; a < 3; ++a) r[a] = cen[a] - b->X[a];\n                cross(b->om, r, w);",
          "for (int a = 0; a < 3; ++a) r[a] = cen[a] - b->X[a];\n                cross(r, b->om, w);")],
        ["marker_velocity"]),
}


def _run_pin(P, orc, name):
    {
        "constant_force": lambda: P.pin_constant_force(orc),
        "settling": lambda: P.pin_settling_first_step(orc),
        "spin": lambda: P.pin_spin_pose(orc),
        "torque": lambda: P.pin_torque_in_turned_pose(orc),
        "marker_velocity": lambda: P.pin_rigid_boundary_velocity(orc),
        "membrane_displacement": lambda: P.pin_membrane_first_step(orc, 0),
        "membrane_printed": lambda: P.pin_membrane_first_step(orc, 1),
    }[name]()


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_reject_planted_mistake(orc, tmp_path, mutant):
    P = _pins()
    repl, must_fail = MUTANTS[mutant]
    so = orc.build_variant(repl, str(tmp_path), name=mutant)
    with orc.use_library(so):
        for pin in must_fail:
            with pytest.raises(AssertionError):
                _run_pin(P, orc, pin)


def test_pins_pass_on_unplanted_copy(orc, tmp_path):
    """The same machinery with no replacement passes every pin, so the failures above come
    from the planted mistakes."""
    P = _pins()
    so = orc.build_variant([], str(tmp_path), name="unplanted")
    with orc.use_library(so):
        for pin in ("constant_force", "settling", "spin", "torque", "marker_velocity",
                    "membrane_displacement", "membrane_printed"):
            _run_pin(P, orc, pin)

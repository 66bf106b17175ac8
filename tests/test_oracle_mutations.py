"""Plants plausible mistakes in copies of the oracle's C source (on the CPU)
and checks that the pins of tests/test_oracle_pins.py catch every one.

Each mutant is the oracle with one textual change (a dropped term, a wrong
sign, power, coefficient or index); it is compiled with the oracle's own
flags into a temporary library, swapped in, and the pins are run until one
fails.  A mutant that survives all pins means the pins are too weak.
"""
import ctypes
import os

import pytest

from oracle import oracle as O
from tests import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "hermite_oracle.c")

# (name, original text, mutated text) -- each original must occur once.
MUTANTS = [
    ("jerk: drop the 3", "const double c3 = 3.0 * rv / s;", "const double c3 = rv / s;"),
    ("jerk: wrong sign of radial term", "mq3 * (wx - c3 * rx)", "mq3 * (wx + c3 * rx)"),
    ("jerk: drop v_ij", "mq3 * (wy - c3 * ry)", "mq3 * (- c3 * ry)"),
    ("r_ij transposed", "const double rx = x[j] - x[i];", "const double rx = x[i] - x[j];"),
    ("v_ij transposed", "const double wz = vz[j] - vz[i];", "const double wz = vz[i] - vz[j];"),
    ("1/s^{3/2} -> 1/s", "m[j] * (q * q * q)", "m[j] * (q * q)"),
    ("softening dropped", "rz * rz + eps2;", "rz * rz;"),
    ("softening doubled", "rz * rz + eps2;", "rz * rz + 2.0 * eps2;"),
    ("potential sign", "const double tph = -(m[j] * q);", "const double tph = (m[j] * q);"),
    ("potential uses m_i", "const double tph = -(m[j] * q);", "const double tph = -(m[i] * q);"),
    ("self term kept", "if (j == i) continue;", "if (j == i && eps2 == 0.0) continue;"),
    ("predictor a/2 -> a/3", "acc[o] / 2.0 * (dt * dt)", "acc[o] / 3.0 * (dt * dt)"),
    ("predictor j/6 -> j/2", "jrk[o] / 6.0 * (dt * dt * dt)", "jrk[o] / 2.0 * (dt * dt * dt)"),
    ("predictor v term dropped", "vel[o] + acc[o] * dt + jrk[o] / 2.0 * (dt * dt);",
     "vel[o] + acc[o] * dt;"),
    ("snap coefficient 3 -> 2", "2.0 * (-3.0 * (a0 - a1)", "2.0 * (-2.0 * (a0 - a1)"),
    ("crackle j0 + j1 -> j0 - j1", "6.0 * (2.0 * (a0 - a1) + (j0 + j1) * h)",
     "6.0 * (2.0 * (a0 - a1) + (j0 - j1) * h)"),
    ("corrector s/24 -> s/12", "s0 / 24.0 * (h * h * h * h)", "s0 / 12.0 * (h * h * h * h)"),
    ("corrector c/120 -> c/24", "c0 / 120.0 * (h * h * h * h * h)", "c0 / 24.0 * (h * h * h * h * h)"),
    ("criterion at t0 (s1 = s0)", "s1[d] = s0 + c0 * h;", "s1[d] = s0;"),
    ("Aarseth |j|^2 -> |j|", "(A * S + J * J)", "(A * S + J)"),
    ("quantise one level too coarse", "k = 1 - e;", "k = -e;"),
    ("growth limit dropped", "if (k_old >= 0 && k < k_old - 1) k = k_old - 1;", ""),
    ("commensurability dropped", "while (k < k_max && (T & ((((int64_t)1) << (tick_bits - k)) - 1)) != 0)",
     "while (0)"),
    ("explicit start-up factor ignored", "eta_init > 0.0 ? eta_init : eta_f;", "eta_f;"),
    ("start-up uses eta for form 1", "form == 0 ? eta : sqrt(eta);\n    const double eta_s",
     "eta;\n    const double eta_s"),
    ("start-up uses |j|/|a|", "const double crit = eta_s * A / J;", "const double crit = eta_s * J / A;"),
    ("select picks t_i = T", "if (t[i] + dt[i] == T) idx[k++]", "if (t[i] == T) idx[k++]"),
    ("energy W without 1/2", "nsum_add(&w, 0.5 * m[i] * phi_scratch[i]);",
     "nsum_add(&w, m[i] * phi_scratch[i]);"),
]

# the pins, as plain calls (parametrised ones with representative arguments)
PINS = [
    P.test_newton_two_body_unsoftened,
    P.test_softened_force_peaks_at_eps_over_sqrt2,
    P.test_acc_is_minus_gradient_of_pot,
    lambda: P.test_jerk_is_time_derivative_of_acc(0.0),
    lambda: P.test_jerk_is_time_derivative_of_acc(0.003),
    P.test_homologous_expansion_jerk_is_minus_2H_acc,
    P.test_rigid_rotation_jerk_is_omega_cross_acc,
    P.test_symmetric_polyhedron,
    P.test_momentum_and_angular_momentum_invariants,
    P.test_self_term_excluded_and_zero_mass,
    P.test_active_subset_and_j_range,
    P.test_predictor_exact_for_cubic_motion,
    P.test_corrector_exact_for_quintic_motion,
    P.test_snap_crackle_from_cubic_acc,
    P.test_aarseth_circular_orbit,
    P.test_aarseth_harmonic_turning_point,
    P.test_quantize_examples,
    P.test_select_definition,
    P.test_energy_matches_pot_sweep,
    P.test_init_dt_examples,
    P.test_startup_transient_below_integration_error,
    lambda: P.test_kepler_orbit_fourth_order(0.5),
]


def test_mutants_are_listed_against_real_text():
    src = open(SRC).read()
    for name, old, _ in MUTANTS:
        assert src.count(old) == 1, name


def test_unmutated_oracle_passes_the_pins():
    for pin in PINS:
        pin()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_every_mutant_is_caught(tmp_path, name, old, new):
    src = open(SRC).read().replace(old, new)
    csrc = tmp_path / "mutant.c"
    csrc.write_text(src)
    lib_path = O.compile_source(str(csrc), str(tmp_path / "libmutant.so"))
    saved = O._lib
    O._lib = O.configure(ctypes.CDLL(lib_path))
    caught = None
    try:
        for pin in PINS:
            try:
                pin()
            except AssertionError:
                caught = getattr(pin, "__name__", "pin")
                break
    finally:
        O._lib = saved
    assert caught is not None, "mutant '%s' survived every pin" % name

"""The oracle's pins have teeth: each test plants one plausible mistake in a
temporary copy of the oracle's C source (never in the oracle itself),
builds it, and runs the pin that should catch it against that build.  The
pin must fail.  Mistakes: a dropped or doubled term, a wrong sign, an
off-by-one window, a wrong constant, a short jump."""
import contextlib
import os
import shutil
import subprocess

import pytest

import oracle as O
import test_oracle_energy as EP
import test_oracle_lfsr as LP
import test_oracle_pins as PP

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "cmc_oracle.c")
HDR = os.path.join(ROOT, "oracle", "cmc_oracle.h")


@contextlib.contextmanager
def planted(tmp_path, old, new):
    """The oracle built with `old` replaced by `new` (exactly one place)."""
    src = open(SRC).read()
    assert src.count(old) == 1, old
    d = tmp_path / "mutant"
    d.mkdir()
    shutil.copy(HDR, d / "cmc_oracle.h")
    (d / "cmc_oracle.c").write_text(src.replace(old, new))
    so = str(d / "liboracle_mutant.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", so,
                    str(d / "cmc_oracle.c"), "-lm"], check=True)
    saved = O.lib()
    O._lib = O.load(so)
    try:
        yield
    finally:
        O._lib = saved


MUTANTS = {
    # potential: M_k without star k (an exclusive prefix)
    "potential_exclusive_prefix": ("    kadd(&M, m[k]);\n    mcum[k] = kval(&M);",
                                   "    mcum[k] = kval(&M);\n    kadd(&M, m[k]);",
                                   lambda: PP.test_potential_brute_force(O, 0)),
    # Q(r) with the centrifugal term's sign flipped
    "q_sign": ("  return 2.0 * E - 2.0 * phi[k] - J2 / (r[k] * r[k]);",
               "  return 2.0 * E - 2.0 * phi[k] + J2 / (r[k] * r[k]);",
               lambda: PP.test_kepler_turning_points_and_time_fraction(O, -0.5, 0.7)),
    # the kick given to the second star with the wrong sign
    "kick_sign": ("      n2[d] = vcm[d] - fa * wn[d];",
                  "      n2[d] = vcm[d] + fa * wn[d];",
                  lambda: PP.test_relax_conservation_and_special_angles(O)),
    # deflection angle twice too large
    "beta_factor": ("  double b = 0.5 * PI * sqrt(dt / tp);",
                    "  double b = PI * sqrt(dt / tp);",
                    lambda: PP.test_dt_rule(O)),
    # Henon velocity unit
    "velocity_unit": ("  const double vscale = sqrt(16.0 / (3.0 * PI));",
                      "  const double vscale = 16.0 / (3.0 * PI);",
                      lambda: PP.test_plummer_energy_and_virial(O)),
    # core density: the window's own edge star counted
    "core_window": ("    for (int64_t k = a + 1; k <= a + 5; ++k) inner += m[k];",
                    "    for (int64_t k = a + 1; k <= a + 6; ++k) inner += m[k];",
                    lambda: PP.test_core_uniform_sphere(O)),
    # energy correction: the whole work instead of its mean over the step
    "correction_half": ("    const double dT = 0.5 * ((phi_new_at_old",
                        "    const double dT = 1.0 * ((phi_new_at_old",
                        EP.test_corrected_steps_conserve_energy),
    # energy correction: the potential's change at the new radius added
    "correction_sign": ("- (phi[q] - phi_old_at_new));",
                        "+ (phi[q] - phi_old_at_new));",
                        EP.test_corrected_steps_conserve_energy),
    # LFSR113: a wrong shift in the third component
    "lfsr_shift": ("static const int lfsr_q[4] = {6, 2, 13, 3};",
                   "static const int lfsr_q[4] = {6, 2, 12, 3};",
                   lambda: LP.test_component_full_period(2, 28)),
    # LFSR113 streams one squaring short (2^79 apart)
    "stream_spacing": ("    for (int t = 0; t < 80; ++t) mat_square(col); /* one stream: 2^80 steps */",
                       "    for (int t = 0; t < 79; ++t) mat_square(col); /* one stream: 2^80 steps */",
                       LP.test_jump_composition_and_streams),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_catches_planted_mistake(tmp_path, name):
    old, new, pin = MUTANTS[name]
    with planted(tmp_path, old, new):
        with pytest.raises(AssertionError):
            pin()


def test_unplanted_build_passes(tmp_path):
    """The same build path without a change passes every pin used above."""
    with planted(tmp_path, "#define PI 3.14159265358979323846",
                 "#define PI 3.14159265358979323846"):
        for _, _, pin in MUTANTS.values():
            pin()

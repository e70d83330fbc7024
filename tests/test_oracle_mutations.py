"""The oracle's pins are sharp enough: every planted mistake in a copy of the oracle fails one.

Each mutant is a textual edit of ``oracle/oracle.c`` (a dropped term, a wrong sign, an index off
by one, a conjugated or swapped operand) compiled on the CPU into a temporary library. The pin
tests of ``test_oracle_pins`` are then run against it; at least one must fail. The real oracle is
never modified.
"""
import os
import subprocess
import tempfile

import pytest

import oracle
from oracle import build as obuild

from . import test_oracle_pins as pins

MUTANTS = {
    "charge_coeff_sign": ("cplx t = -q * pw / (double)m;", "cplx t = q * pw / (double)m;"),
    "charge_coeff_index": ("cplx t = -q * pw / (double)m;", "cplx t = -q * pw / (double)(m + 1);"),
    "dropped_log_term": ("ks_add(&acc[0], q * log(cabs(z)));", "(void)z;"),
    "dipole_power_off_by_one": ("cplx pw = inv;                     /* (y - c)^-(m+1) at m = 0 */",
                                "cplx pw = 1.0;"),
    "dipole_conjugated_normal": ("cplx t = delta * nrm * pw;", "cplx t = delta * conj(nrm) * pw;"),
    "green_sign": ("*q = w[i] * d1[i]; *delta = -w[i] * d2[i];",
                   "*q = w[i] * d1[i]; *delta = w[i] * d2[i];"),
    "eval_conjugated_offset": ("cplx pw = 1.0, dz = x - c;", "cplx pw = 1.0, dz = c - x;"),
    "swapped_strength_densities": ("case ORACLE_D: *q = 0.0; *delta = w[i] * d1[i];",
                                   "case ORACLE_D: *q = 0.0; *delta = d1[i];"),
    "multipole_dipole_sign": ("cplx t = -delta * nrm * pw;", "cplx t = delta * nrm * pw;"),
    "multipole_charge_index": ("t += -q * pw / (double)k;", "t += -q * pw / (double)(k + 1);"),
    "eval_multipole_log_dropped": ("ks_add(&s, coef[0] * log(cabs(z)));", "(void)0;"),
    "point_potential_dipole_sign": ("ks_add(&s, delta * creal(pt(src_nrm, i) / z));",
                                    "ks_add(&s, -delta * creal(pt(src_nrm, i) / z));"),
}

PIN_CALLS = [
    (pins.test_circle_single_layer_interior_is_exact, {"k": 3}),
    (pins.test_circle_single_layer_exterior_converges_in_p, {}),
    (pins.test_circle_double_layer_jump, {"k": 2}),
    (pins.test_gauss_identity_starfish, {}),
    (pins.test_green_representation_starfish, {}),
    (pins.test_center_at_target_reduces_to_plain_quadrature, {}),
    (pins.test_single_source_taylor_remainder, {"p": 3}),
    (pins.test_multipole_far_field_bound, {"kind": 3}),
    (pins.test_local_expansion_near_bound, {"kind": 3}),
]


def _build_mutant(tmp, name, old, new):
    src = open(obuild.SRC).read()
    assert src.count(old) >= 1, f"mutation {name} does not apply"
    path = os.path.join(tmp, f"{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new, 1))
    lib = os.path.join(tmp, f"lib{name}.so")
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-fopenmp", "-fcx-limited-range", "-fPIC",
                           "-shared", path, "-o", lib, "-lm"])
    return lib


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    old, new = MUTANTS[name]
    saved = oracle.lib()
    with tempfile.TemporaryDirectory() as tmp:
        mutant = oracle.load(_build_mutant(tmp, name, old, new))
        oracle._lib = mutant
        failed = []
        try:
            for fn, kw in PIN_CALLS:
                try:
                    fn(**kw)
                except AssertionError:
                    failed.append(fn.__name__)
        finally:
            oracle._lib = saved
    assert failed, f"no pin catches mutant {name}"

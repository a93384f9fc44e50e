"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Each mutant is a one-line edit of ``oracle/hsvd_oracle.c`` (a sign, an index,
a dropped factor, the printed forms of the garbled passages), compiled to a
temporary library that replaces the oracle's for the duration of the test.
"""
import os
import subprocess

import pytest

import oracle
import pins

MUTANTS = {
    # the printed theta denominator -a_ii + hyp a_jj, trigonometric case
    "theta_sign_trig": ("double zeta = (ajj - aii) / two_aij;",
                        "double zeta = (-aii - ajj) / two_aij;"),
    # the printed theta denominator, hyperbolic case
    "theta_sign_hyp": ("double zeta = -num / two_aij;", "double zeta = (ajj - aii) / two_aij;"),
    # larger root instead of the smaller one
    "larger_root": ("tt = sg / (az + s);\n        }\n        double tsq",
                    "tt = sg * (az + s);\n        }\n        double tsq"),
    "cosh_formula": ("*c = 1.0 / sqrt(omt * opt);", "*c = 1.0 / sqrt(1.0 + tt * tt);"),
    "dropped_hyp_in_update": ("gi[q] = fma(ht, y, x) * c;", "gi[q] = fma(t, y, x) * c;"),
    "dropped_c_in_v": ("vi[q] = fma(ht, y, x) * c;", "vi[q] = fma(ht, y, x);"),
    "wrong_new_diag": ("st->d[i] = dot(r, gi, gi);", "st->d[i] = dot(r, gj, gj);"),
    "skip_not_strict": ("return fabs(aij) < tol * (sqrt(aii) * sqrt(ajj));",
                        "return fabs(aij) <= tol * (sqrt(aii) * sqrt(ajj));"),
    # Alg. 4.4 as printed (strict comparison)
    "stepper_strict": ("if (s[0] + s[1] >= r - 1) {", "if (s[0] + s[1] > r - 1) {"),
    "stepper_half": ("s[0] -= r / 2;", "s[0] -= r / 2 - 1;"),
    "sort_direction": ("while (m >= 0 && d[m] < key) {", "while (m >= 0 && d[m] > key) {"),
    "lambda_sign": ("if (lambda) lambda[c] = (q < p) ? d[q] : -d[q];",
                    "if (lambda) lambda[c] = (q < p) ? -d[q] : d[q];"),
    "hyp_from_sign": ("int hyp = ((i < st->p) == (j < st->p)) ? -1 : 1;",
                      "int hyp = ((i < st->p) == (j < st->p)) ? 1 : -1;"),
    "code_table": ("if (fabs(t) > tthresh) return 3;", "if (fabs(t) > tthresh) return 1;"),
    "roundrobin_shift": ("L[m] = 1 + ((m - 1 + step) % (r - 1));", "L[m] = 1 + ((m + step) % (r - 1));"),
    "u_transposed": ("U[(size_t)c * n + row] = Gw[(size_t)c * r + row] / s;",
                     "U[(size_t)c * n + row] = Gw[(size_t)row * r + c] / s;"),
}

# pins that evaluate orderings only, safe to run on a stepper that leaves the
# index range (the solve would index out of bounds with it)
ORDERING_ONLY = {"stepper_strict", "stepper_half", "roundrobin_shift"}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique or missing: {name}"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    hdr = os.path.join(oracle.HERE, "hsvd_oracle.h")
    (tmp_path / "hsvd_oracle.h").write_text(open(hdr).read())
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", str(so), str(mut), "-lm"])
    saved = oracle._lib
    oracle._lib = oracle.load(str(so))
    try:
        pin_set = ([pins.pin_modmod, pins.pin_modmod_vs_appendix, pins.pin_roundrobin]
                   if name in ORDERING_ONLY else pins.ALL_PINS)
        caught = []
        for pin in pin_set:
            try:
                pin()
            except AssertionError:
                caught.append(pin.__name__)
        assert caught, f"mutant {name} passed every pin"
    finally:
        oracle._lib = saved

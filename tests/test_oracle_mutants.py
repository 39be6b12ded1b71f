"""Planted mistakes in a copy of the oracle must fail its pins.

Each mutant is a plausible slip (a misread coefficient, a dropped power of
h, a wrong sign, a swapped mass index, a double-counted pair, the star added
first).  The copy is compiled into a temporary library and the pin suite is
run against it in a subprocess; every mutant must make at least one pin fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hermite_oracle.c")

MUTANTS = {
    "corrector_3_10": ("(3.0 / 20.0)", "(3.0 / 10.0)"),
    "corrector_jerk_power": ("(7.0 * j0[k] + 2.0 * jk[k]) * h3 / 60.0",
                             "(7.0 * j0[k] + 2.0 * jk[k]) * h2 / 60.0"),
    "corrector_v_sign": ("vc[k] = vp[k] - 0.5 * (a0[k] - ak[k]) * h",
                         "vc[k] = vp[k] - 0.5 * (a0[k] + ak[k]) * h"),
    "predictor_v_power": ("0.5 * j0[k] * h2;", "0.5 * j0[k] * h;"),
    "jerk_sign": ("J[c] = u[c] * s3 - 3.0 * ru * s2 * A[c];",
                  "J[c] = u[c] * s3 + 3.0 * ru * s2 * A[c];"),
    "reaction_mass_index": ("a[3 * j + c] = a[3 * j + c] - m[i] * A[c];",
                            "a[3 * j + c] = a[3 * j + c] - m[j] * A[c];"),
    "potential_double_count": ("pot = pot + m[i] * m[j]", "pot = pot + 2.0 * m[i] * m[j]"),
    "star_first": ("    for (int i = 1; i < n; ++i)\n        for (int j = i + 1; j < n; ++j)\n"
                   "            pair_accumulate(i, j, m, x, v, a, jk);\n"
                   "    for (int j = 1; j < n; ++j)\n        pair_accumulate(0, j, m, x, v, a, jk);\n",
                   "    for (int j = 1; j < n; ++j)\n        pair_accumulate(0, j, m, x, v, a, jk);\n"
                   "    for (int i = 1; i < n; ++i)\n        for (int j = i + 1; j < n; ++j)\n"
                   "            pair_accumulate(i, j, m, x, v, a, jk);\n"),
    "timestep_radial_factor": ("J[c] = mu * (u[c] / (r2 * rn) - 3.0 * ru * r[c] / (r2 * r2 * rn));",
                               "J[c] = mu * (u[c] / (r2 * rn) - 2.0 * ru * r[c] / (r2 * r2 * rn));"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found: the oracle changed"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so),
                           str(mut), "-lm", "-lpthread"])
    env = dict(os.environ, FEWBODY_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"

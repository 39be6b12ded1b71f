"""Planted mistakes in a copy of the oracle must fail its pins.

Each mutant is a plausible slip (a misread coefficient, a dropped power of
h, a wrong sign, a swapped mass index, a double-counted pair, the star added
first, a misread stop rule, stall threshold or step cap; for MVS a wrong
Kepler mu, a dropped or reversed reflex drift, a whole kick, the star in the
kick, a wrong f function, a wrong mass; for Cash-Karp a misread tableau
entry, stale stage velocities, a loose acceptance test).  The copy is
compiled into a temporary library and the pin suite of the mutated source is
run against it in a subprocess; every mutant must make at least one pin
fail, and the unmutated copy must pass.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = {"hermite": os.path.join(ROOT, "oracle", "hermite_oracle.c"),
           "mvs": os.path.join(ROOT, "oracle", "mvs_oracle.c"),
           "rkck": os.path.join(ROOT, "oracle", "rkck_oracle.c")}
PINS = {"hermite": "test_oracle_pins.py", "mvs": "test_oracle_mvs.py", "rkck": "test_oracle_rkck.py"}

# name -> (source, text, replacement)
MUTANTS = {
    "corrector_3_10": ("hermite", "(3.0 / 20.0)", "(3.0 / 10.0)"),
    "corrector_jerk_power": ("hermite", "(7.0 * j0[k] + 2.0 * jk[k]) * h3 / 60.0",
                             "(7.0 * j0[k] + 2.0 * jk[k]) * h2 / 60.0"),
    "corrector_v_sign": ("hermite", "vc[k] = vp[k] - 0.5 * (a0[k] - ak[k]) * h",
                         "vc[k] = vp[k] - 0.5 * (a0[k] + ak[k]) * h"),
    "predictor_v_power": ("hermite", "0.5 * j0[k] * h2;", "0.5 * j0[k] * h;"),
    "jerk_sign": ("hermite", "J[c] = u[c] * s3 - 3.0 * ru * s2 * A[c];",
                  "J[c] = u[c] * s3 + 3.0 * ru * s2 * A[c];"),
    "reaction_mass_index": ("hermite", "a[3 * j + c] = a[3 * j + c] - m[i] * A[c];",
                            "a[3 * j + c] = a[3 * j + c] - m[j] * A[c];"),
    "potential_double_count": ("hermite", "pot = pot + m[i] * m[j]", "pot = pot + 2.0 * m[i] * m[j]"),
    "star_first": ("hermite",
                   "    for (int i = 1; i < n; ++i)\n        for (int j = i + 1; j < n; ++j)\n"
                   "            pair_accumulate(i, j, m, x, v, a, jk);\n"
                   "    for (int j = 1; j < n; ++j)\n        pair_accumulate(0, j, m, x, v, a, jk);\n",
                   "    for (int j = 1; j < n; ++j)\n        pair_accumulate(0, j, m, x, v, a, jk);\n"
                   "    for (int i = 1; i < n; ++i)\n        for (int j = i + 1; j < n; ++j)\n"
                   "            pair_accumulate(i, j, m, x, v, a, jk);\n"),
    "timestep_radial_factor": ("hermite",
                               "J[c] = mu * (u[c] / (r2 * rn) - 3.0 * ru * r[c] / (r2 * r2 * rn));",
                               "J[c] = mu * (u[c] / (r2 * rn) - 2.0 * ru * r[c] / (r2 * r2 * rn));"),
    # Stop rules: the Hill radius without its factor 3 or without m0, or from
    # one planet's distance alone; distances from the origin instead of the
    # star (for both rules, or for the ejection test only); only adjacent
    # planet pairs tested; a stall threshold ten times too high; one step
    # too many before MAXSTEPS.
    "hill_factor_3": ("hermite", "cbrt((m[i] + m[j]) / (3.0 * m[0]))", "cbrt((m[i] + m[j]) / m[0])"),
    "hill_star_mass": ("hermite", "cbrt((m[i] + m[j]) / (3.0 * m[0]))", "cbrt((m[i] + m[j]) / 3.0)"),
    "hill_one_distance": ("hermite", "0.5 * (rs[i] + rs[j])", "rs[i]"),
    "distance_from_origin": ("hermite", "d[c] = x[3 * i + c] - x[c];", "d[c] = x[3 * i + c];"),
    "eject_from_origin": ("hermite", "if (rs[i] > r_eject)",
                          "if (sqrt(x[3 * i] * x[3 * i] + x[3 * i + 1] * x[3 * i + 1] + "
                          "x[3 * i + 2] * x[3 * i + 2]) > r_eject)"),
    "encounter_adjacent_pairs_only": ("hermite",
                                      "for (int j = i + 1; j < n; ++j) {\n                double d[3];",
                                      "for (int j = i + 1; j < n && j < i + 2; ++j) {\n                double d[3];"),
    "stall_threshold": ("hermite", "!(*dt_next >= 1e-12 * fabs(t_end))", "!(*dt_next >= 1e-11 * fabs(t_end))"),
    "max_steps_off_by_one": ("hermite", "if (*steps >= max_steps) {", "if (*steps > max_steps) {"),
    # MVS: the two-body mu of Jacobi-style splittings, a dropped or reversed
    # reflex drift, a whole kick where half belongs, the star in the kick, a
    # wrong f function and the wrong mass in the star's velocity.
    "mvs_kepler_mu": ("mvs", "ora_kepler_drift(m[0], Q + 3 * i, V + 3 * i, dt)",
                      "ora_kepler_drift(m[0] + m[i], Q + 3 * i, V + 3 * i, dt)"),
    "mvs_no_reflex_drift": ("mvs", "Q[3 * i + c] += h * P[c] / m[0];", "Q[3 * i + c] += 0.0 * P[c] / m[0];"),
    "mvs_reflex_sign": ("mvs", "Q[3 * i + c] += h * P[c] / m[0];", "Q[3 * i + c] -= h * P[c] / m[0];"),
    "mvs_whole_first_kick": ("mvs", "kick(n, m, Q, V, 0.5 * dt);\n    for (int i = 1;",
                             "kick(n, m, Q, V, dt);\n    for (int i = 1;"),
    "mvs_kick_includes_star": ("mvs", "for (int j = 1; j < n; ++j) {\n            if (j == i)",
                               "for (int j = 0; j < n; ++j) {\n            if (j == i)"),
    "mvs_f_function": ("mvs", "const double f = 1.0 - (a / r0) * (1.0 - c);",
                       "const double f = 1.0 - (a / r0) * (1.0 + c);"),
    "mvs_star_velocity_mass": ("mvs", "v[c] = Vc[c] - sp / m[0];", "v[c] = Vc[c] - sp / M;"),
    # RKCK: a misread coupling coefficient, fifth- and fourth-order weights,
    # stages that reuse the step's starting velocity, a loose acceptance test.
    "rk_coupling_a52": ("rkck", "5.0 / 2.0", "2.0 / 5.0"),
    "rk_weight_b6": ("rkck", "512.0 / 1771.0", "521.0 / 1771.0"),
    "rk_weight_bs5": ("rkck", "277.0 / 14336.0", "227.0 / 14336.0"),
    "rk_stage_velocity": ("rkck", "kx[s][k] = vs[k];", "kx[s][k] = v[k];"),
    "rk_acceptance": ("rkck", "if (!(E <= 1.0)) {", "if (!(E <= 1e3)) {"),
}


def build_and_run_pins(tmp_path, which, old=None, new=None):
    """Compile the oracle with `which`'s source mutated (old -> new; no
    mutation when old is None) and the other source unchanged; run that
    source's pin suite against it.  Returns the pytest process."""
    srcs = []
    for key, path in SOURCES.items():
        text = open(path).read()
        if key == which and old is not None:
            assert text.count(old) == 1, "mutation site not found: the oracle changed"
            text = text.replace(old, new)
        out = tmp_path / os.path.basename(path)
        out.write_text(text)
        srcs.append(str(out))
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so),
                           *srcs, "-lm", "-lpthread"])
    env = dict(os.environ, FEWBODY_ORACLE_LIB=str(so))
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", PINS[which])],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)


@pytest.mark.parametrize("which", sorted(SOURCES))
def test_unmutated_copy_passes(which, tmp_path):
    """Control: the same build route without a mutation passes the pins, so
    a mutant's failure is the mutation's doing."""
    r = build_and_run_pins(tmp_path, which)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    which, old, new = MUTANTS[name]
    r = build_and_run_pins(tmp_path, which, old, new)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"

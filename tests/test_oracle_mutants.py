"""The oracle's pins must be sensitive: each plausible slip below, planted
in a copy of the oracle's C source (on the CPU), must make at least one pin
test fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nbody_oracle.c")

# (name, exact text in the source, replacement)
MUTANTS = [
    ("beta_drops_alpha2", "(vv + ra) * rinv2 + alpha * alpha", "(vv + ra) * rinv2"),
    ("jerk_sign", "mr3 * w[d] - 3.0 * alpha * A", "mr3 * w[d] + 3.0 * alpha * A"),
    ("snap_6alpha_to_3", "- 6.0 * alpha * J", "- 3.0 * alpha * J"),
    ("snap_beta_coeff", "- 3.0 * beta * A", "- 2.0 * beta * A"),
    ("alpha_unsoftened", "const double alpha = rv * rinv2;",
     "const double alpha = rv / (r2 - eps2 + 1e-300);"),
    ("acc_transposed_r", "r[d] = x[3 * j + d] - x[3 * i + d];", "r[d] = x[3 * i + d] - x[3 * j + d];"),
    ("pot_self_term", "if (j == i)\n                continue;", "if (0)\n                continue;"),
    ("crackle_9beta", "- 9.0 * beta * J", "- 6.0 * beta * J"),
    ("crackle_gamma_4alpha3", "(3.0 * beta - 4.0 * alpha * alpha)", "(3.0 * beta - 3.0 * alpha * alpha)"),
    ("crackle_gamma_3va", "(3.0 * va + rj) * rinv2", "(va + rj) * rinv2"),
    ("init_step_order", "st->eta_init * A1 / A2", "st->eta_init * sqrt(A1 / A2)"),
    ("predict_h4", "sn[e] * h4 / 24.0 + cr[e] * h5 / 120.0", "sn[e] * h4 / 12.0 + cr[e] * h5 / 120.0"),
    ("predict_vel_crackle", "cr[e] * h4 / 24.0;", "cr[e] * h4 / 6.0;"),
    ("corrector_h2", "h * h / 10.0 * (j1[d] - j0[d])", "h * h / 12.0 * (j1[d] - j0[d])"),
    ("corrector_pos_sign", "h * h * h / 120.0 * (j1[d] + j0[d])", "h * h * h / 120.0 * (j1[d] - j0[d])"),
    ("interp_168", "168.0 * h * D1", "160.0 * h * D1"),
    ("interp_crk_half", "xx * h * h / 2.0", "xx * h * h"),
    ("criterion_cuberoot", "eta * cbrt(A1 / A4)", "eta * sqrt(A1 / A4)"),
    ("criterion_A4_terms", "norm3(cr) * norm3(a5) + norm3(pp) * norm3(pp)", "norm3(pp) * norm3(pp)"),
    ("block_no_commensurability", "fmod(t_new, 2.0 * dt_old) == 0.0", "1"),
    ("block_round_up", "dt = ldexp(1.0, e - 1);", "dt = ldexp(1.0, e);"),
    ("energy_double_count", "for (int64_t j = i + 1; j < j1; ++j)", "for (int64_t j = off[c]; j < j1; ++j) if (j != i)"),
    ("energy_kinetic_half", "k += 0.5 * m[i]", "k += m[i]"),
    ("run_pairs_nact_squared", "p += (double)cnt[c] * (double)(off[c + 1] - off[c]);",
     "p += (double)cnt[c] * (double)cnt[c];"),
    ("run_hist_round_up", "while ((INT64_C(1) << (b + 1)) <= cnt[c])", "while ((INT64_C(1) << b) < cnt[c])"),
    ("run_counts_before_recap", "    orc_recap(st, t_target);\n    for (;;) {", "    for (;;) {"),
]

PINS = ["tests/test_oracle_force.py", "tests/test_oracle_integrator.py"]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11",
                           "-shared", "-fPIC", "-o", str(lib), str(mut), "-lm"])
    env = dict(os.environ, NBODY_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"

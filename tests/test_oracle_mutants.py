"""Planted-mistake checks for the oracle's pins (CPU only).

Each mutant is a copy of the oracle's C source with one plausible mistake (a
dropped term, a wrong sign, a transposed index, a missing clip...).  It is
compiled into a temporary library and run against a quick subset of the pins
in ``test_oracle_pins``; every mutant must make at least one of them fail.
This shows the pins would catch such mistakes in the real oracle.
"""
import concurrent.futures
import os
import subprocess
import sys
import tempfile


import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gapsafe_oracle.c")

MUTANTS = {
    "gap_drops_l1_term": ("double G = 0.5 * R2 + lambda * l1 - lambda * alpha * Ry",
                          "double G = 0.5 * R2 - lambda * alpha * Ry"),
    "soft_threshold_sign": ("if (x > u) return x - u;", "if (x > u) return x + u;"),
    "cd_transposed_index": ("        const double* xj = X + (int64_t)j * ldx;\n        double z",
                            "        const double* xj = X + (int64_t)j;\n        double z"),
    "alpha_not_clipped": ("    if (alpha > 1.0 / M) alpha = 1.0 / M;\n", ""),
    "residual_update_sign": ("for (int i = 0; i < n; ++i) rho[i] -= d * xj[i];",
                             "for (int i = 0; i < n; ++i) rho[i] += d * xj[i];"),
    "dual_norm_no_abs": ("if (fabs(c_out[k]) > M) M = fabs(c_out[k]);",
                         "if (c_out[k] > M) M = c_out[k];"),
    "cd_step_norm_not_squared": ("double z = beta[j] + col_dot(n, xj, rho) / nrm2[j];",
                                 "double z = beta[j] + col_dot(n, xj, rho) / sqrt(nrm2[j]);"),
    "grid_exponent": ("-delta * (double)t / (double)(T - 1)", "-delta * (double)t / (double)T"),
    "radius_halved": ("double radius_s = sqrt(2.0 * Gp) / lambda",
                      "double radius_s = sqrt(0.25 * Gp) / lambda"),
    "dual_wrong_sign": ("double D = 0.5 * yy - 0.5 * lambda * lambda * d2;",
                        "double D = 0.5 * yy + 0.5 * lambda * lambda * d2;"),
    "lambda_max_not_abs": ("if (fabs(xty[j]) > lmax) lmax = fabs(xty[j]);",
                           "if (xty[j] > lmax) lmax = xty[j];"),
    "gap_bound_drops_y_rho_error": ("                lambda * fabs(alpha_s) * gamma_m(n) * yn * rnorm +\n", ""),
    "dome_normal_flipped": ("  double wx = (xty / lambda - alpha * cj) / Rh;\n  double mu_p",
                            "  double wx = (alpha * cj - xty / lambda) / Rh;\n  double mu_p"),
    "dome_drops_ratio_factor": ("double s2 = (xn * xn - wx * wx) * (1.0 - a * a);",
                                "double s2 = (xn * xn - wx * wx);"),
    "st3_center_on_wrong_side": ("      shift = ref->sstar * ratio / (ref->nstar * ref->nstar);",
                                 "      shift = -ref->sstar * ratio / (ref->nstar * ref->nstar);"),
    "static_radius_drops_lambda_max": ("      rad = sqrt(yy) * fabs(1.0 / lambda - 1.0 / lmx);",
                                       "      rad = sqrt(yy) * fabs(1.0 / lambda - 1.0 / (2.0 * lmx));"),
    "screen_drops_zero_test": ("keep_safe[k] = (nrm2[j] > 0.0 && mu_s >= 1.0 - 4.0 * ORC_U) ? 1 : 0;",
                               "keep_safe[k] = (nrm2[j] > 0.0 && mu_s >= 1.5) ? 1 : 0;"),
}

# Runs in a child process so that a mutant that loops for long is cut off.
CHILD = r"""
import sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
import oracle, test_oracle_pins as T
orc = oracle.Oracle(oracle._declare(__import__('ctypes').CDLL({lib!r})))
checks = [
  lambda: T.test_grid(orc),
  lambda: T.test_lambda_max_gives_zero(orc),
  lambda: T.test_orthonormal_soft_threshold(orc, 0),
  lambda: T.test_pass_gap_matches_definition(orc),
  lambda: T.test_inflated_test_is_superset(orc),
  lambda: T.test_weak_duality_random_points(orc),
  lambda: T.test_prop3_sequential_identity(orc),
  lambda: T.test_brute_force_tiny(orc, 20, 6, 2),
  lambda: T.test_kkt_at_tight_solution(orc, "c0"),
  lambda: T.test_safety_invariant(orc),
  lambda: T.test_rounding_bound_covers_cancelling_y_rho(orc),
  lambda: T.test_dome_support_matches_brute_force(orc),
  lambda: T.test_dome_contains_dual_optimum_and_lies_in_sphere(orc),
  lambda: T.test_comparison_rules_hold_dual_optimum(orc, "st3"),
  lambda: T.test_comparison_rules_hold_dual_optimum(orc, "static"),
  lambda: T.test_static_safe_critical_ratio(orc),
]
failed = 0
for c in checks:          # one failing pin is enough
    try:
        c()
    except BaseException:
        failed += 1
        break
print("FAILED_CHECKS", failed)
"""


def _run_mutant(name, td):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    if old not in src:
        return name, "anchor not found"
    msrc = os.path.join(td, name + ".c")
    open(msrc, "w").write(src.replace(old, new, 1))
    lib = oracle.build(msrc, os.path.join(td, name + ".so"))
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    try:
        out = subprocess.run([sys.executable, "-c", code], capture_output=True,
                             text=True, timeout=240).stdout
    except subprocess.TimeoutExpired:
        return name, None  # the mutant stopped converging: caught
    line = [ln for ln in out.splitlines() if ln.startswith("FAILED_CHECKS")]
    if not line:
        return name, "child crashed without a verdict: " + out[-500:]
    if int(line[0].split()[1]) == 0:
        return name, "passed every pin"
    return name, None


def test_every_mutant_is_caught():
    with tempfile.TemporaryDirectory() as td, \
            concurrent.futures.ThreadPoolExecutor(max_workers=6) as pool:
        results = list(pool.map(lambda m: _run_mutant(m, td), sorted(MUTANTS)))
    escaped = {name: why for name, why in results if why is not None}
    assert not escaped, escaped

"""The oracle's pins must catch plausible mistakes.  Each case plants one
mistake in a copy of oracle/rmo.c (on the CPU), builds it, and runs the pins
that should notice against the mutant: they must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rmo.c")

MUTANTS = {
    "R_prefactor": ("const ld scale = 1.0L / (2.0L * (ld)pw->a);", "const ld scale = 1.0L / ((ld)pw->a);",
                    "test_oracle_R.py::test_rank_one_single_pole"),
    "R_pole_sign": ("const ld d = 1.0L / ((ld)pw->Ek[k] - (ld)E);", "const ld d = 1.0L / ((ld)E - (ld)pw->Ek[k]);",
                    "test_oracle_R.py::test_exact_rational"),
    "R_index": ("for (int j = 0; j <= i; ++j) row[j] += wi * (ld)wk[j];",
                "for (int j = 0; j <= i; ++j) row[j] += wi * (ld)wk[i];",
                "test_oracle_R.py::test_exact_rational"),
    "cf2_sign": ("return (1.0L + I * v) / rho;", "return (1.0L - I * v) / rho;",
                 "test_oracle_asymptotics.py::test_wronskian_sample"),
    "cf1_sign_tracking": ("if (den < 0) sg = -sg;", "if (den < 0) sg = sg;",
                          "test_oracle_asymptotics.py::test_coulomb_vs_mpmath"),
    "taylor_term": ("B * dm1 * h * h * h + C * dm2 * h * h * h * h;", "B * dm1 * h * h * h;",
                    "test_oracle_asymptotics.py::test_coulomb_vs_mpmath"),
    "closed_sign": ("return (1.0L - w) / r;", "return (1.0L + w) / r;",
                    "test_oracle_asymptotics.py::test_closed_neutral_s_wave"),
    "match_b_sign": ("(a * Cpm - b * Cm);", "(a * Cpm + b * Cm);",
                     "test_oracle_K_S.py::test_single_channel_ion_closed_form"),
    "match_rhs_sign": ("- (i == oj ? s : 0.0L);", "+ (i == oj ? s : 0.0L);",
                       "test_oracle_K_S.py::test_neutral_s_wave_closed_form"),
    "lu_back_sub": ("for (int j = r + 1; j < n; ++j) x[r] -= LU[(size_t)r * n + j] * x[j];",
                    "for (int j = r + 2; j < n; ++j) x[r] -= LU[(size_t)r * n + j] * x[j];",
                    "test_oracle_K_S.py::test_full_and_reduced_formulations_agree"),
    "K_rows": ("K[(size_t)i * n + j] = (double)Y[(size_t)open_idx[i] * no + j];",
               "K[(size_t)i * n + j] = (double)Y[(size_t)i * no + j];",
               "test_oracle_K_S.py::test_channel_permutation_covariance"),
    "S_formula": ("rhs[(size_t)i * no + j] = (i == j ? 1.0L : 0.0L) + I * kji;",
                  "rhs[(size_t)i * no + j] = (i == j ? 1.0L : 0.0L) - I * kji;",
                  "test_oracle_K_S.py::test_S_unitary_symmetric_and_T_identity"),
    "omega_target_index": ("pw->target[open_idx[j]]] += half_g * t2;", "pw->target[open_idx[i]]] += half_g * t2;",
                           "test_oracle_K_S.py::test_omega_from_T_identity_by_target"),
    "cond1_row_norm": ("for (int i = 0; i < n; ++i) s += fabsl(A[(size_t)i * n + j]);",
                       "for (int i = 0; i < n; ++i) s += fabsl(A[(size_t)j * n + i]);",
                       "test_oracle_K_S.py::test_cond1_estimate_bounds_true_condition_number"),
    "cond1_transposed_solve": ("lu_solve(LU, n, piv, y, 1);", "lu_solve(LU, n, piv, y, 0);",
                               "test_oracle_K_S.py::test_cond1_estimate_bounds_true_condition_number"),
    "omega_half_g": ("const ld half_g = 0.5L * (ld)pw->g;", "const ld half_g = (ld)pw->g;",
                     "test_oracle_K_S.py::test_single_channel_ion_closed_form"),
    # long-range coupling and Numerov propagation
    "coupling_factor": ("q[(size_t)i * n + j] = 2.0L * u;", "q[(size_t)i * n + j] = u;",
                        "test_oracle_coupling.py::test_coupled_propagation_against_mpmath"),
    "coupling_power": ("ld rp = 1.0L / (r * r);", "ld rp = 1.0L / r;",
                       "test_oracle_coupling.py::test_coupled_propagation_against_mpmath"),
    "numerov_weight": ("(10.0L * h * h / 12.0L) * qy", "(11.0L * h * h / 12.0L) * qy",
                       "test_oracle_coupling.py::test_uncoupled_propagation_converges_to_analytic"),
    "numerov_derivative": ("(((2.0L * Z1[t] - Y1[t]) - (2.0L * Zc[t] - Y[t])) / (2.0L * h))",
                           "((Z1[t] - Zc[t]) / (2.0L * h))",
                           "test_oracle_coupling.py::test_uncoupled_propagation_converges_to_analytic"),
    # multichannel quantum-defect operation
    "mqdt_cot_sign": ("out[2] = -e / W + f * cot;", "out[2] = -e / W - f * cot;",
                      "test_oracle_mqdt.py::test_pair_against_kummer_and_tricomi"),
    "mqdt_norm_A": ("expl(logN + 0.5L * logA", "expl(logN + logA",
                    "test_oracle_mqdt.py::test_pair_continues_the_open_functions_across_threshold"),
    "mqdt_tan_sign": ("Mc[(size_t)i * nc + i] += s / c;", "Mc[(size_t)i * nc + i] -= s / c;",
                      "test_oracle_mqdt.py::test_elimination_reproduces_the_physical_K"),
    "mqdt_series": ("-2.0L * z * cm1 - eps * cm2", "-2.0L * z * cm1 + eps * cm2",
                    "test_oracle_mqdt.py::test_pair_against_kummer_and_tricomi"),
    "mqdt_minv_sign": ("(i == j ? 1.0L : 0.0L) - I * (ld)K[(size_t)i * n + j];",
                       "(i == j ? 1.0L : 0.0L) + I * (ld)K[(size_t)i * n + j];",
                       "test_oracle_mqdt.py::test_fine_point_uses_the_four_surrounding_coarse_points"),
    "mqdt_sform_phase": ("C[(size_t)k * nc + l] = (k == l ? cs - I * sn : 0.0L) - SU(ci[k], ci[l]);",
                         "C[(size_t)k * nc + l] = (k == l ? cs + I * sn : 0.0L) - SU(ci[k], ci[l]);",
                         "test_oracle_mqdt.py::test_s_form_elimination"),
    "mqdt_window": ("int st0 = k - 1;", "int st0 = k - 3;",
                    "test_oracle_mqdt.py::test_fine_point_uses_the_four_surrounding_coarse_points"),
    "mqdt_member_floor": ("const double numin = fnumin > l + 0.1 ? fnumin : l + 0.1;",
                          "const double numin = fnumin > l ? fnumin : l;",
                          "test_oracle_mqdt.py::test_member_rule"),
    "mqdt_coarse_last": ("if (((j - s0) % ieq == 0 || j == s1 - 1) && !flag[j] && !avoid[j])",
                         "if (((j - s0) % ieq == 0) && !flag[j] && !avoid[j])",
                         "test_oracle_mqdt.py::test_coarse_points_and_every_point_coarse"),
    "mqdt_qetest_scale":("const double tol = qetest * pw->z * pw->z;", "const double tol = qetest;",
                          "test_oracle_mqdt.py::test_qetest_reuses_the_interpolant_within_its_energy_step"),
    "taylor_start_binomial": ("for (int t = 1; t <= p; ++t) binom = binom * (ld)(lam + t) / (ld)t;",
                              "for (int t = 1; t <= p; ++t) binom = binom * (ld)(lam + t - 1) / (ld)t;",
                              "test_oracle_coupling.py::test_coupled_propagation_against_mpmath"),
    "stabilise_alpha": ("acc -= Z[(size_t)i * m + a] * alpha[(size_t)a * m + j];",
                        "acc += Z[(size_t)i * m + a] * alpha[(size_t)a * m + j];",
                        "test_oracle_coupling.py::test_coupled_K_symmetric_and_recombination_invariant"),
    "coupled_match_rhs": ("B[(size_t)i * no + j] = acc - (ld)phi[(size_t)i * ld2 + n + j];",
                          "B[(size_t)i * no + j] = acc + (ld)phi[(size_t)i * ld2 + n + j];",
                          "test_oracle_coupling.py::test_uncoupled_K_converges_to_plain_matching"),
    "stabilise_last_step": ("s <= N - 3 && stabilise(", "s <= N - 2 && stabilise(",
                            "test_oracle_coupling.py::test_recombination_at_last_allowed_step"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new, pin = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old}"
    mut = src.replace(old, new, 1)
    c = tmp_path / "rmo_mut.c"
    c.write_text(mut)
    so = tmp_path / "librmo_mut.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-std=c11", "-fPIC", "-shared", "-I",
                           os.path.join(ROOT, "oracle"), str(c), "-o", str(so), "-lm"])
    env = dict(os.environ, RMO_SO=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", pin.split("::")[0]), "-k", pin.split("::")[1]],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"mutant {name} survived {pin}:\n{r.stdout[-2000:]}"

"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake (a dropped factor, a flipped sign, a
swapped ratio, a wrong index) into a private copy of the oracle's C source,
builds it in a temporary directory and runs the pin tests against it: at
least one pin must fail.  The real oracle is never modified."""
import os
import subprocess

import pytest

import oracle as O
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(O.__file__), "mcg_oracle.c")

PINS = [
    pins.test_mmr_with_exact_eigenpairs_equals_abs_A,
    pins.test_mmr_apply_on_sparse_workload_vs_dense_definition,
    pins.test_spmv_matches_scipy,
    pins.test_pcg_with_exact_indefinite_preconditioner_two_iterations,
    lambda: pins.test_pcg_matches_scipy_cg("jacobi"),
    pins.test_pcg_indefinite_preconditioner_energy_norm_monotone,
    pins.test_plain_minres_matches_scipy_minres,
    pins.test_preconditioned_minres_matches_scipy_and_phibar_is_Minv_residual,
    lambda: pins.test_minres_cg_laplace2d_matches_direct_solve(1e-3),
    pins.test_ildl0_reproduces_A_on_its_pattern,
    pins.test_ildl0_is_exact_ldlt_without_fill,
    pins.test_pcg_smw_preconditioner_with_exact_A_is_exact_inverse,
    pins.test_cct_apply_matches_dense_product,
    pins.test_pcg_cct_matches_scipy_cg,
    pins.test_pcg_cct_exact_inverse_factor_one_iteration,
    pins.test_stagnation_status_and_window,
    pins.test_keep_best_returns_smallest_true_residual_iterate,
    pins.test_zero_inner_budget_returns_x0_with_maxit,
    lambda: pins.test_ildlp_without_dropping_is_lapack_bunch_kaufman(
        lambda: pins.saddle(10, 10, 5, h_scale=0.01)),
    lambda: pins.test_ildlp_without_dropping_is_lapack_bunch_kaufman(
        lambda: pins.rand_sym_indefinite(30, 5, 1)[0]),
    pins.test_ildlp_drop_and_fill_limits,
    lambda: pins.test_ildlp_sweeps_are_the_truncated_neumann_series(11),
    pins.test_ildlp_sweeps_become_exact_at_the_factor_depth,
    lambda: [pins.test_ildlp_reproduces_A_on_its_kept_positions(*c) for c in
             ((11, 1.0, 0.05), (12, 2.0, 0.2), (13, 1.0, 0.3), (14, 3.0, 1e-2), (15, 0.5, 0.1),
              (None, 0.0, 1e-2))],
    pins.test_minres_cg_with_ildlp_on_a_saddle_point_system,
]

MUTANTS = {
    "mmr_drop_factor_2": ("s[j] *= 2.0 * fabs(lam[j]);", "s[j] *= 1.0 * fabs(lam[j]);"),
    "mmr_sign": ("q[i] += acc;", "q[i] -= acc;"),
    "spmv_wrong_index": ("s += val[p] * x[col[p]];", "s += val[p] * x[i];"),
    "lanczos_sign": ("y[i] -= f * r1[i];", "y[i] += f * r1[i];"),
    "givens_delta_sign": ("double delta = cs * dbar + sn * alfa;",
                          "double delta = cs * dbar - sn * alfa;"),
    "w_drop_eps_term": ("w[i] = (v[i] - oldeps * w1[i] - delta * w2[i]) / gamma;",
                        "w[i] = (v[i] - delta * w2[i]) / gamma;"),
    "cg_beta_inverted": ("double beta = rho_new / rho;", "double beta = rho / rho_new;"),
    "cg_r_update_sign": ("z[i] += alpha * p[i]; r[i] -= alpha * q[i];",
                         "z[i] += alpha * p[i]; r[i] += alpha * q[i];"),
    "ildl_drop_d": ("if (pim >= 0) s -= l_val[pim] * d[m] * l_val[q];",
                    "if (pim >= 0) s -= l_val[pim] * l_val[q];"),
    "ildl_solve_transposed": ("t[l_col[p]] -= l_val[p] * ti;", "t[l_col[p]] -= l_val[p] * t[l_col[p]];"),
    "smw_sign": ("double c = -2.0 * dot(n, vj, g) / P->lam[j];",
                 "double c = 2.0 * dot(n, vj, g) / P->lam[j];"),
    # C C^T second level: the product order swapped (C^T C g), and C g in
    # place of C^T g (scatter into the row instead of the column)
    "cct_swapped_order": (
        """      double *u = (double *)calloc((size_t)n, sizeof(double));
      for (int32_t i = 0; i < n; ++i)
        for (int32_t p = pc->c_ptr[i]; p < pc->c_ptr[i + 1]; ++p)
          u[pc->c_col[p]] += pc->c_val[p] * g[i];
      orc_spmv(n, pc->c_ptr, pc->c_col, pc->c_val, u, t);""",
        """      double *u = (double *)calloc((size_t)n, sizeof(double));
      orc_spmv(n, pc->c_ptr, pc->c_col, pc->c_val, g, u);
      memset(t, 0, sizeof(double) * (size_t)n);
      for (int32_t i = 0; i < n; ++i)
        for (int32_t p = pc->c_ptr[i]; p < pc->c_ptr[i + 1]; ++p)
          t[pc->c_col[p]] += pc->c_val[p] * u[i];"""),
    "cct_wrong_scatter": ("u[pc->c_col[p]] += pc->c_val[p] * g[i];",
                          "u[i] += pc->c_val[p] * g[pc->c_col[p]];"),
    # failure handling: the best iterate not restored, stagnation never
    # declared, a zero inner budget treated as a converged inner solve
    "keep_best_ignored": ("if (status != ORC_OK && o->keep_best) {",
                          "if (0 && status != ORC_OK && o->keep_best) {"),
    "stagnation_never": ("if (o->stag_window > 0 && since_best >= o->stag_window) "
                         "{ status = ORC_STAGNATION; break; }", ""),
    "zero_budget_accepted": ("if (s == ORC_MAXIT && *budget > 0) s = ORC_OK;",
                             "if (s == ORC_MAXIT && *budget >= 0) s = ORC_OK;"),
    # pivoted incomplete LDL^T: the 2x2 solve, the Bunch-Kaufman test, the
    # 2x2 Schur update, the fill limit, the 2x2 pivot's diagonal, the 1x1 update
    "ildlp_2x2_solve_sign": ("u[i] = (e * x - b * y) / det;", "u[i] = (e * x + b * y) / det;"),
    "ildlp_bk_rule": ("if (absakk * rowmax >= alpha * colmax * colmax) {",
                      "if (absakk * rowmax >= alpha * colmax) {"),
    "ildlp_schur_2x2": ("double u2 = S->doff[s] * a + S->dd[s + 1] * b;",
                        "double u2 = S->doff[s] * b + S->dd[s + 1] * a;"),
    "ildlp_fill_limit": ("int32_t lim = (int32_t)ceil(fill * (double)m_a);",
                         "int32_t lim = (int32_t)ceil(2.0 * fill * (double)m_a);"),
    # a 2x2 pivot's first diagonal read without checking that the Schur
    # column touched it (a value left from an earlier column)
    "ildlp_stale_diagonal": ("double a = m1[c] ? w1[c] : 0.0,", "double a = w1[c],"),
    # the 1x1 Schur update without D
    # the Jacobi sweeps: reading the buffer being written (the sweep before
    # last), an in-place backward sweep
    "ildlp_sweeps_wrong_buffer": ("for (int32_t p = F->l_ptr[i]; p < F->l_ptr[i + 1]; ++p) s -= F->l_val[p] * a[F->l_col[p]];",
                                  "for (int32_t p = F->l_ptr[i]; p < F->l_ptr[i + 1]; ++p) s -= F->l_val[p] * b[F->l_col[p]];"),
    "ildlp_sweeps_in_place": ("b[F->l_col[p]] -= F->l_val[p] * a[i];",
                              "b[F->l_col[p]] -= F->l_val[p] * b[i];"),
    "ildlp_schur_1x1_no_d": ("double coef = S->dd[j] * rw->e[q].val;",
                             "double coef = rw->e[q].val;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found: " + name
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", so, str(path), "-lm"])
    caught = []
    with O.use_library(so):
        for pin in PINS:
            try:
                pin()
            except AssertionError:
                caught.append(getattr(pin, "__name__", "pin"))
            except Exception:          # the mutant crashed a pin: also caught
                caught.append("error")
    assert caught, "no pin failed for mutant " + name

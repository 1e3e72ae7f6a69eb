"""The pins catch plausible mistakes.  Each case plants one mistake in a copy
of the oracle's source (a flipped sign, a dropped term, a swapped index or
operand), builds it, and runs the named pins against that build in a child
process: at least one of them must fail.  CPU only; the oracle in the
repository is not touched."""
import os
import subprocess
import sys

import pytest

from oracle import build as OB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nhdc_oracle.c")
T = "tests/test_oracle.py::"

# (what, original text, mistaken text, pins that must catch it)
MUTANTS = [
    ("Coriolis term with the wrong sign",
     "(zeta_e + m->fe[e])", "(zeta_e - m->fe[e])",
     [T + "test_vn_tendency_of_sheared_solid_body_rotation"]),
    ("vertical advection of vn dropped",
     " - obar * dvdz;", ";",
     [T + "test_vn_tendency_of_sheared_solid_body_rotation"]),
    ("normal gradient from c2 to c1",
     "(p[g->edge_cells[ne + e]] - p[g->edge_cells[e]])",
     "(p[g->edge_cells[e]] - p[g->edge_cells[ne + e]])",
     [T + "test_divergence_of_gradient_exact_for_quadratic_on_regular_lattice"]),
    ("kinetic-energy gradient from c2 to c1",
     "(AT(m->kc, k, nc, c2) - AT(m->kc, k, nc, c1))", "(AT(m->kc, k, nc, c1) - AT(m->kc, k, nc, c2))",
     [T + "test_vn_tendency_of_sheared_solid_body_rotation"]),
    ("horizontal advection of w with the wrong sign",
     "= -hadv - AT(m->omega", "= hadv - AT(m->omega",
     [T + "test_w_tendency_of_advected_ascent"]),
    ("divergence damping with the wrong sign",
     "+ p->div_damp * abar * gdiv;", "- p->div_damp * abar * gdiv;",
     [T + "test_divergence_damping_removes_divergence"]),
    ("reference profile interpolated from the wrong levels",
     "gw[i] * theta_ref[i] + (1.0 - gw[i]) * theta_ref[i - 1]",
     "gw[i] * theta_ref[i - 1] + (1.0 - gw[i]) * theta_ref[i]",
     [T + "test_column_matches_dense_solve_of_implicit_equations[20-3]"]),
    ("explicit weight 1 + beta instead of 1 - beta",
     "double pterm = (1.0 - beta)", "double pterm = (1.0 + beta)",
     [T + "test_column_matches_dense_solve_of_implicit_equations[20-3]"]),
    ("tridiagonal diagonal with the wrong sign",
     "tb[i - 1] = 1.0 + ga[i]", "tb[i - 1] = 1.0 - ga[i]",
     [T + "test_column_matches_dense_solve_of_implicit_equations[20-3]"]),
    ("theta flux carried with rho instead of theta",
     "AT(m->hfl, k, ne, e) = AT(the, k, ne, e) * f;", "AT(m->hfl, k, ne, e) = AT(rhoe, k, ne, e) * f;",
     [T + "test_gravity_wave_frequency_r2b3"]),
    ("mass flux without the layer depth",
     "AT(vnx, k, ne, e) * AT(m->dz_e, k, ne, e);", "AT(vnx, k, ne, e);",
     [T + "test_gravity_wave_frequency_r2b3"]),
    ("upwind value from the downwind cell",
     "int64_t up = u[e] >= 0.0 ?", "int64_t up = u[e] < 0.0 ?",
     [T + "test_upwind_takes_the_upwind_cell"]),
    ("upwind displacement reversed",
     "d[x] = a * (g->edge_x[x * ne + e] - g->cell_x[x * nc + up])",
     "d[x] = a * (g->cell_x[x * nc + up] - g->edge_x[x * ne + e])",
     [T + "test_upwind_edge_value_exact_for_linear_field_on_a_plane"]),
    ("sponge multiplies instead of divides",
     "wp[i] * (1.0 / (1.0 + dt * p->w_damp[i]))", "wp[i] * (1.0 + dt * p->w_damp[i])",
     [T + "test_column_sponge_damps_the_solved_w[20-3]"]),
    ("deformation with the trace added",
     "double d2 = 2.0 * s2 - tr * tr;", "double d2 = 2.0 * s2 + tr * tr;",
     [T + "test_deformation_exact_for_linear_field_on_a_plane"]),
    ("diffusion with the wrong sign",
     "u[e] = u[e] + dt * ke * lap[e];", "u[e] = u[e] - dt * ke * lap[e];",
     [T + "test_each_damping_option_removes_energy_where_it_acts"]),
    ("Smagorinsky coefficient without the cell area",
     "kh[c] = cs2 * g->cell_area[c] * kh[c];", "kh[c] = cs2 * kh[c];",
     [T + "test_smagorinsky_coefficient_scales_with_cell_area"]),
    ("tracer flux from the downwind cell",
     "const int64_t up = F[e] >= 0.0 ?", "const int64_t up = F[e] < 0.0 ?",
     [T + "test_tracer_transport_does_not_grow_noise"]),
    ("tracer gradient without the arc weight",
     "double dq = wgt * (q[nb] - q[c]);", "double dq = (q[nb] - q[c]);",
     [T + "test_tracer_gradient_exact_for_linear_and_zero_for_constant"]),
    ("PPM upward mean with the wrong curvature sign",
     "aT + 0.5 * c * (da + a6", "aT + 0.5 * c * (da - a6",
     [T + "test_ppm_column_exact_for_quadratic_under_uniform_advection[0.37-uneven]"]),
    ("PPM upwind cell swapped",
     "const int up = W[i] > 0.0 ? i : i - 1;", "const int up = W[i] > 0.0 ? i - 1 : i;",
     [T + "test_ppm_column_exact_for_quadratic_under_uniform_advection[0.37-uneven]"]),
    ("Perot operator without the edge lengths",
     "{0.0, 0.0, 0.0};\n        for (int j = 0; j < 3; ++j) {\n            int64_t e = g->cell_edges[j * nc + c];\n"
     "            double wgt = g->cell_sign[j * nc + c] * g->edge_length[e] * u[e];",
     "{0.0, 0.0, 0.0};\n        for (int j = 0; j < 3; ++j) {\n            int64_t e = g->cell_edges[j * nc + c];\n"
     "            double wgt = g->cell_sign[j * nc + c] * u[e];",
     [T + "test_perot_exact_for_uniform_vector_on_a_plane"]),
    ("the step's Perot reconstruction without the edge lengths",
     "g->edge_length[e] * u[e];\n                for (int d = 0; d < 3; ++d) v[d] += wgt * (a *",
     "u[e];\n                for (int d = 0; d < 3; ++d) v[d] += wgt * (a *",
     [T + "test_solid_body_rotation_convergence"]),
    ("kinetic energy without the tangential velocity",
     "0.5 * (un * un + ut * ut);", "0.5 * (un * un);",
     [T + "test_vn_tendency_of_sheared_solid_body_rotation"]),
    ("contravariant correction without the tangential slope",
     "AT(m->vnh, i, ne, e) * AT(m->snh, i, ne, e) +", "AT(m->vnh, i, ne, e) * AT(m->snh, i, ne, e) + 0.0 *",
     [T + "test_contravariant_correction_over_linear_terrain"]),
    ("Thomas back substitution with the next row's factor",
     "x[i] = dp[i] - cp[i] * x[i + 1];", "x[i] = dp[i] - cp[i + 1] * x[i + 1];",
     [T + "test_thomas_matches_lapack"]),
    ("mass-flux accumulators summing the substeps instead of averaging them",
     "m->facc[i] += m->flx[i] / nsub;", "m->facc[i] += m->flx[i];",
     [T + "test_flux_accumulators_average_the_substeps"]),
    ("Exner coefficient of the column inverted",
     "B[k] = dt * (rd / cvd) * pi_n[k]", "B[k] = dt * (cvd / rd) * pi_n[k]",
     [T + "test_column_matches_dense_solve_of_implicit_equations"]),
    ("theta_v from the inverse of the linearised state equation",
     "(cvd / rd) * (rt / pi_n[k])", "(rd / cvd) * (rt / pi_n[k])",
     [T + "test_column_matches_dense_solve_of_implicit_equations"]),
    ("sub-diagonal with the level below's Exner coefficient",
     "ta[i - 1] = -ga[i] * B[i - 1] * al[i - 1];", "ta[i - 1] = -ga[i] * B[i] * al[i - 1];",
     [T + "test_column_matches_dense_solve_of_implicit_equations"]),
    ("reference-state buoyancy dropped from the explicit w",
     "(ppn[i - 1] - ppn[i]) / dzh[i] + thph[i] * dref[i];", "(ppn[i - 1] - ppn[i]) / dzh[i];",
     [T + "test_column_matches_dense_solve_of_implicit_equations"]),
    ("ground w set to zero instead of the contravariant correction",
     "wp[N] = wcc[N];", "wp[N] = 0.0;",
     [T + "test_column_matches_dense_solve_of_implicit_equations"]),
    ("pressure gradient without its terrain correction",
     "AT(gp, k, ne, e) = gl - AT(m->sn, k, ne, e) * dz2;", "AT(gp, k, ne, e) = gl;",
     [T + "test_terrain_corrected_gradient_of_height_only_field"]),
    ("corrector weights the other way round",
     "(1.0 - cv) * AT(m->tvn0, k, ne, e) + cv * AT(m->tvn1, k, ne, e)",
     "cv * AT(m->tvn0, k, ne, e) + (1.0 - cv) * AT(m->tvn1, k, ne, e)",
     [T + "test_corrector_weights_the_two_tendencies"]),
    ("corrector's tendencies taken at the old state",
     "vt_phase(m, m->vns, m->ws, m->tvn1, m->tw1, m->wcc1);",
     "vt_phase(m, m->vn, m->w, m->tvn1, m->tw1, m->wcc1);",
     [T + "test_corrector_weights_the_two_tendencies"]),
    ("corrector column's interface density without the predicted state",
     "m->rho_i[i] = 0.5 * (m->rho[i] + m->rhos[i]);", "m->rho_i[i] = m->rho[i];",
     [T + "test_substep_of_a_horizontally_uniform_column"]),
    ("w tendency weights the other way round",
     "m->twm[i] = (1.0 - cv) * m->tw0[i] + cv * m->tw1[i];",
     "m->twm[i] = cv * m->tw0[i] + (1.0 - cv) * m->tw1[i];",
     [T + "test_substep_of_a_horizontally_uniform_column"]),
    ("Exner history from the predicted state",
     "for (int64_t i = 0; i < NC; ++i) m->pi_prev[i] = m->pi[i] - m->pi_ref[i];",
     "for (int64_t i = 0; i < NC; ++i) m->pi_prev[i] = m->pis[i] - m->pi_ref[i];",
     [T + "test_substep_of_a_horizontally_uniform_column"]),
    ("Exner extrapolation with the weights the other way round",
     "m->pix[i] = (1.0 + eps) * pp - eps * m->pi_prev[i];",
     "m->pix[i] = (1.0 - eps) * pp + eps * m->pi_prev[i];",
     [T + "test_substep_equals_its_steps_composed"]),
    ("divergence damping of the old vn instead of the predicted one",
     "or_op_div(g, m->vns + (int64_t)k * ne, m->dvs + (int64_t)k * nc);",
     "or_op_div(g, m->vn + (int64_t)k * ne, m->dvs + (int64_t)k * nc);",
     [T + "test_substep_equals_its_steps_composed"]),
    ("corrector fluxes carried by the predicted vn",
     "flux_phase(m, m->vnn, dt);", "flux_phase(m, m->vns, dt);",
     [T + "test_substep_equals_its_steps_composed"]),
    ("corrector pressure gradient weighted by the old theta_v",
     "0.5 * (AT(m->thvs, k, nc, c1) + AT(m->thvs, k, nc, c2));",
     "0.5 * (AT(m->thv, k, nc, c1) + AT(m->thv, k, nc, c2));",
     [T + "test_substep_equals_its_steps_composed"]),
    ("upwind edge density from the predicted state",
     "or_op_upwind(g, m->rho + oc, m->grad_r + 3 * oc,", "or_op_upwind(g, m->rhos + oc, m->grad_r + 3 * oc,",
     [T + "test_substep_equals_its_steps_composed[upwind]"]),
    ("theta_v's upwind gradient computed from rho",
     "or_op_cell_grad(&m->g, m->thv + (int64_t)k * nc,", "or_op_cell_grad(&m->g, m->rho + (int64_t)k * nc,",
     [T + "test_substep_equals_its_steps_composed[upwind]"]),
    ("diffusion over a substep's dt instead of the step's",
     "if (m->p.smag > 0.0) diffusion_phase(m, dt);", "if (m->p.smag > 0.0) diffusion_phase(m, dts);",
     [T + "test_step_with_every_damping_option_equals_its_parts_composed"]),
    ("diffusion with the corrector's tangential velocity instead of the new vn's",
     "    perot_phase(m, m->vn);\n    for (int k = 0; k < N; ++k) {\n        double *u = m->vn",
     "    for (int k = 0; k < N; ++k) {\n        double *u = m->vn",
     [T + "test_step_with_every_damping_option_equals_its_parts_composed"]),
    ("fourth-order damping added instead of subtracted",
     "if (damp4) v = v - c4 * AT(m->g4, k, ne, e);", "if (damp4) v = v + c4 * AT(m->g4, k, ne, e);",
     [T + "test_step_with_every_damping_option_equals_its_parts_composed"]),
    ("fourth-order damping of the old vn",
     "or_op_graddiv2(g, m->vns + (int64_t)k * ne,", "or_op_graddiv2(g, m->vn + (int64_t)k * ne,",
     [T + "test_step_with_every_damping_option_equals_its_parts_composed"]),
    ("tracer transport from the density at the step's end",
     "r0 = AT(m->rho0, k, nc, c);", "r0 = AT(m->rho, k, nc, c);",
     [T + "test_step_with_tracers_equals_its_parts_composed"]),
    ("vertical tracer pass with the last substep's flux instead of the average",
     "for (int i = 0; i <= N; ++i) c_W[i] = AT(m->wacc, i, nc, c);",
     "for (int i = 0; i <= N; ++i) c_W[i] = AT(m->vflux, i, nc, c);",
     [T + "test_step_with_tracers_equals_its_parts_composed"]),
    ("horizontal tracer update without the density change",
     "AT(qs, k, nc, c) = (r0 * qk[c] - dt * hT) / rsc;", "AT(qs, k, nc, c) = (r0 * qk[c] - dt * hT) / r0;",
     [T + "test_step_with_tracers_equals_its_parts_composed"]),
    ("vertical derivative of the pressure gradient upside down",
     "(AT(px, ka, nc, c) - AT(px, kb, nc, c)) /", "(AT(px, kb, nc, c) - AT(px, ka, nc, c)) /",
     [T + "test_terrain_corrected_gradient_of_height_only_field"]),
]


def _run_mutant(workdir, old, new, pins, threads):
    """Build the oracle with one planted mistake and run the named pins
    against it in a child pytest; returns (build ok, pytest return code, output)."""
    src = open(SRC).read()
    mutant = os.path.join(workdir, "nhdc_oracle.c")
    with open(mutant, "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(workdir, "liboracle_mutant.so")
    r = subprocess.run(OB.command(mutant, so), capture_output=True, text=True)
    if r.returncode != 0:
        return False, r.returncode, r.stderr
    env = dict(os.environ, ORACLE_SO=so, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return True, r.returncode, r.stdout


@pytest.fixture(scope="module")
def mutant_runs(tmp_path_factory):
    """All planted mistakes, built and run a few at a time (each child with
    a share of the cores), so that builds and start-up overlap."""
    from concurrent.futures import ThreadPoolExecutor
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 8))
    workers = max(1, min(4, cores // 2))
    threads = max(1, cores // workers)
    dirs = {m[0]: str(tmp_path_factory.mktemp("mutant")) for m in MUTANTS}
    with ThreadPoolExecutor(max_workers=workers) as ex:
        futs = {m[0]: ex.submit(_run_mutant, dirs[m[0]], m[1], m[2], m[3], threads) for m in MUTANTS}
        return {k: f.result() for k, f in futs.items()}


@pytest.mark.parametrize("what,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(mutant_runs, what, old, new, pins):
    assert open(SRC).read().count(old) == 1, f"the text to change is not unique in the oracle: {old!r}"
    built, rc, out = mutant_runs[what]
    assert built, out
    assert rc == 1 and "failed" in out, (what, out[-2000:])

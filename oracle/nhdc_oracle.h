/*
 * nhdc_oracle.h -- plain, slow FP64 CPU oracle of the nonhydrostatic
 * dynamical-core substep.  TEST INFRASTRUCTURE ONLY: the tests, the smoke
 * check and the CPU baseline of the benchmark call it; the product library
 * never links, loads or includes anything from this directory, and this
 * directory includes nothing of the product.
 *
 * What it computes.  The paper runs ICON's nonhydrostatic atmosphere on the
 * icosahedral-triangular C grid with a terrain-following hybrid height
 * coordinate (Sec. 2), normal velocity on triangle edges (Table 2 counts it as
 * 1.5 variables per cell) and indirect addressing over triangles and their
 * hexagon/pentagon dual (Sec. 3.2).  It prints no equation of the dynamical
 * core, so the discretisation below is this project's own specification of
 * an ICON-style substep (vector-invariant momentum equation, Exner pressure,
 * predictor-corrector horizontal step, vertically implicit w/Exner solve):
 *
 *   operators, per level, sums in slot order; each fixed metric divisor enters
 *   as its reciprocal (1/x, one IEEE quotient) times the sum or difference:
 *     D(F)_c = (1/A_c) sum_j s(c,e_j) l_ej F_ej        G(p)_e = (p_c2 - p_c1) (1/d_e)
 *     T(q)_e = (q_v2 - q_v1) (1/l_e)                   Z(u)_v = (1/A_v) sum_ring sigma d_e u_e
 *     M(q)_c = (1/3) sum_j q_ej   E(p)_e = (p_c1+p_c2)/2   P(p)_v = (1/valence) sum_ring p_c
 *     Perot vector V_c = radial-free part of (1/A_c) sum_j s l u a (x_e - x_c),
 *     vt_e = (V_c1 + V_c2)/2 . t_e
 *   vertical: z_k = (zh_k + zh_k+1)/2, dz_k = zh_k - zh_k+1, linear interpolation
 *     to half levels with g_i = (z_i-1 - zh_i)/(z_i-1 - z_i); boundary half levels
 *     copy the adjacent full level; edge metrics average their two cells;
 *     slopes from cell (and vertex-averaged) heights.
 *   velocity tendencies VT(vn, w) -> (T_vn, T_w, w_cc): kinetic-energy gradient,
 *     (vorticity + Coriolis) x tangential velocity, contravariant vertical
 *     advection of vn; horizontal and vertical advection of w.
 *   one substep: extrapolated Exner perturbation and its terrain-corrected
 *     normal gradient; predictor vn*, fluxes, divergences, column solve; VT on
 *     the predicted state; corrector vn with averaged tendencies and
 *     divergence damping; fluxes; column solve about state n with interface
 *     values averaged between n and *; FP64 mass-flux accumulation.
 *   edge values of rho and theta_v in the fluxes: the centred average E, or
 *     (option) second-order upwind: psi_up + grad(psi)_up . d, where up is
 *     the cell the normal flux comes from, grad the cell's Green-Gauss
 *     gradient (1/A_c) sum_j s l psi_ej n (radial part removed) with psi_ej
 *     interpolated along the dual arc to the edge midpoint, and d the
 *     displacement from the upwind cell centre to the midpoint of the edge
 *     midpoint's back trajectory over the substep, a (x_e - x_up) -
 *     dt/2 (vn n + vt t).
 *   column solve: explicit parts, tridiagonal system in w on interior half
 *     levels (Thomas, no pivoting), then rho, Exner, theta_v updates; theta_v
 *     from the linearised equation of state so that rho*theta_v is in flux form.
 *   damping and diffusion around the substep (each optional, off by default):
 *     fourth-order divergence damping in the corrector, -c4 Abar^2
 *       G(D(G(D(vn*)))) next to the second-order term c Abar G(D(vn*));
 *     a Rayleigh sponge on w in both column solves: the solved w at interior
 *       half level i is multiplied by 1/(1 + dt r_i) before the mass, Exner
 *       and theta_v updates use it (r_i a given rate profile, 1/s);
 *     Smagorinsky diffusion of vn once per step, after the substeps, with the
 *       step's dt: vn += dt K_e L(vn), L(vn) = G(D(vn)) - T(Z(vn)) the C-grid
 *       vector Laplacian, K_e the mean of the two cells' K_c = c_s^2 A_c |Def|
 *       capped at Abar/(25 dt); |Def|^2 = tension^2 + shear^2 of the cell's
 *       velocity-gradient tensor (Green-Gauss over its edges of vn n + vt t,
 *       projected on the cell's tangent plane).
 *   tracer transport (when tracers are set), once per step after the substeps,
 *     with the step's averaged mass fluxes Facc (edges) and Wacc (half levels)
 *     and the density rho^n at the start of the step:
 *     horizontal: T_e = Facc_e r_up, r_up = q_up + grad(q)_up . a (x_e - x_up),
 *       up = c1 if Facc_e >= 0 else c2, grad the Green-Gauss gradient in
 *       difference form (1/A) sum_j s l w_j (q_nb - q_c) n (w_j the arc
 *       fraction from the cell to the edge midpoint), radial part removed;
 *       rho* = rho^n - dt D(Facc)/dz, (rho q)* = rho^n q - dt D(T)/dz;
 *     vertical: piecewise parabolic on q* = (rho q)* / rho*: interface values
 *       by the non-uniform-grid cubic of Colella and Woodward (1984) at
 *       interfaces 2..N-2, linear next to the lid and the ground; flux
 *       Wacc times the parabola's mean over the swept fraction
 *       c = |Wacc| dt/(rho* dz) of the upwind cell (c capped at 1);
 *       q^{n+1} = ((rho q)* - dt dG/dz) / (rho* - dt dWacc/dz).
 *
 * Every array is FP64, level-major [k][entity]; connectivity slot-major.
 * Built with -O2 -ffp-contract=off (no fused multiply-add), OpenMP over
 * entities within each phase only; results do not depend on thread count.
 */
#ifndef NHDC_ORACLE_H
#define NHDC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_LEV 512

typedef struct or_grid {
    int64_t nc, ne, nv;
    double radius;
    const int32_t *cell_edges, *cell_verts, *cell_cells; /* [3][nc] */
    const int8_t *cell_sign;                             /* [3][nc] */
    const int32_t *edge_cells, *edge_verts;              /* [2][ne] */
    const int32_t *vert_edges, *vert_cells;              /* [6][nv] */
    const int8_t *vert_sign;                             /* [6][nv] */
    const int32_t *vert_valence;                         /* [nv] */
    const double *cell_x, *cell_area;                    /* [3][nc], [nc] */
    const double *edge_x, *edge_normal, *edge_tangent;   /* [3][ne] */
    const double *edge_length, *dual_length;             /* [ne] */
    const double *dual_frac;  /* [ne] the edge midpoint's position along the dual arc c1 -> c2 */
    const double *vert_x, *vert_area;                    /* [3][nv], [nv] */
} or_grid;

typedef struct or_params {
    double radius, omega, grav, rd, cpd, p00;
    double beta;      /* implicit weight of the vertical solve */
    double wgt_corr;  /* corrector weight of the new tendency */
    double extrap;    /* Exner-perturbation extrapolation factor */
    double div_damp;  /* divergence damping coefficient */
    int upwind;       /* edge values of rho and theta_v in the fluxes: 0 centred average,
                         1 second-order upwind (cell gradient at the upwind cell, evaluated
                         at the back-trajectory midpoint of the edge) */
    double div_damp4; /* fourth-order divergence damping coefficient (times Abar^2); 0 off */
    double smag;      /* Smagorinsky constant c_s of the horizontal diffusion of vn; 0 off */
    const double *w_damp; /* [N+1] Rayleigh damping rate of w per half level [1/s]; NULL off */
} or_params;

typedef struct or_model or_model;

/* The model keeps pointers to the grid arrays (caller keeps them alive) and
 * copies zh [N+1][nc], pi_ref and theta_ref [N][nc]. NULL on bad input. */
or_model *or_create(const or_grid *g, int nlev, const double *zh, const double *pi_ref,
                    const double *theta_ref, const or_params *p);
void or_free(or_model *m);
/* pi_prev may be NULL: it is then pi - pi_ref (first extrapolation = identity). */
int or_set_state(or_model *m, const double *vn, const double *w, const double *rho,
                 const double *pi, const double *theta_v, const double *pi_prev);
int or_get_state(const or_model *m, double *vn, double *w, double *rho, double *pi,
                 double *theta_v, double *pi_prev);
int or_get_flux(const or_model *m, double *facc, double *wacc);
/* tracers: nt mixing ratios [nt][N][nc] (copied; nt = 0 removes them); they
 * are transported at the end of every step */
int or_tracers_set(or_model *m, int nt, const double *q);
int or_tracers_get(const or_model *m, double *q);
/* step(dt, nsub): nsub substeps of dt/nsub; the flux accumulators are zeroed first. */
int or_step(or_model *m, double dt, int nsub);
/* velocity tendencies of (vn, w) with the model's metrics; outputs [N][ne], [N+1][nc] x2.
 * vt_out (optional, [N][ne]) receives the reconstructed tangential velocity. */
int or_vt(or_model *m, const double *vn, const double *w, double *tvn, double *tw, double *wcc,
          double *vt_out);
/* terrain-corrected normal gradient of a full-level cell field [N][nc] -> [N][ne] */
int or_pgrad(or_model *m, const double *p, double *gp);
/* dry mass sum_c,k A_c dz_c,k rho_c,k and sum A dz rho theta_v (Kahan, fixed order) */
int or_diag(const or_model *m, double *mass, double *rho_theta);

/* Single-level operators on a grid (arrays of one level). */
void or_op_div(const or_grid *g, const double *f_e, double *out_c);
void or_op_grad(const or_grid *g, const double *p_c, double *out_e);
void or_op_tgrad(const or_grid *g, const double *q_v, double *out_e);
void or_op_curl(const or_grid *g, const double *u_e, double *out_v);
void or_op_cell_avg(const or_grid *g, const double *q_e, double *out_c);
void or_op_vert_avg(const or_grid *g, const double *p_c, double *out_v);
/* horizontal gradient of a cell field: Green-Gauss over the cell's edges
 * with edge values interpolated along the dual arc to the edge midpoint,
 * p_c1 + f (p_c2 - p_c1), minus its component along the cell's radial unit
 * vector radial_c [3][nc] (the model passes the unit cell centres):
 * out [3][nc], per metre */
void or_op_cell_grad(const or_grid *g, const double *p_c, const double *radial_c, double *out);
/* second-order upwind edge values of a cell field with its gradient [3][nc]:
 * psi_up + grad_up . (a (x_e - x_up) - dt/2 (u n + vt t)), up = c1 if u >= 0
 * else c2; u, vt the normal and tangential velocity [ne]; out [ne] */
void or_op_upwind(const or_grid *g, const double *p_c, const double *grad, const double *u,
                  const double *vt, double dt, double *out_e);
/* the C-grid vector Laplacian G(D(u)) - T(Z(u)) of an edge field [ne] -> [ne] */
void or_op_vector_laplacian(const or_grid *g, const double *u, double *out_e);
/* the fourth-order divergence operator G(D(G(D(u)))) of an edge field [ne] -> [ne] */
void or_op_graddiv2(const or_grid *g, const double *u, double *out_e);
/* horizontal deformation magnitude per cell (tension^2 + shear^2)^(1/2) of the
 * edge velocities u n + vt t: the Green-Gauss tensor (1/A) sum_j s l (u n + vt t) n^T,
 * projected on the cell's tangent plane by P = I - x x^T (x the unit cell
 * centre), |Def|^2 = 2 |sym(P G P)|^2 - tr(P G P)^2.  Needs edge_normal. */
void or_op_deformation(const or_grid *g, const double *u, const double *vt, double *out_c);
/* difference-form Green-Gauss gradient of a cell field (tracer transport),
 * radial part removed: out [3][nc]; needs edge_normal and dual_frac */
void or_op_tracer_grad(const or_grid *g, const double *q, double *out);
/* linear reconstruction of a cell field toward each of the cell's edges:
 * out[j][c] = q_c + grad_c . a (x_e(j) - x_c) */
void or_op_tracer_recon(const or_grid *g, const double *q, const double *grad, double *out);
/* PPM interface values a[N+1] of a column of cell means q[N] with thicknesses dz[N] */
int or_ppm_faces(int nlev, const double *dz, const double *q, double *a);
/* vertical PPM transport of one column over dt: density rho[N], mass flux
 * W[N+1] (upward positive, 0 at lid and ground), mixing ratio q[N] ->
 * q_out[N] and (optional) rho_out[N] */
int or_ppm_column(int nlev, double dt, const double *dz, const double *rho, const double *W,
                  const double *q, double *q_out, double *rho_out);
/* Perot reconstruction with explicit positions [3][n] (metres) and cell radial
 * unit vectors: out_vc [3][nc] cell vectors, out_vt [ne] tangential velocity. */
void or_op_perot(const or_grid *g, const double *pos_c, const double *pos_e,
                 const double *radial_c, const double *u_e, double *out_vc, double *out_vt);

/* Tridiagonal solve without pivoting: a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = r[i]. */
int or_thomas(int n, const double *a, const double *b, const double *c, const double *r,
              double *x);

/* One column of the vertically implicit solve (all arrays of this column,
 * contiguous, top to bottom).  Inputs: half-level heights zh[N+1], reference
 * pi_ref/theta_ref[N]; linearisation state pi_n, rho_n, thv_n[N]; interface
 * state rho_i, thv_i[N]; w_n[N+1]; w tendency tw[N+1]; contravariant
 * correction wcc[N+1]; horizontal divergences div_rho, div_th[N].  Outputs
 * w[N+1], rho, pi, thv[N] and the vertical mass flux at half levels vflux[N+1]. */
int or_column(int nlev, double dt, const or_params *p, const double *zh, const double *pi_ref,
              const double *theta_ref, const double *pi_n, const double *rho_n,
              const double *thv_n, const double *rho_i, const double *thv_i, const double *w_n,
              const double *tw, const double *wcc, const double *div_rho, const double *div_th,
              double *w_out, double *rho_out, double *pi_out, double *thv_out, double *vflux);

#ifdef __cplusplus
}
#endif
#endif

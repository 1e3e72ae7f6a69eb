/* nhcase.h -- native helpers of the synthetic case generator (host only).
 * Arrays are level-major [k][i]; connectivity slot-major, as in nhgrid.h.
 * Every function returns 0 on success, -1 on a bad argument, and
 * nhcase_columns returns -2 if a column's balance iteration did not converge. */
#ifndef NHCASE_H
#define NHCASE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nhcase_column_args {
    int64_t n_cells;
    int32_t n_lev;          /* N full levels; N+1 half levels */
    int32_t balanced;       /* 1: discrete hydrostatic balance; 0: analytic profile at full levels */
    const double *zeta;     /* [N+1] flat-terrain half-level heights, top to bottom */
    const double *h;        /* [n_cells] surface height */
    double z_flat;          /* levels are flat above this height */
    double decay_scale;     /* sinh decay scale of the terrain signal */
    double grav, cpd, rd, p00;
    double t0;              /* isothermal background temperature */
    double t_ref_top, t_ref_delta, t_ref_scale; /* T_ref(z) = top + delta*exp(-z/scale) */
} nhcase_column_args;

typedef struct nhcase_grid_args {
    int64_t n_cells, n_edges;
    double radius;
    const int32_t *cell_edges;  /* [3][n_cells] */
    const int8_t *cell_sign;    /* [3][n_cells] */
    const int32_t *edge_cells;  /* [2][n_edges] */
    const double *cell_x;       /* [3][n_cells] */
    const double *cell_area;    /* [n_cells] */
    const double *edge_x;       /* [3][n_edges] */
    const double *edge_normal;  /* [3][n_edges] */
    const double *edge_length;  /* [n_edges] */
} nhcase_grid_args;

int nhcase_terrain(const double *cell_x, int64_t n, int lmax, const double *coef, double *out);
int nhcase_columns(const nhcase_column_args *a, double *zh, double *pi_ref, double *theta_ref,
                   double *pi, double *theta_v, double *rho);
int nhcase_smooth_noise(const nhcase_grid_args *g, int n_lev, int passes, double *x);

#ifdef __cplusplus
}
#endif
#endif

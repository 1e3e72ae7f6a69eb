/*
 * nhdc_oracle.c -- plain FP64 CPU oracle of the dynamical-core substep.
 * TEST INFRASTRUCTURE ONLY (see nhdc_oracle.h for what it computes and who
 * may call it).  Plain loops, one formula per statement, sums in slot order,
 * no fused multiply-add (built with -ffp-contract=off), OpenMP over entities.
 * Operators scale by the reciprocal of each fixed metric length, area,
 * valence or count (1/d_e, 1/l_e, 1/A_c, 1/A_v, 1/valence, 1/3), each the
 * IEEE quotient 1/x: the definitions read (1/A) times a sum and a difference
 * times 1/length, and these metric factors are constant through a run.
 *
 * Index conventions: full level k = 0..N-1 top to bottom; half level i =
 * 0..N, half level i is the top interface of full level i, i = N the ground.
 */
#include "nhdc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct or_model {
    or_grid g;
    or_params p;
    int N;
    /* metrics */
    double *zh, *pi_ref, *theta_ref; /* [N+1][nc], [N][nc] x2 */
    double *z, *dz;                  /* [N][nc] */
    double *dzh, *gw, *dref;         /* [N+1][nc], interior half levels only */
    double *dz_e;                    /* [N][ne] */
    double *gw_e;                    /* [N+1][ne] */
    double *sn;                      /* [N][ne] slope of full levels */
    double *snh, *sth;               /* [N+1][ne] normal / tangential slope of half levels */
    double *fe;                      /* [ne] Coriolis parameter */
    /* state */
    double *vn, *w, *rho, *pi, *thv, *pi_prev;
    double *facc, *wacc;
    /* work */
    double *vt, *vnh, *vth, *kc, *zv, *omega, *wv, *pcx, *pcy, *pcz, *ke, *ae;
    double *tvn0, *tw0, *wcc0, *tvn1, *tw1, *wcc1;
    double *gp, *dpz, *pix, *the, *rhoe, *flx, *hfl, *divr, *divt, *vns, *dvs;
    double *ws, *rhos, *pis, *thvs, *vnn, *vflux, *rho_i, *thv_i, *twm;
    double *grad_r, *grad_t; /* [N][3][nc] cell gradients of rho and theta_v (upwind option) */
    double *rhoe_u, *the_u;  /* [N][ne] upwind edge values (upwind option) */
    double *g4;              /* [N][ne] G(D(G(D(vn*)))) (fourth-order divergence damping) */
    double *kh, *lap;        /* [N][nc] Smagorinsky K_c, [N][ne] vector Laplacian of vn */
    /* tracers: nt mixing ratios [nt][N][nc], carried by the step's averaged mass fluxes */
    int nt;
    double *q, *rho0;        /* tracers; density at the start of the step [N][nc] */
};

#define AT(a, k, n, i) ((a)[(int64_t)(k) * (n) + (i)])

static double *alloc(int64_t n) { return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

/* ------------------------------------------------------------------------ */
/* single-level operators                                                    */
/* ------------------------------------------------------------------------ */

void or_op_div(const or_grid *g, const double *f, double *out) {
    const int64_t nc = g->nc;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j) {
            int64_t e = g->cell_edges[j * nc + c];
            s += g->cell_sign[j * nc + c] * g->edge_length[e] * f[e];
        }
        out[c] = s * (1.0 / g->cell_area[c]);
    }
}

void or_op_grad(const or_grid *g, const double *p, double *out) {
    const int64_t ne = g->ne;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e)
        out[e] = (p[g->edge_cells[ne + e]] - p[g->edge_cells[e]]) * (1.0 / g->dual_length[e]);
}

void or_op_tgrad(const or_grid *g, const double *q, double *out) {
    const int64_t ne = g->ne;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e)
        out[e] = (q[g->edge_verts[ne + e]] - q[g->edge_verts[e]]) * (1.0 / g->edge_length[e]);
}

void or_op_curl(const or_grid *g, const double *u, double *out) {
    const int64_t nv = g->nv;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int j = 0; j < g->vert_valence[v]; ++j) {
            int64_t e = g->vert_edges[j * nv + v];
            s += g->vert_sign[j * nv + v] * g->dual_length[e] * u[e];
        }
        out[v] = s * (1.0 / g->vert_area[v]);
    }
}

void or_op_cell_avg(const or_grid *g, const double *q, double *out) {
    const int64_t nc = g->nc;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j) s += q[g->cell_edges[j * nc + c]];
        out[c] = s * (1.0 / 3.0);
    }
}

void or_op_vert_avg(const or_grid *g, const double *p, double *out) {
    const int64_t nv = g->nv;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int j = 0; j < g->vert_valence[v]; ++j) s += p[g->vert_cells[j * nv + v]];
        out[v] = s * (1.0 / g->vert_valence[v]);
    }
}

void or_op_cell_grad(const or_grid *g, const double *p, const double *rc, double *out) {
    const int64_t nc = g->nc, ne = g->ne;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < 3; ++j) {
            int64_t e = g->cell_edges[j * nc + c];
            double p1 = p[g->edge_cells[e]], p2 = p[g->edge_cells[ne + e]];
            double pe = p1 + g->dual_frac[e] * (p2 - p1);
            double wgt = g->cell_sign[j * nc + c] * g->edge_length[e] * pe;
            for (int d = 0; d < 3; ++d) v[d] += wgt * g->edge_normal[d * ne + e];
        }
        for (int d = 0; d < 3; ++d) v[d] = v[d] * (1.0 / g->cell_area[c]);
        double r = v[0] * rc[c] + v[1] * rc[nc + c] + v[2] * rc[2 * nc + c];
        for (int d = 0; d < 3; ++d) out[d * nc + c] = v[d] - r * rc[d * nc + c];
    }
}

void or_op_upwind(const or_grid *g, const double *p, const double *grad, const double *u,
                  const double *vt, double dt, double *out) {
    const int64_t nc = g->nc, ne = g->ne;
    const double a = g->radius;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        int64_t up = u[e] >= 0.0 ? g->edge_cells[e] : g->edge_cells[ne + e];
        double d[3];
        for (int x = 0; x < 3; ++x)
            d[x] = a * (g->edge_x[x * ne + e] - g->cell_x[x * nc + up]) -
                   0.5 * dt * (u[e] * g->edge_normal[x * ne + e] + vt[e] * g->edge_tangent[x * ne + e]);
        out[e] = p[up] + (grad[up] * d[0] + grad[nc + up] * d[1] + grad[2 * nc + up] * d[2]);
    }
}

void or_op_perot(const or_grid *g, const double *pc, const double *pe, const double *rc,
                 const double *u, double *vc, double *vt) {
    const int64_t nc = g->nc, ne = g->ne;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < 3; ++j) {
            int64_t e = g->cell_edges[j * nc + c];
            double wgt = g->cell_sign[j * nc + c] * g->edge_length[e] * u[e];
            for (int d = 0; d < 3; ++d) v[d] += wgt * (pe[d * ne + e] - pc[d * nc + c]);
        }
        for (int d = 0; d < 3; ++d) v[d] = v[d] * (1.0 / g->cell_area[c]);
        double r = v[0] * rc[c] + v[1] * rc[nc + c] + v[2] * rc[2 * nc + c];
        for (int d = 0; d < 3; ++d) vc[d * nc + c] = v[d] - r * rc[d * nc + c];
    }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
        double s = 0.0;
        for (int d = 0; d < 3; ++d)
            s += 0.5 * (vc[d * nc + c1] + vc[d * nc + c2]) * g->edge_tangent[d * ne + e];
        vt[e] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* model set-up: metrics derived from the half-level heights                  */
/* ------------------------------------------------------------------------ */

void or_op_vector_laplacian(const or_grid *g, const double *u, double *out) {
    const int64_t nc = g->nc, ne = g->ne, nv = g->nv;
    double *d = alloc(nc), *z = alloc(nv), *gd = alloc(ne), *tz = alloc(ne);
    or_op_div(g, u, d);
    or_op_curl(g, u, z);
    or_op_grad(g, d, gd);
    or_op_tgrad(g, z, tz);
    for (int64_t e = 0; e < ne; ++e) out[e] = gd[e] - tz[e];
    free(d);
    free(z);
    free(gd);
    free(tz);
}

void or_op_graddiv2(const or_grid *g, const double *u, double *out) {
    const int64_t nc = g->nc, ne = g->ne;
    double *d = alloc(nc), *gd = alloc(ne), *d2 = alloc(nc);
    or_op_div(g, u, d);
    or_op_grad(g, d, gd);
    or_op_div(g, gd, d2);
    or_op_grad(g, d2, out);
    free(d);
    free(gd);
    free(d2);
}

void or_op_deformation(const or_grid *g, const double *u, const double *vt, double *out) {
    const int64_t nc = g->nc, ne = g->ne;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        /* Green-Gauss velocity-gradient tensor G[a][b] = (1/A) sum_j s l V_a n_b */
        double G[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        for (int j = 0; j < 3; ++j) {
            int64_t e = g->cell_edges[j * nc + c];
            double sl = g->cell_sign[j * nc + c] * g->edge_length[e];
            for (int a = 0; a < 3; ++a) {
                double va = u[e] * g->edge_normal[a * ne + e] + vt[e] * g->edge_tangent[a * ne + e];
                double wa = sl * va;
                for (int b = 0; b < 3; ++b) G[a][b] += wa * g->edge_normal[b * ne + e];
            }
        }
        double ia = 1.0 / g->cell_area[c];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) G[a][b] = G[a][b] * ia;
        /* projection on the tangent plane: M = P G P, P = I - x x^T */
        const double x[3] = {g->cell_x[c], g->cell_x[nc + c], g->cell_x[2 * nc + c]};
        double q[3], H[3][3], r[3], M[3][3];
        for (int b = 0; b < 3; ++b) q[b] = x[0] * G[0][b] + x[1] * G[1][b] + x[2] * G[2][b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) H[a][b] = G[a][b] - x[a] * q[b];
        for (int a = 0; a < 3; ++a) r[a] = H[a][0] * x[0] + H[a][1] * x[1] + H[a][2] * x[2];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[a][b] = H[a][b] - r[a] * x[b];
        /* tension^2 + shear^2 = 2 |sym M|^2 - (tr M)^2 */
        double tr = M[0][0] + M[1][1] + M[2][2];
        double s2 = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double sab = 0.5 * (M[a][b] + M[b][a]);
                s2 += sab * sab;
            }
        double d2 = 2.0 * s2 - tr * tr;
        out[c] = d2 > 0.0 ? sqrt(d2) : 0.0;
    }
}

void or_op_tracer_grad(const or_grid *g, const double *q, double *out) {
    const int64_t nc = g->nc;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < 3; ++j) {
            int64_t e = g->cell_edges[j * nc + c];
            int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[g->ne + e];
            int64_t nb = c1 == c ? c2 : c1;
            /* the edge value's offset from this cell's value along the dual arc */
            double wgt = c1 == c ? g->dual_frac[e] : 1.0 - g->dual_frac[e];
            double dq = wgt * (q[nb] - q[c]);
            double sl = g->cell_sign[j * nc + c] * g->edge_length[e];
            for (int d = 0; d < 3; ++d) v[d] += (sl * dq) * g->edge_normal[d * g->ne + e];
        }
        double ia = 1.0 / g->cell_area[c];
        for (int d = 0; d < 3; ++d) v[d] = v[d] * ia;
        const double x[3] = {g->cell_x[c], g->cell_x[nc + c], g->cell_x[2 * nc + c]};
        double r = v[0] * x[0] + v[1] * x[1] + v[2] * x[2];
        for (int d = 0; d < 3; ++d) out[d * nc + c] = v[d] - r * x[d];
    }
}

void or_op_tracer_recon(const or_grid *g, const double *q, const double *grad, double *out) {
    const int64_t nc = g->nc, ne = g->ne;
    const double a = g->radius;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c)
        for (int j = 0; j < 3; ++j) {
            int64_t e = g->cell_edges[j * nc + c];
            double s = 0.0;
            for (int d = 0; d < 3; ++d)
                s += grad[d * nc + c] * (a * (g->edge_x[d * ne + e] - g->cell_x[d * nc + c]));
            out[j * nc + c] = q[c] + s;
        }
}

int or_ppm_faces(int N, const double *dz, const double *q, double *a) {
    if (N < 2) return -1;
    a[0] = q[0];
    a[N] = q[N - 1];
    /* the two interfaces next to the lid and the ground: linear between centres */
    for (int i = 1; i < N; ++i)
        if (i == 1 || i == N - 1 || N < 4)
            a[i] = q[i - 1] + (dz[i - 1] / (dz[i - 1] + dz[i])) * (q[i] - q[i - 1]);
    /* interior interfaces: the cubic through four cell means on a non-uniform
       grid (Colella and Woodward 1984, their interface and mean-slope formulas) */
    for (int i = 2; i <= N - 2 && N >= 4; ++i) {
        const int j = i - 1; /* interface between cells j and j+1 */
        const double d0 = dz[j - 1], d1 = dz[j], d2 = dz[j + 1], d3 = dz[j + 2];
        const double q0 = q[j - 1], q1 = q[j], q2 = q[j + 1], q3 = q[j + 2];
        /* mean slopes of cells j and j+1 */
        double sj = d1 / (d0 + d1 + d2) *
                    ((2.0 * d0 + d1) / (d2 + d1) * (q2 - q1) + (d1 + 2.0 * d2) / (d0 + d1) * (q1 - q0));
        double sk = d2 / (d1 + d2 + d3) *
                    ((2.0 * d1 + d2) / (d3 + d2) * (q3 - q2) + (d2 + 2.0 * d3) / (d1 + d2) * (q2 - q1));
        double lin = q1 + d1 / (d1 + d2) * (q2 - q1);
        double t1 = 2.0 * d2 * d1 / (d1 + d2) * ((d0 + d1) / (2.0 * d1 + d2) - (d3 + d2) / (2.0 * d2 + d1)) *
                    (q2 - q1);
        double t2 = d1 * (d0 + d1) / (2.0 * d1 + d2) * sk;
        double t3 = d2 * (d2 + d3) / (d1 + 2.0 * d2) * sj;
        a[i] = lin + (t1 - t2 + t3) / (d0 + d1 + d2 + d3);
    }
    return 0;
}

int or_ppm_column(int N, double dt, const double *dz, const double *rho, const double *W,
                  const double *q, double *q_out, double *rho_out) {
    if (N < 2 || N > OR_MAX_LEV) return -1;
    double a[OR_MAX_LEV + 1], G[OR_MAX_LEV + 1];
    or_ppm_faces(N, dz, q, a);
    G[0] = G[N] = 0.0;
    for (int i = 1; i < N; ++i) {
        /* upward flux (W > 0) sweeps the top of cell i, downward the bottom of cell i-1 */
        const int up = W[i] > 0.0 ? i : i - 1;
        const double aT = a[up], aB = a[up + 1];
        const double da = aB - aT, a6 = 6.0 * (q[up] - 0.5 * (aT + aB));
        double c = fabs(W[i]) * dt / (rho[up] * dz[up]);
        c = c < 1.0 ? c : 1.0;
        const double mean = W[i] > 0.0 ? aT + 0.5 * c * (da + a6 * (1.0 - (2.0 / 3.0) * c))
                                       : aB - 0.5 * c * (da - a6 * (1.0 - (2.0 / 3.0) * c));
        G[i] = W[i] * mean;
    }
    for (int k = 0; k < N; ++k) {
        double rq = rho[k] * q[k] - dt * (G[k] - G[k + 1]) / dz[k];
        double rn = rho[k] - dt * (W[k] - W[k + 1]) / dz[k];
        q_out[k] = rq / rn;
        if (rho_out) rho_out[k] = rn;
    }
    return 0;
}

or_model *or_create(const or_grid *g, int N, const double *zh, const double *pi_ref,
                    const double *theta_ref, const or_params *p) {
    if (!g || !zh || !pi_ref || !theta_ref || !p || N < 2 || N > OR_MAX_LEV) return NULL;
    if ((p->upwind || p->smag > 0.0) && !g->edge_normal) return NULL;
    or_model *m = (or_model *)calloc(1, sizeof(or_model));
    if (!m) return NULL;
    m->g = *g;
    m->p = *p;
    m->N = N;
    const int64_t nc = g->nc, ne = g->ne, nv = g->nv;
    const int64_t NC = (int64_t)N * nc, NC1 = (int64_t)(N + 1) * nc;
    const int64_t NE = (int64_t)N * ne, NE1 = (int64_t)(N + 1) * ne;
    const int64_t NV = (int64_t)N * nv, NV1 = (int64_t)(N + 1) * nv;
    double **cells[] = {&m->pi_ref, &m->theta_ref, &m->z, &m->dz, &m->rho, &m->pi, &m->thv,
                        &m->pi_prev, &m->kc, &m->dpz, &m->pix, &m->divr, &m->divt, &m->dvs,
                        &m->rhos, &m->pis, &m->thvs, &m->rho_i, &m->thv_i, &m->pcx, &m->pcy,
                        &m->pcz};
    double **cells1[] = {&m->zh, &m->dzh, &m->gw, &m->dref, &m->w, &m->wacc, &m->omega,
                         &m->tw0, &m->wcc0, &m->tw1, &m->wcc1, &m->ws, &m->vflux, &m->twm};
    double **edges[] = {&m->dz_e, &m->sn, &m->vn, &m->facc, &m->vt, &m->ke, &m->tvn0, &m->tvn1,
                        &m->gp, &m->the, &m->rhoe, &m->flx, &m->hfl, &m->vns, &m->vnn};
    double **edges1[] = {&m->gw_e, &m->snh, &m->sth, &m->vnh, &m->vth, &m->ae};
    int ok = 1;
    for (size_t i = 0; i < sizeof(cells) / sizeof(*cells); ++i) ok &= (*cells[i] = alloc(NC)) != NULL;
    for (size_t i = 0; i < sizeof(cells1) / sizeof(*cells1); ++i) ok &= (*cells1[i] = alloc(NC1)) != NULL;
    for (size_t i = 0; i < sizeof(edges) / sizeof(*edges); ++i) ok &= (*edges[i] = alloc(NE)) != NULL;
    for (size_t i = 0; i < sizeof(edges1) / sizeof(*edges1); ++i) ok &= (*edges1[i] = alloc(NE1)) != NULL;
    ok &= (m->zv = alloc(NV)) != NULL;
    ok &= (m->wv = alloc(NV1)) != NULL;
    ok &= (m->fe = alloc(ne)) != NULL;
    if (p->upwind) {
        ok &= (m->grad_r = alloc(3 * NC)) != NULL;
        ok &= (m->grad_t = alloc(3 * NC)) != NULL;
        ok &= (m->rhoe_u = alloc(NE)) != NULL;
        ok &= (m->the_u = alloc(NE)) != NULL;
    }
    if (p->div_damp4 != 0.0) ok &= (m->g4 = alloc(NE)) != NULL;
    if (p->smag > 0.0) {
        ok &= (m->kh = alloc(NC)) != NULL;
        ok &= (m->lap = alloc(NE)) != NULL;
    }
    if (!ok) {
        or_free(m);
        return NULL;
    }
    memcpy(m->zh, zh, sizeof(double) * NC1);
    memcpy(m->pi_ref, pi_ref, sizeof(double) * NC);
    memcpy(m->theta_ref, theta_ref, sizeof(double) * NC);

    /* cell metrics */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        for (int k = 0; k < N; ++k) {
            AT(m->z, k, nc, c) = 0.5 * (AT(m->zh, k, nc, c) + AT(m->zh, k + 1, nc, c));
            AT(m->dz, k, nc, c) = AT(m->zh, k, nc, c) - AT(m->zh, k + 1, nc, c);
        }
        for (int i = 1; i < N; ++i) {
            double za = AT(m->z, i - 1, nc, c), zb = AT(m->z, i, nc, c);
            AT(m->dzh, i, nc, c) = za - zb;
            AT(m->gw, i, nc, c) = (za - AT(m->zh, i, nc, c)) / (za - zb);
            double g = AT(m->gw, i, nc, c);
            double threfh = g * AT(m->theta_ref, i, nc, c) + (1.0 - g) * AT(m->theta_ref, i - 1, nc, c);
            AT(m->dref, i, nc, c) = -p->grav / (p->cpd * threfh);
        }
    }
    /* vertex-averaged half-level heights (temporary, in wv) */
    for (int i = 0; i <= N; ++i) or_op_vert_avg(g, m->zh + (int64_t)i * nc, m->wv + (int64_t)i * nv);
    /* edge metrics */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
        int64_t v1 = g->edge_verts[e], v2 = g->edge_verts[ne + e];
        for (int k = 0; k < N; ++k) {
            AT(m->dz_e, k, ne, e) = 0.5 * (AT(m->dz, k, nc, c1) + AT(m->dz, k, nc, c2));
            AT(m->sn, k, ne, e) = (AT(m->z, k, nc, c2) - AT(m->z, k, nc, c1)) * (1.0 / g->dual_length[e]);
        }
        for (int i = 0; i <= N; ++i) {
            if (i > 0 && i < N) AT(m->gw_e, i, ne, e) = 0.5 * (AT(m->gw, i, nc, c1) + AT(m->gw, i, nc, c2));
            AT(m->snh, i, ne, e) = (AT(m->zh, i, nc, c2) - AT(m->zh, i, nc, c1)) * (1.0 / g->dual_length[e]);
            AT(m->sth, i, ne, e) = (AT(m->wv, i, nv, v2) - AT(m->wv, i, nv, v1)) * (1.0 / g->edge_length[e]);
        }
        m->fe[e] = 2.0 * p->omega * g->edge_x[2 * ne + e];
    }
    memset(m->wv, 0, sizeof(double) * NV1);
    return m;
}

void or_free(or_model *m) {
    if (!m) return;
    double *all[] = {m->zh, m->pi_ref, m->theta_ref, m->z, m->dz, m->dzh, m->gw, m->dref,
                     m->dz_e, m->gw_e, m->sn, m->snh, m->sth, m->fe, m->vn, m->w, m->rho, m->pi,
                     m->thv, m->pi_prev, m->facc, m->wacc, m->vt, m->vnh, m->vth, m->kc, m->zv,
                     m->omega, m->wv, m->pcx, m->pcy, m->pcz, m->ke, m->ae, m->tvn0, m->tw0,
                     m->wcc0, m->tvn1, m->tw1, m->wcc1, m->gp, m->dpz, m->pix, m->the, m->rhoe,
                     m->flx, m->hfl, m->divr, m->divt, m->vns, m->dvs, m->ws, m->rhos, m->pis,
                     m->thvs, m->vnn, m->vflux, m->rho_i, m->thv_i, m->twm, m->grad_r,
                     m->grad_t, m->rhoe_u, m->the_u, m->g4, m->kh, m->lap, m->q, m->rho0};
    for (size_t i = 0; i < sizeof(all) / sizeof(*all); ++i) free(all[i]);
    free(m);
}

int or_set_state(or_model *m, const double *vn, const double *w, const double *rho,
                 const double *pi, const double *thv, const double *pi_prev) {
    if (!m || !vn || !w || !rho || !pi || !thv) return -1;
    const int64_t nc = m->g.nc, ne = m->g.ne, N = m->N;
    memcpy(m->vn, vn, sizeof(double) * N * ne);
    memcpy(m->w, w, sizeof(double) * (N + 1) * nc);
    memcpy(m->rho, rho, sizeof(double) * N * nc);
    memcpy(m->pi, pi, sizeof(double) * N * nc);
    memcpy(m->thv, thv, sizeof(double) * N * nc);
    if (pi_prev) memcpy(m->pi_prev, pi_prev, sizeof(double) * N * nc);
    else
        for (int64_t i = 0; i < N * nc; ++i) m->pi_prev[i] = m->pi[i] - m->pi_ref[i];
    memset(m->facc, 0, sizeof(double) * N * ne);
    memset(m->wacc, 0, sizeof(double) * (N + 1) * nc);
    return 0;
}

int or_get_state(const or_model *m, double *vn, double *w, double *rho, double *pi, double *thv,
                 double *pi_prev) {
    if (!m) return -1;
    const int64_t nc = m->g.nc, ne = m->g.ne, N = m->N;
    if (vn) memcpy(vn, m->vn, sizeof(double) * N * ne);
    if (w) memcpy(w, m->w, sizeof(double) * (N + 1) * nc);
    if (rho) memcpy(rho, m->rho, sizeof(double) * N * nc);
    if (pi) memcpy(pi, m->pi, sizeof(double) * N * nc);
    if (thv) memcpy(thv, m->thv, sizeof(double) * N * nc);
    if (pi_prev) memcpy(pi_prev, m->pi_prev, sizeof(double) * N * nc);
    return 0;
}

int or_get_flux(const or_model *m, double *facc, double *wacc) {
    if (!m) return -1;
    const int64_t nc = m->g.nc, ne = m->g.ne, N = m->N;
    if (facc) memcpy(facc, m->facc, sizeof(double) * N * ne);
    if (wacc) memcpy(wacc, m->wacc, sizeof(double) * (N + 1) * nc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* velocity tendencies                                                       */
/* ------------------------------------------------------------------------ */

/* tangential velocity m->vt from the Perot reconstruction, level by level */
static void perot_phase(or_model *m, const double *vn) {
    const or_grid *g = &m->g;
    const int64_t nc = g->nc, ne = g->ne;
    const int N = m->N;
    const double a = g->radius;
    for (int k = 0; k < N; ++k) {
        const double *u = vn + (int64_t)k * ne;
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            double v[3] = {0.0, 0.0, 0.0};
            const double xc[3] = {g->cell_x[c], g->cell_x[nc + c], g->cell_x[2 * nc + c]};
            for (int j = 0; j < 3; ++j) {
                int64_t e = g->cell_edges[j * nc + c];
                double wgt = g->cell_sign[j * nc + c] * g->edge_length[e] * u[e];
                for (int d = 0; d < 3; ++d) v[d] += wgt * (a * (g->edge_x[d * ne + e] - xc[d]));
            }
            for (int d = 0; d < 3; ++d) v[d] = v[d] * (1.0 / g->cell_area[c]);
            double r = v[0] * xc[0] + v[1] * xc[1] + v[2] * xc[2];
            AT(m->pcx, k, nc, c) = v[0] - r * xc[0];
            AT(m->pcy, k, nc, c) = v[1] - r * xc[1];
            AT(m->pcz, k, nc, c) = v[2] - r * xc[2];
        }
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < ne; ++e) {
            int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
            double vx = 0.5 * (AT(m->pcx, k, nc, c1) + AT(m->pcx, k, nc, c2));
            double vy = 0.5 * (AT(m->pcy, k, nc, c1) + AT(m->pcy, k, nc, c2));
            double vz = 0.5 * (AT(m->pcz, k, nc, c1) + AT(m->pcz, k, nc, c2));
            AT(m->vt, k, ne, e) = vx * g->edge_tangent[e] + vy * g->edge_tangent[ne + e] +
                                  vz * g->edge_tangent[2 * ne + e];
        }
    }
}

static void vt_phase(or_model *m, const double *vn, const double *w, double *tvn, double *tw,
                     double *wcc) {
    const or_grid *g = &m->g;
    const int64_t nc = g->nc, ne = g->ne, nv = g->nv;
    const int N = m->N;

    /* 1. tangential velocity from the Perot reconstruction */
    perot_phase(m, vn);
    /* 2. vn and vt at half levels; kinetic energy at edges */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        for (int i = 0; i <= N; ++i) {
            double hn, ht;
            if (i == 0) {
                hn = AT(vn, 0, ne, e);
                ht = AT(m->vt, 0, ne, e);
            } else if (i == N) {
                hn = AT(vn, N - 1, ne, e);
                ht = AT(m->vt, N - 1, ne, e);
            } else {
                double gg = AT(m->gw_e, i, ne, e);
                hn = gg * AT(vn, i, ne, e) + (1.0 - gg) * AT(vn, i - 1, ne, e);
                ht = gg * AT(m->vt, i, ne, e) + (1.0 - gg) * AT(m->vt, i - 1, ne, e);
            }
            AT(m->vnh, i, ne, e) = hn;
            AT(m->vth, i, ne, e) = ht;
        }
        for (int k = 0; k < N; ++k) {
            double un = AT(vn, k, ne, e), ut = AT(m->vt, k, ne, e);
            AT(m->ke, k, ne, e) = 0.5 * (un * un + ut * ut);
        }
    }
    /* 3. kinetic energy at cells; 4. vorticity at vertices */
    for (int k = 0; k < N; ++k) {
        or_op_cell_avg(g, m->ke + (int64_t)k * ne, m->kc + (int64_t)k * nc);
        or_op_curl(g, vn + (int64_t)k * ne, m->zv + (int64_t)k * nv);
    }
    /* 5. contravariant correction at half levels 1..N (cell average of edge values) */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e)
        for (int i = 1; i <= N; ++i)
            AT(m->ae, i, ne, e) = AT(m->vnh, i, ne, e) * AT(m->snh, i, ne, e) +
                                  AT(m->vth, i, ne, e) * AT(m->sth, i, ne, e);
    for (int64_t c = 0; c < nc; ++c) wcc[c] = 0.0;
    for (int i = 1; i <= N; ++i) or_op_cell_avg(g, m->ae + (int64_t)i * ne, wcc + (int64_t)i * nc);
    /* 6. contravariant vertical velocity, zero at top and ground */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        AT(m->omega, 0, nc, c) = 0.0;
        AT(m->omega, N, nc, c) = 0.0;
        for (int i = 1; i < N; ++i) AT(m->omega, i, nc, c) = AT(w, i, nc, c) - AT(wcc, i, nc, c);
    }
    /* 7. normal-velocity tendency */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
        int64_t v1 = g->edge_verts[e], v2 = g->edge_verts[ne + e];
        for (int k = 0; k < N; ++k) {
            double gradk = (AT(m->kc, k, nc, c2) - AT(m->kc, k, nc, c1)) * (1.0 / g->dual_length[e]);
            double zeta_e = 0.5 * (AT(m->zv, k, nv, v1) + AT(m->zv, k, nv, v2));
            double of1 = 0.5 * (AT(m->omega, k, nc, c1) + AT(m->omega, k + 1, nc, c1));
            double of2 = 0.5 * (AT(m->omega, k, nc, c2) + AT(m->omega, k + 1, nc, c2));
            double obar = 0.5 * (of1 + of2);
            double dvdz = (AT(m->vnh, k, ne, e) - AT(m->vnh, k + 1, ne, e)) / AT(m->dz_e, k, ne, e);
            AT(tvn, k, ne, e) = -gradk + (zeta_e + m->fe[e]) * AT(m->vt, k, ne, e) - obar * dvdz;
        }
    }
    /* 8. w tendency at interior half levels */
    for (int i = 1; i < N; ++i) or_op_vert_avg(g, w + (int64_t)i * nc, m->wv + (int64_t)i * nv);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
        int64_t v1 = g->edge_verts[e], v2 = g->edge_verts[ne + e];
        for (int i = 1; i < N; ++i) {
            double gw_ = (AT(w, i, nc, c2) - AT(w, i, nc, c1)) * (1.0 / g->dual_length[e]);
            double tw_ = (AT(m->wv, i, nv, v2) - AT(m->wv, i, nv, v1)) * (1.0 / g->edge_length[e]);
            AT(m->ae, i, ne, e) = AT(m->vnh, i, ne, e) * gw_ + AT(m->vth, i, ne, e) * tw_;
        }
    }
    for (int i = 1; i < N; ++i) or_op_cell_avg(g, m->ae + (int64_t)i * ne, tw + (int64_t)i * nc);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        AT(tw, 0, nc, c) = 0.0;
        AT(tw, N, nc, c) = 0.0;
        for (int i = 1; i < N; ++i) {
            double hadv = AT(tw, i, nc, c);
            double dwdz = (AT(w, i - 1, nc, c) - AT(w, i + 1, nc, c)) /
                          (AT(m->zh, i - 1, nc, c) - AT(m->zh, i + 1, nc, c));
            AT(tw, i, nc, c) = -hadv - AT(m->omega, i, nc, c) * dwdz;
        }
    }
}

int or_vt(or_model *m, const double *vn, const double *w, double *tvn, double *tw, double *wcc,
          double *vt_out) {
    if (!m || !vn || !w || !tvn || !tw || !wcc) return -1;
    vt_phase(m, vn, w, tvn, tw, wcc);
    if (vt_out) memcpy(vt_out, m->vt, sizeof(double) * m->N * m->g.ne);
    return 0;
}

/* terrain-corrected normal gradient of a full-level cell field */
static void pgrad(or_model *m, const double *px, double *gp) {
    const or_grid *g = &m->g;
    const int64_t nc = g->nc, ne = g->ne;
    const int N = m->N;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < N; ++k) {
            int ka = k == 0 ? 0 : k - 1, kb = k == N - 1 ? N - 1 : k + 1;
            AT(m->dpz, k, nc, c) = (AT(px, ka, nc, c) - AT(px, kb, nc, c)) /
                                   (AT(m->z, ka, nc, c) - AT(m->z, kb, nc, c));
        }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
        for (int k = 0; k < N; ++k) {
            double gl = (AT(px, k, nc, c2) - AT(px, k, nc, c1)) * (1.0 / g->dual_length[e]);
            double dz2 = 0.5 * (AT(m->dpz, k, nc, c1) + AT(m->dpz, k, nc, c2));
            AT(gp, k, ne, e) = gl - AT(m->sn, k, ne, e) * dz2;
        }
    }
}

int or_pgrad(or_model *m, const double *p, double *gp) {
    if (!m || !p || !gp) return -1;
    pgrad(m, p, gp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* column solve                                                              */
/* ------------------------------------------------------------------------ */

int or_thomas(int n, const double *a, const double *b, const double *c, const double *r,
              double *x) {
    if (n < 1 || n > OR_MAX_LEV + 1) return -1;
    double cp[OR_MAX_LEV + 1], dp[OR_MAX_LEV + 1];
    cp[0] = c[0] / b[0];
    dp[0] = r[0] / b[0];
    for (int i = 1; i < n; ++i) {
        double den = b[i] - a[i] * cp[i - 1];
        cp[i] = c[i] / den;
        dp[i] = (r[i] - a[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    return 0;
}

int or_column(int N, double dt, const or_params *p, const double *zh, const double *pi_ref,
              const double *theta_ref, const double *pi_n, const double *rho_n,
              const double *thv_n, const double *rho_i, const double *thv_i, const double *w_n,
              const double *tw, const double *wcc, const double *div_rho, const double *div_th,
              double *w_out, double *rho_out, double *pi_out, double *thv_out, double *vflux) {
    if (N < 2 || N > OR_MAX_LEV) return -1;
    const double beta = p->beta, cpd = p->cpd, rd = p->rd, cvd = p->cpd - p->rd;
    double z[OR_MAX_LEV], dz[OR_MAX_LEV], ppn[OR_MAX_LEV], B[OR_MAX_LEV], Rh[OR_MAX_LEV],
        Ph[OR_MAX_LEV];
    double dzh[OR_MAX_LEV + 1], gw[OR_MAX_LEV + 1], dref[OR_MAX_LEV + 1], rhoh[OR_MAX_LEV + 1],
        thh[OR_MAX_LEV + 1], thph[OR_MAX_LEV + 1], What[OR_MAX_LEV + 1], Fx[OR_MAX_LEV + 1],
        Hx[OR_MAX_LEV + 1], al[OR_MAX_LEV + 1], ga[OR_MAX_LEV + 1], ta[OR_MAX_LEV + 1],
        tb[OR_MAX_LEV + 1], tc[OR_MAX_LEV + 1], tr[OR_MAX_LEV + 1], wp[OR_MAX_LEV + 1];
    for (int k = 0; k < N; ++k) {
        z[k] = 0.5 * (zh[k] + zh[k + 1]);
        dz[k] = zh[k] - zh[k + 1];
        ppn[k] = pi_n[k] - pi_ref[k];
    }
    for (int i = 1; i < N; ++i) {
        dzh[i] = z[i - 1] - z[i];
        gw[i] = (z[i - 1] - zh[i]) / (z[i - 1] - z[i]);
        double threfh = gw[i] * theta_ref[i] + (1.0 - gw[i]) * theta_ref[i - 1];
        dref[i] = -p->grav / (cpd * threfh);
        rhoh[i] = gw[i] * rho_i[i] + (1.0 - gw[i]) * rho_i[i - 1];
        thh[i] = gw[i] * thv_i[i] + (1.0 - gw[i]) * thv_i[i - 1];
        thph[i] = gw[i] * (thv_i[i] - theta_ref[i]) + (1.0 - gw[i]) * (thv_i[i - 1] - theta_ref[i - 1]);
    }
    /* explicit parts at interior half levels; rigid lid and zero ground flux */
    Fx[0] = Fx[N] = Hx[0] = Hx[N] = al[0] = al[N] = 0.0;
    for (int i = 1; i < N; ++i) {
        double pterm = (1.0 - beta) * thh[i] * (ppn[i - 1] - ppn[i]) / dzh[i] + thph[i] * dref[i];
        What[i] = w_n[i] + dt * (tw[i] - cpd * pterm);
        Fx[i] = rhoh[i] * ((1.0 - beta) * w_n[i] - wcc[i]);
        Hx[i] = thh[i] * Fx[i];
        al[i] = beta * rhoh[i] * thh[i];
        ga[i] = dt * cpd * beta * thh[i] / dzh[i];
    }
    for (int k = 0; k < N; ++k) {
        Rh[k] = rho_n[k] - dt * (div_rho[k] + (Fx[k] - Fx[k + 1]) / dz[k]);
        B[k] = dt * (rd / cvd) * pi_n[k] / (rho_n[k] * thv_n[k] * dz[k]);
        Ph[k] = ppn[k] - B[k] * dz[k] * (div_th[k] + (Hx[k] - Hx[k + 1]) / dz[k]);
    }
    /* tridiagonal system in w on half levels 1..N-1 */
    for (int i = 1; i < N; ++i) {
        ta[i - 1] = -ga[i] * B[i - 1] * al[i - 1];
        tb[i - 1] = 1.0 + ga[i] * al[i] * (B[i - 1] + B[i]);
        tc[i - 1] = -ga[i] * B[i] * al[i + 1];
        tr[i - 1] = What[i] - ga[i] * (Ph[i - 1] - Ph[i]);
    }
    or_thomas(N - 1, ta, tb, tc, tr, wp + 1);
    wp[0] = 0.0;
    wp[N] = wcc[N];
    /* Rayleigh sponge: the solved w is damped before the level updates use it */
    if (p->w_damp)
        for (int i = 1; i < N; ++i) wp[i] = wp[i] * (1.0 / (1.0 + dt * p->w_damp[i]));
    for (int i = 0; i <= N; ++i) w_out[i] = wp[i];
    /* implicit vertical mass flux: zero at the lid and the ground */
    double fl[OR_MAX_LEV + 1];
    fl[0] = fl[N] = 0.0;
    for (int i = 1; i < N; ++i) fl[i] = rhoh[i] * wp[i];
    for (int k = 0; k < N; ++k) {
        double rnew = Rh[k] - dt * beta * (fl[k] - fl[k + 1]) / dz[k];
        double ppnew = Ph[k] - B[k] * (al[k] * wp[k] - al[k + 1] * wp[k + 1]);
        double rt = rho_n[k] * thv_n[k];
        rho_out[k] = rnew;
        pi_out[k] = pi_ref[k] + ppnew;
        thv_out[k] = (rt + (cvd / rd) * (rt / pi_n[k]) * (ppnew - ppn[k])) / rnew;
    }
    if (vflux) {
        vflux[0] = vflux[N] = 0.0;
        for (int i = 1; i < N; ++i)
            vflux[i] = rhoh[i] * (beta * wp[i] + (1.0 - beta) * w_n[i] - wcc[i]);
    }
    return 0;
}

/* run or_column on every column of the model (gathers each column contiguously) */
static void column_phase(or_model *m, double dt, const double *rho_i, const double *thv_i,
                         const double *tw, const double *wcc, double *w_o, double *rho_o,
                         double *pi_o, double *thv_o, double *vflux) {
    const int64_t nc = m->g.nc;
    const int N = m->N;
#pragma omp parallel
    {
        double c_zh[OR_MAX_LEV + 1], c_pr[OR_MAX_LEV], c_tr[OR_MAX_LEV], c_pi[OR_MAX_LEV],
            c_rho[OR_MAX_LEV], c_thv[OR_MAX_LEV], c_ri[OR_MAX_LEV], c_ti[OR_MAX_LEV],
            c_w[OR_MAX_LEV + 1], c_tw[OR_MAX_LEV + 1], c_wcc[OR_MAX_LEV + 1], c_dr[OR_MAX_LEV],
            c_dt[OR_MAX_LEV], o_w[OR_MAX_LEV + 1], o_rho[OR_MAX_LEV], o_pi[OR_MAX_LEV],
            o_thv[OR_MAX_LEV], o_fl[OR_MAX_LEV + 1];
#pragma omp for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            for (int i = 0; i <= N; ++i) {
                c_zh[i] = AT(m->zh, i, nc, c);
                c_w[i] = AT(m->w, i, nc, c);
                c_tw[i] = AT(tw, i, nc, c);
                c_wcc[i] = AT(wcc, i, nc, c);
            }
            for (int k = 0; k < N; ++k) {
                c_pr[k] = AT(m->pi_ref, k, nc, c);
                c_tr[k] = AT(m->theta_ref, k, nc, c);
                c_pi[k] = AT(m->pi, k, nc, c);
                c_rho[k] = AT(m->rho, k, nc, c);
                c_thv[k] = AT(m->thv, k, nc, c);
                c_ri[k] = AT(rho_i, k, nc, c);
                c_ti[k] = AT(thv_i, k, nc, c);
                c_dr[k] = AT(m->divr, k, nc, c);
                c_dt[k] = AT(m->divt, k, nc, c);
            }
            or_column(N, dt, &m->p, c_zh, c_pr, c_tr, c_pi, c_rho, c_thv, c_ri, c_ti, c_w, c_tw,
                      c_wcc, c_dr, c_dt, o_w, o_rho, o_pi, o_thv, o_fl);
            for (int i = 0; i <= N; ++i) {
                AT(w_o, i, nc, c) = o_w[i];
                if (vflux) AT(vflux, i, nc, c) = o_fl[i];
            }
            for (int k = 0; k < N; ++k) {
                AT(rho_o, k, nc, c) = o_rho[k];
                AT(pi_o, k, nc, c) = o_pi[k];
                AT(thv_o, k, nc, c) = o_thv[k];
            }
        }
    }
}

/* cell gradients of rho and theta_v of state n, level by level (upwind option) */
static void gradient_phase(or_model *m) {
    const int64_t nc = m->g.nc;
    for (int k = 0; k < m->N; ++k) {
        or_op_cell_grad(&m->g, m->rho + (int64_t)k * nc, m->g.cell_x, m->grad_r + (int64_t)k * 3 * nc);
        or_op_cell_grad(&m->g, m->thv + (int64_t)k * nc, m->g.cell_x, m->grad_t + (int64_t)k * 3 * nc);
    }
}

/* edge fluxes of mass and rho*theta_v, with the flux velocity vnx, and their
 * cell divergences per unit height.  Edge values of rho and theta_v: the
 * centred averages of state n, or (upwind) the upwind cell's value plus its
 * gradient dotted with the displacement to the back-trajectory midpoint, the
 * trajectory following (vnx, vt) over the substep dt. */
static void flux_phase(or_model *m, const double *vnx, double dt) {
    const or_grid *g = &m->g;
    const int64_t nc = g->nc, ne = g->ne;
    const int N = m->N;
    const double *rhoe = m->rhoe, *the = m->the;
    if (m->p.upwind) {
        for (int k = 0; k < N; ++k) {
            const int64_t oe = (int64_t)k * ne, oc = (int64_t)k * nc;
            or_op_upwind(g, m->rho + oc, m->grad_r + 3 * oc, vnx + oe, m->vt + oe, dt, m->rhoe_u + oe);
            or_op_upwind(g, m->thv + oc, m->grad_t + 3 * oc, vnx + oe, m->vt + oe, dt, m->the_u + oe);
        }
        rhoe = m->rhoe_u;
        the = m->the_u;
    }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < N; ++k) {
            double f = AT(rhoe, k, ne, e) * AT(vnx, k, ne, e) * AT(m->dz_e, k, ne, e);
            AT(m->flx, k, ne, e) = f;
            AT(m->hfl, k, ne, e) = AT(the, k, ne, e) * f;
        }
    for (int k = 0; k < N; ++k) {
        or_op_div(g, m->flx + (int64_t)k * ne, m->divr + (int64_t)k * nc);
        or_op_div(g, m->hfl + (int64_t)k * ne, m->divt + (int64_t)k * nc);
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < N; ++k) {
            AT(m->divr, k, nc, c) = AT(m->divr, k, nc, c) / AT(m->dz, k, nc, c);
            AT(m->divt, k, nc, c) = AT(m->divt, k, nc, c) / AT(m->dz, k, nc, c);
        }
}

/* ------------------------------------------------------------------------ */
/* one substep                                                               */
/* ------------------------------------------------------------------------ */

static void substep(or_model *m, double dt, int nsub) {
    const or_grid *g = &m->g;
    const or_params *p = &m->p;
    const int64_t nc = g->nc, ne = g->ne;
    const int N = m->N;
    const int64_t NC = (int64_t)N * nc, NE = (int64_t)N * ne, NC1 = (int64_t)(N + 1) * nc;
    const double cv = p->wgt_corr, eps = p->extrap;

    /* predictor: tendencies of state n */
    vt_phase(m, m->vn, m->w, m->tvn0, m->tw0, m->wcc0);
    /* extrapolated Exner perturbation and its terrain-corrected gradient */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < NC; ++i) {
        double pp = m->pi[i] - m->pi_ref[i];
        m->pix[i] = (1.0 + eps) * pp - eps * m->pi_prev[i];
    }
    pgrad(m, m->pix, m->gp);
    /* edge values of state n, predicted normal velocity */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
        for (int k = 0; k < N; ++k) {
            AT(m->the, k, ne, e) = 0.5 * (AT(m->thv, k, nc, c1) + AT(m->thv, k, nc, c2));
            AT(m->rhoe, k, ne, e) = 0.5 * (AT(m->rho, k, nc, c1) + AT(m->rho, k, nc, c2));
            AT(m->vns, k, ne, e) = AT(m->vn, k, ne, e) +
                                   dt * (AT(m->tvn0, k, ne, e) -
                                         p->cpd * AT(m->the, k, ne, e) * AT(m->gp, k, ne, e));
        }
    }
    if (p->upwind) gradient_phase(m);
    flux_phase(m, m->vns, dt);
    column_phase(m, dt, m->rho, m->thv, m->tw0, m->wcc0, m->ws, m->rhos, m->pis, m->thvs, NULL);

    /* corrector: tendencies of the predicted state */
    vt_phase(m, m->vns, m->ws, m->tvn1, m->tw1, m->wcc1);
    /* divergence of vn* for the damping term */
    for (int k = 0; k < N; ++k) or_op_div(g, m->vns + (int64_t)k * ne, m->dvs + (int64_t)k * nc);
    const double abar = 4.0 * 3.14159265358979323846 * g->radius * g->radius / (double)nc;
    /* fourth-order divergence damping operator of vn* */
    const int damp4 = p->div_damp4 != 0.0;
    if (damp4)
        for (int k = 0; k < N; ++k) or_op_graddiv2(g, m->vns + (int64_t)k * ne, m->g4 + (int64_t)k * ne);
    const double c4 = p->div_damp4 * abar * abar;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
        for (int k = 0; k < N; ++k) {
            double the_s = 0.5 * (AT(m->thvs, k, nc, c1) + AT(m->thvs, k, nc, c2));
            double tend = (1.0 - cv) * AT(m->tvn0, k, ne, e) + cv * AT(m->tvn1, k, ne, e) -
                          p->cpd * the_s * AT(m->gp, k, ne, e);
            double gdiv = (AT(m->dvs, k, nc, c2) - AT(m->dvs, k, nc, c1)) * (1.0 / g->dual_length[e]);
            double v = AT(m->vn, k, ne, e) + dt * tend + p->div_damp * abar * gdiv;
            if (damp4) v = v - c4 * AT(m->g4, k, ne, e);
            AT(m->vnn, k, ne, e) = v;
        }
    }
    flux_phase(m, m->vnn, dt);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < NC; ++i) {
        m->rho_i[i] = 0.5 * (m->rho[i] + m->rhos[i]);
        m->thv_i[i] = 0.5 * (m->thv[i] + m->thvs[i]);
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < NC1; ++i) m->twm[i] = (1.0 - cv) * m->tw0[i] + cv * m->tw1[i];
    /* new Exner perturbation history = pi^n - pi_ref, taken before pi is replaced */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < NC; ++i) m->pi_prev[i] = m->pi[i] - m->pi_ref[i];
    /* the column writes into the * buffers, then the state takes them over */
    column_phase(m, dt, m->rho_i, m->thv_i, m->twm, m->wcc1, m->ws, m->rhos, m->pis, m->thvs,
                 m->vflux);
    memcpy(m->w, m->ws, sizeof(double) * NC1);
    memcpy(m->rho, m->rhos, sizeof(double) * NC);
    memcpy(m->pi, m->pis, sizeof(double) * NC);
    memcpy(m->thv, m->thvs, sizeof(double) * NC);
    memcpy(m->vn, m->vnn, sizeof(double) * NE);
    /* FP64 mass-flux accumulation */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < NE; ++i) m->facc[i] += m->flx[i] / nsub;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < NC1; ++i) m->wacc[i] += m->vflux[i] / nsub;
}

/* Tracer transport over the step dt with the step's averaged mass fluxes:
 * horizontal (flux form, upwind cell's linear reconstruction at the edge
 * midpoint), then vertical (piecewise parabolic, mass-based Courant number),
 * each with the density change of the same fluxes, from the density at the
 * start of the step. */
static void transport_phase(or_model *m, double dt) {
    const or_grid *g = &m->g;
    const int64_t nc = g->nc, ne = g->ne;
    const int N = m->N;
    const int64_t NC = (int64_t)N * nc;
    double *grad = alloc(3 * nc), *rec = alloc(3 * nc), *tf = alloc(ne), *dT = alloc(nc),
           *dF = alloc(nc), *qs = alloc(NC), *rs = alloc(NC);
    for (int t = 0; t < m->nt; ++t) {
        double *q = m->q + (int64_t)t * NC;
        for (int k = 0; k < N; ++k) {
            const double *qk = q + (int64_t)k * nc, *F = m->facc + (int64_t)k * ne;
            or_op_tracer_grad(g, qk, grad);
            or_op_tracer_recon(g, qk, grad, rec);
            for (int64_t e = 0; e < ne; ++e) {
                const int64_t up = F[e] >= 0.0 ? g->edge_cells[e] : g->edge_cells[ne + e];
                int slot = 0;
                while (g->cell_edges[slot * nc + up] != e) ++slot;
                tf[e] = F[e] * rec[slot * nc + up];
            }
            or_op_div(g, tf, dT);
            or_op_div(g, F, dF);
            for (int64_t c = 0; c < nc; ++c) {
                const double dzc = AT(m->dz, k, nc, c), r0 = AT(m->rho0, k, nc, c);
                double hT = dT[c] / dzc, hF = dF[c] / dzc;
                double rsc = r0 - dt * hF;
                AT(rs, k, nc, c) = rsc;
                AT(qs, k, nc, c) = (r0 * qk[c] - dt * hT) / rsc;
            }
        }
#pragma omp parallel
        {
            double c_dz[OR_MAX_LEV], c_r[OR_MAX_LEV], c_q[OR_MAX_LEV], c_W[OR_MAX_LEV + 1],
                c_o[OR_MAX_LEV];
#pragma omp for schedule(static)
            for (int64_t c = 0; c < nc; ++c) {
                for (int k = 0; k < N; ++k) {
                    c_dz[k] = AT(m->dz, k, nc, c);
                    c_r[k] = AT(rs, k, nc, c);
                    c_q[k] = AT(qs, k, nc, c);
                }
                for (int i = 0; i <= N; ++i) c_W[i] = AT(m->wacc, i, nc, c);
                or_ppm_column(N, dt, c_dz, c_r, c_W, c_q, c_o, NULL);
                for (int k = 0; k < N; ++k) AT(q, k, nc, c) = c_o[k];
            }
        }
    }
    free(grad);
    free(rec);
    free(tf);
    free(dT);
    free(dF);
    free(qs);
    free(rs);
}

int or_tracers_set(or_model *m, int nt, const double *q) {
    if (!m || nt < 0 || (nt > 0 && !q) || (nt > 0 && (!m->g.edge_normal || !m->g.dual_frac)))
        return -1;
    const int64_t NC = (int64_t)m->N * m->g.nc;
    free(m->q);
    free(m->rho0);
    m->q = m->rho0 = NULL;
    m->nt = nt;
    if (nt == 0) return 0;
    m->q = alloc(nt * NC);
    m->rho0 = alloc(NC);
    if (!m->q || !m->rho0) return -1;
    memcpy(m->q, q, sizeof(double) * nt * NC);
    return 0;
}

int or_tracers_get(const or_model *m, double *q) {
    if (!m || !q) return -1;
    if (m->nt) memcpy(q, m->q, sizeof(double) * m->nt * (int64_t)m->N * m->g.nc);
    return 0;
}

/* Smagorinsky diffusion of vn over the step dt, level by level: the cell
 * coefficient from the deformation of (vn, vt), its edge mean capped for
 * stability, times the vector Laplacian of the same vn. */
static void diffusion_phase(or_model *m, double dt) {
    const or_grid *g = &m->g;
    const int64_t nc = g->nc, ne = g->ne;
    const int N = m->N;
    const double abar = 4.0 * 3.14159265358979323846 * g->radius * g->radius / (double)nc;
    const double kmax = abar / (25.0 * dt);
    const double cs2 = m->p.smag * m->p.smag;
    perot_phase(m, m->vn);
    for (int k = 0; k < N; ++k) {
        double *u = m->vn + (int64_t)k * ne, *kh = m->kh + (int64_t)k * nc;
        double *lap = m->lap + (int64_t)k * ne;
        or_op_deformation(g, u, m->vt + (int64_t)k * ne, kh);
        for (int64_t c = 0; c < nc; ++c) kh[c] = cs2 * g->cell_area[c] * kh[c];
        or_op_vector_laplacian(g, u, lap);
        for (int64_t e = 0; e < ne; ++e) {
            double ke = 0.5 * (kh[g->edge_cells[e]] + kh[g->edge_cells[ne + e]]);
            ke = ke < kmax ? ke : kmax;
            u[e] = u[e] + dt * ke * lap[e];
        }
    }
}

int or_step(or_model *m, double dt, int nsub) {
    if (!m || !(dt > 0) || !isfinite(dt) || nsub < 1) return -1;
    const int64_t N = m->N;
    memset(m->facc, 0, sizeof(double) * N * m->g.ne);
    memset(m->wacc, 0, sizeof(double) * (N + 1) * m->g.nc);
    const double dts = dt / nsub;
    if (m->nt) memcpy(m->rho0, m->rho, sizeof(double) * N * m->g.nc);
    for (int s = 0; s < nsub; ++s) substep(m, dts, nsub);
    if (m->p.smag > 0.0) diffusion_phase(m, dt);
    if (m->nt) transport_phase(m, dt);
    return 0;
}

/* compensated (Kahan) sums in fixed entity order, single thread */
int or_diag(const or_model *m, double *mass, double *rho_theta) {
    if (!m) return -1;
    const int64_t nc = m->g.nc;
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
    for (int k = 0; k < m->N; ++k)
        for (int64_t c = 0; c < nc; ++c) {
            double vol = m->g.cell_area[c] * AT(m->dz, k, nc, c);
            double x = vol * AT(m->rho, k, nc, c) - c1;
            double t = s1 + x;
            c1 = (t - s1) - x;
            s1 = t;
            double y = vol * AT(m->rho, k, nc, c) * AT(m->thv, k, nc, c) - c2;
            double u = s2 + y;
            c2 = (u - s2) - y;
            s2 = u;
        }
    if (mass) *mass = s1;
    if (rho_theta) *rho_theta = s2;
    return 0;
}

// nhcase.cpp -- heavy per-column and per-level pieces of the synthetic case
// generator (host only, OpenMP).  These build the INPUTS of the dynamical
// core (terrain, vertical coordinate, reference profile, balanced initial
// state, smoothed velocity noise); neither the CPU oracle nor the HIP library
// calls anything here.
//
// The paper runs a terrain-following hybrid height coordinate (Sec. 2) and
// initialises from reanalysis (Sec. 4.1); neither the terrain nor that data is
// available, so seeded synthetic stand-ins of the same shape are built here.

#include <cmath>
#include <cstdint>
#include <vector>

#include "nhcase.h"

extern "C" {

// Real orthonormal spherical harmonics (unit-sphere L2 normalisation, no
// Condon-Shortley phase) summed with the given coefficients, degree 1..lmax,
// order m = -l..l ascending.  Associated Legendre functions come from the
// standard fully normalised three-term recurrences in cos(colatitude).
int nhcase_terrain(const double *cell_x, int64_t n, int lmax, const double *coef, double *out) {
    if (!cell_x || !coef || !out || n < 0 || lmax < 1 || lmax > 200) return -1;
    const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
#pragma omp parallel
    {
        std::vector<double> q((lmax + 1) * (lmax + 1));
        std::vector<double> cm(lmax + 1), sm(lmax + 1);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double x = cell_x[i], y = cell_x[n + i], z = cell_x[2 * n + i];
            double rxy = std::sqrt(x * x + y * y);
            double ct = z, st = rxy;  // cos/sin of colatitude
            double phi = std::atan2(y, x);
            for (int m = 0; m <= lmax; ++m) {
                cm[m] = std::cos(m * phi);
                sm[m] = std::sin(m * phi);
            }
            auto Q = [&](int l, int m) -> double & { return q[l * (lmax + 1) + m]; };
            Q(0, 0) = std::sqrt(inv4pi);
            for (int m = 1; m <= lmax; ++m)
                Q(m, m) = std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * st * Q(m - 1, m - 1);
            for (int m = 0; m < lmax; ++m) Q(m + 1, m) = std::sqrt(2.0 * m + 3.0) * ct * Q(m, m);
            for (int m = 0; m <= lmax; ++m)
                for (int l = m + 2; l <= lmax; ++l) {
                    double a = std::sqrt((4.0 * l * l - 1.0) / (double(l) * l - double(m) * m));
                    double b = std::sqrt(((l - 1.0) * (l - 1.0) - double(m) * m) /
                                         (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
                    Q(l, m) = a * (ct * Q(l - 1, m) - b * Q(l - 2, m));
                }
            double h = 0.0;
            const double r2 = std::sqrt(2.0);
            for (int l = 1; l <= lmax; ++l) {
                const double *c = coef + (l * l - 1);  // m = -l .. l
                for (int m = -l; m <= l; ++m) {
                    double y_lm;
                    if (m == 0) y_lm = Q(l, 0);
                    else if (m > 0) y_lm = r2 * Q(l, m) * cm[m];
                    else y_lm = r2 * Q(l, -m) * sm[-m];
                    h += c[m + l] * y_lm;
                }
            }
            out[i] = h;
        }
    }
    return 0;
}

// Per-column vertical grid, reference profile and initial thermodynamic state.
int nhcase_columns(const nhcase_column_args *a, double *zh, double *pi_ref, double *theta_ref,
                   double *pi, double *theta_v, double *rho) {
    if (!a || !a->zeta || !a->h || !zh || !pi_ref || !theta_ref || !pi || !theta_v || !rho)
        return -1;
    const int64_t nc = a->n_cells;
    const int N = a->n_lev;
    if (nc < 0 || N < 2) return -1;
    const double g = a->grav, cpd = a->cpd, rd = a->rd, p00 = a->p00, T0 = a->t0;
    const double cvd = cpd - rd;
    const double T1 = a->t_ref_top, dT = a->t_ref_delta, hs = a->t_ref_scale;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t c = 0; c < nc; ++c) {
        std::vector<double> z(N), gw(N + 1), dzh(N + 1), pr(N), tr(N), p(N), dref(N + 1);
        // half-level heights: zeta + h * b(zeta), sinh decay flat above zeta_f
        for (int i = 0; i <= N; ++i) {
            double zt = a->zeta[i];
            double b = 0.0;
            if (zt < a->z_flat)
                b = std::sinh((a->z_flat - zt) / a->decay_scale) / std::sinh(a->z_flat / a->decay_scale);
            zh[int64_t(i) * nc + c] = zt + a->h[c] * b;
        }
        for (int k = 0; k < N; ++k)
            z[k] = 0.5 * (zh[int64_t(k) * nc + c] + zh[int64_t(k + 1) * nc + c]);
        // reference profile at full levels (closed form of d(pi)/dz = -g pi/(cpd T_ref))
        for (int k = 0; k < N; ++k) {
            double tref = T1 + dT * std::exp(-z[k] / hs);
            double pref = std::exp(-g / (cpd * T1) *
                                   (z[k] + hs * std::log((T1 + dT * std::exp(-z[k] / hs)) / (T1 + dT))));
            pr[k] = pref;
            tr[k] = tref / pref;
            pi_ref[int64_t(k) * nc + c] = pref;
            theta_ref[int64_t(k) * nc + c] = tref / pref;
        }
        // interpolation weights and reference vertical derivative at interior half levels
        // (0-based half level i sits between full levels i-1 above and i below)
        for (int i = 1; i < N; ++i) {
            double zhi = zh[int64_t(i) * nc + c];
            gw[i] = (z[i - 1] - zhi) / (z[i - 1] - z[i]);
            dzh[i] = z[i - 1] - z[i];
            double threfh = gw[i] * tr[i] + (1.0 - gw[i]) * tr[i - 1];
            dref[i] = -g / (cpd * threfh);
        }
        if (a->balanced) {
            // discrete hydrostatic balance of the resting w-equation, bottom-up
            p[N - 1] = std::exp(-g * z[N - 1] / (cpd * T0));
            for (int i = N - 1; i >= 1; --i) {
                const double gi = gw[i];
                const double thb = T0 / p[i];
                const double ppb = p[i] - pr[i];
                double x = std::exp(-g * z[i - 1] / (cpd * T0));
                int it = 0;
                double last = 0.0;
                for (; it < 60; ++it) {
                    double tha = T0 / x;
                    double thh = gi * thb + (1.0 - gi) * tha;
                    double thp = gi * (thb - tr[i]) + (1.0 - gi) * (tha - tr[i - 1]);
                    double dpp = (x - pr[i - 1]) - ppb;
                    double r = thh * dpp / dzh[i] + thp * dref[i];
                    double dth = -(1.0 - gi) * T0 / (x * x);
                    double dr = dth * dpp / dzh[i] + thh / dzh[i] + dth * dref[i];
                    double dx = r / dr;
                    x -= dx;
                    last = std::fabs(dx);
                    // converged once the update is at the unit-roundoff level of x
                    if (last <= std::ldexp(std::fabs(x), -52)) break;
                }
                if (it == 60 && last > std::ldexp(std::fabs(x), -50)) bad += 1;
                p[i - 1] = x;
            }
        } else {
            for (int k = 0; k < N; ++k) p[k] = std::exp(-g * z[k] / (cpd * T0));
        }
        for (int k = 0; k < N; ++k) {
            double th = T0 / p[k];
            pi[int64_t(k) * nc + c] = p[k];
            theta_v[int64_t(k) * nc + c] = th;
            rho[int64_t(k) * nc + c] = p00 * std::pow(p[k], cvd / rd) / (rd * th);
        }
    }
    return bad ? -2 : 0;
}

// Sign-aware edge smoother: each pass replaces x_e by the normal component of
// the mean of the reconstructed cell vectors of its two cells, then every
// level is rescaled to unit root-mean-square (sum in the given edge order).
int nhcase_smooth_noise(const nhcase_grid_args *gr, int n_lev, int passes, double *x) {
    if (!gr || !x || n_lev < 1 || passes < 0) return -1;
    const int64_t nc = gr->n_cells, ne = gr->n_edges;
    const double a = gr->radius;
#pragma omp parallel
    {
        std::vector<double> vc(3 * nc);
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < n_lev; ++k) {
            double *xk = x + int64_t(k) * ne;
            for (int p = 0; p < passes; ++p) {
                for (int64_t c = 0; c < nc; ++c) {
                    double v[3] = {0.0, 0.0, 0.0};
                    const double xc[3] = {gr->cell_x[c], gr->cell_x[nc + c], gr->cell_x[2 * nc + c]};
                    for (int j = 0; j < 3; ++j) {
                        int64_t e = gr->cell_edges[j * nc + c];
                        double w = gr->cell_sign[j * nc + c] * gr->edge_length[e] * xk[e] * a;
                        for (int d = 0; d < 3; ++d) v[d] += w * (gr->edge_x[d * ne + e] - xc[d]);
                    }
                    double inv = 1.0 / gr->cell_area[c];
                    for (int d = 0; d < 3; ++d) v[d] *= inv;
                    double r = v[0] * xc[0] + v[1] * xc[1] + v[2] * xc[2];
                    for (int d = 0; d < 3; ++d) vc[d * nc + c] = v[d] - r * xc[d];
                }
                for (int64_t e = 0; e < ne; ++e) {
                    int64_t c1 = gr->edge_cells[e], c2 = gr->edge_cells[ne + e];
                    double s = 0.0;
                    for (int d = 0; d < 3; ++d)
                        s += 0.5 * (vc[d * nc + c1] + vc[d * nc + c2]) * gr->edge_normal[d * ne + e];
                    xk[e] = s;
                }
            }
            double ss = 0.0;
            for (int64_t e = 0; e < ne; ++e) ss += xk[e] * xk[e];
            double scale = 1.0 / std::sqrt(ss / double(ne));
            for (int64_t e = 0; e < ne; ++e) xk[e] *= scale;
        }
    }
    return 0;
}

}  // extern "C"

// nhdc_kernels.hip -- FP64 kernels of one dynamical-core substep for gfx950.
//
// Layout: level-major [k][entity] with entities in space-filling-curve order,
// so that at every level neighbouring lanes read neighbouring addresses and
// the indirect gathers of a wavefront hit the same few cache lines.  Every
// kernel gives one lane one horizontal entity and marches it down the column,
// keeping the values of adjacent levels in registers (vertical stencils never
// re-read memory).  No atomics and no scatter: every sum is a gather in fixed
// slot order, so results are bitwise reproducible run to run.
//
// Arithmetic: this file is compiled without floating-point contraction and
// every value is formed with the same operations, in the same order, as the
// discretisation's plain definition (sums in slot order, divisions where the
// operator divides).  Results therefore do not depend on the numbering, the
// tile shape or the launch configuration.
//
// Substep (one predictor, one corrector):
//   vt_edge   tangential velocity from the cell vector reconstruction
//   vertex    vorticity and vertex average of w
//   cell_vt   kinetic energy, contravariant correction, w tendency, div(vn)
//   edge_pred vn tendency, extrapolated Exner gradient, predicted vn, fluxes
//   column    horizontal divergences + implicit w/Exner tridiagonal solve
//   (the same three tendency kernels on the predicted state)
//   edge_corr corrected vn with averaged tendencies + divergence damping, fluxes
//   column    corrector solve and FP64 mass-flux accumulation
#include <hip/hip_runtime.h>

#include "nhdc_internal.h"

#pragma clang fp contract(off)

namespace nhdc {
namespace {

constexpr int BLOCK = 256;
constexpr unsigned NXCD = 8;  // MI355X: 8 accelerator complex dies, each with its own L2

// Workgroups are dispatched round-robin over the XCDs.  Map them so that each
// XCD works on one contiguous range of tiles: neighbouring tiles gather each
// other's values, and then mostly do so through the same L2.
__device__ __forceinline__ int64_t tile_index() {
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned q = nb / NXCD, rem = nb % NXCD;
    const unsigned x = b % NXCD, r = b / NXCD;
    const unsigned start = x * q + (x < rem ? x : rem);
    return int64_t(start + r);
}

__device__ __forceinline__ int64_t gid() { return tile_index() * BLOCK + threadIdx.x; }

inline unsigned nblocks(int64_t n) { return unsigned((n + BLOCK - 1) / BLOCK); }

// ---------------------------------------------------------------------------
// set-up: interpolation weights, reference vertical derivative, vertex heights

__global__ void k_metrics_cell(int64_t nc, int N, const double *__restrict__ zh,
                               const double *__restrict__ theta_ref, double grav, double cpd,
                               double *__restrict__ gw, double *__restrict__ dref) {
    int64_t c = gid();
    if (c >= nc) return;
    gw[c] = 0.0;
    dref[c] = 0.0;
    gw[int64_t(N) * nc + c] = 0.0;
    dref[int64_t(N) * nc + c] = 0.0;
    for (int i = 1; i < N; ++i) {
        double za = 0.5 * (zh[int64_t(i - 1) * nc + c] + zh[int64_t(i) * nc + c]);
        double zb = 0.5 * (zh[int64_t(i) * nc + c] + zh[int64_t(i + 1) * nc + c]);
        double g = (za - zh[int64_t(i) * nc + c]) / (za - zb);
        gw[int64_t(i) * nc + c] = g;
        double th = g * theta_ref[int64_t(i) * nc + c] + (1.0 - g) * theta_ref[int64_t(i - 1) * nc + c];
        dref[int64_t(i) * nc + c] = -grav / (cpd * th);
    }
}

__global__ void k_metrics_vert(Grid g) {
    int64_t v = gid();
    const int64_t nv = g.nv, nc = g.nc;
    if (v >= nv) return;
    for (int i = 0; i <= g.N; ++i) {
        const double *z = g.zh + int64_t(i) * nc;
        double s = 0.0;
        for (int j = 0; j < 6; ++j) s += g.v_m[j * nv + v] * z[g.v_c[j * nv + v]];
        g.zhv[int64_t(i) * nv + v] = s / g.v_val[v];
    }
}

__global__ void k_init_prev(int64_t n, const double *__restrict__ pi, const double *__restrict__ pi_ref,
                            double *__restrict__ prev) {
    int64_t i = gid();
    if (i < n) prev[i] = pi[i] - pi_ref[i];
}

// ---------------------------------------------------------------------------
// velocity tendencies

// Radial-free reconstructed cell vector from the normal velocities of its edges.
struct CellRecon {
    int32_t e[3];
    double sl[3], dv[9], x[3], area;
};

__device__ __forceinline__ void load_recon(const Grid &g, int32_t c, CellRecon &r) {
    const int64_t nc = g.nc;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        r.e[j] = g.c_e[j * nc + c];
        r.sl[j] = g.c_sl[j * nc + c];
        r.x[j] = g.c_x[j * nc + c];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) r.dv[q] = g.c_dv[q * nc + c];
    r.area = g.c_area[c];
}

__device__ __forceinline__ void recon(const CellRecon &r, const double *__restrict__ u, double V[3]) {
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double wgt = r.sl[j] * u[r.e[j]];
#pragma unroll
        for (int d = 0; d < 3; ++d) v[d] += wgt * r.dv[3 * j + d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) v[d] = v[d] / r.area;
    double rr = v[0] * r.x[0] + v[1] * r.x[1] + v[2] * r.x[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) V[d] = v[d] - rr * r.x[d];
}

// vt_e = (V_c1 + V_c2)/2 . t_e
__global__ void __launch_bounds__(BLOCK) k_vt_edge(Grid g, const double *__restrict__ vn,
                                                   double *__restrict__ vt) {
    int64_t e = gid();
    const int64_t ne = g.ne;
    if (e >= ne) return;
    CellRecon r1, r2;
    load_recon(g, g.e_c[e], r1);
    load_recon(g, g.e_c[ne + e], r2);
    const double t0 = g.e_t[e], t1 = g.e_t[ne + e], t2 = g.e_t[2 * ne + e];
    for (int k = 0; k < g.N; ++k) {
        const double *u = vn + int64_t(k) * ne;
        double V1[3], V2[3];
        recon(r1, u, V1);
        recon(r2, u, V2);
        double vx = 0.5 * (V1[0] + V2[0]);
        double vy = 0.5 * (V1[1] + V2[1]);
        double vz = 0.5 * (V1[2] + V2[2]);
        vt[int64_t(k) * ne + e] = vx * t0 + vy * t1 + vz * t2;
    }
}

// vertex vorticity (full levels) and vertex average of w (interior half levels)
__global__ void __launch_bounds__(BLOCK) k_vertex(Grid g, const double *__restrict__ vn,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ zeta,
                                                  double *__restrict__ wv) {
    int64_t v = gid();
    const int64_t nv = g.nv, ne = g.ne, nc = g.nc;
    if (v >= nv) return;
    int32_t ie[6], ic[6];
    double sd[6], m[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        ie[j] = g.v_e[j * nv + v];
        ic[j] = g.v_c[j * nv + v];
        sd[j] = g.v_sd[j * nv + v];
        m[j] = g.v_m[j * nv + v];
    }
    const double area = g.v_area[v], val = g.v_val[v];
    for (int k = 0; k < g.N; ++k) {
        const double *u = vn + int64_t(k) * ne;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) s += sd[j] * u[ie[j]];
        zeta[int64_t(k) * nv + v] = s / area;
    }
    for (int i = 1; i < g.N; ++i) {
        const double *x = w + int64_t(i) * nc;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) s += m[j] * x[ic[j]];
        wv[int64_t(i) * nv + v] = s / val;
    }
}

// Cell part of the tendencies: kinetic energy K_c, contravariant correction
// w_cc, w tendency T_w and (optionally) the divergence of vn.
template <bool WANT_DIV>
__global__ void __launch_bounds__(BLOCK) k_cell_vt(Grid g, const double *__restrict__ vn,
                                                   const double *__restrict__ vt,
                                                   const double *__restrict__ w,
                                                   const double *__restrict__ wv,
                                                   double *__restrict__ kc,
                                                   double *__restrict__ wcc,
                                                   double *__restrict__ tw,
                                                   double *__restrict__ dvn) {
    int64_t c = gid();
    const int64_t nc = g.nc, ne = g.ne, nv = g.nv;
    const int N = g.N;
    if (c >= nc) return;
    int32_t e[3], c1[3], c2[3], v1[3], v2[3];
    double de[3], le[3], sl[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        e[j] = g.c_e[j * nc + c];
        c1[j] = g.e_c[e[j]];
        c2[j] = g.e_c[ne + e[j]];
        v1[j] = g.e_v[e[j]];
        v2[j] = g.e_v[ne + e[j]];
        de[j] = g.e_de[e[j]];
        le[j] = g.e_le[e[j]];
        sl[j] = g.c_sl[j * nc + c];
    }
    const double area = g.c_area[c];
    double vnp[3] = {0.0, 0.0, 0.0}, vtp[3] = {0.0, 0.0, 0.0};  // full level i-1
    wcc[c] = 0.0;
    tw[c] = 0.0;
    for (int i = 0; i <= N; ++i) {
        double vni[3] = {0.0, 0.0, 0.0}, vti[3] = {0.0, 0.0, 0.0};
        if (i < N) {
            double ks = 0.0, ds = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                vni[j] = vn[int64_t(i) * ne + e[j]];
                vti[j] = vt[int64_t(i) * ne + e[j]];
                ks += 0.5 * (vni[j] * vni[j] + vti[j] * vti[j]);
                ds += sl[j] * vni[j];
            }
            kc[int64_t(i) * nc + c] = ks / 3.0;
            if (WANT_DIV) dvn[int64_t(i) * nc + c] = ds / area;
        }
        if (i > 0) {
            const double *zhi = g.zh + int64_t(i) * nc;
            const double *zvi = g.zhv + int64_t(i) * nv;
            double ccs = 0.0, adv = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double hn, ht;
                if (i < N) {
                    double gg = 0.5 * (g.gw[int64_t(i) * nc + c1[j]] + g.gw[int64_t(i) * nc + c2[j]]);
                    hn = gg * vni[j] + (1.0 - gg) * vnp[j];
                    ht = gg * vti[j] + (1.0 - gg) * vtp[j];
                } else {
                    hn = vnp[j];
                    ht = vtp[j];
                }
                double snh = (zhi[c2[j]] - zhi[c1[j]]) / de[j];
                double sth = (zvi[v2[j]] - zvi[v1[j]]) / le[j];
                ccs += hn * snh + ht * sth;
                if (i < N) {
                    const double *wi = w + int64_t(i) * nc;
                    const double *wvi = wv + int64_t(i) * nv;
                    double gw_ = (wi[c2[j]] - wi[c1[j]]) / de[j];
                    double tw_ = (wvi[v2[j]] - wvi[v1[j]]) / le[j];
                    adv += hn * gw_ + ht * tw_;
                }
            }
            double wcci = ccs / 3.0;
            wcc[int64_t(i) * nc + c] = wcci;
            if (i < N) {
                double hadv = adv / 3.0;
                double om = w[int64_t(i) * nc + c] - wcci;
                double dwdz = (w[int64_t(i - 1) * nc + c] - w[int64_t(i + 1) * nc + c]) /
                              (g.zh[int64_t(i - 1) * nc + c] - g.zh[int64_t(i + 1) * nc + c]);
                tw[int64_t(i) * nc + c] = -hadv - om * dwdz;
            } else {
                tw[int64_t(i) * nc + c] = 0.0;
            }
        }
        if (i < N) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                vnp[j] = vni[j];
                vtp[j] = vti[j];
            }
        }
    }
}

// Per-edge constants shared by the two edge kernels.
struct EdgeCtx {
    int32_t c1, c2, v1, v2;
    double de, fe;
};

__device__ __forceinline__ double omega_at(const double *w, const double *wcc, int i, int N,
                                           int64_t nc, int32_t c) {
    if (i <= 0 || i >= N) return 0.0;
    return w[int64_t(i) * nc + c] - wcc[int64_t(i) * nc + c];
}

// vn tendency at (edge, level k); vnh_k / vnh_k1 are vn at half levels k and k+1.
__device__ __forceinline__ double vn_tendency(const Grid &g, const EdgeCtx &ec, int k,
                                              const double *kc, const double *zeta,
                                              double vtk, const double *w, const double *wcc,
                                              double vnh_k, double vnh_k1, double dze) {
    const int64_t nc = g.nc, nv = g.nv;
    const int N = g.N;
    double gradk = (kc[int64_t(k) * nc + ec.c2] - kc[int64_t(k) * nc + ec.c1]) / ec.de;
    double ze = 0.5 * (zeta[int64_t(k) * nv + ec.v1] + zeta[int64_t(k) * nv + ec.v2]);
    double of1 = 0.5 * (omega_at(w, wcc, k, N, nc, ec.c1) + omega_at(w, wcc, k + 1, N, nc, ec.c1));
    double of2 = 0.5 * (omega_at(w, wcc, k, N, nc, ec.c2) + omega_at(w, wcc, k + 1, N, nc, ec.c2));
    double obar = 0.5 * (of1 + of2);
    double dvdz = (vnh_k - vnh_k1) / dze;
    return -gradk + (ze + ec.fe) * vtk - obar * dvdz;
}

// value at half level i from full levels i (below) and i-1 (above), edge weight
__device__ __forceinline__ double half_interp(const Grid &g, const EdgeCtx &ec, int i,
                                              double below, double above) {
    const int64_t nc = g.nc;
    double gg = 0.5 * (g.gw[int64_t(i) * nc + ec.c1] + g.gw[int64_t(i) * nc + ec.c2]);
    return gg * below + (1.0 - gg) * above;
}

__device__ __forceinline__ double exner_x(const Grid &g, const State &s, double eps, int k,
                                          int32_t c) {
    int64_t o = int64_t(k) * g.nc + c;
    double pp = s.pi[o] - g.pi_ref[o];
    return (1.0 + eps) * pp - eps * s.pi_prev[o];
}

__device__ __forceinline__ double dpz_at(const Grid &g, const State &s, double eps, int k,
                                         int32_t c) {
    const int N = g.N;
    const int64_t nc = g.nc;
    int ka = k == 0 ? 0 : k - 1, kb = k == N - 1 ? N - 1 : k + 1;
    double za = 0.5 * (g.zh[int64_t(ka) * nc + c] + g.zh[int64_t(ka + 1) * nc + c]);
    double zb = 0.5 * (g.zh[int64_t(kb) * nc + c] + g.zh[int64_t(kb + 1) * nc + c]);
    return (exner_x(g, s, eps, ka, c) - exner_x(g, s, eps, kb, c)) / (za - zb);
}

__device__ __forceinline__ double edge_dz(const Grid &g, const EdgeCtx &ec, int k) {
    const int64_t nc = g.nc;
    double dz1 = g.zh[int64_t(k) * nc + ec.c1] - g.zh[int64_t(k + 1) * nc + ec.c1];
    double dz2 = g.zh[int64_t(k) * nc + ec.c2] - g.zh[int64_t(k + 1) * nc + ec.c2];
    return 0.5 * (dz1 + dz2);
}

// Predictor on edges: vn tendency of state n, terrain-corrected gradient of
// the extrapolated Exner perturbation, predicted vn, mass and theta fluxes.
__global__ void __launch_bounds__(BLOCK) k_edge_pred(Grid g, State s, Work wk, Params p,
                                                     double dt) {
    int64_t e = gid();
    const int64_t ne = g.ne, nc = g.nc;
    const int N = g.N;
    if (e >= ne) return;
    EdgeCtx ec{g.e_c[e], g.e_c[ne + e], g.e_v[e], g.e_v[ne + e], g.e_de[e], g.fe[e]};
    double vnm = 0.0, vn0 = s.vn[e];  // levels k-1, k
    for (int k = 0; k < N; ++k) {
        const int64_t o = int64_t(k) * ne + e;
        double vn1 = k + 1 < N ? s.vn[o + ne] : vn0;
        double vnh_k = k == 0 ? vn0 : half_interp(g, ec, k, vn0, vnm);
        double vnh_k1 = k + 1 == N ? vn0 : half_interp(g, ec, k + 1, vn1, vn0);
        double dze = edge_dz(g, ec, k);
        double tvn = vn_tendency(g, ec, k, wk.kc, wk.zeta, wk.vt[o], s.w, wk.wcc0, vnh_k, vnh_k1, dze);
        double px1 = exner_x(g, s, p.extrap, k, ec.c1), px2 = exner_x(g, s, p.extrap, k, ec.c2);
        double dpz1 = dpz_at(g, s, p.extrap, k, ec.c1), dpz2 = dpz_at(g, s, p.extrap, k, ec.c2);
        double z1 = 0.5 * (g.zh[int64_t(k) * nc + ec.c1] + g.zh[int64_t(k + 1) * nc + ec.c1]);
        double z2 = 0.5 * (g.zh[int64_t(k) * nc + ec.c2] + g.zh[int64_t(k + 1) * nc + ec.c2]);
        double sn = (z2 - z1) / ec.de;
        double gl = (px2 - px1) / ec.de;
        double dz2 = 0.5 * (dpz1 + dpz2);
        double gp = gl - sn * dz2;
        double the = 0.5 * (s.thv[int64_t(k) * nc + ec.c1] + s.thv[int64_t(k) * nc + ec.c2]);
        double rhe = 0.5 * (s.rho[int64_t(k) * nc + ec.c1] + s.rho[int64_t(k) * nc + ec.c2]);
        double vns = vn0 + dt * (tvn - p.cpd * the * gp);
        double f = rhe * vns * dze;
        wk.tvn0[o] = tvn;
        wk.gp[o] = gp;
        wk.vns[o] = vns;
        wk.flx[o] = f;
        wk.hfl[o] = the * f;
        vnm = vn0;
        vn0 = vn1;
    }
}

// Corrector on edges: vn^{n+1} from the averaged tendencies, the predictor's
// Exner gradient with the predicted theta_v, and divergence damping; fluxes
// with state-n edge values; FP64 flux accumulation.
__global__ void __launch_bounds__(BLOCK) k_edge_corr(Grid g, State s, Work wk, Params p, double dt,
                                                     int nsub, int first) {
    int64_t e = gid();
    const int64_t ne = g.ne, nc = g.nc;
    const int N = g.N;
    if (e >= ne) return;
    EdgeCtx ec{g.e_c[e], g.e_c[ne + e], g.e_v[e], g.e_v[ne + e], g.e_de[e], g.fe[e]};
    const double cv = p.wgt_corr;
    const double dnsub = double(nsub);
    double vnm = 0.0, vn0 = wk.vns[e];  // predicted vn at levels k-1, k
    for (int k = 0; k < N; ++k) {
        const int64_t o = int64_t(k) * ne + e;
        double vn1 = k + 1 < N ? wk.vns[o + ne] : vn0;
        double vnh_k = k == 0 ? vn0 : half_interp(g, ec, k, vn0, vnm);
        double vnh_k1 = k + 1 == N ? vn0 : half_interp(g, ec, k + 1, vn1, vn0);
        double dze = edge_dz(g, ec, k);
        double tvn1 = vn_tendency(g, ec, k, wk.kc, wk.zeta, wk.vt[o], wk.ws, wk.wcc1, vnh_k, vnh_k1, dze);
        double ths = 0.5 * (wk.thvs[int64_t(k) * nc + ec.c1] + wk.thvs[int64_t(k) * nc + ec.c2]);
        double tend = (1.0 - cv) * wk.tvn0[o] + cv * tvn1 - p.cpd * ths * wk.gp[o];
        double gdiv = (wk.dvn[int64_t(k) * nc + ec.c2] - wk.dvn[int64_t(k) * nc + ec.c1]) / ec.de;
        double vnn = s.vn[o] + dt * tend + p.div_damp * g.abar * gdiv;
        double the = 0.5 * (s.thv[int64_t(k) * nc + ec.c1] + s.thv[int64_t(k) * nc + ec.c2]);
        double rhe = 0.5 * (s.rho[int64_t(k) * nc + ec.c1] + s.rho[int64_t(k) * nc + ec.c2]);
        double f = rhe * vnn * dze;
        s.vn[o] = vnn;
        wk.flx[o] = f;
        wk.hfl[o] = the * f;
        double acc = first ? 0.0 : s.facc[o];
        s.facc[o] = acc + f / dnsub;
        vnm = vn0;
        vn0 = vn1;
    }
}

// ---------------------------------------------------------------------------
// column: horizontal divergences, explicit parts, tridiagonal solve in w
// (Thomas, no pivoting; factors and the explicit rho / Exner parts kept in
// global scratch), then rho, Exner and theta_v.  CORR selects the corrector:
// interface state averaged between n and the prediction, averaged w tendency,
// in-place update of the state, Exner history and flux accumulation.
template <bool CORR>
__global__ void __launch_bounds__(BLOCK) k_column(Grid g, State s, Work wk, Params p, double dt,
                                                  int nsub, int first) {
    int64_t c = gid();
    const int64_t nc = g.nc, ne = g.ne;
    const int N = g.N;
    if (c >= nc) return;
    const double beta = p.beta, cpd = p.cpd, rd = p.rd, cvd = p.cpd - p.rd;
    const double cv = p.wgt_corr;
    const double dnsub = double(nsub);
    int32_t e[3];
    double sl[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        e[j] = g.c_e[j * nc + c];
        sl[j] = g.c_sl[j * nc + c];
    }
    const double area = g.c_area[c];
    const double *wcc = CORR ? wk.wcc1 : wk.wcc0;
    double *w_out = CORR ? s.w : wk.ws;
    double *rho_out = CORR ? s.rho : wk.rhos;
    double *thv_out = CORR ? s.thv : wk.thvs;
    auto at = [&](int k) { return int64_t(k) * nc + c; };
    auto rho_if = [&](int k) {
        return CORR ? 0.5 * (s.rho[at(k)] + wk.rhos[at(k)]) : s.rho[at(k)];
    };
    auto thv_if = [&](int k) {
        return CORR ? 0.5 * (s.thv[at(k)] + wk.thvs[at(k)]) : s.thv[at(k)];
    };
    auto twv = [&](int i) {
        return CORR ? (1.0 - cv) * wk.tw0[at(i)] + cv * wk.tw1[at(i)] : wk.tw0[at(i)];
    };
    // ---- forward sweep, top to bottom ----
    // carried: explicit fluxes, alpha, gamma and W-hat of half level k (top of
    // level k); Pi-hat and B of level k-1; alpha of half level k-1; Thomas factors.
    double fx_k = 0.0, hx_k = 0.0, al_k = 0.0, ga_k = 0.0, wh_k = 0.0;
    double ph_prev = 0.0, b_prev = 0.0, al_prev = 0.0, cp_prev = 0.0, dp_prev = 0.0;
    for (int k = 0; k < N; ++k) {
        double fx_b = 0.0, hx_b = 0.0, al_b = 0.0, ga_b = 0.0, wh_b = 0.0;
        const int i = k + 1;  // bottom interface of level k
        if (i < N) {
            double za = 0.5 * (g.zh[at(i - 1)] + g.zh[at(i)]);
            double zb = 0.5 * (g.zh[at(i)] + g.zh[at(i + 1)]);
            double dzh = za - zb;
            double gw = g.gw[at(i)];
            double ti = thv_if(i), ta = thv_if(i - 1);
            double rhoh = gw * rho_if(i) + (1.0 - gw) * rho_if(i - 1);
            double thh = gw * ti + (1.0 - gw) * ta;
            double thph = gw * (ti - g.theta_ref[at(i)]) + (1.0 - gw) * (ta - g.theta_ref[at(i - 1)]);
            double ppa = s.pi[at(i - 1)] - g.pi_ref[at(i - 1)];
            double ppb = s.pi[at(i)] - g.pi_ref[at(i)];
            double wn = s.w[at(i)];
            double pterm = (1.0 - beta) * thh * (ppa - ppb) / dzh + thph * g.dref[at(i)];
            wh_b = wn + dt * (twv(i) - cpd * pterm);
            fx_b = rhoh * ((1.0 - beta) * wn - wcc[at(i)]);
            hx_b = thh * fx_b;
            al_b = beta * rhoh * thh;
            ga_b = dt * cpd * beta * thh / dzh;
        }
        double dz = g.zh[at(k)] - g.zh[at(k + 1)];
        double sr = 0.0, st = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            sr += sl[j] * wk.flx[int64_t(k) * ne + e[j]];
            st += sl[j] * wk.hfl[int64_t(k) * ne + e[j]];
        }
        double divr = sr / area / dz;
        double divt = st / area / dz;
        double rn = s.rho[at(k)], tn = s.thv[at(k)], pn = s.pi[at(k)];
        double ppn = pn - g.pi_ref[at(k)];
        double rh = rn - dt * (divr + (fx_k - fx_b) / dz);
        double bk = dt * (rd / cvd) * pn / (rn * tn * dz);
        double ph = ppn - bk * dz * (divt + (hx_k - hx_b) / dz);
        wk.rh[at(k)] = rh;
        wk.ph[at(k)] = ph;
        if (k >= 1) {  // tridiagonal row of half level k
            double a = -ga_k * b_prev * al_prev;
            double b = 1.0 + ga_k * al_k * (b_prev + bk);
            double cc = -ga_k * bk * al_b;
            double r = wh_k - ga_k * (ph_prev - ph);
            double cpk, dpk;
            if (k == 1) {
                cpk = cc / b;
                dpk = r / b;
            } else {
                double den = b - a * cp_prev;
                cpk = cc / den;
                dpk = (r - a * dp_prev) / den;
            }
            wk.cp[at(k)] = cpk;
            wk.dp[at(k)] = dpk;
            cp_prev = cpk;
            dp_prev = dpk;
        }
        ph_prev = ph;
        b_prev = bk;
        al_prev = al_k;
        fx_k = fx_b;
        hx_k = hx_b;
        al_k = al_b;
        ga_k = ga_b;
        wh_k = wh_b;
    }
    // ---- back substitution, bottom to top, with the level updates ----
    double w_b = wcc[at(N)];          // w at half level k+1; kinematic value at the ground
    double fl_b = 0.0, alw_b = 0.0;   // implicit fluxes at half level k+1 (zero at the ground)
    w_out[at(N)] = w_b;
    for (int k = N - 1; k >= 0; --k) {
        double w_t = 0.0, fl_t = 0.0, alw_t = 0.0;  // half level k (zero at the lid)
        if (k >= 1) {
            // the bottom interior row has no super-diagonal
            w_t = (k == N - 1) ? wk.dp[at(k)] : wk.dp[at(k)] - wk.cp[at(k)] * w_b;
            double gw = g.gw[at(k)];
            double rhoh = gw * rho_if(k) + (1.0 - gw) * rho_if(k - 1);
            double thh = gw * thv_if(k) + (1.0 - gw) * thv_if(k - 1);
            double al = beta * rhoh * thh;
            fl_t = rhoh * w_t;
            alw_t = al * w_t;
            if (CORR) {
                double vf = rhoh * (beta * w_t + (1.0 - beta) * s.w[at(k)] - wcc[at(k)]);
                double acc = first ? 0.0 : s.wacc[at(k)];
                s.wacc[at(k)] = acc + vf / dnsub;
            }
        }
        double dz = g.zh[at(k)] - g.zh[at(k + 1)];
        double rn = s.rho[at(k)], tn = s.thv[at(k)], pn = s.pi[at(k)];
        double ppn = pn - g.pi_ref[at(k)];
        double bk = dt * (rd / cvd) * pn / (rn * tn * dz);
        double rnew = wk.rh[at(k)] - dt * beta * (fl_t - fl_b) / dz;
        double ppnew = wk.ph[at(k)] - bk * (alw_t - alw_b);
        double rt = rn * tn;
        double thnew = (rt + (cvd / rd) * (rt / pn) * (ppnew - ppn)) / rnew;
        if (CORR) {
            s.pi_prev[at(k)] = ppn;
            s.pi[at(k)] = g.pi_ref[at(k)] + ppnew;
        }
        rho_out[at(k)] = rnew;
        thv_out[at(k)] = thnew;
        w_out[at(k)] = w_t;
        w_b = w_t;
        fl_b = fl_t;
        alw_b = alw_t;
    }
    if (CORR && first) {
        s.wacc[at(0)] = 0.0;
        s.wacc[at(N)] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// diagnostics: fixed-order two-level reduction (per-block partials, then one block)

__global__ void k_diag_partial(int64_t nc, int N, const double *__restrict__ area,
                               const double *__restrict__ zh, const double *__restrict__ rho,
                               const double *__restrict__ thv, double *__restrict__ part) {
    __shared__ double s1[BLOCK], s2[BLOCK];
    int64_t c = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (c < nc) {
        for (int k = 0; k < N; ++k) {
            double vol = area[c] * (zh[int64_t(k) * nc + c] - zh[int64_t(k + 1) * nc + c]);
            double r = rho[int64_t(k) * nc + c];
            a += vol * r;
            b += vol * r * thv[int64_t(k) * nc + c];
        }
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

__global__ void k_diag_final(int nparts, const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double s1[BLOCK], s2[BLOCK];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nparts; i += BLOCK) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s1[0];
        out[1] = s2[0];
    }
}

__global__ void k_finite(int64_t n, const double *__restrict__ x, int *__restrict__ flag) {
    int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
    if (i < n && !isfinite(x[i])) flag[0] = 1;  // benign race: every writer stores 1
}

}  // namespace

const char *const kKernelNames[K_NUM] = {"vt_edge", "vertex", "cell_vt", "edge_pred",
                                         "column_pred", "edge_corr", "column_corr"};

hipError_t launch_metrics(const Grid &g, const Params &p, hipStream_t st) {
    hipLaunchKernelGGL(k_metrics_cell, dim3(nblocks(g.nc)), dim3(BLOCK), 0, st, g.nc, g.N, g.zh,
                       g.theta_ref, p.grav, p.cpd, g.gw, g.dref);
    hipLaunchKernelGGL(k_metrics_vert, dim3(nblocks(g.nv)), dim3(BLOCK), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_init_prev(nhdc_ctx *ctx, hipStream_t st) {
    int64_t n = int64_t(ctx->g.N) * ctx->g.nc;
    hipLaunchKernelGGL(k_init_prev, dim3(nblocks(n)), dim3(BLOCK), 0, st, n, ctx->s.pi,
                       ctx->g.pi_ref, ctx->s.pi_prev);
    return hipGetLastError();
}

#define LAUNCH(id, ...)                                      \
    do {                                                     \
        hipError_t e_ = timing_begin(ctx, (id), st);         \
        if (e_ != hipSuccess) return e_;                     \
        hipLaunchKernelGGL(__VA_ARGS__);                     \
        e_ = timing_end(ctx, st);                            \
        if (e_ != hipSuccess) return e_;                     \
    } while (0)

hipError_t launch_substep(nhdc_ctx *ctx, double dt, int nsub, bool first, hipStream_t st) {
    const Grid &g = ctx->g;
    State &s = ctx->s;
    Work &w = ctx->w;
    const Params &p = ctx->p;
    // predictor
    LAUNCH(K_VT_EDGE, k_vt_edge, dim3(nblocks(g.ne)), dim3(BLOCK), 0, st, g, s.vn, w.vt);
    LAUNCH(K_VERTEX, k_vertex, dim3(nblocks(g.nv)), dim3(BLOCK), 0, st, g, s.vn, s.w, w.zeta, w.wv);
    LAUNCH(K_CELL_VT, k_cell_vt<false>, dim3(nblocks(g.nc)), dim3(BLOCK), 0, st, g, s.vn, w.vt,
           s.w, w.wv, w.kc, w.wcc0, w.tw0, w.dvn);
    LAUNCH(K_EDGE_PRED, k_edge_pred, dim3(nblocks(g.ne)), dim3(BLOCK), 0, st, g, s, w, p, dt);
    LAUNCH(K_COLUMN_PRED, k_column<false>, dim3(nblocks(g.nc)), dim3(BLOCK), 0, st, g, s, w, p, dt,
           nsub, int(first));
    // corrector
    LAUNCH(K_VT_EDGE, k_vt_edge, dim3(nblocks(g.ne)), dim3(BLOCK), 0, st, g, w.vns, w.vt);
    LAUNCH(K_VERTEX, k_vertex, dim3(nblocks(g.nv)), dim3(BLOCK), 0, st, g, w.vns, w.ws, w.zeta, w.wv);
    LAUNCH(K_CELL_VT, k_cell_vt<true>, dim3(nblocks(g.nc)), dim3(BLOCK), 0, st, g, w.vns, w.vt,
           w.ws, w.wv, w.kc, w.wcc1, w.tw1, w.dvn);
    LAUNCH(K_EDGE_CORR, k_edge_corr, dim3(nblocks(g.ne)), dim3(BLOCK), 0, st, g, s, w, p, dt,
           nsub, int(first));
    LAUNCH(K_COLUMN_CORR, k_column<true>, dim3(nblocks(g.nc)), dim3(BLOCK), 0, st, g, s, w, p, dt,
           nsub, int(first));
    return hipGetLastError();
}

hipError_t launch_diag(nhdc_ctx *ctx, double *out2, hipStream_t st) {
    const Grid &g = ctx->g;
    unsigned nb = nblocks(g.nc);
    double *part = ctx->w.red;
    hipLaunchKernelGGL(k_diag_partial, dim3(nb), dim3(BLOCK), 0, st, g.nc, g.N, g.c_area, g.zh,
                       ctx->s.rho, ctx->s.thv, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(BLOCK), 0, st, int(nb), part, out2);
    return hipGetLastError();
}

hipError_t launch_finite(nhdc_ctx *ctx, int *flag, hipStream_t st) {
    const Grid &g = ctx->g;
    const State &s = ctx->s;
    const int64_t NC = int64_t(g.N) * g.nc, NC1 = int64_t(g.N + 1) * g.nc, NE = int64_t(g.N) * g.ne;
    const double *arrs[4] = {s.rho, s.pi, s.thv, s.pi_prev};
    for (int i = 0; i < 4; ++i)
        hipLaunchKernelGGL(k_finite, dim3(nblocks(NC)), dim3(BLOCK), 0, st, NC, arrs[i], flag);
    hipLaunchKernelGGL(k_finite, dim3(nblocks(NC1)), dim3(BLOCK), 0, st, NC1, s.w, flag);
    hipLaunchKernelGGL(k_finite, dim3(nblocks(NE)), dim3(BLOCK), 0, st, NE, s.vn, flag);
    return hipGetLastError();
}

}  // namespace nhdc

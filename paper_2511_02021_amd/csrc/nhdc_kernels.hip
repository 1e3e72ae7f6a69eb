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
// w_cc, w tendency T_w and (optionally) the divergence of vn.  The cell, its
// three neighbours and its three vertices are each gathered once per level;
// the own column's w and zh are carried in registers (levels i-1, i, i+1).
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
    int32_t e[3], nb[3], vx[3];
    bool out[3];
    double de[3], le[3], sl[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        e[j] = g.c_e[j * nc + c];
        nb[j] = g.c_n[j * nc + c];
        vx[j] = g.c_v[j * nc + c];
        sl[j] = g.c_sl[j * nc + c];
        out[j] = sl[j] > 0.0;
        de[j] = g.e_de[e[j]];
        le[j] = g.e_le[e[j]];
    }
    const double area = g.c_area[c];
    double vnp[3] = {0.0, 0.0, 0.0}, vtp[3] = {0.0, 0.0, 0.0};  // full level i-1
    double w_m = 0.0, w_0 = w[c], w_p = w[nc + c];               // own w at i-1, i, i+1
    double z_m = 0.0, z_0 = g.zh[c], z_p = g.zh[nc + c];         // own zh at i-1, i, i+1
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
            const bool interior = i < N;
            const int64_t oc = int64_t(i) * nc, ov = int64_t(i) * nv;
            double zn[3], zv[3], gwn[3] = {0.0, 0.0, 0.0}, wnb[3] = {0.0, 0.0, 0.0},
                   wvv[3] = {0.0, 0.0, 0.0};
            double gwc = interior ? g.gw[oc + c] : 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                zn[j] = g.zh[oc + nb[j]];
                zv[j] = g.zhv[ov + vx[j]];
                if (interior) {
                    gwn[j] = g.gw[oc + nb[j]];
                    wnb[j] = w[oc + nb[j]];
                    wvv[j] = wv[ov + vx[j]];
                }
            }
            double ccs = 0.0, adv = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int jn = j == 2 ? 0 : j + 1;
                // edge j runs from vertex slot j to j+1: (v1, v2) in that order when
                // its normal points out of this cell, reversed otherwise
                double zc1 = out[j] ? z_0 : zn[j], zc2 = out[j] ? zn[j] : z_0;
                double zv1 = out[j] ? zv[j] : zv[jn], zv2 = out[j] ? zv[jn] : zv[j];
                double hn, ht;
                if (interior) {
                    double gg = 0.5 * (out[j] ? gwc + gwn[j] : gwn[j] + gwc);
                    hn = gg * vni[j] + (1.0 - gg) * vnp[j];
                    ht = gg * vti[j] + (1.0 - gg) * vtp[j];
                } else {
                    hn = vnp[j];
                    ht = vtp[j];
                }
                double snh = (zc2 - zc1) / de[j];
                double sth = (zv2 - zv1) / le[j];
                ccs += hn * snh + ht * sth;
                if (interior) {
                    double wc1 = out[j] ? w_0 : wnb[j], wc2 = out[j] ? wnb[j] : w_0;
                    double wv1 = out[j] ? wvv[j] : wvv[jn], wv2 = out[j] ? wvv[jn] : wvv[j];
                    double gw_ = (wc2 - wc1) / de[j];
                    double tw_ = (wv2 - wv1) / le[j];
                    adv += hn * gw_ + ht * tw_;
                }
            }
            double wcci = ccs / 3.0;
            wcc[oc + c] = wcci;
            if (interior) {
                double hadv = adv / 3.0;
                double om = w_0 - wcci;
                double dwdz = (w_m - w_p) / (z_m - z_p);
                tw[oc + c] = -hadv - om * dwdz;
            } else {
                tw[oc + c] = 0.0;
            }
        }
        if (i < N) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                vnp[j] = vni[j];
                vtp[j] = vti[j];
            }
        }
        w_m = w_0;
        w_0 = w_p;
        z_m = z_0;
        z_0 = z_p;
        if (i + 2 <= N) {
            w_p = w[int64_t(i + 2) * nc + c];
            z_p = g.zh[int64_t(i + 2) * nc + c];
        }
    }
}

// Edge kernels march one edge down its column.  Per level they gather each
// cell field at c1 and c2 once; values needed at adjacent levels (the Exner
// perturbation and heights for the vertical derivative, interpolation
// weights, contravariant velocity at the two half levels) are carried in
// registers from the previous level.

__device__ __forceinline__ double exner_x(const Grid &g, const State &s, double eps, int k,
                                          int32_t c) {
    int64_t o = int64_t(k) * g.nc + c;
    double pp = s.pi[o] - g.pi_ref[o];
    return (1.0 + eps) * pp - eps * s.pi_prev[o];
}

// Predictor on edges: vn tendency of state n, terrain-corrected gradient of
// the extrapolated Exner perturbation, predicted vn, mass and theta fluxes.
__global__ void __launch_bounds__(BLOCK) k_edge_pred(Grid g, State s, Work wk, Params p,
                                                     double dt) {
    int64_t e = gid();
    const int64_t ne = g.ne, nc = g.nc, nv = g.nv;
    const int N = g.N;
    if (e >= ne) return;
    const int32_t c1 = g.e_c[e], c2 = g.e_c[ne + e], v1 = g.e_v[e], v2 = g.e_v[ne + e];
    const double de = g.e_de[e], fe = g.fe[e], eps = p.extrap;
    // heights zh at k, k+1, k+2; Exner perturbation and full-level heights at k-1, k, k+1
    double h1_0 = g.zh[c1], h1_1 = g.zh[nc + c1], h1_2 = g.zh[2 * nc + c1];
    double h2_0 = g.zh[c2], h2_1 = g.zh[nc + c2], h2_2 = g.zh[2 * nc + c2];
    double p1_m = 0.0, p1_0 = exner_x(g, s, eps, 0, c1), p1_p = exner_x(g, s, eps, 1, c1);
    double p2_m = 0.0, p2_0 = exner_x(g, s, eps, 0, c2), p2_p = exner_x(g, s, eps, 1, c2);
    double z1_m = 0.0, z1_0 = 0.5 * (h1_0 + h1_1), z1_p = 0.5 * (h1_1 + h1_2);
    double z2_m = 0.0, z2_0 = 0.5 * (h2_0 + h2_1), z2_p = 0.5 * (h2_1 + h2_2);
    double gk1 = 0.0, gk2 = 0.0;   // interpolation weights at half level k
    double om1 = 0.0, om2 = 0.0;   // contravariant vertical velocity at half level k
    double vnm = 0.0, vn0 = s.vn[e];
    for (int k = 0; k < N; ++k) {
        const int64_t o = int64_t(k) * ne + e, oc = int64_t(k) * nc, ov = int64_t(k) * nv;
        const bool last = k + 1 == N;
        double vn1 = vn0, gb1 = 0.0, gb2 = 0.0, omb1 = 0.0, omb2 = 0.0;
        if (!last) {
            const int64_t ob = oc + nc;
            vn1 = s.vn[o + ne];
            gb1 = g.gw[ob + c1];
            gb2 = g.gw[ob + c2];
            omb1 = s.w[ob + c1] - wk.wcc0[ob + c1];
            omb2 = s.w[ob + c2] - wk.wcc0[ob + c2];
        }
        double vnh_k = vn0, vnh_k1 = vn0;
        if (k > 0) {
            double gg = 0.5 * (gk1 + gk2);
            vnh_k = gg * vn0 + (1.0 - gg) * vnm;
        }
        if (!last) {
            double gg = 0.5 * (gb1 + gb2);
            vnh_k1 = gg * vn1 + (1.0 - gg) * vn0;
        }
        double dz1 = h1_0 - h1_1, dz2 = h2_0 - h2_1;
        double dze = 0.5 * (dz1 + dz2);
        double gradk = (wk.kc[oc + c2] - wk.kc[oc + c1]) / de;
        double ze = 0.5 * (wk.zeta[ov + v1] + wk.zeta[ov + v2]);
        double of1 = 0.5 * (om1 + omb1);
        double of2 = 0.5 * (om2 + omb2);
        double obar = 0.5 * (of1 + of2);
        double dvdz = (vnh_k - vnh_k1) / dze;
        double tvn = -gradk + (ze + fe) * wk.vt[o] - obar * dvdz;
        // vertical derivative of the extrapolated perturbation, one-sided at the ends
        double pa1 = k == 0 ? p1_0 : p1_m, pb1 = last ? p1_0 : p1_p;
        double za1 = k == 0 ? z1_0 : z1_m, zb1 = last ? z1_0 : z1_p;
        double pa2 = k == 0 ? p2_0 : p2_m, pb2 = last ? p2_0 : p2_p;
        double za2 = k == 0 ? z2_0 : z2_m, zb2 = last ? z2_0 : z2_p;
        double dpz1 = (pa1 - pb1) / (za1 - zb1);
        double dpz2 = (pa2 - pb2) / (za2 - zb2);
        double sn = (z2_0 - z1_0) / de;
        double gl = (p2_0 - p1_0) / de;
        double dzp = 0.5 * (dpz1 + dpz2);
        double gp = gl - sn * dzp;
        double the = 0.5 * (s.thv[oc + c1] + s.thv[oc + c2]);
        double rhe = 0.5 * (s.rho[oc + c1] + s.rho[oc + c2]);
        double vns = vn0 + dt * (tvn - p.cpd * the * gp);
        double f = rhe * vns * dze;
        wk.tvn0[o] = tvn;
        wk.gp[o] = gp;
        wk.vns[o] = vns;
        wk.flx[o] = f;
        wk.hfl[o] = the * f;
        // shift the level windows
        vnm = vn0;
        vn0 = vn1;
        gk1 = gb1;
        gk2 = gb2;
        om1 = omb1;
        om2 = omb2;
        p1_m = p1_0;
        p1_0 = p1_p;
        p2_m = p2_0;
        p2_0 = p2_p;
        z1_m = z1_0;
        z1_0 = z1_p;
        z2_m = z2_0;
        z2_0 = z2_p;
        h1_0 = h1_1;
        h1_1 = h1_2;
        h2_0 = h2_1;
        h2_1 = h2_2;
        if (k + 2 < N) {
            p1_p = exner_x(g, s, eps, k + 2, c1);
            p2_p = exner_x(g, s, eps, k + 2, c2);
            h1_2 = g.zh[int64_t(k + 3) * nc + c1];
            h2_2 = g.zh[int64_t(k + 3) * nc + c2];
            z1_p = 0.5 * (h1_1 + h1_2);
            z2_p = 0.5 * (h2_1 + h2_2);
        }
    }
}

// Corrector on edges: vn^{n+1} from the averaged tendencies, the predictor's
// Exner gradient with the predicted theta_v, and divergence damping; fluxes
// with state-n edge values; FP64 flux accumulation.
__global__ void __launch_bounds__(BLOCK) k_edge_corr(Grid g, State s, Work wk, Params p, double dt,
                                                     int nsub, int first) {
    int64_t e = gid();
    const int64_t ne = g.ne, nc = g.nc, nv = g.nv;
    const int N = g.N;
    if (e >= ne) return;
    const int32_t c1 = g.e_c[e], c2 = g.e_c[ne + e], v1 = g.e_v[e], v2 = g.e_v[ne + e];
    const double de = g.e_de[e], fe = g.fe[e];
    const double cv = p.wgt_corr;
    const double dnsub = double(nsub);
    double h1_0 = g.zh[c1], h2_0 = g.zh[c2];  // zh at level k
    double gk1 = 0.0, gk2 = 0.0, om1 = 0.0, om2 = 0.0;
    double vnm = 0.0, vn0 = wk.vns[e];  // predicted vn at levels k-1, k
    for (int k = 0; k < N; ++k) {
        const int64_t o = int64_t(k) * ne + e, oc = int64_t(k) * nc, ov = int64_t(k) * nv;
        const bool last = k + 1 == N;
        double vn1 = vn0, gb1 = 0.0, gb2 = 0.0, omb1 = 0.0, omb2 = 0.0;
        if (!last) {
            const int64_t ob = oc + nc;
            vn1 = wk.vns[o + ne];
            gb1 = g.gw[ob + c1];
            gb2 = g.gw[ob + c2];
            omb1 = wk.ws[ob + c1] - wk.wcc1[ob + c1];
            omb2 = wk.ws[ob + c2] - wk.wcc1[ob + c2];
        }
        double vnh_k = vn0, vnh_k1 = vn0;
        if (k > 0) {
            double gg = 0.5 * (gk1 + gk2);
            vnh_k = gg * vn0 + (1.0 - gg) * vnm;
        }
        if (!last) {
            double gg = 0.5 * (gb1 + gb2);
            vnh_k1 = gg * vn1 + (1.0 - gg) * vn0;
        }
        double h1_b = g.zh[oc + nc + c1], h2_b = g.zh[oc + nc + c2];
        double dz1 = h1_0 - h1_b, dz2 = h2_0 - h2_b;
        double dze = 0.5 * (dz1 + dz2);
        double gradk = (wk.kc[oc + c2] - wk.kc[oc + c1]) / de;
        double ze = 0.5 * (wk.zeta[ov + v1] + wk.zeta[ov + v2]);
        double of1 = 0.5 * (om1 + omb1);
        double of2 = 0.5 * (om2 + omb2);
        double obar = 0.5 * (of1 + of2);
        double dvdz = (vnh_k - vnh_k1) / dze;
        double tvn1 = -gradk + (ze + fe) * wk.vt[o] - obar * dvdz;
        double ths = 0.5 * (wk.thvs[oc + c1] + wk.thvs[oc + c2]);
        double tend = (1.0 - cv) * wk.tvn0[o] + cv * tvn1 - p.cpd * ths * wk.gp[o];
        double gdiv = (wk.dvn[oc + c2] - wk.dvn[oc + c1]) / de;
        double vnn = s.vn[o] + dt * tend + p.div_damp * g.abar * gdiv;
        double the = 0.5 * (s.thv[oc + c1] + s.thv[oc + c2]);
        double rhe = 0.5 * (s.rho[oc + c1] + s.rho[oc + c2]);
        double f = rhe * vnn * dze;
        s.vn[o] = vnn;
        wk.flx[o] = f;
        wk.hfl[o] = the * f;
        double acc = first ? 0.0 : s.facc[o];
        s.facc[o] = acc + f / dnsub;
        vnm = vn0;
        vn0 = vn1;
        gk1 = gb1;
        gk2 = gb2;
        om1 = omb1;
        om2 = omb2;
        h1_0 = h1_b;
        h2_0 = h2_b;
    }
}

// ---------------------------------------------------------------------------
// column: horizontal divergences, explicit parts, tridiagonal solve in w
// (Thomas, no pivoting; factors and the explicit rho / Exner parts kept in
// global scratch), then rho, Exner and theta_v.  One lane per column, 64
// adjacent columns per wavefront, levels in sequence; values of the level
// above and below are carried in registers, and the interpolation weight and
// reference derivative are recomputed from zh and theta_ref rather than read.
// CORR selects the corrector: interface state averaged between n and the
// prediction, averaged w tendency, in-place update of the state, Exner
// history and flux accumulation.
template <bool CORR>
__global__ void __launch_bounds__(BLOCK) k_column(Grid g, State s, Work wk, Params p, double dt,
                                                  int nsub, int first) {
    int64_t c = gid();
    const int64_t nc = g.nc, ne = g.ne;
    const int N = g.N;
    if (c >= nc) return;
    const double beta = p.beta, cpd = p.cpd, rd = p.rd, cvd = p.cpd - p.rd, grav = p.grav;
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
    // values of one full level
    struct Lev {
        double rn, tn, pn, prf, trf, ri, ti;
    };
    auto load = [&](int k) {
        Lev L;
        L.rn = s.rho[at(k)];
        L.tn = s.thv[at(k)];
        L.pn = s.pi[at(k)];
        L.prf = g.pi_ref[at(k)];
        L.trf = g.theta_ref[at(k)];
        if (CORR) {
            L.ri = 0.5 * (L.rn + wk.rhos[at(k)]);
            L.ti = 0.5 * (L.tn + wk.thvs[at(k)]);
        } else {
            L.ri = L.rn;
            L.ti = L.tn;
        }
        return L;
    };
    auto twv = [&](int i) {
        return CORR ? (1.0 - cv) * wk.tw0[at(i)] + cv * wk.tw1[at(i)] : wk.tw0[at(i)];
    };
    // ---- forward sweep, top to bottom ----
    // carried: explicit fluxes, alpha, gamma and W-hat of half level k (top of
    // level k); Pi-hat and B of level k-1; alpha of half level k-1; Thomas
    // factors; level k and zh at k, k+1, k+2.
    double fx_k = 0.0, hx_k = 0.0, al_k = 0.0, ga_k = 0.0, wh_k = 0.0;
    double ph_prev = 0.0, b_prev = 0.0, al_prev = 0.0, cp_prev = 0.0, dp_prev = 0.0;
    Lev cur = load(0), nxt = cur;
    double h0 = g.zh[at(0)], h1 = g.zh[at(1)], h2 = g.zh[at(2)];
    for (int k = 0; k < N; ++k) {
        double fx_b = 0.0, hx_b = 0.0, al_b = 0.0, ga_b = 0.0, wh_b = 0.0;
        const int i = k + 1;  // bottom interface of level k
        if (i < N) {
            nxt = load(i);
            double za = 0.5 * (h0 + h1);
            double zb = 0.5 * (h1 + h2);
            double dzh = za - zb;
            double gw = (za - h1) / (za - zb);
            double rhoh = gw * nxt.ri + (1.0 - gw) * cur.ri;
            double thh = gw * nxt.ti + (1.0 - gw) * cur.ti;
            double thph = gw * (nxt.ti - nxt.trf) + (1.0 - gw) * (cur.ti - cur.trf);
            double threfh = gw * nxt.trf + (1.0 - gw) * cur.trf;
            double dref = -grav / (cpd * threfh);
            double ppa = cur.pn - cur.prf;
            double ppb = nxt.pn - nxt.prf;
            double wn = s.w[at(i)];
            double pterm = (1.0 - beta) * thh * (ppa - ppb) / dzh + thph * dref;
            wh_b = wn + dt * (twv(i) - cpd * pterm);
            fx_b = rhoh * ((1.0 - beta) * wn - wcc[at(i)]);
            hx_b = thh * fx_b;
            al_b = beta * rhoh * thh;
            ga_b = dt * cpd * beta * thh / dzh;
        }
        double dz = h0 - h1;
        double sr = 0.0, st = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            sr += sl[j] * wk.flx[int64_t(k) * ne + e[j]];
            st += sl[j] * wk.hfl[int64_t(k) * ne + e[j]];
        }
        double divr = sr / area / dz;
        double divt = st / area / dz;
        double ppn = cur.pn - cur.prf;
        double rh = cur.rn - dt * (divr + (fx_k - fx_b) / dz);
        double bk = dt * (rd / cvd) * cur.pn / (cur.rn * cur.tn * dz);
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
        cur = nxt;
        h0 = h1;
        h1 = h2;
        if (k + 3 <= N) h2 = g.zh[at(k + 3)];
    }
    // ---- back substitution, bottom to top, with the level updates ----
    double w_b = wcc[at(N)];          // w at half level k+1; kinematic value at the ground
    double fl_b = 0.0, alw_b = 0.0;   // implicit fluxes at half level k+1 (zero at the ground)
    w_out[at(N)] = w_b;
    double hb = g.zh[at(N)], hk = g.zh[at(N - 1)];  // zh at k+1, k
    Lev lk = load(N - 1);
    for (int k = N - 1; k >= 0; --k) {
        double w_t = 0.0, fl_t = 0.0, alw_t = 0.0;  // half level k (zero at the lid)
        double ha = 0.0;
        Lev la = lk;
        if (k >= 1) {
            ha = g.zh[at(k - 1)];
            la = load(k - 1);
            // the bottom interior row has no super-diagonal
            w_t = (k == N - 1) ? wk.dp[at(k)] : wk.dp[at(k)] - wk.cp[at(k)] * w_b;
            double za = 0.5 * (ha + hk);
            double zb = 0.5 * (hk + hb);
            double gw = (za - hk) / (za - zb);
            double rhoh = gw * lk.ri + (1.0 - gw) * la.ri;
            double thh = gw * lk.ti + (1.0 - gw) * la.ti;
            double al = beta * rhoh * thh;
            fl_t = rhoh * w_t;
            alw_t = al * w_t;
            if (CORR) {
                double vf = rhoh * (beta * w_t + (1.0 - beta) * s.w[at(k)] - wcc[at(k)]);
                double acc = first ? 0.0 : s.wacc[at(k)];
                s.wacc[at(k)] = acc + vf / dnsub;
            }
        }
        double dz = hk - hb;
        double ppn = lk.pn - lk.prf;
        double bk = dt * (rd / cvd) * lk.pn / (lk.rn * lk.tn * dz);
        double rnew = wk.rh[at(k)] - dt * beta * (fl_t - fl_b) / dz;
        double ppnew = wk.ph[at(k)] - bk * (alw_t - alw_b);
        double rt = lk.rn * lk.tn;
        double thnew = (rt + (cvd / rd) * (rt / lk.pn) * (ppnew - ppn)) / rnew;
        if (CORR) {
            s.pi_prev[at(k)] = ppn;
            s.pi[at(k)] = lk.prf + ppnew;
        }
        rho_out[at(k)] = rnew;
        thv_out[at(k)] = thnew;
        w_out[at(k)] = w_t;
        w_b = w_t;
        fl_b = fl_t;
        alw_b = alw_t;
        hb = hk;
        hk = ha;
        lk = la;
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

// nhdc_runtime.hip -- host side of libnhdc: context, validation, stencil
// coefficients, device memory, state transfer, the step driver, level-tile
// autotuning and per-kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "nhdc_host.h"
#include "nhdc_internal.h"

// host-side coefficients are formed without contraction, as the operators form them
#pragma clang fp contract(off)

using namespace nhdc;

namespace nhdc {

int set_err(std::string &err, int code, const std::string &msg) {
    err = msg;
    return code;
}

int hip_fail(std::string &err, hipError_t e, const char *where) {
    return set_err(err, NHDC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

void *dev_alloc(const Allocator &a, size_t bytes) {
    void *p = nullptr;
    if (a.alloc) {
        p = a.alloc(bytes, a.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    return p;
}

void dev_free(const Allocator &a, void *p) {
    if (!p) return;
    if (a.free_) a.free_(p, a.user);
    else (void)hipFree(p);
}

hipError_t timing_begin(Timing *tm, int id, hipStream_t st) {
    if (!tm || !tm->on) return hipSuccess;
    size_t slot = tm->ids.size();
    while (tm->ev.size() < 2 * (slot + 1)) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        tm->ev.push_back(e);
    }
    tm->ids.push_back(id);
    return hipEventRecord(tm->ev[2 * slot], st);
}

hipError_t timing_end(Timing *tm, hipStream_t st) {
    if (!tm || !tm->on) return hipSuccess;
    return hipEventRecord(tm->ev[2 * (tm->ids.size() - 1) + 1], st);
}

const FormOps &form_ops(int precision) {
    static const FormOps fp64{launch_substep_fp64, launch_diffusion_fp64, launch_tracers_fp64,
                              launch_persistent_fp64, persistent_blocks_per_cu_fp64};
    static const FormOps mixed{launch_substep_mixed, launch_diffusion_mixed, launch_tracers_mixed,
                               launch_persistent_mixed, persistent_blocks_per_cu_mixed};
    static const FormOps vn32{launch_substep_mixed_vn32, launch_diffusion_mixed_vn32,
                              launch_tracers_mixed_vn32, launch_persistent_mixed_vn32,
                              persistent_blocks_per_cu_mixed_vn32};
    return precision == NHDC_MIXED ? mixed : precision == NHDC_MIXED_VN32 ? vn32 : fp64;
}

hipError_t run_step(const Launcher &L, const double *dt, int nsub, Timing *tm, hipStream_t st) {
    const FormOps &f = form_ops(L.precision);
    Sub sub;
    for (int i = 0; i < L.n; ++i) sub.dt[i] = dt[i] / nsub;
    for (int i = L.n; i < MAX_INST; ++i) sub.dt[i] = 0.0;
    sub.nsub = nsub;
    Sub whole = sub;  // the step's dt per instance (diffusion, tracers)
    for (int i = 0; i < L.n; ++i) whole.dt[i] = dt[i];
    if (L.tracers) {
        hipError_t e = f.tracers(L, whole, 0, tm, st);
        if (e != hipSuccess) return e;
    }
    for (int s = 0; s < nsub; ++s) {
        sub.first = s == 0;
        sub.last = s == nsub - 1;
        hipError_t e = f.substep(L, sub, tm, st);
        if (e != hipSuccess) return e;
    }
    if (L.smag) {  // the diffusion of vn over the whole step
        hipError_t e = f.diffusion(L, whole, tm, st);
        if (e != hipSuccess) return e;
    }
    if (L.tracers) {  // tracer transport with the step's averaged mass fluxes
        hipError_t e = f.tracers(L, whole, 1, tm, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t run_step_persistent(const Launcher &L, const PMaps *d_pm, int grid, const double *dt,
                               int nsub, hipStream_t st) {
    Sub sub;
    for (int i = 0; i < L.n; ++i) sub.dt[i] = dt[i] / nsub;
    for (int i = L.n; i < MAX_INST; ++i) sub.dt[i] = 0.0;
    sub.nsub = nsub;
    sub.first = 1;
    sub.last = nsub == 1;
    Sub whole = sub;
    for (int i = 0; i < L.n; ++i) whole.dt[i] = dt[i];
    const FormOps &f = form_ops(L.precision);
    hipError_t e = hipSuccess;
    if (L.tracers) e = f.tracers(L, whole, 0, nullptr, st);
    if (e != hipSuccess) return e;
    e = f.persistent(L, d_pm, sub, grid, st);
    if (e != hipSuccess) return e;
    if (L.smag) e = f.diffusion(L, whole, nullptr, st);
    if (e != hipSuccess) return e;
    if (L.tracers) e = f.tracers(L, whole, 1, nullptr, st);
    return e;
}

void rebuild_maps(Launcher &L, const std::vector<nhdc_ctx *> &ctxs, const Tune &t) {
    std::vector<const Grid *> grids;
    for (auto *c : ctxs) grids.push_back(&c->g);
    L.col_width = 0;
    int nmax = 0;
    for (auto *g : grids) nmax = g->N > nmax ? g->N : nmax;
    if (t.col_mode == 1)  // the level-parallel column: BLOCK lanes over col_width columns
        L.col_width = stg_width(nmax, device_max_lds(ctxs.empty() ? 0 : ctxs[0]->device));
    for (int k = 0; k < KIND_NUM; ++k) {
        const int ent = k == KIND_COLUMN ? L.col_width : 0;
        build_map(L.maps[k], L.nblocks[k], Kind(k), grids.data(), int(grids.size()), t, ent);
        L.block[k] = ent ? BLOCK : kind_block(Kind(k), t);
        L.dyn_lds[k] = ent ? stg_lds(ent, nmax)
                     : k == KIND_COLUMN ? occupancy_lds(t.col_waves, L.block[k]) : 0u;
    }
    Tune tt = t;
    tt.blk_col = BLOCK;
    tt.col_mode = 0;
    build_map(L.trmap, L.trblocks, KIND_COLUMN, grids.data(), int(grids.size()), tt);
}

// The descriptor of one instance in the precision of its work arrays.
template <class RT>
static Inst<RT> make_inst(const nhdc_ctx *c, const Work<RT> &w) {
    Inst<RT> I;
    I.g = c->g;
    I.s = c->s;
    I.w = w;
    I.p = c->p;
    I.tr = c->tr;
    return I;
}

int upload_insts(Launcher &L, const std::vector<nhdc_ctx *> &ctxs, std::string &err) {
    const int n = int(ctxs.size());
    const int prec = ctxs[0]->precision;
    std::vector<char> host;
    if (fp32_stencils(prec)) {
        std::vector<Inst<float>> v;
        for (auto *c : ctxs) v.push_back(make_inst<float>(c, c->wf));
        const char *b = reinterpret_cast<const char *>(v.data());
        host.assign(b, b + v.size() * sizeof(Inst<float>));
    } else {
        std::vector<Inst<double>> v;
        for (auto *c : ctxs) v.push_back(make_inst<double>(c, c->wd));
        const char *b = reinterpret_cast<const char *>(v.data());
        host.assign(b, b + v.size() * sizeof(Inst<double>));
    }
    if (L.d_insts) {
        hipError_t e = hipDeviceSynchronize();  // no launch may still read the old descriptors
        if (e != hipSuccess) return hip_fail(err, e, "instance descriptors: sync");
        dev_free(L.al, L.d_insts);
        L.d_insts = nullptr;
    }
    L.d_insts = dev_alloc(L.al, host.size());
    if (!L.d_insts) return set_err(err, NHDC_ENOMEM, "instance descriptors: allocation failed");
    hipError_t e = hipMemcpy(L.d_insts, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(err, e, "instance descriptors: hipMemcpy");
    L.precision = prec;
    L.n = n;
    L.upwind = L.div4 = L.smag = L.sponge = L.tracers = L.vt_two = false;
    L.cvt_lds = true;
    for (auto *c : ctxs) {
        L.cvt_lds = L.cvt_lds && c->g.cvt_ok != 0;
        L.vt_two = L.vt_two || c->g.eb_max > BLOCK;
        L.tracers = L.tracers || c->tr.nt > 0;
        L.sponge = L.sponge || c->g.w_damp != nullptr;
        L.upwind = L.upwind || c->p.upwind != 0;
        L.div4 = L.div4 || c->p.div_damp4 != 0.0;
        L.smag = L.smag || c->p.smag > 0.0;
    }
    return NHDC_OK;
}

// ---- state snapshot (autotuning runs real steps) ----
// the state's arrays and their sizes in bytes
static void state_arrays(nhdc_ctx *c, std::vector<std::pair<double *, size_t>> &out) {
    const size_t NC = size_t(c->g.N) * c->g.nc * 8, NC1 = size_t(c->g.N + 1) * c->g.nc * 8,
                 NE = size_t(c->g.N) * c->g.ne * 8;
    const size_t NEV = size_t(c->g.N) * c->g.ne * size_t(vn_bytes(c->precision));
    out = {{c->s.vn, NEV}, {c->s.w, NC1}, {c->s.rho, NC}, {c->s.pi, NC}, {c->s.thv, NC},
           {c->s.pi_prev, NC}, {c->s.facc, NE}, {c->s.wacc, NC1}, {c->s.px, NC}};
    if (c->tr.nt) out.push_back({c->tr.q, size_t(c->tr.nt) * NC});
}

static int snapshot(const Allocator &al, const std::vector<nhdc_ctx *> &ctxs,
                    std::vector<void *> &buf, bool restore, hipStream_t st, std::string &err) {
    size_t q = 0;
    for (auto *c : ctxs) {
        std::vector<std::pair<double *, size_t>> arr;
        state_arrays(c, arr);
        for (auto &a : arr) {
            hipError_t e;
            if (!restore) {
                void *b = dev_alloc(al, a.second);
                if (!b) {
                    for (void *x : buf) dev_free(al, x);
                    buf.clear();
                    return set_err(err, NHDC_ENOMEM, "autotune: no memory for the state snapshot");
                }
                buf.push_back(b);
                e = hipMemcpyAsync(b, a.first, a.second, hipMemcpyDeviceToDevice, st);
            } else {
                e = hipMemcpyAsync(a.first, buf[q++], a.second, hipMemcpyDeviceToDevice, st);
            }
            if (e != hipSuccess) return hip_fail(err, e, "autotune: state copy");
        }
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(err, e, "autotune: sync");
    if (restore) {
        for (void *x : buf) dev_free(al, x);
        buf.clear();
    }
    return NHDC_OK;
}

// ---- JSON cache: one entry per line,
// "key": [lt_edge, lt_cell, lt_vert, block_column, block_vertex, column_waves, ms, column_mode] ----
constexpr int kBest = 8;
static bool cache_lookup(const char *path, const std::string &key, double best[kBest]) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line, pat = "\"" + key + "\":";
    while (std::getline(f, line)) {
        size_t p = line.find(pat);
        if (p == std::string::npos) continue;
        size_t a = line.find('[', p), b = line.find(']', p);
        if (a == std::string::npos || b == std::string::npos) return false;
        std::string body = line.substr(a + 1, b - a - 1);
        for (char &ch : body)
            if (ch == ',') ch = ' ';
        std::istringstream is(body);
        for (int i = 0; i < kBest; ++i)
            if (!(is >> best[i])) return false;
        return valid_block(int(best[3])) && valid_block(int(best[4])) && valid_waves(int(best[5])) &&
               valid_col_mode(int(best[7]));
    }
    return false;
}

static void cache_store(const char *path, const std::string &key, const double best[kBest]) {
    if (!path) return;
    std::vector<std::string> entries;
    {
        std::ifstream f(path);
        std::string line, pat = "\"" + key + "\":";
        while (f && std::getline(f, line)) {
            if (line.find("\":") == std::string::npos || line.find(pat) != std::string::npos) continue;
            while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
            entries.push_back(line);
        }
    }
    char buf[512];
    std::snprintf(buf, sizeof(buf), "  \"%s\": [%d, %d, %d, %d, %d, %d, %.6f, %d]", key.c_str(),
                  int(best[0]), int(best[1]), int(best[2]), int(best[3]), int(best[4]), int(best[5]),
                  best[6], int(best[7]));
    entries.push_back(buf);
    std::ofstream f(path, std::ios::trunc);
    f << "{\n";
    for (size_t i = 0; i < entries.size(); ++i)
        f << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
    f << "}\n";
}

int autotune(Launcher &L, Tune &tune, const std::vector<nhdc_ctx *> &ctxs, const double *dt,
             int nsub, const char *cache_path, double *best_out, hipStream_t st,
             std::string &err, const Stepper &stepper, const char *path_tag) {
    std::ostringstream ks;
    ks << (L.precision == NHDC_MIXED ? "mixed" : L.precision == NHDC_MIXED_VN32 ? "mixed_vn32" : "fp64")
       << "|" << path_tag << "|";
    for (size_t i = 0; i < ctxs.size(); ++i)
        ks << (i ? "," : "") << ctxs[i]->g.nc << "x" << ctxs[i]->g.N;
    const std::string key = ks.str();
    double best[kBest];
    auto apply = [&](const Tune &t) -> hipError_t {
        rebuild_maps(L, ctxs, t);
        return stepper.prepare ? stepper.prepare(t) : hipSuccess;
    };
    if (cache_lookup(cache_path, key, best)) {
        tune.lt_edge = int(best[0]);
        tune.lt_cell = int(best[1]);
        tune.lt_vert = int(best[2]);
        tune.blk_col = int(best[3]);
        tune.blk_vert = int(best[4]);
        tune.col_waves = int(best[5]);
        tune.col_mode = int(best[7]);
        hipError_t e = apply(tune);
        if (e != hipSuccess) return hip_fail(err, e, "autotune: set-up");
        if (best_out)
            for (int i = 0; i < kBest; ++i) best_out[i] = best[i];
        return NHDC_OK;
    }
    std::vector<void *> snap;
    int rc = snapshot(L.al, ctxs, snap, false, st, err);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        snapshot(L.al, ctxs, snap, true, st, err);
        return set_err(err, NHDC_EHIP, "autotune: hipEventCreate failed");
    }
    auto measure = [&](const Tune &t, double &ms) -> int {
        hipError_t e = apply(t);
        if (e == hipSuccess) e = stepper.step(dt, nsub, st);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < 2 && e == hipSuccess; ++r) e = stepper.step(dt, nsub, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float f = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
        if (e != hipSuccess) return hip_fail(err, e, "autotune: timed step");
        ms = f / 2.0;
        return NHDC_OK;
    };
    // coordinate search: each parameter in turn over its candidates, keeping
    // the best so far (the column mode first, as it changes what the column
    // block shapes mean; level tiles of edges, cells, vertices; block sizes
    // of the column and vertex kernels, when the path takes them)
    Tune bt = tune;
    double bms = 0.0;
    rc = measure(bt, bms);
    const int cand_m[] = {0, 1};
    const int cand_ec[] = {0, 48, 32, 16, 8, 4};
    const int cand_v[] = {0, 32, 16, 8, 4};
    const int cand_b[] = {256, 128, 64};
    const int cand_w[] = {3, 0, 2};
    const int nparam = stepper.block_sizes ? 7 : 3;
    for (int pi = 0; pi < nparam && !rc; ++pi) {
        // parameter order: [mode,] tiles e, c, v [, block column, block vertex, waves]
        const int param = stepper.block_sizes ? (pi == 0 ? 6 : pi - 1) : pi;
        const int *cand = param == 6 ? cand_m : param < 2 ? cand_ec : param == 2 ? cand_v
                        : param < 5 ? cand_b : cand_w;
        const int ncand = param == 6 ? 2 : param < 2 ? 6 : param == 2 ? 5 : 3;
        for (int q = 0; q < ncand; ++q) {
            Tune t = bt;
            int &slot = param == 0 ? t.lt_edge : param == 1 ? t.lt_cell : param == 2 ? t.lt_vert
                      : param == 3 ? t.blk_col : param == 4 ? t.blk_vert : param == 5 ? t.col_waves
                      : t.col_mode;
            if (slot == cand[q]) continue;
            slot = cand[q];
            double ms = 0.0;
            if ((rc = measure(t, ms))) break;
            if (ms < bms) {
                bms = ms;
                bt = t;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::string err2;
    int rc2 = snapshot(L.al, ctxs, snap, true, st, err2);
    if (rc) {  // the launches go back to the shapes they had (the last candidate's are set)
        (void)apply(tune);
        return rc;
    }
    if (rc2) return set_err(err, rc2, err2);
    tune = bt;
    hipError_t e = apply(tune);
    if (e != hipSuccess) return hip_fail(err, e, "autotune: set-up");
    best[0] = tune.lt_edge;
    best[1] = tune.lt_cell;
    best[2] = tune.lt_vert;
    best[3] = tune.blk_col;
    best[4] = tune.blk_vert;
    best[5] = tune.col_waves;
    best[6] = bms;
    best[7] = tune.col_mode;
    cache_store(cache_path, key, best);
    if (best_out)
        for (int i = 0; i < kBest; ++i) best_out[i] = best[i];
    return NHDC_OK;
}

void free_context(nhdc_ctx *ctx) {
    if (hipSetDevice(ctx->device) == hipSuccess) {
        (void)hipDeviceSynchronize();  // no pending work may touch the memory
        for (hipEvent_t e : ctx->tm.ev) (void)hipEventDestroy(e);
        dev_free(ctx->al, ctx->L.d_insts);
        for (void *q : ctx->allocs) dev_free(ctx->al, q);
        for (void *q : ctx->tr_allocs) dev_free(ctx->al, q);
        dev_free(ctx->al, ctx->arena);
    }
    delete ctx;
}

}  // namespace nhdc

namespace {

int set_err(nhdc_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

#define HIP_TRY(ctx, call)                                                  \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) return nhdc::hip_fail((ctx)->err, e_, #call); \
    } while (0)

// Arrays carved from the arena start on 2 MiB boundaries (measured faster
// than packing them at 256 bytes).
constexpr size_t kArenaAlign = size_t(2) << 20;

// Bytes of the arena: every array nhdc_upload_grid allocates, in its order,
// each rounded to kArenaAlign (cell_vt's block tables counted whether or not
// the grid's blocks fit them).
size_t arena_bytes(const nhdc_grid *g, const nhdc_vertical *v, const nhdc_params *p, int precision) {
    const int64_t nc = g->n_cells, ne = g->n_edges, nv = g->n_verts, N = v->n_lev;
    const int64_t NC = N * nc, NC1 = (N + 1) * nc, NE = N * ne, NV = N * nv, NV1 = (N + 1) * nv;
    const int64_t nbc = (nc + BLOCK - 1) / BLOCK, nbe = (ne + BLOCK - 1) / BLOCK;
    size_t total = 0;
    auto add = [&](int64_t n, size_t size) {
        total += (size_t(n > 0 ? n : 1) * size + kArenaAlign - 1) & ~(kArenaAlign - 1);
    };
    const bool f32 = fp32_stencils(precision);
    const size_t rt = f32 ? 4 : 8, vb = size_t(vn_bytes(precision));
    // connectivity and block tables (int32)
    for (int i = 0; i < 3; ++i) add(3 * nc, 4);                        // c_e, c_n, c_v
    add(nbc * CVT_E, 4); add(nbc * CVT_V, 4); add(nbc * CVT_X, 4); add(3 * nbc, 4);
    for (int i = 0; i < 3; ++i) add(3 * nc, 4);                        // c_el, c_vl, c_nl
    add(3 * nc, 4);                                                    // c_ns
    add(2 * ne, 4);                                                    // e_c
    add(nbe * 2 * BLOCK, 4); add(nbe, 4); add(2 * ne, 4);              // eb_cells, eb_n, e_loc
    add(2 * ne, 4); add(6 * nv, 4); add(6 * nv, 4);                    // e_v, v_e, v_c
    // FP64 coefficients, and their FP32 copies in the mixed forms
    const int64_t geo[] = {3 * nc, 9 * nc, 3 * nc, nc, nc, ne, ne, 3 * ne, ne, 6 * nv, 6 * nv, nv, nv};
    for (int64_t n : geo) add(n, 8);
    if (f32)
        for (int i = 0; i < 13; ++i)
            if (i != 3) add(geo[i], 4);                                // (no FP32 cell area)
    // heights and reference profiles
    add(NC1, 8); add(NC, 8); add(NC, 8); add(NV1, 8);
    if (p->upwind) { add(3 * ne, 8); add(3 * ne, 8); }
    if (g->edge_normal) add(3 * ne, 8);
    if (g->dual_frac) add(ne, 8);
    if (v->w_damp) add(N + 1, 8);
    add(2 * (N + 1) + 2 * N, 4);                                       // flat-top rows
    // state and accumulators
    for (int i = 0; i < 5; ++i) add(NC, 8);                            // rho, pi, thv, pi_prev, px
    add(NC1, 8); add(NC1, 8);                                          // w, wacc
    add(vb == 4 ? (NE + 1) / 2 : NE, 8); add(NE, 8);                   // vn, facc
    // work arrays
    add(NC, rt); add(NC, rt);                                          // kc, dvn
    for (int i = 0; i < 4; ++i) add(NC1, rt);                          // wcc0, tw0, wcc1, tw1
    add(NE, rt); add(NE, rt);                                          // vt, tvn0
    add(NV, rt); add(NV1, rt);                                         // zeta, wv
    add(NC, 8); add(NC, 8); add(NC1, 8);                               // rhos, thvs, ws
    add(vb == 4 ? (NE + 1) / 2 : NE, 8);                               // vns
    add(2 * NC, 8); add(2 * NC1, 8); add(2 * NE, 8);                   // rp, cd, fh
    if (p->upwind) add(6 * NC, 8);
    if (p->div_damp4 != 0.0) add(NC, rt);
    if (p->smag > 0.0) add(NC, rt);
    add(2 * nbc + 2, 8); add(1, 4);                                    // reduction partials, flag
    return total;
}

// Device array of n elements: carved from the context's arena while it has
// room, else a device allocation of its own.
template <class T>
int dalloc(nhdc_ctx *ctx, T **p, int64_t n, bool arena = true) {
    size_t bytes = size_t(n > 0 ? n : 1) * sizeof(T);
    const size_t carve = (bytes + kArenaAlign - 1) & ~(kArenaAlign - 1);
    if (arena && ctx->arena && ctx->arena_used + carve <= ctx->arena_size) {
        *p = reinterpret_cast<T *>(ctx->arena + ctx->arena_used);
        ctx->arena_used += carve;
        return NHDC_OK;
    }
    void *q = dev_alloc(ctx->al, bytes);
    if (!q)
        return set_err(ctx, NHDC_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                             " bytes failed" + (ctx->al.alloc ? " (caller's allocator)" : ""));
    ctx->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return NHDC_OK;
}

template <class T>
int upload(nhdc_ctx *ctx, T **p, const T *host, int64_t n) {
    int rc = dalloc(ctx, p, n);
    if (rc) return rc;
    HIP_TRY(ctx, hipMemcpy(*p, host, size_t(n) * sizeof(T), hipMemcpyHostToDevice));
    return NHDC_OK;
}

// FP32 copy of a device FP64 array
int upload_f32(nhdc_ctx *ctx, float **p, const double *dsrc, int64_t n) {
    int rc = dalloc(ctx, p, n);
    if (rc) return rc;
    HIP_TRY(ctx, launch_to_float(dsrc, *p, n, nullptr));
    return NHDC_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0; }

// The FP32-vn variant's conversions at the boundary: FP64 vn (host or
// device) into the FP32 store, and the FP32 store out as FP64; host data
// pass through a temporary device buffer.  Synchronous on `s` when a host
// buffer is involved.
int vn_to_f32(nhdc_ctx *ctx, const double *src, bool on_device, hipStream_t s) {
    const int64_t NE = int64_t(ctx->g.N) * ctx->g.ne;
    float *dst = reinterpret_cast<float *>(ctx->s.vn);
    if (on_device) {
        HIP_TRY(ctx, launch_to_float(src, dst, NE, s));
        return NHDC_OK;
    }
    double *tmp = static_cast<double *>(dev_alloc(ctx->al, size_t(NE) * 8));
    if (!tmp) return set_err(ctx, NHDC_ENOMEM, "init_state: no memory to convert vn");
    hipError_t e = hipMemcpyAsync(tmp, src, size_t(NE) * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_to_float(tmp, dst, NE, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(ctx->al, tmp);
    if (e != hipSuccess) return nhdc::hip_fail(ctx->err, e, "init_state: vn to FP32");
    return NHDC_OK;
}

int vn_to_f64(nhdc_ctx *ctx, double *dst, bool on_device, hipStream_t s) {
    const int64_t NE = int64_t(ctx->g.N) * ctx->g.ne;
    const float *src = reinterpret_cast<const float *>(ctx->s.vn);
    if (on_device) {
        HIP_TRY(ctx, launch_to_double(src, dst, NE, s));
        return NHDC_OK;
    }
    double *tmp = static_cast<double *>(dev_alloc(ctx->al, size_t(NE) * 8));
    if (!tmp) return set_err(ctx, NHDC_ENOMEM, "get_state: no memory to convert vn");
    hipError_t e = launch_to_double(src, tmp, NE, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dst, tmp, size_t(NE) * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(ctx->al, tmp);
    if (e != hipSuccess) return nhdc::hip_fail(ctx->err, e, "get_state: vn to FP64");
    return NHDC_OK;
}

int validate(nhdc_ctx *ctx, const nhdc_grid *g, const nhdc_vertical *v) {
    const int64_t nc = g->n_cells, ne = g->n_edges, nv = g->n_verts;
    if (nc <= 0 || ne <= 0 || nv <= 0) return set_err(ctx, NHDC_EGRID, "grid: empty");
    if (nv - ne + nc != 2) return set_err(ctx, NHDC_EGRID, "grid: Euler characteristic is not 2");
    if (nc > INT32_MAX / 3 || ne > INT32_MAX / 3 || nv > INT32_MAX / 3)
        return set_err(ctx, NHDC_EGRID, "grid: too many entities for int32 indices");
    if (!(g->radius > 0)) return set_err(ctx, NHDC_EGRID, "grid: radius must be positive");
    const int N = v->n_lev;
    if (N < 2 || N > NHDC_MAX_LEV) return set_err(ctx, NHDC_EINVAL, "vertical: n_lev out of range");
    for (int64_t c = 0; c < nc; ++c) {
        if (!finite_pos(g->cell_area[c])) return set_err(ctx, NHDC_EGRID, "grid: cell area <= 0");
        for (int j = 0; j < 3; ++j) {
            int64_t e = g->cell_edges[j * nc + c];
            if (e < 0 || e >= ne) return set_err(ctx, NHDC_EGRID, "grid: cell_edges out of range");
            int8_t s = g->cell_sign[j * nc + c];
            int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
            if (!((s == 1 && c1 == c) || (s == -1 && c2 == c)))
                return set_err(ctx, NHDC_EGRID, "grid: cell_sign inconsistent with edge_cells");
        }
    }
    std::vector<uint8_t> seen(ne, 0);
    for (int64_t c = 0; c < nc; ++c)
        for (int j = 0; j < 3; ++j) seen[g->cell_edges[j * nc + c]]++;
    for (int64_t e = 0; e < ne; ++e) {
        if (seen[e] != 2) return set_err(ctx, NHDC_EGRID, "grid: edge not shared by exactly two cells");
        for (int s = 0; s < 2; ++s) {
            int64_t c = g->edge_cells[s * ne + e], vv = g->edge_verts[s * ne + e];
            if (c < 0 || c >= nc) return set_err(ctx, NHDC_EGRID, "grid: edge_cells out of range");
            if (vv < 0 || vv >= nv) return set_err(ctx, NHDC_EGRID, "grid: edge_verts out of range");
        }
        if (g->edge_cells[e] == g->edge_cells[ne + e])
            return set_err(ctx, NHDC_EGRID, "grid: edge with identical cells");
        if (!finite_pos(g->edge_length[e]) || !finite_pos(g->dual_length[e]))
            return set_err(ctx, NHDC_EGRID, "grid: edge length <= 0");
    }
    for (int64_t vtx = 0; vtx < nv; ++vtx) {
        int val = g->vert_valence[vtx];
        if (val != 5 && val != 6) return set_err(ctx, NHDC_EGRID, "grid: valence not 5 or 6");
        if (!finite_pos(g->vert_area[vtx])) return set_err(ctx, NHDC_EGRID, "grid: dual area <= 0");
        for (int j = 0; j < 6; ++j) {
            int64_t e = g->vert_edges[j * nv + vtx], c = g->vert_cells[j * nv + vtx];
            if (j < val) {
                if (e < 0 || e >= ne || c < 0 || c >= nc)
                    return set_err(ctx, NHDC_EGRID, "grid: vertex ring index out of range");
                int8_t s = g->vert_sign[j * nv + vtx];
                bool is2 = g->edge_verts[ne + e] == vtx, is1 = g->edge_verts[e] == vtx;
                if (!((s == 1 && is2) || (s == -1 && is1)))
                    return set_err(ctx, NHDC_EGRID, "grid: vert_sign inconsistent with edge_verts");
            } else if (e != -1 || c != -1) {
                return set_err(ctx, NHDC_EGRID, "grid: pentagon pad slot must be -1");
            }
        }
    }
    for (int64_t c = 0; c < nc; ++c) {
        for (int i = 0; i < N; ++i) {
            double a = v->zh[int64_t(i) * nc + c], b = v->zh[int64_t(i + 1) * nc + c];
            if (!(std::isfinite(a) && std::isfinite(b) && a > b))
                return set_err(ctx, NHDC_EGRID, "vertical: zh not strictly decreasing");
            if (!finite_pos(v->pi_ref[int64_t(i) * nc + c]) || !finite_pos(v->theta_ref[int64_t(i) * nc + c]))
                return set_err(ctx, NHDC_EGRID, "vertical: reference state must be positive");
        }
    }
    return NHDC_OK;
}

template <class RT>
int alloc_work(nhdc_ctx *ctx, Work<RT> &W) {
    const int64_t nc = ctx->g.nc, ne = ctx->g.ne, nv = ctx->g.nv, N = ctx->g.N;
    const int64_t NC = N * nc, NC1 = (N + 1) * nc, NE = N * ne, NV = N * nv, NV1 = (N + 1) * nv;
    int rc;
    RT **rt_c[] = {&W.kc, &W.dvn};
    RT **rt_c1[] = {&W.wcc0, &W.tw0, &W.wcc1, &W.tw1};
    RT **rt_e[] = {&W.vt, &W.tvn0};
    for (auto q : rt_c)
        if ((rc = dalloc(ctx, q, NC))) return rc;
    for (auto q : rt_c1)
        if ((rc = dalloc(ctx, q, NC1))) return rc;
    for (auto q : rt_e)
        if ((rc = dalloc(ctx, q, NE))) return rc;
    if ((rc = dalloc(ctx, &W.zeta, NV))) return rc;
    if ((rc = dalloc(ctx, &W.wv, NV1))) return rc;
    HIP_TRY(ctx, hipMemset(W.wv, 0, sizeof(RT) * NV1));
    double **d_c[] = {&W.rhos, &W.thvs};
    for (auto q : d_c)
        if ((rc = dalloc(ctx, q, NC))) return rc;
    if ((rc = dalloc(ctx, &W.ws, NC1))) return rc;
    if ((rc = dalloc(ctx, &W.vns, vn_bytes(ctx->precision) == 4 ? (NE + 1) / 2 : NE))) return rc;
    // pairs of doubles read and written together
    if ((rc = dalloc(ctx, &W.rp, 2 * NC))) return rc;
    if ((rc = dalloc(ctx, &W.cd, 2 * NC1))) return rc;
    if ((rc = dalloc(ctx, &W.fh, 2 * NE))) return rc;
    if (ctx->p.upwind) {
        if ((rc = dalloc(ctx, &W.gq, 6 * NC))) return rc;
    }
    if (ctx->p.div_damp4 != 0.0 && (rc = dalloc(ctx, &W.dd4, NC))) return rc;
    if (ctx->p.smag > 0.0 && (rc = dalloc(ctx, &W.kh, NC))) return rc;
    return NHDC_OK;
}

int timing_collect(nhdc_ctx *ctx, hipStream_t s) {
    Timing &t = ctx->tm;
    if (!t.on) return NHDC_OK;
    HIP_TRY(ctx, hipStreamSynchronize(s));
    for (size_t i = 0; i < t.ids.size(); ++i) {
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]));
        t.total_ms[t.ids[i]] += ms;
        t.launches[t.ids[i]] += 1;
    }
    t.ids.clear();
    return NHDC_OK;
}

}  // namespace

extern "C" {

int nhdc_create(nhdc_ctx **out, int precision, int device) {
    if (!out) return NHDC_EINVAL;
    *out = nullptr;
    if (precision != NHDC_FP64 && precision != NHDC_MIXED && precision != NHDC_MIXED_VN32)
        return NHDC_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return NHDC_EHIP;
    }
    nhdc_ctx *ctx = new (std::nothrow) nhdc_ctx;
    if (!ctx) return NHDC_ENOMEM;
    ctx->device = device;
    ctx->precision = precision;
    *out = ctx;
    return NHDC_OK;
}

int nhdc_set_allocator(nhdc_ctx *ctx, void *(*alloc)(size_t bytes, void *user),
                       void (*free_)(void *ptr, void *user), void *user) {
    if (!ctx) return NHDC_EINVAL;
    if ((alloc == nullptr) != (free_ == nullptr))
        return set_err(ctx, NHDC_EINVAL, "set_allocator: give both callbacks or neither");
    if (ctx->grid_ready || !ctx->allocs.empty() || ctx->arena)
        return set_err(ctx, NHDC_ESTATE, "set_allocator: must come before nhdc_upload_grid");
    ctx->al = Allocator{alloc, free_, alloc ? user : nullptr};
    ctx->L.al = ctx->al;
    return NHDC_OK;
}

int nhdc_upload_grid(nhdc_ctx *ctx, const nhdc_grid *g, const nhdc_vertical *v,
                     const nhdc_params *prm) {
    if (!ctx) return NHDC_EINVAL;
    if (!g || !v || !prm) return set_err(ctx, NHDC_EINVAL, "upload_grid: NULL argument");
    if (ctx->grid_ready) return set_err(ctx, NHDC_ESTATE, "upload_grid: grid already uploaded");
    const void *need[] = {g->cell_edges, g->cell_sign, g->edge_cells, g->edge_verts, g->vert_edges,
                          g->vert_cells, g->vert_sign, g->vert_valence, g->cell_x, g->cell_area,
                          g->edge_x, g->edge_tangent, g->edge_length, g->dual_length,
                          g->vert_area, v->zh, v->pi_ref, v->theta_ref};
    for (const void *q : need)
        if (!q) return set_err(ctx, NHDC_EINVAL, "upload_grid: NULL array");
    if (!(prm->beta >= 0.5 && prm->beta <= 1.0) || !(prm->cpd > prm->rd && prm->rd > 0) ||
        !(prm->grav > 0) || !std::isfinite(prm->omega) || !std::isfinite(prm->extrap) ||
        !std::isfinite(prm->wgt_corr) || !std::isfinite(prm->div_damp) ||
        (prm->upwind != 0 && prm->upwind != 1) || !(prm->div_damp4 >= 0.0) ||
        !std::isfinite(prm->div_damp4) || !(prm->smag >= 0.0) || !std::isfinite(prm->smag))
        return set_err(ctx, NHDC_EINVAL, "upload_grid: bad parameters");
    if (prm->smag > 0.0 && !g->edge_normal)
        return set_err(ctx, NHDC_EINVAL, "upload_grid: the diffusion option needs edge_normal");
    if (prm->upwind && (!g->edge_normal || !g->dual_frac))
        return set_err(ctx, NHDC_EINVAL, "upload_grid: the upwind option needs edge_normal and dual_frac");
    if (g->dual_frac)
        for (int64_t e = 0; e < g->n_edges; ++e)
            if (!(g->dual_frac[e] > 0.0 && g->dual_frac[e] < 1.0))
                return set_err(ctx, NHDC_EGRID, "grid: dual_frac outside (0, 1)");
    int rc = validate(ctx, g, v);
    if (rc) return rc;
    if (v->w_damp)
        for (int i = 0; i <= v->n_lev; ++i)
            if (!(v->w_damp[i] >= 0.0) || !std::isfinite(v->w_damp[i]))
                return set_err(ctx, NHDC_EINVAL, "upload_grid: w_damp must be finite and >= 0");
    HIP_TRY(ctx, hipSetDevice(ctx->device));

    const int64_t nc = g->n_cells, ne = g->n_edges, nv = g->n_verts;
    const int N = v->n_lev;
    const double a = g->radius;
    Grid &G = ctx->g;
    G.nc = nc;
    G.ne = ne;
    G.nv = nv;
    G.N = N;
    G.radius = a;
    G.abar = 4.0 * 3.14159265358979323846 * a * a / double(nc);
    ctx->p = Params{prm->omega, prm->grav, prm->rd, prm->cpd, prm->p00, prm->beta,
                    prm->wgt_corr, prm->extrap, prm->div_damp, prm->upwind, prm->div_damp4,
                    prm->smag};
    if (fp32_stencils(ctx->precision)) {
        // the mixed forms: one allocation for the arrays below (without it,
        // no memory for one piece, each array is allocated on its own).  The
        // FP64 form keeps separate allocations: from one range it measured
        // the same or slower.
        const size_t want = arena_bytes(g, v, prm, ctx->precision);
        ctx->arena = static_cast<char *>(dev_alloc(ctx->al, want));
        ctx->arena_size = ctx->arena ? want : 0;
        ctx->arena_used = 0;
    }

    // ---- stencil coefficients on the host (each formed exactly as the
    // operators form it, so device sums see the same operands) ----
    std::vector<double> c_sl(3 * nc), c_dv(9 * nc), v_sd(6 * nv), v_m(6 * nv), v_ival(nv), fe(ne);
    std::vector<double> c_ia(nc), e_ide(ne), e_ile(ne), v_ia(nv);
    for (int64_t c = 0; c < nc; ++c) c_ia[c] = 1.0 / g->cell_area[c];
    for (int64_t e = 0; e < ne; ++e) {
        e_ide[e] = 1.0 / g->dual_length[e];
        e_ile[e] = 1.0 / g->edge_length[e];
    }
    for (int64_t v = 0; v < nv; ++v) v_ia[v] = 1.0 / g->vert_area[v];
    std::vector<int32_t> v_e(6 * nv), v_c(6 * nv);
    for (int64_t c = 0; c < nc; ++c) {
        const double xc[3] = {g->cell_x[c], g->cell_x[nc + c], g->cell_x[2 * nc + c]};
        for (int j = 0; j < 3; ++j) {
            int64_t e = g->cell_edges[j * nc + c];
            c_sl[j * nc + c] = g->cell_sign[j * nc + c] * g->edge_length[e];
            for (int q = 0; q < 3; ++q) c_dv[(3 * j + q) * nc + c] = a * (g->edge_x[q * ne + e] - xc[q]);
        }
    }
    for (int64_t vtx = 0; vtx < nv; ++vtx) {
        int val = g->vert_valence[vtx];
        v_ival[vtx] = 1.0 / double(val);
        for (int j = 0; j < 6; ++j) {
            bool real = j < val;
            int64_t e = real ? g->vert_edges[j * nv + vtx] : g->vert_edges[vtx];
            int64_t c = real ? g->vert_cells[j * nv + vtx] : g->vert_cells[vtx];
            v_e[j * nv + vtx] = int32_t(e);
            v_c[j * nv + vtx] = int32_t(c);
            v_sd[j * nv + vtx] = real ? g->vert_sign[j * nv + vtx] * g->dual_length[e] : 0.0;
            v_m[j * nv + vtx] = real ? 1.0 : 0.0;
        }
    }
    for (int64_t e = 0; e < ne; ++e) fe[e] = 2.0 * prm->omega * g->edge_x[2 * ne + e];
    // neighbours and vertex slots of every cell, from its edges: edge slot j runs
    // from vertex slot j to j+1 counter-clockwise, i.e. from v1 to v2 when the
    // normal points out of the cell (s = +1) and from v2 to v1 otherwise.
    std::vector<int32_t> c_n(3 * nc), c_v(3 * nc);
    for (int64_t c = 0; c < nc; ++c) {
        int32_t first[3], second[3];
        for (int j = 0; j < 3; ++j) {
            int64_t e = g->cell_edges[j * nc + c];
            bool out = g->cell_sign[j * nc + c] > 0;
            c_n[j * nc + c] = out ? g->edge_cells[ne + e] : g->edge_cells[e];
            first[j] = out ? g->edge_verts[e] : g->edge_verts[ne + e];
            second[j] = out ? g->edge_verts[ne + e] : g->edge_verts[e];
            c_v[j * nc + c] = first[j];
        }
        for (int j = 0; j < 3; ++j)
            if (second[j] != first[(j + 1) % 3])
                return set_err(ctx, NHDC_EGRID,
                               "grid: cell edges are not a counter-clockwise chain of its vertices");
    }
    if ((rc = upload(ctx, &G.c_e, g->cell_edges, 3 * nc))) return rc;
    if ((rc = upload(ctx, &G.c_n, c_n.data(), 3 * nc))) return rc;
    if ((rc = upload(ctx, &G.c_v, c_v.data(), 3 * nc))) return rc;
    {
        // each block of BLOCK consecutive cells: its distinct edges and
        // vertices and the neighbours outside it, ascending, if they fit
        const int64_t nblk = (nc + BLOCK - 1) / BLOCK;
        std::vector<int32_t> be(static_cast<size_t>(nblk) * CVT_E), bv(static_cast<size_t>(nblk) * CVT_V);
        std::vector<int32_t> bx(static_cast<size_t>(nblk) * CVT_X), bn(static_cast<size_t>(3 * nblk));
        std::vector<int32_t> el(static_cast<size_t>(3 * nc)), vl(static_cast<size_t>(3 * nc));
        std::vector<int32_t> nl(static_cast<size_t>(3 * nc));
        std::vector<int32_t> ue, uv, ux;
        bool fits = true;
        for (int64_t b = 0; b < nblk && fits; ++b) {
            const int64_t c0 = b * BLOCK, c1 = std::min<int64_t>(nc, c0 + BLOCK);
            ue.clear();
            uv.clear();
            ux.clear();
            for (int64_t c = c0; c < c1; ++c)
                for (int j = 0; j < 3; ++j) {
                    ue.push_back(g->cell_edges[j * nc + c]);
                    uv.push_back(c_v[size_t(j * nc + c)]);
                    const int32_t x = c_n[size_t(j * nc + c)];
                    if (x < c0 || x >= c1) ux.push_back(x);
                }
            for (auto *u : {&ue, &uv, &ux}) {
                std::sort(u->begin(), u->end());
                u->erase(std::unique(u->begin(), u->end()), u->end());
            }
            if (ue.size() > size_t(CVT_E) || uv.size() > size_t(CVT_V) || ux.size() > size_t(CVT_X)) {
                fits = false;
                break;
            }
            bn[size_t(b)] = int32_t(ue.size());
            bn[size_t(nblk + b)] = int32_t(uv.size());
            bn[size_t(2 * nblk + b)] = int32_t(ux.size());
            for (int j = 0; j < CVT_E; ++j) be[size_t(b * CVT_E + j)] = j < int(ue.size()) ? ue[size_t(j)] : ue[0];
            for (int j = 0; j < CVT_V; ++j) bv[size_t(b * CVT_V + j)] = j < int(uv.size()) ? uv[size_t(j)] : uv[0];
            for (int j = 0; j < CVT_X; ++j)
                bx[size_t(b * CVT_X + j)] = j < int(ux.size()) ? ux[size_t(j)] : (ux.empty() ? int32_t(c0) : ux[0]);
            for (int64_t c = c0; c < c1; ++c)
                for (int j = 0; j < 3; ++j) {
                    const size_t s = size_t(j * nc + c);
                    el[s] = int32_t(std::lower_bound(ue.begin(), ue.end(), g->cell_edges[s]) - ue.begin());
                    vl[s] = int32_t(std::lower_bound(uv.begin(), uv.end(), c_v[s]) - uv.begin());
                    const int32_t x = c_n[s];
                    nl[s] = (x >= c0 && x < c1)
                                ? int32_t(x - c0)
                                : int32_t(BLOCK + (std::lower_bound(ux.begin(), ux.end(), x) - ux.begin()));
                }
        }
        G.cvt_ok = fits ? 1 : 0;
        if (fits) {
            if ((rc = upload(ctx, &G.cb_e, be.data(), nblk * CVT_E))) return rc;
            if ((rc = upload(ctx, &G.cb_v, bv.data(), nblk * CVT_V))) return rc;
            if ((rc = upload(ctx, &G.cb_x, bx.data(), nblk * CVT_X))) return rc;
            if ((rc = upload(ctx, &G.cb_n, bn.data(), 3 * nblk))) return rc;
            if ((rc = upload(ctx, &G.c_el, el.data(), 3 * nc))) return rc;
            if ((rc = upload(ctx, &G.c_vl, vl.data(), 3 * nc))) return rc;
            if ((rc = upload(ctx, &G.c_nl, nl.data(), 3 * nc))) return rc;
        }
    }
    {
        // the slot of each shared edge in the neighbour across it
        std::vector<int32_t> c_ns(3 * nc);
        for (int64_t c = 0; c < nc; ++c)
            for (int j = 0; j < 3; ++j) {
                const int64_t e = g->cell_edges[j * nc + c], nb = c_n[j * nc + c];
                int s = 0;
                while (s < 3 && g->cell_edges[s * nc + nb] != e) ++s;
                if (s == 3) return set_err(ctx, NHDC_EGRID, "grid: a neighbour does not share the edge");
                c_ns[j * nc + c] = s;
            }
        if ((rc = upload(ctx, &G.c_ns, c_ns.data(), 3 * nc))) return rc;
    }
    if ((rc = upload(ctx, &G.e_c, g->edge_cells, 2 * ne))) return rc;
    {
        // each block of BLOCK consecutive edges: its distinct cells, ascending
        const int64_t nblk = (ne + BLOCK - 1) / BLOCK;
        std::vector<int32_t> cells(static_cast<size_t>(nblk) * 2 * BLOCK);
        std::vector<int32_t> cnt(static_cast<size_t>(nblk)), loc(static_cast<size_t>(2 * ne));
        std::vector<int32_t> u;
        u.reserve(2 * BLOCK);
        for (int64_t b = 0; b < nblk; ++b) {
            const int64_t e0 = b * BLOCK, e1 = std::min<int64_t>(ne, e0 + BLOCK);
            u.clear();
            for (int64_t e = e0; e < e1; ++e) {
                u.push_back(g->edge_cells[e]);
                u.push_back(g->edge_cells[ne + e]);
            }
            std::sort(u.begin(), u.end());
            u.erase(std::unique(u.begin(), u.end()), u.end());
            cnt[size_t(b)] = int32_t(u.size());
            for (int j = 0; j < 2 * BLOCK; ++j)
                cells[size_t(b) * 2 * BLOCK + size_t(j)] = j < int(u.size()) ? u[size_t(j)] : u[0];
            for (int64_t e = e0; e < e1; ++e)
                for (int s = 0; s < 2; ++s)
                    loc[size_t(s * ne + e)] = int32_t(
                        std::lower_bound(u.begin(), u.end(), g->edge_cells[s * ne + e]) - u.begin());
        }
        G.eb_max = *std::max_element(cnt.begin(), cnt.end());
        if ((rc = upload(ctx, &G.eb_cells, cells.data(), nblk * 2 * BLOCK))) return rc;
        if ((rc = upload(ctx, &G.eb_n, cnt.data(), nblk))) return rc;
        if ((rc = upload(ctx, &G.e_loc, loc.data(), 2 * ne))) return rc;
    }
    if ((rc = upload(ctx, &G.e_v, g->edge_verts, 2 * ne))) return rc;
    if ((rc = upload(ctx, &G.v_e, v_e.data(), 6 * nv))) return rc;
    if ((rc = upload(ctx, &G.v_c, v_c.data(), 6 * nv))) return rc;
    Geo<double> &D = G.gd;
    if ((rc = upload(ctx, &D.c_sl, c_sl.data(), 3 * nc))) return rc;
    if ((rc = upload(ctx, &D.c_dv, c_dv.data(), 9 * nc))) return rc;
    if ((rc = upload(ctx, &D.c_x, g->cell_x, 3 * nc))) return rc;
    if ((rc = upload(ctx, &D.c_area, g->cell_area, nc))) return rc;
    if ((rc = upload(ctx, &D.c_ia, c_ia.data(), nc))) return rc;
    if ((rc = upload(ctx, &D.e_ide, e_ide.data(), ne))) return rc;
    if ((rc = upload(ctx, &D.e_ile, e_ile.data(), ne))) return rc;
    if ((rc = upload(ctx, &D.e_t, g->edge_tangent, 3 * ne))) return rc;
    if ((rc = upload(ctx, &D.fe, fe.data(), ne))) return rc;
    if ((rc = upload(ctx, &D.v_sd, v_sd.data(), 6 * nv))) return rc;
    if ((rc = upload(ctx, &D.v_m, v_m.data(), 6 * nv))) return rc;
    if ((rc = upload(ctx, &D.v_ival, v_ival.data(), nv))) return rc;
    if ((rc = upload(ctx, &D.v_ia, v_ia.data(), nv))) return rc;
    const int64_t NC = int64_t(N) * nc, NC1 = int64_t(N + 1) * nc, NE = int64_t(N) * ne;
    const int64_t NV1 = int64_t(N + 1) * nv;
    if ((rc = upload(ctx, &G.zh, v->zh, NC1))) return rc;
    if ((rc = upload(ctx, &G.pi_ref, v->pi_ref, NC))) return rc;
    if ((rc = upload(ctx, &G.theta_ref, v->theta_ref, NC))) return rc;
    if ((rc = dalloc(ctx, &G.zhv, NV1))) return rc;
    if (prm->upwind) {
        // displacements from the two cell centres to the edge midpoint, formed
        // as the flux reconstruction forms them
        std::vector<double> d1(3 * ne), d2(3 * ne);
        for (int64_t e = 0; e < ne; ++e) {
            const int64_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
            for (int x = 0; x < 3; ++x) {
                d1[x * ne + e] = a * (g->edge_x[x * ne + e] - g->cell_x[x * nc + c1]);
                d2[x * ne + e] = a * (g->edge_x[x * ne + e] - g->cell_x[x * nc + c2]);
            }
        }
        if ((rc = upload(ctx, &G.e_d1, d1.data(), 3 * ne))) return rc;
        if ((rc = upload(ctx, &G.e_d2, d2.data(), 3 * ne))) return rc;
    }
    // normals and arc fractions whenever the grid has them (the upwind,
    // diffusion and tracer options read them)
    if (g->edge_normal)
        if ((rc = upload(ctx, &G.e_n, g->edge_normal, 3 * ne))) return rc;
    if (g->dual_frac)
        if ((rc = upload(ctx, &G.e_frac, g->dual_frac, ne))) return rc;
    if (v->w_damp)
        if ((rc = upload(ctx, &G.w_damp, v->w_damp, int64_t(N) + 1))) return rc;
    HIP_TRY(ctx, launch_metrics(G, nullptr));
    {
        // the flat top of the height coordinate, level by level from the lid
        // (rows: zh, zhv at N+1 half levels; pi_ref, theta_ref at N levels)
        const int64_t n_rows = 2 * (int64_t(N) + 1) + 2 * int64_t(N);
        int32_t *d_nf = nullptr;
        if ((rc = dalloc(ctx, &d_nf, n_rows))) return rc;
        HIP_TRY(ctx, hipMemset(d_nf, 0, sizeof(int32_t) * size_t(n_rows)));
        int32_t *nf_zh = d_nf, *nf_zhv = d_nf + N + 1, *nf_pr = d_nf + 2 * (N + 1), *nf_tr = nf_pr + N;
        HIP_TRY(ctx, launch_level_nonflat(G.zh, nc, N + 1, nf_zh, nullptr));
        HIP_TRY(ctx, launch_level_nonflat(G.zhv, nv, N + 1, nf_zhv, nullptr));
        HIP_TRY(ctx, launch_level_nonflat(G.pi_ref, nc, N, nf_pr, nullptr));
        HIP_TRY(ctx, launch_level_nonflat(G.theta_ref, nc, N, nf_tr, nullptr));
        std::vector<int32_t> nf(static_cast<size_t>(n_rows));
        HIP_TRY(ctx, hipMemcpy(nf.data(), d_nf, sizeof(int32_t) * nf.size(), hipMemcpyDeviceToHost));
        const int32_t *h_zh = nf.data(), *h_zhv = h_zh + N + 1, *h_pr = h_zhv + N + 1, *h_tr = h_pr + N;
        G.flat_c = 0;
        while (G.flat_c <= N && h_zh[G.flat_c] == 0) ++G.flat_c;
        G.flat_v = 0;
        while (G.flat_v <= N && h_zhv[G.flat_v] == 0) ++G.flat_v;
        G.flat_r = 0;
        while (G.flat_r < N && h_pr[G.flat_r] == 0 && h_tr[G.flat_r] == 0) ++G.flat_r;
    }
    if (fp32_stencils(ctx->precision)) {
        Geo<float> &F = G.gf;
        if ((rc = upload_f32(ctx, &F.c_sl, D.c_sl, 3 * nc))) return rc;
        if ((rc = upload_f32(ctx, &F.c_dv, D.c_dv, 9 * nc))) return rc;
        if ((rc = upload_f32(ctx, &F.c_x, D.c_x, 3 * nc))) return rc;
        if ((rc = upload_f32(ctx, &F.c_ia, D.c_ia, nc))) return rc;
        if ((rc = upload_f32(ctx, &F.e_ide, D.e_ide, ne))) return rc;
        if ((rc = upload_f32(ctx, &F.e_ile, D.e_ile, ne))) return rc;
        if ((rc = upload_f32(ctx, &F.e_t, D.e_t, 3 * ne))) return rc;
        if ((rc = upload_f32(ctx, &F.fe, D.fe, ne))) return rc;
        if ((rc = upload_f32(ctx, &F.v_sd, D.v_sd, 6 * nv))) return rc;
        if ((rc = upload_f32(ctx, &F.v_m, D.v_m, 6 * nv))) return rc;
        if ((rc = upload_f32(ctx, &F.v_ival, D.v_ival, nv))) return rc;
        if ((rc = upload_f32(ctx, &F.v_ia, D.v_ia, nv))) return rc;
    }

    // ---- state, accumulators and work arrays ----
    State &S = ctx->s;
    double **cellsN[] = {&S.rho, &S.pi, &S.thv, &S.pi_prev, &S.px};
    for (auto q : cellsN)
        if ((rc = dalloc(ctx, q, NC))) return rc;
    if ((rc = dalloc(ctx, &S.w, NC1))) return rc;
    if ((rc = dalloc(ctx, &S.wacc, NC1))) return rc;
    // the stored normal velocity: FP64, or FP32 (half the bytes) in the FP32-vn variant
    if ((rc = dalloc(ctx, &S.vn, vn_bytes(ctx->precision) == 4 ? (NE + 1) / 2 : NE))) return rc;
    if ((rc = dalloc(ctx, &S.facc, NE))) return rc;
    if (fp32_stencils(ctx->precision)) rc = alloc_work<float>(ctx, ctx->wf);
    else rc = alloc_work<double>(ctx, ctx->wd);
    if (rc) return rc;
    if ((rc = dalloc(ctx, &ctx->red, 2 * ((nc + BLOCK - 1) / BLOCK) + 2))) return rc;
    if ((rc = dalloc(ctx, &ctx->flag, 1))) return rc;
    HIP_TRY(ctx, hipDeviceSynchronize());
    std::vector<nhdc_ctx *> one{ctx};
    if ((rc = upload_insts(ctx->L, one, ctx->err))) return rc;
    const Grid *gp = &ctx->g;
    ctx->tune = default_tune(&gp, 1);
    rebuild_maps(ctx->L, one, ctx->tune);
    ctx->grid_ready = true;
    return NHDC_OK;
}

int nhdc_init_state(nhdc_ctx *ctx, const nhdc_state_view *st, void *stream) {
    if (!ctx) return NHDC_EINVAL;
    if (!st) return set_err(ctx, NHDC_EINVAL, "init_state: NULL state");
    if (!ctx->grid_ready) return set_err(ctx, NHDC_ESTATE, "init_state: no grid uploaded");
    if (!st->vn || !st->w || !st->rho || !st->pi || !st->theta_v)
        return set_err(ctx, NHDC_EINVAL, "init_state: NULL field");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid &G = ctx->g;
    const size_t NC = size_t(G.N) * G.nc * 8, NC1 = size_t(G.N + 1) * G.nc * 8,
                 NE = size_t(G.N) * G.ne * 8;
    hipMemcpyKind kind = st->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (vn_bytes(ctx->precision) == 4) {  // FP64 in, stored in FP32
        int rc = vn_to_f32(ctx, st->vn, st->on_device != 0, s);
        if (rc) return rc;
    } else {
        HIP_TRY(ctx, hipMemcpyAsync(ctx->s.vn, st->vn, NE, kind, s));
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->s.w, st->w, NC1, kind, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->s.rho, st->rho, NC, kind, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->s.pi, st->pi, NC, kind, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->s.thv, st->theta_v, NC, kind, s));
    if (st->pi_prev) HIP_TRY(ctx, hipMemcpyAsync(ctx->s.pi_prev, st->pi_prev, NC, kind, s));
    else HIP_TRY(ctx, launch_init_prev(ctx->g, ctx->s, s));
    HIP_TRY(ctx, launch_exner_x(ctx->g, ctx->s, ctx->p.extrap, s));
    HIP_TRY(ctx, hipMemsetAsync(ctx->s.facc, 0, NE, s));
    HIP_TRY(ctx, hipMemsetAsync(ctx->s.wacc, 0, NC1, s));
    if (!st->on_device) HIP_TRY(ctx, hipStreamSynchronize(s));
    ctx->state_ready = true;
    return NHDC_OK;
}

int nhdc_step(nhdc_ctx *ctx, double dt, int nsub, void *stream) {
    if (!ctx) return NHDC_EINVAL;
    if (!(dt > 0) || !std::isfinite(dt)) return set_err(ctx, NHDC_EINVAL, "step: dt must be positive and finite");
    if (nsub < 1) return set_err(ctx, NHDC_EINVAL, "step: nsubsteps must be >= 1");
    if (!ctx->state_ready) return set_err(ctx, NHDC_ESTATE, "step: state not initialised");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->tm.ids.clear();
    HIP_TRY(ctx, run_step(ctx->L, &dt, nsub, &ctx->tm, s));
    return timing_collect(ctx, s);
}

int nhdc_set_block_sizes(nhdc_ctx *ctx, int column, int vertex, int column_waves) {
    if (!ctx) return NHDC_EINVAL;
    if (!ctx->grid_ready) return set_err(ctx, NHDC_ESTATE, "set_block_sizes: no grid uploaded");
    if (!valid_block(column) || !valid_block(vertex) || !valid_waves(column_waves))
        return set_err(ctx, NHDC_EINVAL,
                       "set_block_sizes: block sizes must be 64, 128 or 256 and column_waves 0, 2 or 3");
    ctx->tune.blk_col = column;
    ctx->tune.blk_vert = vertex;
    ctx->tune.col_waves = column_waves;
    std::vector<nhdc_ctx *> one{ctx};
    rebuild_maps(ctx->L, one, ctx->tune);
    return NHDC_OK;
}

int nhdc_set_column_mode(nhdc_ctx *ctx, int mode) {
    if (!ctx) return NHDC_EINVAL;
    if (!ctx->grid_ready) return set_err(ctx, NHDC_ESTATE, "set_column_mode: no grid uploaded");
    if (!valid_col_mode(mode))
        return set_err(ctx, NHDC_EINVAL, "set_column_mode: mode must be 0 (stream) or 1 (levels)");
    ctx->tune.col_mode = mode;
    std::vector<nhdc_ctx *> one{ctx};
    rebuild_maps(ctx->L, one, ctx->tune);
    return NHDC_OK;
}

int nhdc_get_shapes(const nhdc_ctx *ctx, int *shapes) {
    if (!ctx || !shapes) return NHDC_EINVAL;
    if (!ctx->grid_ready) return NHDC_ESTATE;
    tune_shapes(ctx->tune, shapes);
    return NHDC_OK;
}

int nhdc_set_tiles(nhdc_ctx *ctx, int lt_edge, int lt_cell, int lt_vert) {
    if (!ctx) return NHDC_EINVAL;
    if (!ctx->grid_ready) return set_err(ctx, NHDC_ESTATE, "set_tiles: no grid uploaded");
    if (lt_edge < 0 || lt_cell < 0 || lt_vert < 0)
        return set_err(ctx, NHDC_EINVAL, "set_tiles: tiles must be >= 0");
    ctx->tune.lt_edge = lt_edge;
    ctx->tune.lt_cell = lt_cell;
    ctx->tune.lt_vert = lt_vert;
    std::vector<nhdc_ctx *> one{ctx};
    rebuild_maps(ctx->L, one, ctx->tune);
    return NHDC_OK;
}

int nhdc_autotune(nhdc_ctx *ctx, double dt, int nsub, const char *cache_path, double *best,
                  void *stream) {
    if (!ctx) return NHDC_EINVAL;
    if (!(dt > 0) || !std::isfinite(dt) || nsub < 1)
        return set_err(ctx, NHDC_EINVAL, "autotune: bad dt or nsubsteps");
    if (!ctx->state_ready) return set_err(ctx, NHDC_ESTATE, "autotune: state not initialised");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    std::vector<nhdc_ctx *> one{ctx};
    Stepper stepper;
    const Launcher &L = ctx->L;
    stepper.step = [&L](const double *d, int ns, hipStream_t st) { return run_step(L, d, ns, nullptr, st); };
    return autotune(ctx->L, ctx->tune, one, &dt, nsub, cache_path, best,
                    static_cast<hipStream_t>(stream), ctx->err, stepper, "launches");
}

int nhdc_get_state(nhdc_ctx *ctx, const nhdc_state_view *dst, void *stream) {
    if (!ctx) return NHDC_EINVAL;
    if (!dst) return set_err(ctx, NHDC_EINVAL, "get_state: NULL view");
    if (!ctx->state_ready) return set_err(ctx, NHDC_ESTATE, "get_state: state not initialised");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid &G = ctx->g;
    const size_t NC = size_t(G.N) * G.nc * 8, NC1 = size_t(G.N + 1) * G.nc * 8,
                 NE = size_t(G.N) * G.ne * 8;
    hipMemcpyKind kind = dst->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (dst->vn && vn_bytes(ctx->precision) == 4) {  // stored in FP32, FP64 out
        int rc = vn_to_f64(ctx, dst->vn, dst->on_device != 0, s);
        if (rc) return rc;
    } else if (dst->vn) {
        HIP_TRY(ctx, hipMemcpyAsync(dst->vn, ctx->s.vn, NE, kind, s));
    }
    if (dst->w) HIP_TRY(ctx, hipMemcpyAsync(dst->w, ctx->s.w, NC1, kind, s));
    if (dst->rho) HIP_TRY(ctx, hipMemcpyAsync(dst->rho, ctx->s.rho, NC, kind, s));
    if (dst->pi) HIP_TRY(ctx, hipMemcpyAsync(dst->pi, ctx->s.pi, NC, kind, s));
    if (dst->theta_v) HIP_TRY(ctx, hipMemcpyAsync(dst->theta_v, ctx->s.thv, NC, kind, s));
    if (dst->pi_prev) HIP_TRY(ctx, hipMemcpyAsync(dst->pi_prev, ctx->s.pi_prev, NC, kind, s));
    if (!dst->on_device) HIP_TRY(ctx, hipStreamSynchronize(s));
    return NHDC_OK;
}

int nhdc_get_mass_flux(nhdc_ctx *ctx, double *facc, double *wacc, int on_device, void *stream) {
    if (!ctx) return NHDC_EINVAL;
    if (!ctx->state_ready) return set_err(ctx, NHDC_ESTATE, "get_mass_flux: state not initialised");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid &G = ctx->g;
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (facc) HIP_TRY(ctx, hipMemcpyAsync(facc, ctx->s.facc, size_t(G.N) * G.ne * 8, kind, s));
    if (wacc) HIP_TRY(ctx, hipMemcpyAsync(wacc, ctx->s.wacc, size_t(G.N + 1) * G.nc * 8, kind, s));
    if (!on_device) HIP_TRY(ctx, hipStreamSynchronize(s));
    return NHDC_OK;
}

int nhdc_diag(nhdc_ctx *ctx, double *mass, double *rho_theta, void *stream) {
    if (!ctx) return NHDC_EINVAL;
    if (!ctx->state_ready) return set_err(ctx, NHDC_ESTATE, "diag: state not initialised");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *out = ctx->red + 2 * ((ctx->g.nc + BLOCK - 1) / BLOCK);
    HIP_TRY(ctx, launch_diag(ctx->g, ctx->s, ctx->red, out, s));
    double h[2];
    HIP_TRY(ctx, hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (mass) *mass = h[0];
    if (rho_theta) *rho_theta = h[1];
    return NHDC_OK;
}

int nhdc_check_finite(nhdc_ctx *ctx, void *stream) {
    if (!ctx) return NHDC_EINVAL;
    if (!ctx->state_ready) return set_err(ctx, NHDC_ESTATE, "check_finite: state not initialised");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipMemsetAsync(ctx->flag, 0, sizeof(int), s));
    HIP_TRY(ctx, launch_finite(ctx->g, ctx->s, vn_bytes(ctx->precision), ctx->flag, s));
    int h = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&h, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (h) return set_err(ctx, NHDC_EUNSTABLE, "check_finite: non-finite value in the state");
    return NHDC_OK;
}

int nhdc_sizes(const nhdc_ctx *ctx, int64_t *n_cells, int64_t *n_edges, int64_t *n_verts,
               int32_t *n_lev) {
    if (!ctx || !ctx->grid_ready) return NHDC_ESTATE;
    if (n_cells) *n_cells = ctx->g.nc;
    if (n_edges) *n_edges = ctx->g.ne;
    if (n_verts) *n_verts = ctx->g.nv;
    if (n_lev) *n_lev = ctx->g.N;
    return NHDC_OK;
}

int nhdc_set_timing(nhdc_ctx *ctx, int enable) {
    if (!ctx) return NHDC_EINVAL;
    ctx->tm.on = enable != 0;
    ctx->tm.ids.clear();
    for (int k = 0; k < K_NUM; ++k) {
        ctx->tm.total_ms[k] = 0.0;
        ctx->tm.launches[k] = 0;
    }
    return NHDC_OK;
}

int nhdc_kernel_count(void) { return K_NUM; }

int nhdc_kernel_stats(const nhdc_ctx *ctx, int index, const char **name, double *total_ms,
                      int64_t *launches) {
    if (!ctx || index < 0 || index >= K_NUM) return NHDC_EINVAL;
    if (name) *name = kKernelNames[index];
    if (total_ms) *total_ms = ctx->tm.total_ms[index];
    if (launches) *launches = ctx->tm.launches[index];
    return NHDC_OK;
}

const char *nhdc_last_error(const nhdc_ctx *ctx) { return ctx ? ctx->err.c_str() : context_free_error(); }

int nhdc_set_tracers(nhdc_ctx *ctx, int n_tracers, const double *q, int on_device, void *stream) {
    if (!ctx) return NHDC_EINVAL;
    if (!ctx->grid_ready) return set_err(ctx, NHDC_ESTATE, "set_tracers: no grid uploaded");
    if (n_tracers < 0 || n_tracers > NHDC_MAX_TRACERS)
        return set_err(ctx, NHDC_EINVAL, "set_tracers: n_tracers out of range");
    if (n_tracers > 0 && !q) return set_err(ctx, NHDC_EINVAL, "set_tracers: NULL tracers");
    if (ctx->in_batches > 0)
        return set_err(ctx, NHDC_ESTATE, "set_tracers: the context is part of a live batch");
    if (n_tracers > 0 && (!ctx->g.e_n || !ctx->g.e_frac))
        return set_err(ctx, NHDC_EINVAL, "set_tracers: the grid was uploaded without edge_normal and dual_frac");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipStreamSynchronize(s));
    HIP_TRY(ctx, hipDeviceSynchronize());
    for (void *p : ctx->tr_allocs) dev_free(ctx->al, p);
    ctx->tr_allocs.clear();
    ctx->tr = Tracers{};
    if (n_tracers > 0) {
        const int64_t NC = int64_t(ctx->g.N) * ctx->g.nc;
        double **arr[] = {&ctx->tr.q, &ctx->tr.rec, &ctx->tr.qs, &ctx->tr.rs, &ctx->tr.rho0};
        const int64_t len[] = {n_tracers * NC, 3 * n_tracers * NC, n_tracers * NC, NC, NC};
        for (int i = 0; i < 5; ++i) {
            int rc = dalloc(ctx, arr[i], len[i], false);
            if (rc) return rc;
            ctx->allocs.pop_back();  // owned by the tracer list, freed on replacement
            ctx->tr_allocs.push_back(*arr[i]);
        }
        ctx->tr.nt = n_tracers;
        HIP_TRY(ctx, hipMemcpyAsync(ctx->tr.q, q, sizeof(double) * n_tracers * NC,
                                    on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
    }
    std::vector<nhdc_ctx *> one{ctx};
    return upload_insts(ctx->L, one, ctx->err);
}

int nhdc_get_tracers(nhdc_ctx *ctx, double *q, int on_device, void *stream) {
    if (!ctx) return NHDC_EINVAL;
    if (!q) return set_err(ctx, NHDC_EINVAL, "get_tracers: NULL buffer");
    if (ctx->tr.nt == 0) return NHDC_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = sizeof(double) * ctx->tr.nt * size_t(ctx->g.N) * ctx->g.nc;
    HIP_TRY(ctx, hipMemcpyAsync(q, ctx->tr.q, bytes,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!on_device) HIP_TRY(ctx, hipStreamSynchronize(s));
    return NHDC_OK;
}

int nhdc_n_tracers(const nhdc_ctx *ctx) { return ctx ? ctx->tr.nt : NHDC_EINVAL; }

void nhdc_destroy(nhdc_ctx *ctx) {
    if (!ctx) return;
    if (ctx->in_batches > 0) {
        // a live batch still holds the context's descriptor and device
        // memory: the last nhdc_batch_destroy releases them
        ctx->destroy_pending = true;
        return;
    }
    free_context(ctx);
}

}  // extern "C"

// nhdc_batch.hip -- many independent instances advanced together: one launch
// per kernel over all instances, a whole step captured once into a HIP graph
// and replayed, level tiles from the autotuner.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "nhdc_host.h"
#include "nhdc_internal.h"

using namespace nhdc;

struct nhdc_batch {
    int device = 0;
    std::vector<nhdc_ctx *> ctxs;
    Launcher L;
    Tune tune;
    hipStream_t cap = nullptr;          // private stream used only for graph capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<double> graph_dt;       // the step the graph holds
    int graph_nsub = 0;
    Tune graph_tune;
    std::string err;
};

namespace {

void drop_graph(nhdc_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_dt.clear();
}

bool graph_matches(const nhdc_batch *b, const double *dt, int nsub) {
    if (!b->exec || b->graph_nsub != nsub) return false;
    if (b->graph_tune.lt_edge != b->tune.lt_edge || b->graph_tune.lt_cell != b->tune.lt_cell ||
        b->graph_tune.lt_vert != b->tune.lt_vert)
        return false;
    for (size_t i = 0; i < b->ctxs.size(); ++i)
        if (b->graph_dt[i] != dt[i]) return false;
    return true;
}

// Capture one step (nsub substeps x 10 launches over all instances) into a graph.
int capture(nhdc_batch *b, const double *dt, int nsub) {
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(b->err, e, "batch: hipStreamBeginCapture");
    hipError_t le = run_step(b->L, dt, nsub, nullptr, b->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(b->err, le, "batch: launch during capture");
    }
    if (e != hipSuccess) return hip_fail(b->err, e, "batch: hipStreamEndCapture");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return hip_fail(b->err, e, "batch: hipGraphInstantiate");
    }
    b->graph_dt.assign(dt, dt + b->ctxs.size());
    b->graph_nsub = nsub;
    b->graph_tune = b->tune;
    return NHDC_OK;
}

int check_dt(nhdc_batch *b, const double *dt, int nsub) {
    if (!dt) return set_err(b->err, NHDC_EINVAL, "batch: dt is NULL");
    if (nsub < 1) return set_err(b->err, NHDC_EINVAL, "batch: nsubsteps must be >= 1");
    for (size_t i = 0; i < b->ctxs.size(); ++i)
        if (!(dt[i] > 0) || !std::isfinite(dt[i]))
            return set_err(b->err, NHDC_EINVAL, "batch: dt must be positive and finite");
    return NHDC_OK;
}

}  // namespace

extern "C" {

int nhdc_batch_create(nhdc_batch **out, nhdc_ctx *const *inst, int n) {
    if (!out) return NHDC_EINVAL;
    *out = nullptr;
    if (!inst || n < 1 || n > MAX_INST) return NHDC_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!inst[i] || !inst[i]->grid_ready || !inst[i]->state_ready || inst[i]->destroy_pending)
            return NHDC_ESTATE;
        if (inst[i]->device != inst[0]->device || inst[i]->precision != inst[0]->precision)
            return NHDC_EINVAL;
        for (int j = 0; j < i; ++j)
            if (inst[j] == inst[i]) return NHDC_EINVAL;  // each instance once
    }
    nhdc_batch *b = new (std::nothrow) nhdc_batch;
    if (!b) return NHDC_ENOMEM;
    b->device = inst[0]->device;
    b->ctxs.assign(inst, inst + n);
    b->L.al = inst[0]->al;  // the batch's descriptors come from its first instance's allocator
    if (hipSetDevice(b->device) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return NHDC_EHIP;
    }
    if (upload_insts(b->L, b->ctxs, b->err) != NHDC_OK) {
        (void)hipStreamDestroy(b->cap);
        delete b;
        return NHDC_ENOMEM;
    }
    rebuild_maps(b->L, b->ctxs, b->tune);
    for (auto *c : b->ctxs) ++c->in_batches;
    *out = b;
    return NHDC_OK;
}

int nhdc_batch_step(nhdc_batch *b, const double *dt, int nsub, int nsteps, void *stream) {
    if (!b) return NHDC_EINVAL;
    int rc = check_dt(b, dt, nsub);
    if (rc) return rc;
    if (nsteps < 0) return set_err(b->err, NHDC_EINVAL, "batch: nsteps must be >= 0");
    if (hipSetDevice(b->device) != hipSuccess) return set_err(b->err, NHDC_EHIP, "batch: hipSetDevice");
    if (!graph_matches(b, dt, nsub) && (rc = capture(b, dt, nsub))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < nsteps; ++i) {
        hipError_t e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) return hip_fail(b->err, e, "batch: hipGraphLaunch");
    }
    return NHDC_OK;
}

int nhdc_batch_set_tiles(nhdc_batch *b, int lt_edge, int lt_cell, int lt_vert) {
    if (!b) return NHDC_EINVAL;
    if (lt_edge < 0 || lt_cell < 0 || lt_vert < 0)
        return set_err(b->err, NHDC_EINVAL, "batch: tiles must be >= 0");
    b->tune.lt_edge = lt_edge;
    b->tune.lt_cell = lt_cell;
    b->tune.lt_vert = lt_vert;
    rebuild_maps(b->L, b->ctxs, b->tune);
    return NHDC_OK;
}

int nhdc_batch_autotune(nhdc_batch *b, const double *dt, int nsub, const char *cache_path,
                        double *best, void *stream) {
    if (!b) return NHDC_EINVAL;
    int rc = check_dt(b, dt, nsub);
    if (rc) return rc;
    if (hipSetDevice(b->device) != hipSuccess) return set_err(b->err, NHDC_EHIP, "batch: hipSetDevice");
    drop_graph(b);
    return autotune(b->L, b->tune, b->ctxs, dt, nsub, cache_path, best,
                    static_cast<hipStream_t>(stream), b->err);
}

const char *nhdc_batch_last_error(const nhdc_batch *b) { return b ? b->err.c_str() : "no batch"; }

void nhdc_batch_destroy(nhdc_batch *b) {
    if (!b) return;
    if (hipSetDevice(b->device) == hipSuccess) {
        (void)hipDeviceSynchronize();  // replays still in flight read the descriptors
        drop_graph(b);
        dev_free(b->L.al, b->L.d_insts);
        if (b->cap) (void)hipStreamDestroy(b->cap);
    }
    for (auto *c : b->ctxs) {
        --c->in_batches;
        if (c->in_batches == 0 && c->destroy_pending) free_context(c);
    }
    delete b;
}

}  // extern "C"

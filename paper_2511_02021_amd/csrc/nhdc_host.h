// nhdc_host.h -- host helpers shared by contexts and batches.
#pragma once
#include <string>
#include <vector>

#include "nhdc_internal.h"

namespace nhdc {
int set_err(std::string &err, int code, const std::string &msg);
int hip_fail(std::string &err, hipError_t e, const char *where);
// enqueue one step (nsub substeps) of every instance of L; dt[i] per instance
hipError_t run_step(const Launcher &L, const double *dt, int nsub, Timing *tm, hipStream_t st);
void rebuild_maps(Launcher &L, const std::vector<nhdc_ctx *> &ctxs, const Tune &t);
int upload_insts(Launcher &L, const std::vector<nhdc_ctx *> &ctxs, std::string &err);
int autotune(Launcher &L, Tune &tune, const std::vector<nhdc_ctx *> &ctxs, const double *dt,
             int nsub, const char *cache_path, double *best_out, hipStream_t st,
             std::string &err);
}  // namespace nhdc

// nhdc_util.hip -- set-up and diagnostic kernels of libnhdc (not on the step
// path): vertex heights, FP32 copies of coefficients, the initial Exner
// history and extrapolated perturbation, the deterministic mass sums and the
// finiteness check.  No contraction, so the metrics equal their plain FP64
// definitions.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "nhdc_internal.h"

#pragma clang fp contract(off)

namespace nhdc {
namespace {

__device__ __forceinline__ int64_t lin() { return int64_t(blockIdx.x) * BLOCK + threadIdx.x; }

inline unsigned nb(int64_t n) { return unsigned((n + BLOCK - 1) / BLOCK); }

__global__ void k_metrics_vert(int64_t nv, int64_t nc, int N, const int32_t *__restrict__ v_c,
                               const double *__restrict__ v_m, const double *__restrict__ v_ival,
                               const double *__restrict__ zh, double *__restrict__ zhv) {
    int64_t v = lin();
    if (v >= nv) return;
    for (int i = 0; i <= N; ++i) {
        const double *z = zh + int64_t(i) * nc;
        double s = 0.0;
        for (int j = 0; j < 6; ++j) s += v_m[j * nv + v] * z[v_c[j * nv + v]];
        zhv[int64_t(i) * nv + v] = s * v_ival[v];
    }
}

__global__ void k_level_nonflat(const double *__restrict__ a, int64_t n, int32_t *__restrict__ out) {
    const int lvl = int(blockIdx.y);
    const int64_t j = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
    const double *row = a + int64_t(lvl) * n;
    const bool d = j < n && __double_as_longlong(row[j]) != __double_as_longlong(row[0]);
    if (__ballot(d) != 0 && (threadIdx.x & 63u) == 0) atomicOr(out + lvl, 1);
}

__global__ void k_to_float(const double *__restrict__ src, float *__restrict__ dst, int64_t n) {
    int64_t i = lin();
    if (i < n) dst[i] = float(src[i]);
}

__global__ void k_to_double(const float *__restrict__ src, double *__restrict__ dst, int64_t n) {
    int64_t i = lin();
    if (i < n) dst[i] = double(src[i]);
}

__global__ void k_init_prev(int64_t n, const double *__restrict__ pi, const double *__restrict__ pi_ref,
                            double *__restrict__ prev) {
    int64_t i = lin();
    if (i < n) prev[i] = pi[i] - pi_ref[i];
}

// extrapolated Exner perturbation of the next predictor
__global__ void k_exner_x(int64_t n, const double *__restrict__ pi, const double *__restrict__ pi_ref,
                          const double *__restrict__ prev, double eps, double *__restrict__ px) {
    int64_t i = lin();
    if (i < n) {
        double pp = pi[i] - pi_ref[i];
        px[i] = (1.0 + eps) * pp - eps * prev[i];
    }
}

// fixed-order two-level reduction: per-block partials, then one block
__global__ void k_diag_partial(int64_t nc, int N, const double *__restrict__ area,
                               const double *__restrict__ zh, const double *__restrict__ rho,
                               const double *__restrict__ thv, double *__restrict__ part) {
    __shared__ double s1[BLOCK], s2[BLOCK];
    int64_t c = lin();
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

template <class T>
__global__ void k_finite(int64_t n, const T *__restrict__ x, int *__restrict__ flag) {
    int64_t i = lin();
    if (i < n && !isfinite(x[i])) flag[0] = 1;  // benign race: every writer stores 1
}

}  // namespace

hipError_t launch_metrics(const Grid &g, hipStream_t st) {
    hipLaunchKernelGGL(k_metrics_vert, dim3(nb(g.nv)), dim3(BLOCK), 0, st, g.nv, g.nc, g.N, g.v_c,
                       g.gd.v_m, g.gd.v_ival, g.zh, g.zhv);
    return hipGetLastError();
}

hipError_t launch_level_nonflat(const double *a, int64_t n, int nlev, int32_t *out, hipStream_t st) {
    hipLaunchKernelGGL(k_level_nonflat, dim3(nb(n), unsigned(nlev)), dim3(BLOCK), 0, st, a, n, out);
    return hipGetLastError();
}

hipError_t launch_to_float(const double *src, float *dst, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_to_float, dim3(nb(n)), dim3(BLOCK), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_to_double(const float *src, double *dst, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_to_double, dim3(nb(n)), dim3(BLOCK), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_init_prev(const Grid &g, const State &s, hipStream_t st) {
    int64_t n = int64_t(g.N) * g.nc;
    hipLaunchKernelGGL(k_init_prev, dim3(nb(n)), dim3(BLOCK), 0, st, n, s.pi, g.pi_ref, s.pi_prev);
    return hipGetLastError();
}

hipError_t launch_exner_x(const Grid &g, const State &s, double eps, hipStream_t st) {
    int64_t n = int64_t(g.N) * g.nc;
    hipLaunchKernelGGL(k_exner_x, dim3(nb(n)), dim3(BLOCK), 0, st, n, s.pi, g.pi_ref, s.pi_prev, eps,
                       s.px);
    return hipGetLastError();
}

hipError_t launch_diag(const Grid &g, const State &s, double *part, double *out2, hipStream_t st) {
    unsigned n = nb(g.nc);
    hipLaunchKernelGGL(k_diag_partial, dim3(n), dim3(BLOCK), 0, st, g.nc, g.N, g.gd.c_area, g.zh,
                       s.rho, s.thv, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(BLOCK), 0, st, int(n), part, out2);
    return hipGetLastError();
}

hipError_t launch_finite(const Grid &g, const State &s, int vn_size, int *flag, hipStream_t st) {
    const int64_t NC = int64_t(g.N) * g.nc, NC1 = int64_t(g.N + 1) * g.nc, NE = int64_t(g.N) * g.ne;
    const double *arrs[4] = {s.rho, s.pi, s.thv, s.pi_prev};
    for (int i = 0; i < 4; ++i)
        hipLaunchKernelGGL(k_finite<double>, dim3(nb(NC)), dim3(BLOCK), 0, st, NC, arrs[i], flag);
    hipLaunchKernelGGL(k_finite<double>, dim3(nb(NC1)), dim3(BLOCK), 0, st, NC1, s.w, flag);
    if (vn_size == 4)
        hipLaunchKernelGGL(k_finite<float>, dim3(nb(NE)), dim3(BLOCK), 0, st, NE,
                           reinterpret_cast<const float *>(s.vn), flag);
    else
        hipLaunchKernelGGL(k_finite<double>, dim3(nb(NE)), dim3(BLOCK), 0, st, NE, s.vn, flag);
    return hipGetLastError();
}

// ---- the allocation-free mass sums (nhdc_diag_noalloc) ----
// The per-block partials live in a fixed device array of this file, one copy
// per GPU for the life of the process.  Host code never passes the array's
// name to a kernel: it looks up the array's device address once per device
// and passes that.
constexpr int64_t NOALLOC_PARTS = (NHDC_NOALLOC_MAX_CELLS + BLOCK - 1) / BLOCK;
static __device__ __align__(256) double scratch[2 * NOALLOC_PARTS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_ptr[MAX_DEVICES] = {};
thread_local std::string free_err;  // message of the last failed context-free call
}  // namespace

const char *context_free_error() { return free_err.empty() ? "no context" : free_err.c_str(); }

// The device address of this device's scratch array, looked up on the first
// call on each device (with that device current).
static hipError_t device_scratch(int dev, double **out) {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

const char *const kKernelNames[K_NUM] = {"vt_edge",   "vertex",      "cell_vt",
                                         "edge_pred", "column_pred", "edge_corr",
                                         "column_corr", "cell_grad", "div4",
                                         "smag_cell",   "smag_edge",   "tr_save",
                                         "tr_recon",    "tr_horiz",    "tr_vert"};

int device_max_lds(int device) {
    static std::mutex mu;
    static int cached[MAX_DEVICES] = {};
    if (device < 0 || device >= MAX_DEVICES) return 65536;
    std::lock_guard<std::mutex> lock(mu);
    if (!cached[device]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess || v <= 0)
            v = 65536;
        cached[device] = v;
    }
    return cached[device];
}

int kind_block(Kind kind, const Tune &t) {
    const int b = kind == KIND_COLUMN ? t.blk_col : kind == KIND_VERT ? t.blk_vert : BLOCK;
    return valid_block(b) ? b : BLOCK;
}

void build_map(Map &m, int64_t &nblocks, Kind kind, const Grid *const *grids, int n,
               const Tune &t, int entities) {
    const int64_t B = entities > 0 ? entities : kind_block(kind, t);
    m.n = n;
    m.off[0] = 0;
    for (int i = 0; i < n; ++i) {
        const Grid &g = *grids[i];
        int64_t ent = kind == KIND_EDGE ? g.ne : kind == KIND_VERT ? g.nv : g.nc;
        int lt = kind == KIND_EDGE ? t.lt_edge : kind == KIND_VERT ? t.lt_vert
               : kind == KIND_CELL ? t.lt_cell : 0;
        if (lt <= 0 || lt > g.N) lt = g.N;
        int64_t nbe = (ent + B - 1) / B;
        int64_t tiles = (g.N + lt - 1) / lt;
        m.nbe[i] = int32_t(nbe);
        m.lt[i] = lt;
        m.off[i + 1] = int32_t(m.off[i] + nbe * tiles);
    }
    nblocks = m.off[n];
}

}  // namespace nhdc

extern "C" int nhdc_diag_noalloc(int64_t n_cells, int32_t n_lev, const double *cell_area,
                                 const double *zh, const double *rho, const double *theta_v,
                                 double *out, void *stream) {
    using namespace nhdc;
    if (!cell_area || !zh || !rho || !theta_v || !out) {
        free_err = "diag_noalloc: NULL array";
        return NHDC_EINVAL;
    }
    if (n_cells < 1 || n_lev < 1 || n_lev > NHDC_MAX_LEV) {
        free_err = "diag_noalloc: n_cells must be >= 1 and n_lev in 1.." + std::to_string(NHDC_MAX_LEV);
        return NHDC_EINVAL;
    }
    if (n_cells > NHDC_NOALLOC_MAX_CELLS) {
        free_err = "diag_noalloc: " + std::to_string(n_cells) + " cells exceed the static scratch of " +
                   std::to_string(int64_t(NHDC_NOALLOC_MAX_CELLS)) + " cells";
        return NHDC_ETOOBIG;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= MAX_DEVICES)) e = hipErrorInvalidDevice;
    double *part = nullptr;
    if (e == hipSuccess) e = device_scratch(dev, &part);
    if (e != hipSuccess) {
        free_err = std::string("diag_noalloc: scratch address: ") + hipGetErrorString(e);
        return NHDC_EHIP;
    }
    // every partial the final pass reads is written first by this call, so
    // nothing needs clearing; the kernels are those of nhdc_diag
    const unsigned n = nb(n_cells);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_diag_partial, dim3(n), dim3(BLOCK), 0, st, int64_t(n_cells), int(n_lev),
                       cell_area, zh, rho, theta_v, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(BLOCK), 0, st, int(n), part, out);
    e = hipGetLastError();
    if (e != hipSuccess) {
        free_err = std::string("diag_noalloc: launch: ") + hipGetErrorString(e);
        return NHDC_EHIP;
    }
    return NHDC_OK;
}

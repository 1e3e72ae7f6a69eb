"""Benchmark: dynamical-core cell-level updates per second on one MI355X.

A step is one dynamical-core step (dt, 5 substeps; each substep = velocity
tendencies, predictor, column solve, tendencies of the prediction, corrector,
column solve) over the whole grid; a cell-level update is one cell at one
full level through one substep.  Inputs are synthetic (seeded recipe with the
paper's grid and level counts) and resident in HBM before timing.

Default workload (the value): R2B8 (5 242 880 cells, the paper's 10 km grid),
90 stretched levels to 75 km over seeded random-harmonic terrain, dt = 22.5 s,
FP64 plain form, 2 warm-up steps then 48 timed steps (a 50-step run).  The
same line carries the FP32-mixed form on the same workload (throughput,
speedup, per-field error against FP64 next to the FP32-rounding floor), the
roofline of the dominant kernel (algorithmic bytes / average duration from
HIP events on the stream the kernels run on) with the whole-substep
accounting (bytes per cell-level-substep of the compulsory and the practical
two-phase budgets, and counted bytes, times the rate), and, under forms, the
other workloads: R2B6x90 in both forms with the options, R2B7x90 mixed with
its per-field error after 100 steps, and the batch of 16 uneven instances
against 16 sequential runs.  The CPU oracle is timed on a bounded sample.

--config 3/4/5 runs one of those workloads alone (for its counter passes).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FIELDS = ("vn", "w", "rho", "pi", "theta_v")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the benchmark's metric: the value is cell-level updates/s; the HBM fraction
# of peak is the roofline object, and the FP32-mixed form with its per-field
# error sits under forms
METRIC = "dycore cell-level updates/s, HBM %peak; FP64 vs FP32-mixed at stated err"


def algorithmic_bytes(nc, ne, nv, N, prec="fp64", nsub=5, nt=4):
    """Bytes each kernel must read and write once per launch: every input and
    output array once at its size (cached re-reads of gathered neighbours,
    register-carried levels and column scratch round trips not counted).
    Tendency-side arrays are FP32 in the mixed form; state, fluxes and the
    column are FP64 in both.  The Exner history is written on the last of
    `nsub` substeps only, so it counts 1/nsub per corrector column launch.
    The stored normal velocity (vn, and the predicted vn*) takes 4 bytes in
    the mixed_vn32 variant, 8 otherwise."""
    r = 8 if prec == "fp64" else 4
    vb = 4 if prec == "mixed_vn32" else 8
    C, C1, Ci = N * nc, (N + 1) * nc, (N - 1) * nc        # entity-level counts
    E, V, V1, Vi = N * ne, N * nv, (N + 1) * nv, (N - 1) * nv
    gc = nc * 3 * (4 + 4 + 4 + r) + nc * r                 # c_e, c_n, c_v, c_sl; area
    ge = ne * (2 * 4 + 2 * 4 + 2 * r)                      # e_c, e_v, d_e/l_e or f
    gv = nv * 6 * (4 + 4 + r + r) + 2 * nv * r
    recon = 2 * ne * (3 * 4 + 16 * r) + 3 * ne * r         # two cells' reconstruction coeffs + tangent
    t = {
        "vt_edge": [E * vb + E * r + recon],
        "vertex": [E * vb + Ci * 8 + V * r + Vi * r + gv],
        # vn, vt, w, wv, zh, zhv -> kc, wcc, tw (+ div vn in the corrector)
        "cell_vt": [E * vb + E * r + C1 * 8 + Vi * r + C1 * 8 + V1 * 8 + C * r + 2 * C1 * r + gc + ge,
                    E * vb + E * r + C1 * 8 + Vi * r + C1 * 8 + V1 * 8 + 2 * C * r + 2 * C1 * r + gc + ge],
        # kc, zeta, vt, vn, w, wcc, px, thv, zh -> tvn, vns
        "edge_pred": [C * r + V * r + E * r + E * vb + C1 * 8 + C1 * r + 2 * C * 8 + C1 * 8
                      + E * r + E * vb + ge],
        # kc, zeta, vt, vns, ws, wcc1, thvs, tvn0, px, dvn, vn, thv, rho, zh, facc -> vn, flx, hfl, facc
        "edge_corr": [C * r + V * r + E * r + E * vb + C1 * 8 + C1 * r + C * 8 + E * r + C * 8 + C * r
                      + E * vb + 2 * C * 8 + C1 * 8 + E * 8 + E * vb + 3 * E * 8 + ge],
        # vns, rho, thv, pi, pi_ref, theta_ref, w, wcc, tw, zh -> ws, rhos, thvs
        "column_pred": [E * vb + 5 * C * 8 + C1 * 8 + 2 * C1 * r + C1 * 8 + 2 * C * 8 + gc],
        # flx, hfl, rho, thv, pi, pi_ref, theta_ref, w, rhos, thvs, wcc1, tw0, tw1, zh, wacc
        #   -> w, rho, thv, pi, px, wacc (+ pi_prev on the last substep)
        "column_corr": [2 * E * 8 + 5 * C * 8 + C1 * 8 + 2 * C * 8 + 3 * C1 * r + C1 * 8 + C1 * 8
                        + C1 * 8 + 4 * C * 8 + C * 8 / nsub + C1 * 8 + gc],
        # (upwind option) rho, thv -> their gradients, 3 components each
        "cell_grad": [2 * C * 8 + 6 * C * 8 + gc + ne * (8 + 3 * 8)],
    }
    # builds of the upwind option: the edge kernels also read the six gradient
    # fields and the edge's displacements, normal and tangent; the predictor
    # also reads rho and writes both fluxes, which its column then reads in
    # place of the predicted vn
    upg = 6 * C * 8 + ne * 12 * 8
    t["edge_pred_upwind"] = [t["edge_pred"][0] + upg + C * 8 + 2 * E * 8]
    t["edge_corr_upwind"] = [t["edge_corr"][0] + upg]
    t["column_pred_upwind"] = [t["column_pred"][0] + E * 8]
    t["column_corr_upwind"] = list(t["column_corr"])
    # damping and diffusion options: D(G(div vn*)) per cell; the once-per-step
    # diffusion's cell pass (vn, vt -> div, coefficient) and edge pass
    # (coefficient, div, vorticity, vn -> vn); the corrector's edges also
    # gather D(G(div vn*)); the sponge's rate profile is N+1 values
    t["div4"] = [2 * C * r + nc * (3 * 4 + 3 * 4 + 3 * r + r) + ne * r]
    t["smag_cell"] = [E * 8 + E * r + 2 * C * r + gc + nc * 3 * r + ne * 3 * (8 + r)]
    t["smag_edge"] = [2 * C * r + V * r + 2 * E * 8 + ge + ne * r]
    t["edge_corr_div4"] = [t["edge_corr"][0] + C * r]
    t["column_pred_sponge"] = list(t["column_pred"])
    t["column_corr_sponge"] = list(t["column_corr"])
    # tracers (nt of them, FP64): density kept at the start of the step;
    # reconstruction toward the three edges; horizontal update (mass fluxes,
    # densities, reconstructions, q -> q*, rho*); vertical PPM (q*, rho*,
    # heights, vertical mass flux -> q)
    t["tr_save"] = [2 * C * 8]
    t["tr_recon"] = [nt * (C * 8 + 3 * C * 8) + nc * (3 * 4 * 2 + 3 * 8 + 9 * 8 + 3 * 8 + 8)
                     + ne * (8 + 3 * 8)]
    t["tr_horiz"] = [E * 8 + 2 * C * 8 + C1 * 8 + nt * (5 * C * 8) + nc * (3 * 4 * 3 + 3 * 8 + 8)]
    t["tr_vert"] = [2 * C1 * 8 + C * 8 + nt * 2 * C * 8]
    return {k: sum(v) / len(v) for k, v in t.items()}


KERNEL_SOURCES = ("nhdc_step.inc", "nhdc_fp64.hip", "nhdc_mixed.hip", "nhdc_mixed_vn32.hip",
                  "nhdc_internal.h")


def _code_tokens(src):
    """`src` (C++ source text) without its comments, every run of white space
    made one blank; string and character literals are kept as written."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return re.sub(r"\s+", " ", "".join(out)).strip()


def kernel_source_hash():
    """Identifies the device code of the step kernels (counter summaries taken
    on other code no longer describe them); comments and layout do not count."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_02021_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(_code_tokens(fh.read()).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def _summary_matches(txt, src_hash, numbering):
    """A counter summary describes this run if it was taken on the current
    kernel sources and the same numbering of the grid."""
    m = re.search(r"kernel_source_sha256_16:\s*(\w+)", txt)
    n = re.search(r"^numbering:\s*(\w+)", txt, re.M)
    return bool(m and n and m.group(1) == src_hash and n.group(1) == numbering)


def measured_traffic(kernel, src_hash, precision, numbering="curve", tag="r2b8x90"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of workload `tag`, if it was taken on the current kernel sources
    and numbering; else None."""
    path = os.path.join(ROOT, "profiles", f"dycore_{precision}_{tag}_hbm_counters.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    b = re.search(rf"^{kernel}\s+.*?hbm_bytes_per_launch=([0-9.eE+]+)", txt, re.M)
    if not b or not _summary_matches(txt, src_hash, numbering):
        return None
    return float(b.group(1))


LAUNCHES_PER_STEP = {"vt_edge": 2, "vertex": 2, "cell_vt": 2, "edge_pred": 1, "column_pred": 1,
                     "edge_corr": 1, "column_corr": 1}  # per substep


def step_traffic(src_hash, precision, nsub, numbering="curve", tag="r2b8x90"):
    """HBM bytes of one whole step from the committed counter summary of
    workload `tag` (every kernel's counted bytes per launch x its launches),
    if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"dycore_{precision}_{tag}_hbm_counters.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    if not _summary_matches(txt, src_hash, numbering):
        return None
    total = 0.0
    for k, n in LAUNCHES_PER_STEP.items():
        b = re.search(rf"^{k}\s+.*?hbm_bytes_per_launch=([0-9.eE+]+)", txt, re.M)
        if not b:
            return None
        total += float(b.group(1)) * n * nsub
    return total


def cpu_baseline(case, headline_tag=None):
    """The oracle, as it stands, on one step (5 substeps) of `case` (the
    R2B6x90 workload: the oracle cannot hold the larger grids in host memory,
    and its rate per cell-level is about the same at any size)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    m = oracle.Model(case)
    t0 = time.perf_counter()
    m.step(case.dt, case.nsub)
    el = time.perf_counter() - t0
    units = case.grid.n_cells * case.n_lev * case.nsub
    out = {"value": units / el, "unit": "cell-level updates/s", "cores": threads,
           "kind": "oracle", "seconds": round(el, 2),
           "sample": f"1 step ({case.nsub} substeps) of the R2B{case.grid.k}x{case.n_lev} case of the "
                     f"same recipe (terrain, 90 stretched levels) from its initial state"
                     + (f", standing in for the {headline_tag} workload, which exceeds the oracle's "
                        f"host memory" if headline_tag and headline_tag != "r2b6x90" else "")}
    out["host_cpu"] = host_cpu_model()
    out["logical_cpus"] = os.cpu_count()
    # thread scaling of the oracle on the small flat case (R2B4x20, one step),
    # in child processes with their own OpenMP thread counts
    out["small_case"] = {n: oracle_small_case_rate(n) for n in (1, threads)}
    return out


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_small_case_rate(threads):
    """Cell-level updates/s of the oracle on one step of R2B4x20 (flat, dt
    300 s) with `threads` OpenMP threads, timed in a child process."""
    import subprocess
    code = ("import time, oracle\n"
            "from paper_2511_02021_amd.inputs import case as CS\n"
            "c = CS.config_case(1)\n"
            "m = oracle.Model(c)\n"
            "t = time.perf_counter(); m.step(c.dt, c.nsub); el = time.perf_counter() - t\n"
            "print(c.grid.n_cells * c.n_lev * c.nsub / el, el)\n")
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    if r.returncode != 0:
        return {"error": r.stderr.strip()[-200:]}
    v, el = (float(x) for x in r.stdout.split())
    return {"threads": threads, "value": v, "seconds": round(el, 3)}


def timed_steps(torch, stepper, steps, warmup, stream):
    for _ in range(warmup):
        stepper()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        stepper()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def copy_bandwidth(torch, gib=4, reps=10):
    """Device-to-device copy of `gib` GiB (read + write counted), the best of
    `reps`: the HBM rate a plain streaming kernel reaches on this GPU."""
    n = (gib << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2 * (gib << 30) / (best / 1e3) / 1e9


def stream_rates(torch, gib=4, reps=10):
    """Read-only (a sum) and write-only (a fill) streaming over `gib` GiB, the
    best of `reps` each, in GB/s: with the copy, the rates plain streaming
    kernels reach on this GPU."""
    n = (gib << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    out = {}
    for name, op in (("read", lambda: a.sum()), ("write", lambda: a.fill_(1.0))):
        best = float("inf")
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            op()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        out[name] = (gib << 30) / (best / 1e3) / 1e9
    del a
    torch.cuda.empty_cache()
    return out


def kernel_table(d, case, steps, stream, precision):
    g = case.grid
    d.set_timing(True)
    for _ in range(steps):
        d.step(case.dt, case.nsub, stream)
    stats = d.kernel_stats()
    d.set_timing(False)
    nt = 0 if case.tracers is None else case.tracers.shape[0]
    alg = algorithmic_bytes(g.n_cells, g.n_edges, g.n_verts, case.n_lev, precision, nt=nt)
    if case.params.upwind:
        alg = {k: alg.get(k + "_upwind", v) for k, v in alg.items()}
    if case.params.div_damp4:
        alg["edge_corr"] = alg["edge_corr_div4"]
    kern = {k: {"avg_ms": v[0] / v[1], "launches": v[1], "total": v[0]} for k, v in stats.items()
            if v[1]}
    tot = sum(x["total"] for x in kern.values())
    for k in kern:
        kern[k]["share"] = kern[k]["total"] / tot
        kern[k]["alg_bytes"] = alg[k]
        kern[k]["alg_GBs"] = alg[k] / (kern[k]["avg_ms"] / 1e3) / 1e9
    return kern


def rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def error_table(nhdc, case, steps):
    """Per field: E = rel-L2(mixed - FP64), S = rel-L2 between two FP64 runs
    whose initial states differ by seeded relative noise 2^-24 (the
    FP32-rounding floor), both after `steps` steps from the initial state."""
    import numpy as np
    init = dict(vn=case.vn, w=case.w, rho=case.rho, pi=case.pi, theta_v=case.theta_v)

    def run(prec, state=None):
        d = nhdc.Dycore(case, precision=prec)
        if state is not None:
            d.init_state(*[state[f] for f in FIELDS])
        for _ in range(steps):
            d.step(case.dt, case.nsub)
        s = d.get_state()
        d.close()
        return s

    f64 = run("fp64")
    mix = run("mixed")
    rng = np.random.default_rng(7)
    pert = {k: v * (1.0 + 2.0 ** -24 * rng.standard_normal(v.shape)) for k, v in init.items()}
    f64p = run("fp64", pert)
    out = {}
    for f in FIELDS:
        sig = np.linalg.norm(f64[f] - init[f])
        out[f] = {"E": rel_l2(mix[f], f64[f]), "S": rel_l2(f64p[f], f64[f]),
                  "E_over_signal": float(np.linalg.norm(mix[f] - f64[f]) / max(sig, 1e-300))}
    return out


# bytes per cell-level-substep of the substep's budget (the design-independent
# accounting): the compulsory traffic of an ideal single pass (state n read and
# written, the Exner history, the FP64 flux accumulators read-modify-write, the
# heights and reference profiles) and a practical two-phase design (plus the
# predicted state, the state-n tendencies and the Exner gradient written and
# read, and state n read again by the corrector); edge fields count 1.5 per
# cell-level.  The mixed form's tendency arrays are FP32.
STEP_BUDGET_B = {"fp64": {"compulsory": 152.0, "practical": 332.0},
                 "mixed": {"compulsory": 152.0, "practical": 300.0}}


def step_accounting(rate, precision, counted_b=None):
    """Whole-substep bandwidth of a form running at `rate` cell-level
    updates/s (= cell-level-substeps/s): each budget's bytes x rate, and the
    counted bytes x rate when a counter summary of the same kernel sources
    gives them; each against the 8 TB/s peak."""
    out = {}
    for basis, b in STEP_BUDGET_B[precision].items():
        gbs = b * rate / 1e9
        out[basis] = {"B_per_cell_level_substep": b, "GBs": round(gbs, 1),
                      "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if counted_b is not None:
        gbs = counted_b * rate / 1e9
        out["counted"] = {"B_per_cell_level_substep": round(counted_b, 1), "GBs": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def time_form(args, torch, nhdc, case, prec, stream, steps=None, warmup=None, table=True,
              handover=False):
    """One form on one case: throughput over `steps` timed steps after
    `warmup` untimed ones, then (optionally) the per-kernel table.  With
    `handover`, the wall-clock time of handing the state over from pageable
    host memory before the run and back after it, and the rate that counts
    both beside the timed steps (the timed steps themselves start with the
    state resident in HBM either way)."""
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    g = case.grid
    d = nhdc.Dycore(case, precision=prec, init=not handover)
    if handover:  # nhdc_init_state from host buffers returns once the copies are done
        t0 = time.perf_counter()
        d.init_state(case.vn, case.w, case.rho, case.pi, case.theta_v)
        up_s = time.perf_counter() - t0
    if getattr(args, "column_mode", -1) >= 0:
        d.set_column_mode(args.column_mode)
    ms = timed_steps(torch, lambda: d.step(case.dt, case.nsub, stream), steps, warmup, stream)
    d.check_finite()
    units = g.n_cells * case.n_lev * case.nsub
    out = {"value": units * steps / (ms / 1e3), "ms_per_step": ms / steps}
    if handover:  # nhdc_get_state into host buffers, likewise synchronous
        t0 = time.perf_counter()
        st = d.get_state()
        down_s = time.perf_counter() - t0
        b_in = sum(getattr(case, f).nbytes for f in ("vn", "w", "rho", "pi", "theta_v"))
        b_out = sum(a.nbytes for a in st.values())
        del st
        out["host_handover"] = {
            "bytes_in": b_in, "upload_s": round(up_s, 3), "upload_GBs": round(b_in / up_s / 1e9, 2),
            "bytes_out": b_out, "download_s": round(down_s, 3),
            "download_GBs": round(b_out / down_s / 1e9, 2),
            "pcie_inclusive_value": units * steps / (ms / 1e3 + up_s + down_s),
            "basis": f"the {steps} timed steps plus one upload of the initial state and one "
                     "download of the final state, from and to pageable host memory"}
    if table:
        out["_table"] = kernel_table(d, case, args.timing_steps, stream, prec)
    d.close()
    return out


def error_table_device(torch, nhdc, case, steps, precision="mixed"):
    """Per field: E = rel-L2(mixed - FP64), S = rel-L2 between two FP64 runs
    whose initial states differ by seeded relative noise 2^-24 (the
    FP32-rounding floor), after `steps` steps from the initial state.  The
    norms are taken on the device, so grids of any size fit."""
    dev = torch.device("cuda", 0)
    init = {f: torch.from_numpy(getattr(case, f)).to(dev) for f in FIELDS}

    def run(prec, state=None):
        d = nhdc.Dycore(case, precision=prec)
        if state is not None:
            d.init_state(*[state[f] for f in FIELDS])
        for _ in range(steps):
            d.step(case.dt, case.nsub)
        out = d.get_state_device()
        torch.cuda.synchronize()
        d.close()
        return {f: out[f] for f in FIELDS}

    f64 = run("fp64")
    mix = run(precision)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    pert = {f: v * (1.0 + 2.0 ** -24 * torch.randn(v.shape, generator=gen, device=dev,
                                                      dtype=torch.float64)) for f, v in init.items()}
    f64p = run("fp64", pert)
    del pert
    out = {}
    for f in FIELDS:
        nref = float(torch.linalg.vector_norm(f64[f]))
        sig = float(torch.linalg.vector_norm(f64[f] - init[f]))
        e = float(torch.linalg.vector_norm(mix[f] - f64[f]))
        sf = float(torch.linalg.vector_norm(f64p[f] - f64[f]))
        out[f] = {"E": e / nref, "S": sf / nref, "E_over_signal": e / max(sig, 1e-300)}
    del f64, mix, f64p, init
    torch.cuda.empty_cache()
    return out


def options_forms(args, torch, nhdc, CS, case, stream, plain_ms):
    """The FP64 step with each option set, on `case`, timed as the plain form."""
    import dataclasses
    units = case.grid.n_cells * case.n_lev * case.nsub
    out = {}

    def one(label, ocase):
        r = time_form(args, torch, nhdc, ocase, "fp64", stream)
        tab = r.pop("_table")
        r["cost_vs_plain"] = r["ms_per_step"] / plain_ms
        r["kernels"] = {k: {"avg_ms": round(v["avg_ms"], 5), "alg_GBs": round(v["alg_GBs"], 1)}
                        for k, v in tab.items()}
        log(f"  fp64 {label}: {r['ms_per_step']:.3f} ms/step, {r['value']:.4e} cell-level updates/s")
        return r

    extra = [f for f in args.options.split(",") if f]
    if "upwind" in extra:  # second-order upwind edge values of rho and theta_v
        out["fp64_upwind"] = one("upwind", dataclasses.replace(
            case, params=dataclasses.replace(case.params, upwind=1)))
    if "damped" in extra:  # fourth-order divergence damping, w sponge, Smagorinsky diffusion
        dc = CS.with_damping(case)
        out["fp64_damped"] = one("damped", dc)
        out["fp64_damped"]["options"] = {"div_damp4": dc.params.div_damp4, "smag": dc.params.smag,
                                         "sponge_rate_at_lid": float(dc.w_damp[0]),
                                         "sponge_base_m": CS.DAMPED["sponge_base"]}
    if "tracers" in extra:  # four tracers carried by the step's averaged mass fluxes
        out["fp64_tracers"] = one("tracers", CS.with_tracers(case))
        out["fp64_tracers"]["tracers"] = list(CS.TRACER_NAMES)
    return out


def short_table(tab):
    return {k: {"avg_ms": round(v["avg_ms"], 5), "share": round(v["share"], 4),
                "alg_GBs": round(v["alg_GBs"], 1)} for k, v in tab.items()}


def kernel_roofline(tab, src_hash, prec, tag, numbering):
    """The dominant kernel's algorithmic bytes per launch over its average
    launch time (HIP events on the step's stream), against the 8 TB/s peak;
    traffic = its counted bytes per launch when the counter summary of this
    workload was taken on the current kernel sources."""
    dom = max(tab, key=lambda k: tab[k]["share"])
    achieved = tab[dom]["alg_GBs"]
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom, src_hash, prec, numbering, tag),
            "alg_bytes_per_launch": int(tab[dom]["alg_bytes"]),
            "avg_launch_ms": round(tab[dom]["avg_ms"], 5),
            "basis": "dominant kernel: its algorithmic bytes per launch (every input and output "
                     "array once) / its average launch time"}


def bench_headline(args, torch, nhdc, CS):
    """The headline workload in the FP64 and FP32-mixed forms, with the
    other contract workloads as forms of the same line."""
    stream = torch.cuda.current_stream()
    cfg = args.headline
    tag = f"r2b{CS.CONFIGS[cfg]['k']}x{CS.CONFIGS[cfg]['n_lev']}"
    t0 = time.time()
    case = CS.config_case(cfg, order=args.order)
    g = case.grid
    units_per_step = g.n_cells * case.n_lev * case.nsub
    log(f"case R2B{g.k}x{case.n_lev}: {g.n_cells} cells, {g.n_edges} edges ({time.time() - t0:.1f}s)")
    forms, tables = {}, {}
    want = [f for f in args.forms.split(",") if f]
    for prec in ("fp64", "mixed"):
        forms[prec] = time_form(args, torch, nhdc, case, prec, stream, handover=prec == "fp64")
        tables[prec] = forms[prec].pop("_table")
        log(f"{prec}: {forms[prec]['ms_per_step']:.3f} ms/step, "
            f"{forms[prec]['value']:.4e} cell-level updates/s")
        if "host_handover" in forms[prec]:
            h = forms[prec]["host_handover"]
            log(f"  state from/to host: {h['upload_s']:.2f} s in, {h['download_s']:.2f} s out; "
                f"with them {h['pcie_inclusive_value']:.4e} cell-level updates/s")
    forms["mixed"]["speedup_vs_fp64"] = forms["fp64"]["ms_per_step"] / forms["mixed"]["ms_per_step"]
    if args.error_steps > 0:
        log(f"per-field error of the mixed form, {args.error_steps} steps ...")
        forms["mixed"]["per_field_error"] = error_table_device(torch, nhdc, case, args.error_steps)
        forms["mixed"]["error_steps"] = args.error_steps
    if "vn32" in want:  # the mixed form's variant with vn stored in FP32
        r = time_form(args, torch, nhdc, case, "mixed_vn32", stream)
        tab = r.pop("_table")
        r["speedup_vs_fp64"] = forms["fp64"]["ms_per_step"] / r["ms_per_step"]
        r["speedup_vs_mixed"] = forms["mixed"]["ms_per_step"] / r["ms_per_step"]
        r["kernels"] = short_table(tab)
        log(f"mixed_vn32: {r['ms_per_step']:.3f} ms/step, {r['value']:.4e} cell-level updates/s")
        if args.error_steps > 0:
            r["per_field_error"] = error_table_device(torch, nhdc, case, args.error_steps, "mixed_vn32")
            r["error_steps"] = args.error_steps
        forms["mixed_vn32"] = r
    src_hash = kernel_source_hash()
    kern = tables["fp64"]
    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["share"]):
        log(f"  fp64 {k:12s} {v['avg_ms']:8.4f} ms  share {v['share']:.3f}  {v['alg_GBs']:8.1f} GB/s")
    roofline = kernel_roofline(kern, src_hash, "fp64", tag, args.order)
    counted = step_traffic(src_hash, "fp64", case.nsub, args.order, tag)
    roofline["step"] = step_accounting(forms["fp64"]["value"], "fp64",
                                       None if counted is None else counted / (units_per_step))
    if not args.copy_calibration:  # counter runs keep a single copy: the calibration one
        copy_gbs = copy_bandwidth(torch)
        roofline["copy_GBs"] = round(copy_gbs, 1)
        roofline["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 4)
        rates = stream_rates(torch)
        roofline["read_GBs"] = round(rates["read"], 1)
        roofline["write_GBs"] = round(rates["write"], 1)
        log(f"4 GiB device copy: {copy_gbs:.1f} GB/s; read-only {rates['read']:.1f}, "
            f"write-only {rates['write']:.1f} GB/s")
    mk = tables["mixed"]
    forms["mixed"]["kernels"] = short_table(mk)
    forms["mixed"]["roofline"] = kernel_roofline(mk, src_hash, "mixed", tag, args.order)
    mcount = step_traffic(src_hash, "mixed", case.nsub, args.order, tag)
    forms["mixed"]["roofline"]["step"] = step_accounting(
        forms["mixed"]["value"], "mixed", None if mcount is None else mcount / units_per_step)
    workload = (f"R2B{g.k} ({g.n_cells} cells) x {case.n_lev} levels to 75 km, terrain, "
                f"dt={case.dt:g}s, {case.nsub} substeps, FP64 plain")
    del case
    if "r2b6" in want and cfg != 2:  # the R2B6x90 workload: both forms and the options
        c2 = CS.config_case(2, order=args.order)
        log("R2B6x90 ...")
        r6 = {}
        for prec in ("fp64", "mixed") + (("mixed_vn32",) if "vn32" in want else ()):
            r6[prec] = time_form(args, torch, nhdc, c2, prec, stream)
            r6[prec]["kernels"] = short_table(r6[prec].pop("_table"))
            log(f"  {prec}: {r6[prec]['ms_per_step']:.3f} ms/step, {r6[prec]['value']:.4e}")
        r6.update(options_forms(args, torch, nhdc, CS, c2, stream, r6["fp64"]["ms_per_step"]))
        forms["config2_r2b6x90"] = r6
        del c2
    elif cfg == 2:
        forms.update(options_forms(args, torch, nhdc, CS, CS.config_case(2, order=args.order), stream,
                                   forms["fp64"]["ms_per_step"]))
    if "config1" in want:  # the small flat case: its working set fits the 256 MB Infinity Cache
        c1 = CS.config_case(1, order=args.order)
        r1 = time_form(args, torch, nhdc, c1, "fp64", stream, steps=20, warmup=2, table=False)
        r1["workload"] = "R2B4 (20480 cells) x 20 levels to 30 km, flat, dt=300s, 5 substeps, FP64 plain"
        r1["steps"] = 20
        forms["config1_r2b4x20"] = r1
        log(f"R2B4x20 fp64: {r1['ms_per_step']:.3f} ms/step ({r1['value']:.4e})")
    if "small" in want:
        log("small shares ...")
        forms["small_shares"] = bench_small_shares(args, torch, nhdc, CS, stream)
    if "config3" in want:
        log("R2B7x90 mixed ...")
        forms["config3_r2b7x90_mixed"] = bench_config3(args, torch, nhdc, CS, stream)
    if "config4" in want:
        log("batch of 16 ...")
        forms["config4_batch16"] = bench_batch_form(args, torch, nhdc, CS, stream)
    if args.copy_calibration:  # the run's last device work: the copy the counters are scaled by
        calibration_copy(torch)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(CS.config_case(2, order=args.order), headline_tag=tag)
        log(f"  oracle {cpu['value']:.4e} cell-level updates/s on {cpu['cores']} threads")
    return {
        "metric": METRIC,
        "value": forms["fp64"]["value"],
        "unit": "cell-level updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": forms["fp64"]["ms_per_step"],
        "simulated_s_per_wall_s": CS.CONFIGS[cfg]["dt"] / (forms["fp64"]["ms_per_step"] / 1e3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "cells": g.n_cells, "levels": CS.CONFIGS[cfg]["n_lev"],
                   "substeps": 5, "numbering": args.order, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "kernels": short_table(kern),
        "kernel_source_sha256_16": src_hash,
        **({"column_mode": args.column_mode} if args.column_mode >= 0 else {}),
    }


def bench_small_shares(args, torch, nhdc, CS, stream):
    """Shares of one GPU near the paper's strong-scaling floor (about 10 800
    cells per GPU at 90 levels, Sec. 5): R2B3 (5120 cells), R2B4 (20480) and
    R2B5 (81920) x 90 levels of the R2B6x90 recipe, FP64.  Each with the
    library's starting shapes for its size (level tiles; the level-parallel
    column up to 40960 cells), with whole columns and the streaming column,
    and with the autotuner's shapes; and the two column builds' kernel
    times."""
    out = {}
    for k in (3, 4, 5):
        c = CS.config_case(2, k=k, order=args.order)
        units = c.grid.n_cells * c.n_lev * c.nsub
        d = nhdc.Dycore(c)
        steps = 30
        r = {"workload": f"R2B{k} ({c.grid.n_cells} cells) x {c.n_lev} levels to 75 km, terrain, "
                         f"dt={c.dt:g}s, {c.nsub} substeps, FP64 plain"}

        def run(tag):
            ms = timed_steps(torch, lambda: d.step(c.dt, c.nsub, stream), steps, 3, stream) / steps
            r[tag] = {"ms_per_step": ms, "value": units / (ms / 1e3)}
            return ms

        run("starting_shapes")
        cols = {}
        for mode, name in ((1, "levels"), (0, "stream")):
            d.set_column_mode(mode)
            tab = kernel_table(d, c, 4, stream, "fp64")
            cols[name] = {kk: round(tab[kk]["avg_ms"], 4) for kk in ("column_pred", "column_corr")}
        r["column_kernels_ms"] = cols
        d.set_tiles(0, 0, 0)
        d.set_column_mode(0)
        run("whole_columns_stream")
        best = d.autotune(c.dt, c.nsub)
        run("autotuned")
        r["autotuned"]["shapes"] = {"lt_edge": best[0], "lt_cell": best[1], "lt_vert": best[2],
                                    "column_mode": best[7]}
        d.check_finite()
        d.close()
        r["speedup_starting_vs_whole_stream"] = (r["whole_columns_stream"]["ms_per_step"]
                                                 / r["starting_shapes"]["ms_per_step"])
        log(f"  R2B{k}x90: starting shapes {r['starting_shapes']['ms_per_step']:.3f} ms/step, whole columns "
            f"{r['whole_columns_stream']['ms_per_step']:.3f}, autotuned {r['autotuned']['ms_per_step']:.3f}; "
            f"columns levels {cols['levels']} stream {cols['stream']}")
        out[f"r2b{k}x90"] = r
    return out


def bench_config3(args, torch, nhdc, CS, stream):
    """R2B7x90 in the FP32-mixed form: throughput, and the per-field error
    against FP64 after the workload's 100 steps."""
    case = CS.config_case(3, order=args.order)
    r = time_form(args, torch, nhdc, case, "mixed", stream, table=False)
    f = time_form(args, torch, nhdc, case, "fp64", stream, table=False)
    r["fp64_ms_per_step"] = f["ms_per_step"]
    r["speedup_vs_fp64"] = f["ms_per_step"] / r["ms_per_step"]
    r["workload"] = (f"R2B7 ({case.grid.n_cells} cells) x 90 levels, terrain, dt={case.dt:g}s, "
                     "5 substeps, FP32-mixed")
    log(f"  mixed {r['ms_per_step']:.3f} ms/step ({r['value']:.4e}), fp64 {f['ms_per_step']:.3f}")
    if args.error_steps > 0:
        n = CS.CONFIGS[3]["steps"]
        log(f"  per-field error after {n} steps ...")
        r["per_field_error"] = error_table_device(torch, nhdc, case, n)
        r["error_steps"] = n
    return r


def bench_batch_form(args, torch, nhdc, CS, stream):
    """16 uneven instances (R2B4-R2B6, 30-90 levels), FP32-mixed, one launch
    per kernel over all instances, graph replay, autotuned level tiles; against
    the 16 instances run one after another in the plain FP64 form and in the
    mixed form, each instance for the same 10 steps."""
    cases = CS.batch_cases(order=args.order)
    steps = 10
    units = sum(c.grid.n_cells * c.n_lev * c.nsub for c in cases) * steps
    res = {}
    for prec in ("fp64", "mixed"):
        total = 0.0
        for c in cases:  # sequential, one instance at a time
            d = nhdc.Dycore(c, precision=prec)
            total += timed_steps(torch, lambda: d.step(c.dt, c.nsub, stream), steps, 1, stream)
            d.close()
        res[f"sequential_{prec}_ms"] = total
    ds = [nhdc.Dycore(c, precision="mixed") for c in cases]
    b = nhdc.Batch(ds)
    dts = [c.dt for c in cases]
    best = b.autotune(dts, 5)
    ms = timed_steps(torch, lambda: b.step(dts, 5, 1, stream), steps, 1, stream)
    for d in ds:
        d.check_finite()
    # the persistent path: each step's substeps as one cooperative launch
    b.set_persistent(True)
    pbest = b.autotune(dts, 5)
    pms = timed_steps(torch, lambda: b.step(dts, 5, 1, stream), steps, 1, stream)
    for d in ds:
        d.check_finite()
    grid = b.persistent_grid
    b.close()
    for d in ds:
        d.close()
    out = {"value": units / (ms / 1e3), "ms_per_step": ms / steps, "steps": steps,
           "path": "graph of launches (one launch per kernel over all instances, a step captured once)",
           "instances": [f"R2B{c.grid.k}x{c.n_lev}" for c in cases],
           "shapes": {"lt_edge": best[0], "lt_cell": best[1], "lt_vert": best[2],
                      "block_column": best[3], "block_vertex": best[4], "column_waves": best[5]},
           "speedup_vs_sequential_fp64": res["sequential_fp64_ms"] / ms,
           "speedup_vs_sequential_mixed": res["sequential_mixed_ms"] / ms,
           "sequential_ms": res,
           "persistent": {"value": units / (pms / 1e3), "ms_per_step": pms / steps, "grid_blocks": grid,
                          "shapes": {"lt_edge": pbest[0], "lt_cell": pbest[1], "lt_vert": pbest[2]},
                          "vs_graph": ms / pms,
                          "speedup_vs_sequential_fp64": res["sequential_fp64_ms"] / pms,
                          "speedup_vs_sequential_mixed": res["sequential_mixed_ms"] / pms}}
    log(f"  batch {ms / steps:.3f} ms/step ({out['value']:.4e}); x{out['speedup_vs_sequential_fp64']:.2f} "
        f"vs sequential fp64, x{out['speedup_vs_sequential_mixed']:.2f} vs sequential mixed; "
        f"persistent {pms / steps:.3f} ms/step on {grid} blocks")
    return out


def calibration_copy(torch):
    """One 1 GiB device-to-device copy: a plain copy kernel of known size whose
    counter readings scale the hardware byte counters."""
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: 1 GiB read + 1 GiB written")
    del a, b


def counters_line(args, ms, steps, units, workload):
    """The JSON line of a counter run: how many steps ran in all (warm-up and
    timed), for the per-step byte count."""
    return {"metric": METRIC, "value": units / (ms / 1e3), "unit": "cell-level updates/s",
            "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": ms / steps,
            "steps_run": steps + args.warmup, "counters_run": True, "config": {"workload": workload},
            "tiles_arg": "" if args.tiles == [0, 0, 0] else " --tiles " + ",".join(map(str, args.tiles)),
            "kernel_source_sha256_16": kernel_source_hash()}


def bench_single(args, torch, nhdc, CS, cfg):
    """R2B7x90 (config 3) or R2B8x90 (config 5), FP32-mixed."""
    stream = torch.cuda.current_stream()
    t0 = time.time()
    case = CS.config_case(cfg)
    g = case.grid
    log(f"case R2B{g.k}x{case.n_lev}: {g.n_cells} cells ({time.time() - t0:.1f}s)")
    steps = args.steps if args.steps is not None else CS.CONFIGS[cfg]["steps"] - 2
    d = nhdc.Dycore(case, precision="mixed")
    ms = timed_steps(torch, lambda: d.step(case.dt, case.nsub, stream), steps, args.warmup, stream)
    d.check_finite()
    units = g.n_cells * case.n_lev * case.nsub * steps
    if args.counters:  # only the warm-up and timed steps ran: counted bytes / steps_run
        d.close()
        calibration_copy(torch)
        return counters_line(args, ms, steps, units, f"R2B{g.k}x{case.n_lev} FP32-mixed")
    kern = kernel_table(d, case, args.timing_steps, stream, "mixed")
    d.close()
    dom = max(kern, key=lambda k: kern[k]["share"])
    out = {"metric": METRIC, "value": units / (ms / 1e3),
           "unit": "cell-level updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
           "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": f"R2B{g.k} ({g.n_cells} cells) x {case.n_lev} levels, terrain, "
                                  f"dt={case.dt:g}s, {case.nsub} substeps, FP32-mixed",
                      "cells": g.n_cells, "levels": case.n_lev},
           "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(kern[dom]["alg_GBs"], 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(kern[dom]["alg_GBs"] / HBM_PEAK_GBS, 4), "traffic": None},
           "kernels": {k: {"avg_ms": round(v["avg_ms"], 5), "share": round(v["share"], 4),
                           "alg_GBs": round(v["alg_GBs"], 1)} for k, v in kern.items()}}
    if cfg == 3 and args.error_steps > 0:
        log("per-field error vs FP64 ...")
        out["per_field_error"] = error_table(nhdc, case, CS.CONFIGS[cfg]["steps"])
    return out


def bench_batch(args, torch, nhdc, CS):
    """16 uneven instances (R2B4-R2B6, 30-90 levels), FP32-mixed, one launch
    per kernel over all instances, graph replay, autotuned level tiles; against
    the 16 instances run one after another in the plain FP64 form and in the
    mixed form."""
    stream = torch.cuda.current_stream()
    t0 = time.time()
    cases = CS.batch_cases()
    log(f"16 cases ({time.time() - t0:.1f}s): " + ", ".join(f"R2B{c.grid.k}x{c.n_lev}" for c in cases))
    steps = args.steps if args.steps is not None else 10
    units = sum(c.grid.n_cells * c.n_lev * c.nsub for c in cases) * steps
    res = {}
    if args.counters:  # the batch alone at given tiles: counted bytes / steps_run
        ds = [nhdc.Dycore(c, precision="mixed") for c in cases]
        b = nhdc.Batch(ds)
        b.set_tiles(*args.tiles)
        if args.persistent:
            b.set_persistent(True)
        dts = [c.dt for c in cases]
        ms = timed_steps(torch, lambda: b.step(dts, 5, 1, stream), steps, args.warmup, stream)
        b.close()
        for d in ds:
            d.close()
        calibration_copy(torch)
        return counters_line(args, ms, steps, units, "batch of 16, FP32-mixed, tiles "
                             + ",".join(map(str, args.tiles)))
    for prec in ("fp64", "mixed"):
        total = 0.0
        for c in cases:  # sequential, one instance at a time
            d = nhdc.Dycore(c, precision=prec)
            total += timed_steps(torch, lambda: d.step(c.dt, c.nsub, stream), steps, 1, stream)
            d.close()
        res[f"sequential_{prec}_ms"] = total
    ds = [nhdc.Dycore(c, precision="mixed") for c in cases]
    b = nhdc.Batch(ds)
    dts = [c.dt for c in cases]
    tune_path = os.path.join(ROOT, "gpurun_out", "batch_tiles.json") if os.path.isdir(
        os.path.join(ROOT, "gpurun_out")) else None
    best = b.autotune(dts, 5, cache_path=tune_path)
    log(f"autotuned tiles {best}")
    ms = timed_steps(torch, lambda: b.step(dts, 5, 1, stream), steps, 1, stream)
    for d in ds:
        d.check_finite()
    b.close()
    for d in ds:
        d.close()
    return {"metric": METRIC, "value": units / (ms / 1e3),
            "unit": "cell-level updates/s", "n_gpus": 1, "steps": steps, "warmup": 1,
            "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "batch of 16 instances R2B4-R2B6, 30-90 levels, terrain, "
                                   "FP32-mixed, one launch per kernel + graph replay",
                       "instances": [f"R2B{c.grid.k}x{c.n_lev}" for c in cases],
                       "tiles": {"lt_edge": best[0], "lt_cell": best[1], "lt_vert": best[2]}},
            "speedup_vs_sequential_fp64": res["sequential_fp64_ms"] / ms,
            "speedup_vs_sequential_mixed": res["sequential_mixed_ms"] / ms,
            "sequential_ms": res}


# ---------------------------------------------------------------------------
# rocprofv3 summaries (profiles/): the commands that make the raw CSVs, and the
# reduction of those CSVs to the short text files kept in the repository.

def _prof_cmds(tag, extra):
    """rocprofv3 commands of one profiled workload: a kernel trace, then one
    FETCH_SIZE and one WRITE_SIZE pass over a short run that ends with the
    calibration copy."""
    base = "python3 -u bench.py --error-steps 0 --no-cpu-baseline" + extra
    if "--forms" not in extra:
        base += " --forms none"
    return {
        "trace": f"rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_{tag}trace "
                 f"-o {tag}trace -- {base} --steps 10 --warmup 2 --timing-steps 4 "
                 f"> gpurun_out/prof_{tag}trace.json",
        "fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof_{tag}fetch "
                 f"-o {tag}fetch -- {base} --steps 2 --warmup 1 --timing-steps 1 --copy-calibration "
                 f"> gpurun_out/prof_{tag}fetch.json",
        "write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof_{tag}write "
                 f"-o {tag}write -- {base} --steps 2 --warmup 1 --timing-steps 1 --copy-calibration "
                 f"> gpurun_out/prof_{tag}write.json",
    }


# the profiled workloads: the headline R2B8x90 step (FP64 and mixed); the
# R2B6x90 step with the upwind option next to it; the R2B6x90 damped and
# tracer forms (the kernels only the options run)
PROFILE_SETS = {
    "h": {"tag": "r2b8x90", "cmds": _prof_cmds("h", " --headline 5 --options none --forms vn32")},
    "s": {"tag": "r2b6x90", "cmds": _prof_cmds("s", " --headline 2 --options upwind")},
    "d": {"tag": "r2b6x90", "cmds": _prof_cmds("d", " --headline 2 --options damped,tracers")},
    # the R2B6x90 workload with the level-parallel column (its factors in LDS):
    # the column's bytes without the scratch round trip
    "l": {"tag": "r2b6x90_levels_column",
          "cmds": _prof_cmds("l", " --headline 2 --options none --column-mode 1")},
}
PROFILE_CMDS = {k + kind: c for k, v in PROFILE_SETS.items() for kind, c in v["cmds"].items()}
CONFIG_CMDS = {
    cfg: {"run": f"python3 -u bench.py --config {cfg} --no-cpu-baseline > gpurun_out/bench_c{cfg}.json",
          **{kind: f"rocprofv3 --pmc {ctr} --output-format csv -d gpurun_out/prof_c{cfg}{kind} "
                   f"-o c{cfg}{kind} -- python3 -u bench.py --config {cfg} --steps 3 --warmup 1 "
                   f"--counters --no-cpu-baseline{{tiles}} > gpurun_out/prof_c{cfg}{kind}.json"
             for kind, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE"))}}
    for cfg in (3, 4, 5)}
# kernel traces of the batch of 16 on its two paths (graph of launches,
# persistent launch) over the warm-up and timed steps at fixed tiles: how much
# of a step the GPU spends between launches
BATCH_TRACE_CMDS = {
    path: f"rocprofv3 --kernel-trace --output-format csv -d gpurun_out/prof_b{path} -o b{path} -- "
          f"python3 -u bench.py --config 4 --steps 3 --warmup 1 --counters --no-cpu-baseline"
          f"{' --persistent' if path == 'persistent' else ''} > gpurun_out/prof_b{path}.json"
    for path in ("graph", "persistent")}
# the same workload in a 3-D Hilbert numbering, the bisection's own and a
# random one, against the bisection-curve numbering of the main runs
ORDER_CMDS = {
    o: {"run": f"python3 -u bench.py --headline 2 --options none --order {o} --forms none "
               f"--error-steps 0 --no-cpu-baseline --steps 20 > gpurun_out/bench_o{o}.json",
        **{kind: f"rocprofv3 --pmc {ctr} --output-format csv -d gpurun_out/prof_o{o}{kind} "
                 f"-o o{o}{kind} -- python3 -u bench.py --headline 2 --options none --order {o} "
                 f"--forms none --steps 2 "
                 f"--warmup 1 --timing-steps 1 --error-steps 0 --no-cpu-baseline --copy-calibration "
                 f"> gpurun_out/prof_o{o}{kind}.json"
           for kind, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE"))}}
    for o in ("curve", "sfc", "canonical", "random")}
# instruction issue and texture-addresser activity of the step kernels (FP64
# and mixed R2B6x90 steps): two counter passes over the same short run
ISSUE_CMDS = {
    "issue1": "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SALU "
              "GRBM_GUI_ACTIVE --output-format csv -d gpurun_out/prof_issue1 -o issue1 -- python3 -u "
              "bench.py --headline 2 --options none --forms none --steps 2 --warmup 1 --timing-steps 1 --error-steps 0 "
              "--no-cpu-baseline > gpurun_out/prof_issue1.json",
    "issue2": "rocprofv3 --pmc TA_BUSY_avr SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 "
              "SQ_INSTS_VALU_FMA_F64 GRBM_GUI_ACTIVE --output-format csv -d gpurun_out/prof_issue2 "
              "-o issue2 -- python3 -u bench.py --headline 2 --options none --forms none --steps 2 --warmup 1 --timing-steps 1 "
              "--error-steps 0 --no-cpu-baseline > gpurun_out/prof_issue2.json",
    # L2 read requests to the fabric, and those of less than a full line
    "issue3": "rocprofv3 --pmc TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_BUBBLE_sum --output-format csv "
              "-d gpurun_out/prof_issue3 -o issue3 -- python3 -u bench.py --headline 2 --options none --forms none --steps 2 "
              "--warmup 1 --timing-steps 1 --error-steps 0 --no-cpu-baseline > gpurun_out/prof_issue3.json",
}
CS_TRACERS = ("one", "h2o", "o3", "co2")  # the tracer set the tracer form carries
OPTION_KERNELS = ("div4", "smag_cell", "smag_edge", "column_pred_sponge", "column_corr_sponge",
                  "tr_save", "tr_recon", "tr_horiz", "tr_vert")


def _kernel_id(name):
    """rocprofv3 kernel name -> (kernel id as in kernel_stats, precision); the
    builds of the upwind option get the suffix _upwind."""
    m = re.search(r"k_(vt_edge|vertex|cell_vt|edge_pred|edge_corr|column_stg|column|cell_grad|div4|smag_cell|"
                  r"smag_edge|tr_save|tr_recon|tr_horiz|tr_vert)<(double|float)((?:, (?:true|false))*)"
                  r"(?:, \d+)?>",
                  name)
    if not m:
        return None, None
    k = m.group(1)
    form = "fp64" if m.group(2) == "double" else ("mixed_vn32" if "vn32::" in name else "mixed")
    flags = re.findall(r"true|false", m.group(3))
    upwind = k == "cell_grad"
    if k in ("column", "column_stg"):  # flags: corrector, upwind build, sponge build (either build)
        k = "column_corr" if flags[0] == "true" else "column_pred"
        upwind = flags[1] == "true"
        if flags[2] == "true":
            k += "_sponge"
    elif k in ("edge_pred", "edge_corr"):  # flag: upwind build
        upwind = flags[0] == "true"
    if upwind and k != "cell_grad":
        k += "_upwind"
    return k, form


def _cell_vt_phase(name):
    """k_cell_vt<RT, CORR, LDSM>: the corrector's build when CORR, the second
    template argument, is true (the third selects the LDS-staged build)."""
    m = re.search(r"k_cell_vt<(?:double|float), (true|false), (?:true|false)>", name)
    return "corr" if m and m.group(1) == "true" else "pred"


def _rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _counter(src, kind, name):
    """Per kernel name, the values of counter `name` in dispatch order."""
    from collections import defaultdict
    out = defaultdict(list)
    for r in sorted(_rows(os.path.join(src, f"prof_{kind}", f"{kind}_counter_collection.csv")),
                    key=lambda r: int(r["Dispatch_Id"])):
        if r["Counter_Name"] == name:
            out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return out


def profile_summary(src, dst):
    """Reduce the rocprofv3 CSVs under `src` (made by PROFILE_CMDS and the
    other command tables) to the text summaries under `dst`."""
    done = []
    for key, ps in PROFILE_SETS.items():
        if key != "d" and all(os.path.exists(os.path.join(src, f"prof_{key}{k}.json"))
                              for k in ("trace", "fetch", "write")):
            summarise_set(src, dst, key, ps["tag"])
            done.append(key)
    if all(os.path.exists(os.path.join(src, f"prof_d{k}.json")) for k in ("trace", "fetch", "write")):
        runs = {f"d{k}": json.load(open(os.path.join(src, f"prof_d{k}.json")))
                for k in ("trace", "fetch", "write")}
        cfg = runs["dtrace"]["config"]
        nc, N = cfg["cells"], cfg["levels"]
        wl = f"R2B6x90 ({nc} cells x {N} levels, dt 90 s, 5 substeps)"
        damped_summary(src, dst, runs, runs["dtrace"]["kernel_source_sha256_16"], wl, nc,
                       nc * 3 // 2, nc // 2 + 2, N)
    config_summary(src, dst)
    batch_trace_summary(src, dst)
    order_summary(src, dst)
    if all(os.path.exists(os.path.join(src, f"prof_{k}.json")) for k in ISSUE_CMDS):
        issue_summary(src, dst)
    print(f"wrote summaries of profile sets {done} to {dst}")


def summarise_set(src, dst, key, tag):
    """One profiled workload: per-kernel durations (kernel trace) and HBM
    bytes per launch from FETCH_SIZE / WRITE_SIZE, scaled by what the same
    counters read for the 1 GiB device copy of the calibration."""
    from collections import defaultdict
    cmds = PROFILE_SETS[key]["cmds"]
    runs = {k: json.load(open(os.path.join(src, f"prof_{key}{k}.json"))) for k in cmds}
    hashes = {r["kernel_source_sha256_16"] for r in runs.values()}
    if len(hashes) != 1:
        raise SystemExit(f"profiled runs used different kernel sources: {hashes}")
    src_hash = hashes.pop()
    cfg = runs["trace"]["config"]
    nc, N = cfg["cells"], cfg["levels"]
    ne, nv = nc * 3 // 2, nc // 2 + 2
    wl = (f"{tag.split('_')[0].upper().replace('X', 'x')} ({nc} cells x {N} levels, "
          f"{runs['trace']['config']['workload']})")
    if runs["trace"].get("column_mode", -1) == 1:
        wl += ", level-parallel column"
    numbering = cfg.get("numbering", "curve")
    # ---- kernel trace ----
    stats = _rows(os.path.join(src, f"prof_{key}trace", f"{key}trace_kernel_stats.csv"))
    lines = [f"# rocprofv3 kernel trace: dycore substep kernels, {wl}",
             f"kernel_source_sha256_16: {src_hash}",
             f"numbering: {numbering}",
             f"command: {cmds['trace']}",
             f"summarised by: python3 bench.py --profile-summary gpurun_out",
             "", "## per instantiation (rocprofv3 --stats)",
             f"{'kernel':24s} {'form':10s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'share%':>7s}"]
    agg = defaultdict(lambda: [0.0, 0])
    for r in stats:
        k, prec = _kernel_id(r["Name"])
        if not k:
            continue
        var = f"cell_vt({_cell_vt_phase(r['Name'])})" if k == "cell_vt" else k
        lines.append(f"{var:24s} {prec:10s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['MinNs']) / 1e3:9.2f} {float(r['MaxNs']) / 1e3:9.2f} "
                     f"{float(r['Percentage']):7.2f}")
        agg[(k, prec)][0] += float(r["TotalDurationNs"])
        agg[(k, prec)][1] += int(r["Calls"])
    lines += ["", "## per kernel id, against the HIP-event averages bench.py measured in the same run",
              f"{'kernel':14s} {'form':10s} {'rocprof_avg_us':>15s} {'hip_event_avg_us':>17s} {'diff%':>7s}"]
    ev = {"fp64": dict(runs["trace"]["kernels"]),
          "mixed": runs["trace"]["forms"]["mixed"].get("kernels", {}),
          "mixed_vn32": runs["trace"]["forms"].get("mixed_vn32", {}).get("kernels", {})}
    for k, v in runs["trace"]["forms"].get("fp64_upwind", {}).get("kernels", {}).items():
        if k == "cell_grad" or k in ("edge_pred", "edge_corr", "column_pred", "column_corr"):
            ev["fp64"][k if k == "cell_grad" else k + "_upwind"] = v
    for (k, prec), (tot, n) in sorted(agg.items(), key=lambda kv: (kv[0][1], -kv[1][0])):
        a = tot / n / 1e3
        e = ev.get(prec, {}).get(k, {}).get("avg_ms")
        if e is None:
            lines.append(f"{k:14s} {prec:10s} {a:15.2f} {'-':>17s} {'-':>7s}")
        else:
            lines.append(f"{k:14s} {prec:10s} {a:15.2f} {e * 1e3:17.2f} {100 * (a / (e * 1e3) - 1):7.2f}")
    os.makedirs(dst, exist_ok=True)
    with open(os.path.join(dst, f"dycore_{tag}_kernel_trace.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    # ---- HBM counters ----
    fetch, write = _counter(src, f"{key}fetch", "FETCH_SIZE"), _counter(src, f"{key}write", "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k]
    # the calibration copy: the largest device copy of the profiled run (1 GiB;
    # the state copies of the run are smaller)
    cf, cw = max(fetch[copy[0]]), max(write[copy[0]])
    fs, ws = (1 << 30) / (cf * 1024), (1 << 30) / (cw * 1024)
    for prec in ("fp64", "mixed", "mixed_vn32"):
        alg = algorithmic_bytes(nc, ne, nv, N, prec)
        per = defaultdict(lambda: [[], []])
        for kname, vals in fetch.items():
            k, p = _kernel_id(kname)
            if p != prec:
                continue
            per[k][0] += vals
            per[k][1] += write.get(kname, [])
            if k == "cell_vt":
                var = "cell_vt_" + _cell_vt_phase(kname)
                per[var][0] += vals
                per[var][1] += write.get(kname, [])
        if not per:
            continue
        lines = [f"# rocprofv3 HBM counters: dycore substep kernels, {prec} form, {wl}",
                 f"kernel_source_sha256_16: {src_hash}",
                 f"numbering: {numbering}",
                 f"command (FETCH_SIZE pass): {cmds['fetch']}",
                 f"command (WRITE_SIZE pass): {cmds['write']}",
                 f"summarised by: python3 bench.py --profile-summary gpurun_out",
                 f"calibration: the 1 GiB device-to-device copy (__amd_rocclr_copyBuffer, 1 GiB read + "
                 f"1 GiB written) reads FETCH_SIZE {cf:.1f} KiB and WRITE_SIZE {cw:.1f} KiB per dispatch, "
                 f"so fetch KiB x {fs:.3f} and write KiB x {ws:.3f} give bytes",
                 "units: B/cl = bytes per cell-level (one cell at one full level) per launch", "",
                 f"{'kernel':14s} {'n':>3s} {'fetch_KiB':>12s} {'write_KiB':>12s}  hbm_bytes_per_launch  "
                 f"alg_bytes_per_launch  hbm_B/cl  alg_B/cl  hbm/alg"]
        order = list(alg)
        step_b = 0.0
        for k in sorted(per, key=lambda x: order.index(x) if x in order else order.index("cell_vt")):
            fv, wv = per[k]
            rd = sum(fv) / len(fv)
            wr = sum(wv) / len(wv)
            hbm = rd * 1024 * fs + wr * 1024 * ws
            base = k if k in alg else "cell_vt"
            a = alg[base]
            if k in LAUNCHES_PER_STEP:
                step_b += hbm * LAUNCHES_PER_STEP[k]
            lines.append(f"{k:14s} {len(fv):3d} {rd:12.1f} {wr:12.1f}  hbm_bytes_per_launch={hbm:.4e}  "
                         f"alg_bytes_per_launch={a:.4e}  {hbm / (nc * N):8.1f}  {a / (nc * N):8.1f}  "
                         f"{hbm / a:7.2f}")
        lines += ["", f"substep total (every kernel x its launches per substep): {step_b:.4e} B = "
                      f"{step_b / (nc * N):.1f} B per cell-level-substep"]
        with open(os.path.join(dst, f"dycore_{prec}_{tag}_hbm_counters.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")


def issue_summary(src, dst):
    """profiles/dycore_r2b6x90_issue_counters.txt: per step kernel, the share
    of its cycles in which the texture addresser (the unit every vector memory
    instruction passes) is busy, vector instructions issued per CU-cycle, and
    the FP64 operations, from the two ISSUE_CMDS passes.  A kernel's cycles are
    GRBM_GUI_ACTIVE over the 8 XCDs, whose counts it sums; the chip has 256
    CUs, each issuing at most one wave-wide vector instruction per cycle."""
    import csv
    from collections import defaultdict
    acc = defaultdict(lambda: defaultdict(list))
    meta = {}
    for k in ISSUE_CMDS:
        meta[k] = json.loads(open(os.path.join(src, f"prof_{k}.json")).read().strip().splitlines()[-1])
        f = os.path.join(src, f"prof_{k}", f"{k}_counter_collection.csv")
        for r in csv.DictReader(open(f)):
            kid, prec = _kernel_id(r["Kernel_Name"])
            if kid is None:
                continue
            acc[(kid, prec)][r["Counter_Name"] + "@" + k].append(float(r["Counter_Value"]))
    src_hash = meta["issue1"].get("kernel_source_sha256_16")
    wl = meta["issue1"]["config"]["workload"]
    lines = [f"# rocprofv3 issue counters: dycore substep kernels, {wl}",
             f"kernel_source_sha256_16: {src_hash}",
             f"numbering: {meta['issue1']['config'].get('numbering')}"]
    lines += [f"command ({k}): {ISSUE_CMDS[k]}" for k in ISSUE_CMDS]
    lines += ["summarised by: python3 bench.py --profile-summary gpurun_out",
              "cycles = GRBM_GUI_ACTIVE / 8 (the counter sums the 8 XCDs); TA busy = TA_BUSY_avr / "
              "cycles; VALU/CU-cycle = SQ_INSTS_VALU / (256 x cycles); VMEM/CU-cycle likewise for "
              "SQ_INSTS_VMEM_RD + SQ_INSTS_VMEM_WR; L2_RDREQ = TCC_EA0_RDREQ_sum, of which RDREQ_32B "
              "(32-byte requests) and BUBBLE (TCC_BUBBLE_sum); counts are per dispatch", "",
              f"{'kernel':20s} {'form':5s} {'n':>3s} {'cycles':>9s} {'TA_busy':>8s} {'VALU/CUc':>9s} "
              f"{'VMEM/CUc':>9s} {'VMEM_RD':>10s} {'VMEM_WR':>10s} {'F64_ADD':>10s} {'F64_MUL':>10s} "
              f"{'F64_FMA':>10s} {'L2_RDREQ':>10s} {'RDREQ_32B':>10s} {'BUBBLE':>8s}"]
    def avg(d, name):
        v = d.get(name)
        return sum(v) / len(v) if v else float("nan")
    for (kid, prec) in sorted(acc, key=lambda x: (x[1], x[0])):
        d = acc[(kid, prec)]
        cyc1 = avg(d, "GRBM_GUI_ACTIVE@issue1") / 8.0
        cyc2 = avg(d, "GRBM_GUI_ACTIVE@issue2") / 8.0
        n = len(d.get("GRBM_GUI_ACTIVE@issue1", []))
        ta = avg(d, "TA_BUSY_avr@issue2") / cyc2
        valu = avg(d, "SQ_INSTS_VALU@issue1") / (256.0 * cyc1)
        vmem = (avg(d, "SQ_INSTS_VMEM_RD@issue1") + avg(d, "SQ_INSTS_VMEM_WR@issue1")) / (256.0 * cyc1)
        lines.append(f"{kid:20s} {prec:5s} {n:3d} {cyc1:9.0f} {100 * ta:7.1f}% {100 * valu:8.1f}% "
                     f"{100 * vmem:8.2f}% {avg(d, 'SQ_INSTS_VMEM_RD@issue1'):10.3e} "
                     f"{avg(d, 'SQ_INSTS_VMEM_WR@issue1'):10.3e} {avg(d, 'SQ_INSTS_VALU_ADD_F64@issue2'):10.3e} "
                     f"{avg(d, 'SQ_INSTS_VALU_MUL_F64@issue2'):10.3e} {avg(d, 'SQ_INSTS_VALU_FMA_F64@issue2'):10.3e} "
                     f"{avg(d, 'TCC_EA0_RDREQ_sum@issue3'):10.3e} {avg(d, 'TCC_EA0_RDREQ_32B_sum@issue3'):10.3e} "
                     f"{avg(d, 'TCC_BUBBLE_sum@issue3'):8.0f}")
    with open(os.path.join(dst, "dycore_r2b6x90_issue_counters.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def order_summary(src, dst):
    """profiles/dycore_numbering_r2b6x90.txt: per-kernel time (HIP events)
    and counted HBM bytes of the FP64 step in the space-filling-curve, the
    bisection's and a random numbering."""
    import csv
    from collections import defaultdict

    def bytes_per_launch(tag):
        out = {}
        cal = {}
        acc = {}
        for kind, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
            f = os.path.join(src, f"prof_{tag}{kind}", f"{tag}{kind}_counter_collection.csv")
            vals, copies = defaultdict(list), []
            for r in sorted(csv.DictReader(open(f)), key=lambda r: int(r["Dispatch_Id"])):
                if r["Counter_Name"] != ctr:
                    continue
                if "copyBuffer" in r["Kernel_Name"]:
                    copies.append(float(r["Counter_Value"]))
                    continue
                k, p = _kernel_id(r["Kernel_Name"])
                if k and p == "fp64":
                    vals[k].append(float(r["Counter_Value"]))
            cal[kind] = (1 << 30) / (max(copies) * 1024)
            acc[kind] = {k: sum(v) / len(v) * 1024 * cal[kind] for k, v in vals.items()}
        for k in acc["fetch"]:
            out[k] = acc["fetch"][k] + acc["write"].get(k, 0.0)
        return out

    runs = {}
    for o in ORDER_CMDS:
        runs[o] = (f"o{o}", os.path.join(src, f"bench_o{o}.json"))
    if not all(os.path.exists(p) for _, p in runs.values()) or not all(
            os.path.exists(os.path.join(src, f"prof_o{o}fetch.json")) for o in ORDER_CMDS):
        return
    res, hashes = {}, set()
    for o, (tag, path) in runs.items():
        d = json.loads(open(path).read().strip().splitlines()[-1])
        res[o] = {"ms": d["ms_per_step"], "kern": d["kernels"], "bytes": bytes_per_launch(tag)}
        hashes.add(d.get("kernel_source_sha256_16"))
    if len(hashes) != 1:
        raise SystemExit(f"numbering runs used different kernel sources: {hashes}")
    kernels = [k for k in res["curve"]["kern"] if k in res["random"]["kern"]]
    lines = ["# the FP64 R2B6x90 step in four numberings of cells, edges and vertices: the "
             "continuous curve over the bisection tree (the default), a 3-D Hilbert curve "
             "through the cell centres, the bisection's own order, random",
             f"kernel_source_sha256_16: {hashes.pop()}"]
    for o in ORDER_CMDS:
        lines.append(f"commands ({o}): " + "; ".join(ORDER_CMDS[o][k] for k in ("run", "fetch", "write")))
    lines += ["summarised by: python3 bench.py --profile-summary gpurun_out",
              "per kernel: avg ms per launch (HIP events) / counted HBM bytes per cell-level per launch",
              "", "ms per step: " + ", ".join(f"{o} {r['ms']:.2f}" for o, r in res.items()), "",
              f"{'kernel':12s} " + " ".join(f"{o + ' ms':>14s} {o + ' B/cl':>14s}" for o in res)]
    ncl = 327680 * 90
    for k in kernels:
        row = f"{k:12s} "
        for o, r in res.items():
            b = r["bytes"].get(k)
            row += f"{r['kern'][k]['avg_ms']:14.4f} {(b / ncl if b else float('nan')):14.1f} "
        lines.append(row.rstrip())
    with open(os.path.join(dst, "dycore_numbering_r2b6x90.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("numbering: " + ", ".join(f"{o} {r['ms']:.2f} ms" for o, r in res.items()))


def batch_trace_summary(src, dst):
    """profiles/dycore_config4_batch_paths.txt: per step of the batch of 16,
    the span from the first kernel's start to the last one's end, the sum of
    the kernel durations and the gaps between launches, on the graph path and
    on the persistent path (one launch per step), from the kernel traces."""
    runs = {}
    for path in BATCH_TRACE_CMDS:
        f = os.path.join(src, f"prof_b{path}", f"b{path}_kernel_trace.csv")
        j = os.path.join(src, f"prof_b{path}.json")
        if not (os.path.exists(f) and os.path.exists(j)):
            return
        meta = json.loads(open(j).read().strip().splitlines()[-1])
        rows_ = [r for r in _rows(f) if _kernel_id(r["Kernel_Name"])[0] or "k_persistent" in r["Kernel_Name"]]
        rows_.sort(key=lambda r: int(r["Start_Timestamp"]))
        nsteps = meta["steps_run"]
        per_step = len(rows_) // nsteps
        steps = []
        for i in range(1, nsteps):  # the warm-up step aside
            blk = rows_[i * per_step:(i + 1) * per_step]
            t0 = min(int(r["Start_Timestamp"]) for r in blk)
            t1 = max(int(r["End_Timestamp"]) for r in blk)
            busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in blk)
            steps.append((t1 - t0, busy, len(blk)))
        span = sum(x[0] for x in steps) / len(steps) / 1e6
        busy = sum(x[1] for x in steps) / len(steps) / 1e6
        runs[path] = (span, busy, steps[0][2], meta)
    lines = ["# the batch of 16 (R2B4-R2B6 x 30-90 levels, FP32-mixed) on its two paths: kernel traces",
             f"kernel_source_sha256_16: {runs['graph'][3]['kernel_source_sha256_16']}"]
    lines += [f"command ({p}): {c}" for p, c in BATCH_TRACE_CMDS.items()]
    lines += ["summarised by: python3 bench.py --profile-summary gpurun_out",
              "per step (the timed steps of each trace): span = last kernel end - first kernel start; "
              "busy = sum of kernel durations; gaps = span - busy (one stream: kernels do not overlap)", "",
              f"{'path':12s} {'launches':>9s} {'span_ms':>9s} {'busy_ms':>9s} {'gaps_ms':>8s} {'gaps%':>6s}"]
    for p, (span, busy, n, _) in runs.items():
        lines.append(f"{p:12s} {n:9d} {span:9.3f} {busy:9.3f} {span - busy:8.3f} {100 * (span - busy) / span:6.2f}")
    with open(os.path.join(dst, "dycore_config4_batch_paths.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("batch paths: " + ", ".join(f"{p} span {v[0]:.2f} ms, gaps {v[0] - v[1]:.3f} ms" for p, v in runs.items()))


def config_summary(src, dst):
    """profiles/dycore_config{3,4,5}_hbm.txt: whole-step HBM bytes of each
    workload from its counter passes (every dispatch of a step kernel, summed,
    over the steps that ran), against its unprofiled time per step."""
    import csv
    from collections import defaultdict
    for cfg, cmds in CONFIG_CMDS.items():
        paths = {k: os.path.join(src, f"prof_c{cfg}{k}.json") for k in ("fetch", "write")}
        run = os.path.join(src, f"bench_c{cfg}.json")
        if not all(os.path.exists(p) for p in list(paths.values()) + [run]):
            continue
        meta = {k: json.loads(open(p).read().strip().splitlines()[-1]) for k, p in paths.items()}
        timed = json.loads(open(run).read().strip().splitlines()[-1])
        tot, per, cal = {}, {}, {}
        for kind, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
            f = os.path.join(src, f"prof_c{cfg}{kind}", f"c{cfg}{kind}_counter_collection.csv")
            rows_ = sorted(csv.DictReader(open(f)), key=lambda r: int(r["Dispatch_Id"]))
            acc = defaultdict(float)
            copies = []
            for r in rows_:
                if r["Counter_Name"] != ctr:
                    continue
                if "copyBuffer" in r["Kernel_Name"]:
                    copies.append(float(r["Counter_Value"]))
                    continue
                k, _ = _kernel_id(r["Kernel_Name"])
                if k:
                    acc[k] += float(r["Counter_Value"])
            cal[kind] = (1 << 30) / (max(copies) * 1024)
            per[kind] = {k: v * 1024 * cal[kind] / meta[kind]["steps_run"] for k, v in acc.items()}
            tot[kind] = sum(per[kind].values())
        step_bytes = tot["fetch"] + tot["write"]
        ms = timed["ms_per_step"]
        gbs = step_bytes / (ms / 1e3) / 1e9
        lines = [f"# rocprofv3 HBM counters, whole step: {timed['config']['workload']}",
                 f"kernel_source_sha256_16: {meta['fetch']['kernel_source_sha256_16']}",
                 f"command (time per step, unprofiled): {cmds['run']}",
                 f"command (FETCH_SIZE pass): {cmds['fetch'].format(tiles=meta['fetch']['tiles_arg'])}",
                 f"command (WRITE_SIZE pass): {cmds['write'].format(tiles=meta['write']['tiles_arg'])}",
                 f"summarised by: python3 bench.py --profile-summary gpurun_out",
                 f"calibration: FETCH_SIZE x {cal['fetch']:.3f}, WRITE_SIZE x {cal['write']:.3f} "
                 "(the 1 GiB device copy at the end of each pass)",
                 f"counter passes: {meta['fetch']['steps_run']} steps each (warm-up + timed)", "",
                 f"HBM bytes per step: {step_bytes:.4e}",
                 f"time per step (unprofiled): {ms:.3f} ms",
                 f"HBM rate: {gbs:.1f} GB/s = {100 * gbs / HBM_PEAK_GBS:.1f} % of {HBM_PEAK_GBS:.0f} GB/s",
                 "", f"{'kernel':20s} {'bytes_per_step':>15s} {'share':>7s}"]
        allk = set(per["fetch"]) | set(per["write"])
        for k in sorted(allk, key=lambda x: -(per["fetch"].get(x, 0) + per["write"].get(x, 0))):
            b = per["fetch"].get(k, 0) + per["write"].get(k, 0)
            lines.append(f"{k:20s} {b:15.4e} {b / step_bytes:7.3f}")
        with open(os.path.join(dst, f"dycore_config{cfg}_hbm.txt"), "w") as fo:
            fo.write("\n".join(lines) + "\n")
        print(f"config {cfg}: {gbs:.1f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f} % of peak)")


def damped_summary(src, dst, runs, src_hash, wl, nc, ne, nv, N):
    """Durations and HBM bytes of the kernels only the options run (fourth-
    order damping, the diffusion's two passes, the sponge's column builds,
    the four tracer kernels with four tracers), from runs that time the
    damped and tracer forms next to the plain ones."""
    from collections import defaultdict
    alg = algorithmic_bytes(nc, ne, nv, N, "fp64")
    stats = _rows(os.path.join(src, "prof_dtrace", "dtrace_kernel_stats.csv"))
    dur = {}
    for r in stats:
        k, prec = _kernel_id(r["Name"])
        if prec == "fp64" and k in OPTION_KERNELS:
            dur[k] = (float(r["AverageNs"]) / 1e3, int(r["Calls"]))
    fetch, write = _counter(src, "dfetch", "FETCH_SIZE"), _counter(src, "dwrite", "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k]
    cf, cw = max(fetch[copy[0]]), max(write[copy[0]])
    fs, ws = (1 << 30) / (cf * 1024), (1 << 30) / (cw * 1024)
    per = defaultdict(lambda: [[], []])
    for kname, vals in fetch.items():
        k, p = _kernel_id(kname)
        if p == "fp64" and k in OPTION_KERNELS:
            per[k][0] += vals
            per[k][1] += write.get(kname, [])
    ev = runs["dtrace"]["forms"].get("fp64_damped", {}).get("kernels", {})
    evid = {"div4": "div4", "smag_cell": "smag_cell", "smag_edge": "smag_edge",
            "column_pred_sponge": "column_pred", "column_corr_sponge": "column_corr"}
    evt = runs["dtrace"]["forms"].get("fp64_tracers", {}).get("kernels", {})
    opts = runs["dtrace"]["forms"].get("fp64_damped", {}).get("options", {})
    lines = [f"# rocprofv3: kernels of the damping, diffusion and tracer options, fp64 form, {wl}",
             f"options: {json.dumps(opts, sort_keys=True)}",
             f"kernel_source_sha256_16: {src_hash}",
             f"command (trace): {PROFILE_CMDS['dtrace']}",
             f"command (FETCH_SIZE pass): {PROFILE_CMDS['dfetch']}",
             f"command (WRITE_SIZE pass): {PROFILE_CMDS['dwrite']}",
             f"summarised by: python3 bench.py --profile-summary gpurun_out",
             f"calibration: FETCH_SIZE x {fs:.3f}, WRITE_SIZE x {ws:.3f} (the 1 GiB device copy of the same run)",
             "units: B/cl = bytes per cell-level per launch", "",
             f"{'kernel':20s} {'calls':>5s} {'rocprof_us':>10s} {'hip_event_us':>12s} {'hbm_B/cl':>9s} "
             f"{'alg_B/cl':>9s} {'hbm/alg':>7s} {'alg_GB/s':>9s}"]
    for k in OPTION_KERNELS:
        if k not in dur or k not in per:
            continue
        us, calls = dur[k]
        fv, wv = per[k]
        hbm = sum(fv) / len(fv) * 1024 * fs + sum(wv) / len(wv) * 1024 * ws
        a = alg[k]
        e = (evt.get(k, {}) if k.startswith("tr_") else ev.get(evid[k], {})).get("avg_ms")
        lines.append(f"{k:20s} {calls:5d} {us:10.2f} {('%.2f' % (e * 1e3)) if e else '-':>12s} "
                     f"{hbm / (nc * N):9.1f} {a / (nc * N):9.1f} {hbm / a:7.2f} {a / (us * 1e3):9.1f}")
    lines.append("tracers: " + ", ".join(CS_TRACERS) + " (four, FP64)")
    with open(os.path.join(dst, "dycore_options_r2b6x90_kernels.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 48 of the headline's 50-step run; with --config, "
                         "the workload's own count less the warm-up)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--headline", type=int, default=5, choices=[2, 5],
                    help="workload of the value: 5 = R2B8x90 (default), 2 = R2B6x90")
    ap.add_argument("--config", type=int, default=None, choices=[3, 4, 5],
                    help="one other workload alone (for its counter passes): 3 = R2B7x90 mixed, "
                         "4 = the batch of 16, 5 = R2B8x90 mixed")
    ap.add_argument("--timing-steps", type=int, default=4)
    ap.add_argument("--error-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--order", default="curve", choices=["curve", "sfc", "canonical", "random"],
                    help="numbering of cells, edges and vertices of the default workload: the "
                         "continuous curve over the bisection tree (default), a 3-D Hilbert "
                         "curve through the cell centres, the bisection's own order, or random")
    ap.add_argument("--counters", action="store_true",
                    help="configs 3-5: run only the warm-up and timed steps (no kernel table, "
                         "error table, sequential runs or autotuning), for a hardware-counter pass")
    ap.add_argument("--column-mode", type=int, default=-1, choices=(-1, 0, 1),
                    help="the headline forms' column build: 0 one lane per column, 1 level-parallel "
                         "(-1: the library's starting shapes; profile set l)")
    ap.add_argument("--persistent", action="store_true",
                    help="config 4 with --counters: the persistent path")
    ap.add_argument("--tiles", type=lambda x: [int(v) for v in x.split(",")], default=[0, 0, 0],
                    help="config 4 with --counters: level tiles lt_edge,lt_cell,lt_vert")
    ap.add_argument("--forms", default="vn32,config1,r2b6,small,config3,config4",
                    help="other forms and workloads carried in the line: vn32 (the mixed form with vn "
                         "stored in FP32, same workload), config1 (R2B4x20 FP64), "
                         "r2b6 (R2B6x90 in both forms "
                         "with the options), small (R2B3x90 to R2B5x90 FP64: shares near the paper's "
                         "strong-scaling floor, the column builds and shapes), "
                         "config3 (R2B7x90 mixed with its error after 100 steps), "
                         "config4 (the batch of 16 against sequential runs); 'none' for none")
    ap.add_argument("--options", default="upwind,damped,tracers",
                    help="options timed on the R2B6x90 FP64 step: upwind, damped, tracers; 'none'")
    ap.add_argument("--profile-summary", metavar="DIR",
                    help="reduce the rocprofv3 CSVs under DIR to the summaries in profiles/ and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, copy 1 GiB device-to-device once (a plain copy kernel of "
                         "known size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(args.profile_summary, os.path.join(ROOT, "profiles"))
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs one GPU per process and this benchmark one GPU "
              f"(got --gpus {args.gpus}); the decomposition over several GPUs is designed "
              "but not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2511_02021_amd import nhdc
    from paper_2511_02021_amd.inputs import case as CS
    torch.cuda.set_device(0)
    if args.forms == "none":
        args.forms = ""
    if args.options == "none":
        args.options = ""
    if args.config is None:
        if args.steps is None:
            args.steps = 48
        out = bench_headline(args, torch, nhdc, CS)
    elif args.config == 4:
        out = bench_batch(args, torch, nhdc, CS)
    else:
        out = bench_single(args, torch, nhdc, CS, args.config)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Python binding of libnhdc (include/nhdc.h): argument marshalling only.

Every step of the dynamical core runs in the library's HIP kernels; PyTorch
is used for device memory (tensors handed over by pointer) and for the HIP
stream on which work is enqueued.  There is no CPU fallback: if libnhdc.so is
missing or fails to load, the import of the library raises.
"""
import ctypes as C
import os

import numpy as np

from . import _build

NHDC_FP64, NHDC_MIXED, NHDC_MIXED_VN32 = 0, 1, 2
MAX_INST = 64  # NHDC_MAX_INST: instances of one batch
PRECISIONS = {"fp64": NHDC_FP64, "mixed": NHDC_MIXED, "mixed_vn32": NHDC_MIXED_VN32}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EGRID", -5: "ESTATE", -6: "EUNSTABLE",
          -7: "ETOOBIG"}
NOALLOC_MAX_CELLS = 65536 * 256  # NHDC_NOALLOC_MAX_CELLS
COLUMN_STREAM, COLUMN_LEVELS = 0, 1  # NHDC_COLUMN_STREAM, NHDC_COLUMN_LEVELS

EXPORTS = ("nhdc_create", "nhdc_upload_grid", "nhdc_init_state", "nhdc_step", "nhdc_get_state",
           "nhdc_get_mass_flux", "nhdc_diag", "nhdc_check_finite", "nhdc_sizes",
           "nhdc_set_tiles", "nhdc_autotune", "nhdc_set_timing", "nhdc_kernel_count",
           "nhdc_kernel_stats", "nhdc_last_error", "nhdc_destroy", "nhdc_batch_create",
           "nhdc_batch_step", "nhdc_batch_set_tiles", "nhdc_batch_autotune",
           "nhdc_batch_last_error", "nhdc_batch_destroy", "nhdc_set_tracers", "nhdc_get_tracers",
           "nhdc_n_tracers", "nhdc_diag_noalloc", "nhdc_set_allocator", "nhdc_set_block_sizes",
           "nhdc_batch_set_block_sizes", "nhdc_batch_set_persistent", "nhdc_batch_persistent_grid",
           "nhdc_set_column_mode", "nhdc_batch_set_column_mode", "nhdc_get_shapes",
           "nhdc_batch_get_shapes")


class NhdcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Grid(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_edges", C.c_int64), ("n_verts", C.c_int64),
                ("radius", C.c_double)] + [(n, C.c_void_p) for n in (
                    "cell_edges", "cell_sign", "edge_cells", "edge_verts", "vert_edges",
                    "vert_cells", "vert_sign", "vert_valence", "cell_x", "cell_area", "edge_x",
                    "edge_tangent", "edge_length", "dual_length", "vert_area", "edge_normal",
                    "dual_frac")]


class _Vertical(C.Structure):
    _fields_ = [("n_lev", C.c_int32), ("zh", C.c_void_p), ("pi_ref", C.c_void_p),
                ("theta_ref", C.c_void_p), ("w_damp", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("omega", "grav", "rd", "cpd", "p00", "beta", "wgt_corr",
                                          "extrap", "div_damp")] + [("upwind", C.c_int32)] + [
        ("div_damp4", C.c_double), ("smag", C.c_double)]


class _State(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("vn", "w", "rho", "pi", "theta_v", "pi_prev")] + [
        ("on_device", C.c_int32)]


_LIB = None

# nhdc_set_allocator callbacks: alloc(bytes, user) -> device pointer; free_(ptr, user)
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class TorchAllocator:
    """Device memory of a context from PyTorch's caching allocator
    (nhdc_set_allocator): the library then allocates nothing of its own, and
    torch.cuda.memory_allocated() counts the context's arrays."""

    def __init__(self, device):
        import torch
        self.device = int(device)
        self.live = 0

        def alloc(nbytes, user):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device)
            except Exception:  # out of memory: the library reports ENOMEM
                return None
            self.live += 1
            return p

        def free(ptr, user):
            try:
                torch.cuda.caching_allocator_delete(ptr)
                self.live -= 1
            except Exception:  # interpreter shutdown
                pass

        self.alloc = _ALLOC_FN(alloc)  # kept alive with the context
        self.free = _FREE_FN(free)


def library_path():
    return _build.NHDC_SO


def lib():
    """Load libnhdc.so (building it in-tree if nothing is built yet).

    torch is imported first: its HIP runtime (soname libamdhip64.so.7) is then
    already in the process and libnhdc binds to that same runtime, so streams
    and device pointers from torch are valid in the library.  Loading libnhdc
    first would bring in a second copy of the runtime."""
    global _LIB
    if _LIB is None:
        import torch  # noqa: F401  (HIP runtime first, see above)
        path = _build.ensure(_build.NHDC_SO, _build.build_nhdc)
        L = C.CDLL(path)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        L.nhdc_create.argtypes = [C.POINTER(vp), i, i]
        L.nhdc_upload_grid.argtypes = [vp, vp, vp, vp]
        L.nhdc_init_state.argtypes = [vp, vp, vp]
        L.nhdc_step.argtypes = [vp, d, i, vp]
        L.nhdc_get_state.argtypes = [vp, vp, vp]
        L.nhdc_get_mass_flux.argtypes = [vp, vp, vp, i, vp]
        L.nhdc_set_tracers.argtypes = [vp, i, vp, i, vp]
        L.nhdc_get_tracers.argtypes = [vp, vp, i, vp]
        L.nhdc_n_tracers.argtypes = [vp]
        L.nhdc_diag.argtypes = [vp, vp, vp, vp]
        L.nhdc_check_finite.argtypes = [vp, vp]
        L.nhdc_sizes.argtypes = [vp] + [vp] * 4
        L.nhdc_set_tiles.argtypes = [vp, i, i, i]
        L.nhdc_set_block_sizes.argtypes = [vp, i, i, i]
        L.nhdc_batch_set_block_sizes.argtypes = [vp, i, i, i]
        L.nhdc_set_column_mode.argtypes = [vp, i]
        L.nhdc_get_shapes.argtypes = [vp, vp]
        L.nhdc_batch_get_shapes.argtypes = [vp, vp]
        L.nhdc_batch_set_column_mode.argtypes = [vp, i]
        L.nhdc_batch_set_persistent.argtypes = [vp, i, i]
        L.nhdc_batch_persistent_grid.argtypes = [vp]
        L.nhdc_autotune.argtypes = [vp, d, i, C.c_char_p, C.POINTER(d), vp]
        L.nhdc_batch_create.argtypes = [C.POINTER(vp), C.POINTER(vp), i]
        L.nhdc_batch_step.argtypes = [vp, C.POINTER(d), i, i, vp]
        L.nhdc_batch_set_tiles.argtypes = [vp, i, i, i]
        L.nhdc_batch_autotune.argtypes = [vp, C.POINTER(d), i, C.c_char_p, C.POINTER(d), vp]
        L.nhdc_batch_last_error.argtypes = [vp]
        L.nhdc_batch_last_error.restype = C.c_char_p
        L.nhdc_batch_destroy.argtypes = [vp]
        L.nhdc_batch_destroy.restype = None
        L.nhdc_set_timing.argtypes = [vp, i]
        L.nhdc_kernel_count.argtypes = []
        L.nhdc_kernel_stats.argtypes = [vp, i, C.POINTER(C.c_char_p), C.POINTER(d),
                                        C.POINTER(C.c_int64)]
        L.nhdc_diag_noalloc.argtypes = [C.c_int64, C.c_int32] + [vp] * 6
        L.nhdc_set_allocator.argtypes = [vp, _ALLOC_FN, _FREE_FN, vp]
        L.nhdc_last_error.argtypes = [vp]
        L.nhdc_last_error.restype = C.c_char_p
        L.nhdc_destroy.argtypes = [vp]
        L.nhdc_destroy.restype = None
        _LIB = L
    return _LIB


def _np_ptr(a):
    assert isinstance(a, np.ndarray) and a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def _best_tuple(best):
    """The autotuner's 8 reported values: shapes as ints, the time as a float."""
    return tuple(int(x) for x in best[:6]) + (best[6], int(best[7]))


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def params_struct(p):
    return _Params(p.omega, p.grav, p.rd, p.cpd, p.p00, p.beta, p.wgt_corr, p.extrap, p.div_damp,
                   int(p.upwind), p.div_damp4, p.smag)


class Dycore:
    """One dynamical-core instance resident on a GPU."""

    def __init__(self, case, precision="fp64", device=0, init=True, allocator=None):
        """allocator: None (the library's hipMalloc), "torch" (PyTorch's
        caching allocator) or an object whose `alloc` and `free` are
        nhdc_set_allocator callbacks (ctypes functions it keeps alive)."""
        self.L = lib()
        self.case = case
        self.grid = case.grid
        self.N = case.n_lev
        self.device = device
        self.precision = precision
        h = C.c_void_p()
        rc = self.L.nhdc_create(C.byref(h), PRECISIONS[precision], int(device))
        if rc != 0:
            raise NhdcError(rc, "nhdc_create failed (no usable HIP device?)")
        self.h = h
        self.allocator = None
        if allocator == "torch":
            self.allocator = TorchAllocator(device)
        elif allocator is not None and hasattr(allocator, "alloc") and hasattr(allocator, "free"):
            self.allocator = allocator  # an object with nhdc_set_allocator callbacks
        elif allocator is not None:
            raise ValueError(f"unknown allocator {allocator!r}")
        if self.allocator is not None:
            self._check(self.L.nhdc_set_allocator(self.h, self.allocator.alloc,
                                                  self.allocator.free, None))
        g = case.grid
        keep = {}

        def arr(name, dtype):
            keep[name] = np.ascontiguousarray(getattr(g, name), dtype=dtype)
            return _np_ptr(keep[name])

        gs = _Grid(g.n_cells, g.n_edges, g.n_verts, g.radius,
                   arr("cell_edges", np.int32), arr("cell_sign", np.int8),
                   arr("edge_cells", np.int32), arr("edge_verts", np.int32),
                   arr("vert_edges", np.int32), arr("vert_cells", np.int32),
                   arr("vert_sign", np.int8), arr("vert_valence", np.int32),
                   arr("cell_x", np.float64), arr("cell_area", np.float64),
                   arr("edge_x", np.float64), arr("edge_tangent", np.float64),
                   arr("edge_length", np.float64), arr("dual_length", np.float64),
                   arr("vert_area", np.float64), arr("edge_normal", np.float64),
                   arr("dual_frac", np.float64))
        zh = np.ascontiguousarray(case.zh, dtype=np.float64)
        pr = np.ascontiguousarray(case.pi_ref, dtype=np.float64)
        tr = np.ascontiguousarray(case.theta_ref, dtype=np.float64)
        wd = None if case.w_damp is None else np.ascontiguousarray(case.w_damp, dtype=np.float64)
        vs = _Vertical(self.N, _np_ptr(zh), _np_ptr(pr), _np_ptr(tr),
                       None if wd is None else _np_ptr(wd))
        ps = params_struct(case.params)
        self._check(self.L.nhdc_upload_grid(self.h, C.byref(gs), C.byref(vs), C.byref(ps)))
        if init:
            self.init_state(case.vn, case.w, case.rho, case.pi, case.theta_v)
        if getattr(case, "tracers", None) is not None:
            self.set_tracers(case.tracers)

    # -- helpers ------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise NhdcError(rc, self.L.nhdc_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.L.nhdc_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @property
    def shapes(self):
        nc, ne, N = self.grid.n_cells, self.grid.n_edges, self.N
        return dict(vn=(N, ne), w=(N + 1, nc), rho=(N, nc), pi=(N, nc), theta_v=(N, nc),
                    pi_prev=(N, nc))

    # -- state ----------------------------------------------------------------
    def init_state(self, vn, w, rho, pi, theta_v, pi_prev=None, stream=None):
        """Host numpy arrays or device torch tensors (float64, contiguous)."""
        fields = [vn, w, rho, pi, theta_v, pi_prev]
        names = ["vn", "w", "rho", "pi", "theta_v", "pi_prev"]
        on_dev = not isinstance(vn, np.ndarray)
        keep, ptrs = [], []
        for n, f in zip(names, fields):
            if f is None:
                ptrs.append(None)
                continue
            if on_dev:
                assert f.is_cuda and f.dtype.is_floating_point and f.element_size() == 8
                f = f.contiguous()
                assert tuple(f.shape) == self.shapes[n], (n, tuple(f.shape))
                keep.append(f)
                ptrs.append(C.c_void_p(f.data_ptr()))
            else:
                a = np.ascontiguousarray(f, dtype=np.float64)
                assert a.shape == self.shapes[n], (n, a.shape)
                keep.append(a)
                ptrs.append(_np_ptr(a))
        st = _State(*ptrs, int(on_dev))
        self._check(self.L.nhdc_init_state(self.h, C.byref(st),
                                           _stream_ptr(stream) if on_dev else None))
        self._keep = keep

    def step(self, dt, nsub, stream=None):
        self._check(self.L.nhdc_step(self.h, float(dt), int(nsub), _stream_ptr(stream)))

    def get_state(self):
        """Host copy of the prognostic state (numpy, float64)."""
        out = {n: np.empty(s) for n, s in self.shapes.items()}
        st = _State(*[_np_ptr(out[n]) for n in ("vn", "w", "rho", "pi", "theta_v", "pi_prev")], 0)
        self._check(self.L.nhdc_get_state(self.h, C.byref(st), _stream_ptr(None)))
        return out

    def get_state_device(self, stream=None):
        import torch
        dev = torch.device("cuda", self.device)
        out = {n: torch.empty(s, dtype=torch.float64, device=dev) for n, s in self.shapes.items()}
        st = _State(*[C.c_void_p(out[n].data_ptr()) for n in
                      ("vn", "w", "rho", "pi", "theta_v", "pi_prev")], 1)
        self._check(self.L.nhdc_get_state(self.h, C.byref(st), _stream_ptr(stream)))
        return out

    def mass_flux(self):
        N, nc, ne = self.N, self.grid.n_cells, self.grid.n_edges
        facc, wacc = np.empty((N, ne)), np.empty((N + 1, nc))
        self._check(self.L.nhdc_get_mass_flux(self.h, _np_ptr(facc), _np_ptr(wacc), 0,
                                              _stream_ptr(None)))
        return facc, wacc

    def set_tracers(self, q):
        """Tracer mixing ratios [n, N, n_cells] (numpy, FP64); n = 0 removes them."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        n = q.shape[0] if q.size else 0
        if n:
            assert q.shape[1:] == (self.N, self.grid.n_cells)
        self._check(self.L.nhdc_set_tracers(self.h, int(n), _np_ptr(q) if n else None, 0,
                                            _stream_ptr(None)))

    def get_tracers(self):
        n = self.L.nhdc_n_tracers(self.h)
        out = np.empty((n, self.N, self.grid.n_cells))
        if n:
            self._check(self.L.nhdc_get_tracers(self.h, _np_ptr(out), 0, _stream_ptr(None)))
        return out

    def diag(self):
        m, r = C.c_double(), C.c_double()
        self._check(self.L.nhdc_diag(self.h, C.byref(m), C.byref(r), _stream_ptr(None)))
        return m.value, r.value

    def check_finite(self):
        self._check(self.L.nhdc_check_finite(self.h, _stream_ptr(None)))

    def set_tiles(self, lt_edge=0, lt_cell=0, lt_vert=0):
        """Levels per lane of the marching kernels (0 = whole column)."""
        self._check(self.L.nhdc_set_tiles(self.h, int(lt_edge), int(lt_cell), int(lt_vert)))

    def set_block_sizes(self, column=256, vertex=64, column_waves=3):
        """Lanes per block of the column and vertex kernels (64, 128, 256) and
        the column kernel's waves per SIMD (2, 3; 0 = uncapped); the
        defaults are the library's."""
        self._check(self.L.nhdc_set_block_sizes(self.h, int(column), int(vertex), int(column_waves)))

    def set_column_mode(self, mode):
        """Column solver build: COLUMN_STREAM (one lane per column, the
        starting build above 40960 cells) or COLUMN_LEVELS (levels shared
        among lanes, the factors in LDS; the starting build up to 40960
        cells); the same results to the bit."""
        self._check(self.L.nhdc_set_column_mode(self.h, int(mode)))

    @property
    def shapes_in_use(self):
        """(lt_edge, lt_cell, lt_vert, block_column, block_vertex,
        column_waves, column_mode) of the launches now."""
        out = (C.c_int * 7)()
        self._check(self.L.nhdc_get_shapes(self.h, out))
        return tuple(out)

    def autotune(self, dt, nsub, cache_path=None, stream=None):
        """Search the column mode, level tiles and block sizes by timing whole
        steps; the state is restored.  Returns (lt_edge, lt_cell, lt_vert,
        block_column, block_vertex, column_waves, ms_per_step, column_mode)."""
        best = (C.c_double * 8)()
        path = cache_path.encode() if cache_path else None
        self._check(self.L.nhdc_autotune(self.h, float(dt), int(nsub), path, best,
                                         _stream_ptr(stream)))
        return _best_tuple(best)

    def set_timing(self, on):
        self._check(self.L.nhdc_set_timing(self.h, int(bool(on))))

    def kernel_stats(self):
        """{kernel name: (total ms, launches)} accumulated while timing is on."""
        out = {}
        for k in range(self.L.nhdc_kernel_count()):
            name, ms, n = C.c_char_p(), C.c_double(), C.c_int64()
            self._check(self.L.nhdc_kernel_stats(self.h, k, C.byref(name), C.byref(ms), C.byref(n)))
            out[name.value.decode()] = (ms.value, n.value)
        return out


def diag_noalloc(cell_area, zh, rho, theta_v, out, stream=None):
    """nhdc_diag_noalloc: the global sums (mass, rho*theta_v) of caller-held
    device tensors (float64, contiguous; zh [N+1][nc], rho and theta_v
    [N][nc]) into the device tensor out[2], enqueued on the stream; the
    library allocates nothing."""
    L = lib()
    nc = int(cell_area.numel())
    n_lev = int(rho.shape[0]) if rho.dim() == 2 else 0
    for t in (cell_area, zh, rho, theta_v, out):
        assert t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous()
    assert tuple(zh.shape) == (n_lev + 1, nc) and tuple(theta_v.shape) == tuple(rho.shape)
    assert tuple(rho.shape) == (n_lev, nc) and out.numel() >= 2
    rc = L.nhdc_diag_noalloc(nc, n_lev, *[C.c_void_p(t.data_ptr()) for t in
                                          (cell_area, zh, rho, theta_v, out)], _stream_ptr(stream))
    if rc != 0:
        raise NhdcError(rc, L.nhdc_last_error(None).decode())


class Batch:
    """Several Dycore instances (same device and precision, any sizes) advanced
    together: one launch per kernel over all of them, each step replayed from a
    captured HIP graph.  The batch keeps its members alive; closing a member
    while the batch lives defers the release of its device memory to the
    batch's close."""

    def __init__(self, dycores):
        self.L = lib()
        self.members = list(dycores)
        arr = (C.c_void_p * len(self.members))(*[d.h for d in self.members])
        h = C.c_void_p()
        rc = self.L.nhdc_batch_create(C.byref(h), arr, len(self.members))
        if rc != 0:
            raise NhdcError(rc, "nhdc_batch_create failed (instances must share device and "
                                "precision, have grid and state, and number 1..64)")
        self.h = h

    def _check(self, rc):
        if rc != 0:
            raise NhdcError(rc, self.L.nhdc_batch_last_error(self.h).decode())

    def _dts(self, dt):
        dts = [float(x) for x in (dt if hasattr(dt, "__len__") else [dt] * len(self.members))]
        assert len(dts) == len(self.members)
        return (C.c_double * len(dts))(*dts)

    def step(self, dt, nsub, nsteps=1, stream=None):
        self._check(self.L.nhdc_batch_step(self.h, self._dts(dt), int(nsub), int(nsteps),
                                           _stream_ptr(stream)))

    def set_tiles(self, lt_edge=0, lt_cell=0, lt_vert=0):
        self._check(self.L.nhdc_batch_set_tiles(self.h, int(lt_edge), int(lt_cell), int(lt_vert)))

    def set_block_sizes(self, column=256, vertex=64, column_waves=3):
        self._check(self.L.nhdc_batch_set_block_sizes(self.h, int(column), int(vertex),
                                                      int(column_waves)))

    def set_column_mode(self, mode):
        self._check(self.L.nhdc_batch_set_column_mode(self.h, int(mode)))

    @property
    def shapes_in_use(self):
        out = (C.c_int * 7)()
        self._check(self.L.nhdc_batch_get_shapes(self.h, out))
        return tuple(out)

    def set_persistent(self, on=True, blocks_per_cu=0):
        """Run each step's substeps as one persistent cooperative launch."""
        self._check(self.L.nhdc_batch_set_persistent(self.h, int(bool(on)), int(blocks_per_cu)))

    @property
    def persistent_grid(self):
        return self.L.nhdc_batch_persistent_grid(self.h)

    def autotune(self, dt, nsub, cache_path=None, stream=None):
        """As Dycore.autotune, over the batch on its current path."""
        best = (C.c_double * 8)()
        path = cache_path.encode() if cache_path else None
        self._check(self.L.nhdc_batch_autotune(self.h, self._dts(dt), int(nsub), path, best,
                                               _stream_ptr(stream)))
        return _best_tuple(best)

    def close(self):
        if getattr(self, "h", None):
            self.L.nhdc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def exported_symbols(path=None):
    """Names of the nhdc_* symbols the shared library exports (no GPU needed)."""
    import subprocess
    path = path or _build.NHDC_SO
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True,
                         check=True).stdout
    return sorted({ln.split()[-1] for ln in out.splitlines() if " T nhdc_" in ln})


def header_symbols():
    """Function names declared in include/nhdc.h."""
    import re
    src = open(os.path.join(_build.INCLUDE, "nhdc.h")).read()
    return sorted(set(re.findall(r"\b(nhdc_[a-z_]+)\s*\(", src)))

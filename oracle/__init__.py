"""Plain FP64 CPU oracle of the dynamical-core substep (ctypes binding of
liboracle.so).  TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke
check and the CPU-baseline leg of the benchmark, never by the product."""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None
_GRID_PTRS = ("cell_edges", "cell_verts", "cell_cells", "cell_sign", "edge_cells", "edge_verts",
              "vert_edges", "vert_cells", "vert_sign", "vert_valence", "cell_x", "cell_area",
              "edge_x", "edge_normal", "edge_tangent", "edge_length", "dual_length", "dual_frac",
              "vert_x", "vert_area")


class OrGrid(C.Structure):
    _fields_ = [("nc", C.c_int64), ("ne", C.c_int64), ("nv", C.c_int64), ("radius", C.c_double)] + [
        (n, C.c_void_p) for n in _GRID_PTRS]


class OrParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("radius", "omega", "grav", "rd", "cpd", "p00", "beta",
                                          "wgt_corr", "extrap", "div_damp")] + [("upwind", C.c_int)] + [
        ("div_damp4", C.c_double), ("smag", C.c_double), ("w_damp", C.c_void_p)]


def lib():
    global _LIB
    if _LIB is None:
        # ORACLE_SO: another build of the oracle (the tests of the pins
        # themselves load builds with planted mistakes this way)
        path = os.environ.get("ORACLE_SO", _build.SO)
        if path == _build.SO and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        vp, d, i = C.c_void_p, C.c_double, C.c_int
        L.or_create.restype = vp
        L.or_create.argtypes = [vp, i, vp, vp, vp, vp]
        L.or_free.argtypes = [vp]
        L.or_free.restype = None
        L.or_set_state.argtypes = [vp] * 7
        L.or_get_state.argtypes = [vp] * 7
        L.or_get_flux.argtypes = [vp] * 3
        L.or_step.argtypes = [vp, d, i]
        L.or_vt.argtypes = [vp] * 7
        L.or_pgrad.argtypes = [vp] * 3
        L.or_diag.argtypes = [vp] * 3
        for f in ("or_op_div", "or_op_grad", "or_op_tgrad", "or_op_curl", "or_op_cell_avg",
                  "or_op_vert_avg"):
            getattr(L, f).argtypes = [vp, vp, vp]
            getattr(L, f).restype = None
        L.or_op_cell_grad.argtypes = [vp, vp, vp, vp]
        L.or_op_cell_grad.restype = None
        L.or_op_upwind.argtypes = [vp] * 5 + [d, vp]
        L.or_op_upwind.restype = None
        for f in ("or_op_vector_laplacian", "or_op_graddiv2"):
            getattr(L, f).argtypes = [vp, vp, vp]
            getattr(L, f).restype = None
        L.or_op_deformation.argtypes = [vp] * 4
        L.or_op_deformation.restype = None
        L.or_op_tracer_grad.argtypes = [vp] * 3
        L.or_op_tracer_grad.restype = None
        L.or_op_tracer_recon.argtypes = [vp] * 4
        L.or_op_tracer_recon.restype = None
        L.or_ppm_faces.argtypes = [i, vp, vp, vp]
        L.or_ppm_column.argtypes = [i, d] + [vp] * 6
        L.or_tracers_set.argtypes = [vp, i, vp]
        L.or_tracers_get.argtypes = [vp, vp]
        L.or_op_perot.argtypes = [vp] * 7
        L.or_op_perot.restype = None
        L.or_thomas.argtypes = [i] + [vp] * 5
        L.or_column.argtypes = [i, d] + [vp] * 19
        _LIB = L
    return _LIB


def _p(a):
    if a is None:
        return None
    assert isinstance(a, np.ndarray) and a.flags.c_contiguous, "array must be C-contiguous"
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _GridHandle:
    """Keeps the numpy arrays alive behind an or_grid struct."""

    def __init__(self, grid):
        self.arrays = {}
        for n in _GRID_PTRS:
            a = np.ascontiguousarray(getattr(grid, n))
            self.arrays[n] = a
        self.s = OrGrid(grid.n_cells, grid.n_edges, grid.n_verts, grid.radius,
                        *[_p(self.arrays[n]) for n in _GRID_PTRS])

    @property
    def ref(self):
        return C.byref(self.s)


def params_struct(p, w_damp=None):
    """or_params of a case's Params; w_damp (a C-contiguous FP64 array the
    caller keeps alive) is the per-half-level Rayleigh rate of w, or None."""
    return OrParams(p.radius, p.omega, p.grav, p.rd, p.cpd, p.p00, p.beta, p.wgt_corr, p.extrap,
                    p.div_damp, int(p.upwind), p.div_damp4, p.smag, _p(w_damp))


class Model:
    """The oracle's model of one case: metrics from the case's heights, state
    from the case (or set later)."""

    def __init__(self, case, params=None):
        self.grid = case.grid
        self.N = case.n_lev
        self.params = params if params is not None else case.params
        self._g = _GridHandle(case.grid)
        self._wd = None if case.w_damp is None else _f64(case.w_damp)
        self._pp = params_struct(self.params, self._wd)
        self._keep = [_f64(case.zh), _f64(case.pi_ref), _f64(case.theta_ref)]
        self.pi_ref = self._keep[1]
        self.h = lib().or_create(self._g.ref, self.N, *[_p(a) for a in self._keep],
                                 C.byref(self._pp))
        if not self.h:
            raise RuntimeError("or_create failed")
        self.set_state(case.vn, case.w, case.rho, case.pi, case.theta_v)
        self.nt = 0
        if getattr(case, "tracers", None) is not None:
            self.set_tracers(case.tracers)

    def set_tracers(self, q):
        q = _f64(q)
        self.nt = q.shape[0] if q.size else 0
        if lib().or_tracers_set(self.h, self.nt, _p(q) if self.nt else None) != 0:
            raise RuntimeError("or_tracers_set failed")

    def tracers(self):
        out = np.empty((self.nt, self.N, self.grid.n_cells))
        lib().or_tracers_get(self.h, _p(out))
        return out

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_free(self.h)
            self.h = None

    def set_state(self, vn, w, rho, pi, theta_v, pi_prev=None):
        arrs = [_f64(a) for a in (vn, w, rho, pi, theta_v)]
        pp = _f64(pi_prev) if pi_prev is not None else None
        rc = lib().or_set_state(self.h, *[_p(a) for a in arrs], _p(pp))
        if rc != 0:
            raise RuntimeError("or_set_state failed")

    def state(self):
        nc, ne, N = self.grid.n_cells, self.grid.n_edges, self.N
        out = dict(vn=np.empty((N, ne)), w=np.empty((N + 1, nc)), rho=np.empty((N, nc)),
                   pi=np.empty((N, nc)), theta_v=np.empty((N, nc)), pi_prev=np.empty((N, nc)))
        lib().or_get_state(self.h, *[_p(out[k]) for k in ("vn", "w", "rho", "pi", "theta_v",
                                                           "pi_prev")])
        return out

    def flux(self):
        nc, ne, N = self.grid.n_cells, self.grid.n_edges, self.N
        facc, wacc = np.empty((N, ne)), np.empty((N + 1, nc))
        lib().or_get_flux(self.h, _p(facc), _p(wacc))
        return facc, wacc

    def step(self, dt, nsub):
        rc = lib().or_step(self.h, float(dt), int(nsub))
        if rc != 0:
            raise RuntimeError("or_step failed")

    def vt(self, vn, w):
        nc, ne, N = self.grid.n_cells, self.grid.n_edges, self.N
        tvn, tw, wcc, vt = np.empty((N, ne)), np.empty((N + 1, nc)), np.empty((N + 1, nc)), \
            np.empty((N, ne))
        vn, w = _f64(vn), _f64(w)
        lib().or_vt(self.h, _p(vn), _p(w), _p(tvn), _p(tw), _p(wcc), _p(vt))
        return tvn, tw, wcc, vt

    def pgrad(self, p):
        out = np.empty((self.N, self.grid.n_edges))
        p = _f64(p)
        lib().or_pgrad(self.h, _p(p), _p(out))
        return out

    def diag(self):
        m, rt = C.c_double(), C.c_double()
        lib().or_diag(self.h, C.byref(m), C.byref(rt))
        return m.value, rt.value


# ---- single-level operators -------------------------------------------------

def _op(name, grid, x, n_out):
    h = _GridHandle(grid)
    x = _f64(x)
    out = np.empty(n_out)
    getattr(lib(), name)(h.ref, _p(x), _p(out))
    return out


def div(grid, f):
    return _op("or_op_div", grid, f, grid.n_cells)


def grad(grid, p):
    return _op("or_op_grad", grid, p, grid.n_edges)


def tgrad(grid, q):
    return _op("or_op_tgrad", grid, q, grid.n_edges)


def curl(grid, u):
    return _op("or_op_curl", grid, u, grid.n_verts)


def cell_avg(grid, q):
    return _op("or_op_cell_avg", grid, q, grid.n_cells)


def vert_avg(grid, p):
    return _op("or_op_vert_avg", grid, p, grid.n_verts)


def cell_grad(grid, p, radial_c=None):
    """Green-Gauss horizontal gradient of a cell field, [3][n_cells] per metre;
    radial_c (default: the unit cell centres) is the direction removed."""
    h = _GridHandle(grid)
    p = _f64(p)
    rc = _f64(grid.cell_x if radial_c is None else radial_c)
    out = np.empty((3, grid.n_cells))
    lib().or_op_cell_grad(h.ref, _p(p), _p(rc), _p(out))
    return out


def upwind(grid, p, grad, u, vt, dt):
    """Second-order upwind edge values of a cell field (one level)."""
    h = _GridHandle(grid)
    p, grad, u, vt = (_f64(a) for a in (p, grad, u, vt))
    out = np.empty(grid.n_edges)
    lib().or_op_upwind(h.ref, _p(p), _p(grad), _p(u), _p(vt), float(dt), _p(out))
    return out


def vector_laplacian(grid, u):
    """G(D(u)) - T(Z(u)) of an edge field (one level)."""
    return _op("or_op_vector_laplacian", grid, u, grid.n_edges)


def graddiv2(grid, u):
    """G(D(G(D(u)))) of an edge field (one level)."""
    return _op("or_op_graddiv2", grid, u, grid.n_edges)


def deformation(grid, u, vt):
    """Horizontal deformation magnitude per cell of the edge velocities u n + vt t."""
    h = _GridHandle(grid)
    u, vt = _f64(u), _f64(vt)
    out = np.empty(grid.n_cells)
    lib().or_op_deformation(h.ref, _p(u), _p(vt), _p(out))
    return out


def tracer_grad(grid, q):
    """Difference-form Green-Gauss gradient of a cell field, [3][n_cells]."""
    h = _GridHandle(grid)
    q = _f64(q)
    out = np.empty((3, grid.n_cells))
    lib().or_op_tracer_grad(h.ref, _p(q), _p(out))
    return out


def tracer_recon(grid, q, grad):
    """Linear reconstruction toward each of a cell's edges, [3][n_cells]."""
    h = _GridHandle(grid)
    q, grad = _f64(q), _f64(grad)
    out = np.empty((3, grid.n_cells))
    lib().or_op_tracer_recon(h.ref, _p(q), _p(grad), _p(out))
    return out


def ppm_faces(dz, q):
    dz, q = _f64(dz), _f64(q)
    a = np.empty(len(q) + 1)
    if lib().or_ppm_faces(len(q), _p(dz), _p(q), _p(a)) != 0:
        raise RuntimeError("or_ppm_faces failed")
    return a


def ppm_column(dt, dz, rho, W, q):
    """Vertical PPM transport of one column: returns (q_out, rho_out)."""
    dz, rho, W, q = (_f64(a) for a in (dz, rho, W, q))
    qo, ro = np.empty(len(q)), np.empty(len(q))
    if lib().or_ppm_column(len(q), float(dt), _p(dz), _p(rho), _p(W), _p(q), _p(qo), _p(ro)) != 0:
        raise RuntimeError("or_ppm_column failed")
    return qo, ro


def perot(grid, pos_c, pos_e, radial_c, u):
    h = _GridHandle(grid)
    pos_c, pos_e, radial_c, u = (_f64(a) for a in (pos_c, pos_e, radial_c, u))
    vc, vt = np.empty((3, grid.n_cells)), np.empty(grid.n_edges)
    lib().or_op_perot(h.ref, _p(pos_c), _p(pos_e), _p(radial_c), _p(u), _p(vc), _p(vt))
    return vc, vt


def thomas(a, b, c, r):
    a, b, c, r = (_f64(x) for x in (a, b, c, r))
    x = np.empty_like(r)
    rc = lib().or_thomas(int(r.size), _p(a), _p(b), _p(c), _p(r), _p(x))
    if rc != 0:
        raise RuntimeError("or_thomas failed")
    return x


def column(params, dt, zh, pi_ref, theta_ref, pi_n, rho_n, thv_n, rho_i, thv_i, w_n, tw, wcc,
           div_rho, div_th, w_damp=None):
    N = len(pi_ref)
    ins = [_f64(a) for a in (zh, pi_ref, theta_ref, pi_n, rho_n, thv_n, rho_i, thv_i, w_n, tw, wcc,
                             div_rho, div_th)]
    w, rho, pi, thv, fl = np.empty(N + 1), np.empty(N), np.empty(N), np.empty(N), np.empty(N + 1)
    wd = None if w_damp is None else _f64(w_damp)
    pp = params_struct(params, wd)
    rc = lib().or_column(N, float(dt), C.byref(pp), *[_p(a) for a in ins], _p(w), _p(rho), _p(pi),
                         _p(thv), _p(fl))
    if rc != 0:
        raise RuntimeError("or_column failed")
    return dict(w=w, rho=rho, pi=pi, theta_v=thv, vflux=fl)

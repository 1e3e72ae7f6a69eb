"""ctypes binding of the icosahedral grid builder (include/nhgrid.h).

The grid is returned as numpy arrays copied out of the native object, with
the slot-major layout of the C side: ``cell_edges[j, c]`` is edge slot j of
cell c, vectors are ``[3, n]``.
"""
import ctypes as C
from dataclasses import dataclass

import numpy as np

from .. import _build

ORDERS = {"canonical": 0, "sfc": 1, "random": 2, "curve": 3}
EARTH_RADIUS = 6371229.0


class _View(C.Structure):
    _fields_ = [("k", C.c_int32), ("order", C.c_int32),
                ("n_cells", C.c_int64), ("n_edges", C.c_int64), ("n_verts", C.c_int64),
                ("radius", C.c_double)] + [
        (name, C.c_void_p) for name in (
            "cell_edges", "cell_verts", "cell_cells", "cell_sign", "edge_cells", "edge_verts",
            "vert_edges", "vert_cells", "vert_sign", "vert_valence", "cell_x", "cell_area",
            "edge_x", "edge_normal", "edge_tangent", "edge_length", "dual_length", "dual_frac",
            "vert_x", "vert_area", "canon_cell", "canon_edge", "canon_vert")]


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = C.CDLL(_build.ensure(_build.INPUTS_SO, _build.build_inputs))
        _LIB.nhgrid_build.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_void_p)]
        _LIB.nhgrid_reorder.argtypes = [C.c_void_p, C.c_int, C.c_uint64]
        _LIB.nhgrid_get_view.argtypes = [C.c_void_p, C.POINTER(_View)]
        _LIB.nhgrid_free.argtypes = [C.c_void_p]
        _LIB.nhgrid_free.restype = None
        _LIB.nhgrid_last_error.restype = C.c_char_p
        _LIB.nhgrid_counts.argtypes = [C.c_int] + [C.POINTER(C.c_int64)] * 3
        _LIB.nhgrid_counts.restype = None
    return _LIB


def grid_counts(k):
    """(n_cells, n_edges, n_verts) of R2Bk from the closed forms."""
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    lib().nhgrid_counts(k, C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


@dataclass
class Grid:
    k: int
    order: str
    radius: float
    n_cells: int
    n_edges: int
    n_verts: int
    cell_edges: np.ndarray
    cell_verts: np.ndarray
    cell_cells: np.ndarray
    cell_sign: np.ndarray
    edge_cells: np.ndarray
    edge_verts: np.ndarray
    vert_edges: np.ndarray
    vert_cells: np.ndarray
    vert_sign: np.ndarray
    vert_valence: np.ndarray
    cell_x: np.ndarray
    cell_area: np.ndarray
    edge_x: np.ndarray
    edge_normal: np.ndarray
    edge_tangent: np.ndarray
    edge_length: np.ndarray
    dual_length: np.ndarray
    dual_frac: np.ndarray
    vert_x: np.ndarray
    vert_area: np.ndarray
    canon_cell: np.ndarray
    canon_edge: np.ndarray
    canon_vert: np.ndarray


def _copy(ptr, ctype, shape):
    n = int(np.prod(shape))
    if n == 0:
        return np.zeros(shape, dtype=np.ctypeslib.as_ctypes_type(ctype))
    arr = np.ctypeslib.as_array(C.cast(ptr, C.POINTER(ctype)), shape=(n,))
    return arr.copy().reshape(shape)


def _snapshot(h):
    v = _View()
    rc = lib().nhgrid_get_view(h, C.byref(v))
    if rc != 0:
        raise RuntimeError(lib().nhgrid_last_error().decode())
    nc, ne, nv = v.n_cells, v.n_edges, v.n_verts
    i32, i8, f64 = C.c_int32, C.c_int8, C.c_double
    return Grid(
        k=v.k, order={v_: k_ for k_, v_ in ORDERS.items()}[v.order], radius=v.radius,
        n_cells=nc, n_edges=ne, n_verts=nv,
        cell_edges=_copy(v.cell_edges, i32, (3, nc)), cell_verts=_copy(v.cell_verts, i32, (3, nc)),
        cell_cells=_copy(v.cell_cells, i32, (3, nc)), cell_sign=_copy(v.cell_sign, i8, (3, nc)),
        edge_cells=_copy(v.edge_cells, i32, (2, ne)), edge_verts=_copy(v.edge_verts, i32, (2, ne)),
        vert_edges=_copy(v.vert_edges, i32, (6, nv)), vert_cells=_copy(v.vert_cells, i32, (6, nv)),
        vert_sign=_copy(v.vert_sign, i8, (6, nv)), vert_valence=_copy(v.vert_valence, i32, (nv,)),
        cell_x=_copy(v.cell_x, f64, (3, nc)), cell_area=_copy(v.cell_area, f64, (nc,)),
        edge_x=_copy(v.edge_x, f64, (3, ne)), edge_normal=_copy(v.edge_normal, f64, (3, ne)),
        edge_tangent=_copy(v.edge_tangent, f64, (3, ne)),
        edge_length=_copy(v.edge_length, f64, (ne,)), dual_length=_copy(v.dual_length, f64, (ne,)),
        dual_frac=_copy(v.dual_frac, f64, (ne,)),
        vert_x=_copy(v.vert_x, f64, (3, nv)), vert_area=_copy(v.vert_area, f64, (nv,)),
        canon_cell=_copy(v.canon_cell, i32, (nc,)), canon_edge=_copy(v.canon_edge, i32, (ne,)),
        canon_vert=_copy(v.canon_vert, i32, (nv,)))


def build_grid(k, order="canonical", seed=0, radius=EARTH_RADIUS, with_canonical=False):
    """Build R2Bk and renumber it ('canonical', 'sfc' or 'random').  With
    ``with_canonical`` the canonical-order grid is returned as well, as the
    pair (canonical, renumbered)."""
    h = C.c_void_p()
    rc = lib().nhgrid_build(int(k), float(radius), C.byref(h))
    if rc != 0:
        raise RuntimeError(lib().nhgrid_last_error().decode())
    try:
        canon = _snapshot(h) if (with_canonical or order == "canonical") else None
        if order == "canonical":
            g = canon
        else:
            rc = lib().nhgrid_reorder(h, ORDERS[order], int(seed))
            if rc != 0:
                raise RuntimeError(lib().nhgrid_last_error().decode())
            g = _snapshot(h)
        return (canon, g) if with_canonical else g
    finally:
        lib().nhgrid_free(h)


def permute_grid_fields(grid, fields, kind):
    """Map arrays given in canonical numbering (last axis = entity) to the
    numbering of ``grid``.  kind: 'cell', 'edge' or 'vert'."""
    canon = {"cell": grid.canon_cell, "edge": grid.canon_edge, "vert": grid.canon_vert}[kind]
    return [np.ascontiguousarray(f[..., canon]) for f in fields]

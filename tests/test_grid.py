"""Grid builder and renumbering: closed-form counts (Table 2 sizes), topology
of the icosahedral triangle grid and its hexagon/pentagon dual (Sec. 3.2),
geometry identities, and renumbering invariants."""
import numpy as np
import pytest

from paper_2511_02021_amd.inputs import grid as G

A = G.EARTH_RADIUS
SPHERE = 4.0 * np.pi * A * A


@pytest.fixture(scope="module", params=[0, 1, 3, 4])
def g(request):
    return G.build_grid(request.param)


def test_closed_form_counts_and_table2_sizes():
    for k in range(10):
        nc, ne, nv = G.grid_counts(k)
        assert nc == 20 * 4 ** (k + 1) and ne == 30 * 4 ** (k + 1) and nv == 10 * 4 ** (k + 1) + 2
        assert nv - ne + nc == 2          # Euler characteristic of the sphere
        assert 2 * ne == 3 * nc           # edges = 1.5 x cells (vn counts 1.5 variables)
    # Table 2: 10 km grid 0.05e8 cells, 1.25 km grid 3.36e8 cells
    assert round(G.grid_counts(8)[0] / 1e8, 2) == 0.05
    assert G.grid_counts(8)[0] == 5242880
    nc11 = 20 * 4 ** 12
    assert round(nc11 / 1e8, 2) == 3.36
    assert G.grid_counts(4) == (20480, 30720, 10242)


def test_built_counts_match_closed_forms(g):
    assert (g.n_cells, g.n_edges, g.n_verts) == G.grid_counts(g.k)
    assert g.n_verts - g.n_edges + g.n_cells == 2


def test_twelve_pentagons(g):
    val = g.vert_valence
    assert (val == 5).sum() == 12 and (val == 6).sum() == g.n_verts - 12
    pad = g.vert_edges[5] < 0
    assert np.array_equal(pad, val == 5)
    assert np.all(g.vert_cells[5][pad] < 0) and np.all(g.vert_sign[5][pad] == 0)


def test_areas_tile_the_sphere(g):
    assert abs(g.cell_area.sum() / SPHERE - 1) < 1e-12
    assert abs(g.vert_area.sum() / SPHERE - 1) < 1e-12
    assert np.all(g.cell_area > 0) and np.all(g.vert_area > 0)


def test_edge_topology_and_signs(g):
    nc = g.n_cells
    c1, c2 = g.edge_cells
    assert np.all(c1 < c2)  # canonical numbering: c1 is the lower id
    # every edge appears in exactly two cells, with opposite signs
    cnt = np.bincount(g.cell_edges.ravel(), minlength=g.n_edges)
    assert np.all(cnt == 2)
    sign_sum = np.zeros(g.n_edges)
    np.add.at(sign_sum, g.cell_edges.ravel(), g.cell_sign.ravel().astype(float))
    assert np.all(sign_sum == 0)
    for j in range(3):
        e = g.cell_edges[j]
        own = np.arange(nc)
        assert np.all(np.where(g.cell_sign[j] > 0, c1[e] == own, c2[e] == own))
        # neighbour across slot j is the other cell of that edge
        other = np.where(c1[e] == own, c2[e], c1[e])
        assert np.array_equal(other, g.cell_cells[j])
        # edge slot j joins vertex slots j and j+1
        va, vb = g.cell_verts[j], g.cell_verts[(j + 1) % 3]
        ev = g.edge_verts[:, e]
        assert np.all(((ev[0] == va) & (ev[1] == vb)) | ((ev[0] == vb) & (ev[1] == va)))


def test_geometry_identities(g):
    n, t, x = g.edge_normal, g.edge_tangent, g.edge_x
    assert np.allclose((n * n).sum(0), 1, atol=1e-14, rtol=0)
    assert np.abs((n * t).sum(0)).max() < 1e-14
    assert np.abs((n * x).sum(0)).max() < 1e-14
    v1, v2 = g.edge_verts
    chord = g.vert_x[:, v2] - g.vert_x[:, v1]
    # n is perpendicular to the primal edge chord; t points from v1 to v2
    assert np.abs((n * chord).sum(0)).max() < 1e-14
    assert np.all((t * chord).sum(0) > 0)
    c1, c2 = g.edge_cells
    assert np.all((n * (g.cell_x[:, c2] - g.cell_x[:, c1])).sum(0) > 0)
    assert np.all(g.edge_length > 0) and np.all(g.dual_length > 0)
    # circumcentres are equidistant from the three corners
    d = np.stack([(g.cell_x * g.vert_x[:, g.cell_verts[j]]).sum(0) for j in range(3)])
    assert np.abs(d - d[0]).max() < 1e-14
    # triangles counter-clockwise seen from outside
    p0, p1, p2 = (g.vert_x[:, g.cell_verts[j]] for j in range(3))
    assert np.all((np.cross(p1 - p0, p2 - p0, axis=0) * p0).sum(0) > 0)


def test_vertex_rings_counter_clockwise(g):
    nv = g.n_verts
    xv = g.vert_x
    for v in range(0, nv, max(1, nv // 500)):
        m = g.vert_valence[v]
        es = g.vert_edges[:m, v]
        assert es[0] == es.min()
        other = np.where(g.edge_verts[0, es] == v, g.edge_verts[1, es], g.edge_verts[0, es])
        d = g.vert_x[:, other] - np.outer(xv[:, v], xv[:, v] @ g.vert_x[:, other])
        ang = np.arctan2(xv[:, v] @ np.cross(d[:, 0], d, axis=0), d[:, 0] @ d)
        ang = np.where(ang < 0, ang + 2 * np.pi, ang)
        assert np.all(np.diff(ang) > 0)
        for j in range(m):
            cell = g.vert_cells[j, v]
            assert es[j] in g.cell_edges[:, cell] and es[(j + 1) % m] in g.cell_edges[:, cell]
            sgn = 1 if g.edge_verts[1, es[j]] == v else -1
            assert g.vert_sign[j, v] == sgn


def _mapped_back(gr, canon):
    """Tables of a renumbered grid expressed in canonical ids and order."""
    ic = np.argsort(gr.canon_cell)
    ie = np.argsort(gr.canon_edge)
    iv = np.argsort(gr.canon_vert)
    out = dict(
        cell_edges=np.where(gr.cell_edges >= 0, gr.canon_edge[gr.cell_edges], -1)[:, ic],
        cell_verts=gr.canon_vert[gr.cell_verts][:, ic],
        cell_cells=gr.canon_cell[gr.cell_cells][:, ic],
        cell_sign=gr.cell_sign[:, ic],
        edge_cells=gr.canon_cell[gr.edge_cells][:, ie],
        edge_verts=gr.canon_vert[gr.edge_verts][:, ie],
        vert_edges=np.where(gr.vert_edges >= 0, gr.canon_edge[np.maximum(gr.vert_edges, 0)], -1)[:, iv],
        vert_cells=np.where(gr.vert_cells >= 0, gr.canon_cell[np.maximum(gr.vert_cells, 0)], -1)[:, iv],
        vert_sign=gr.vert_sign[:, iv], cell_x=gr.cell_x[:, ic], cell_area=gr.cell_area[ic],
        edge_normal=gr.edge_normal[:, ie], dual_length=gr.dual_length[ie],
        vert_area=gr.vert_area[iv])
    return out


@pytest.mark.parametrize("order", ["sfc", "random", "curve"])
def test_renumbering_is_a_relabelling(order):
    canon, gr = G.build_grid(4, order=order, seed=7, with_canonical=True)
    for m in (gr.canon_cell, gr.canon_edge, gr.canon_vert):
        assert np.array_equal(np.sort(m), np.arange(m.size))
    back = _mapped_back(gr, canon)
    for name, arr in back.items():
        assert np.array_equal(arr, getattr(canon, name)), name


def test_sfc_locality_beats_random():
    def near(gr, w=256):
        c = np.arange(gr.n_cells)
        return (np.abs(gr.cell_cells - c) < w).mean()
    sfc = G.build_grid(5, order="sfc")
    rnd = G.build_grid(5, order="random", seed=1)
    assert near(sfc) > 0.9 and near(rnd) < 0.01
    # edges numbered by first touch: a cell's three edge ids are close together
    spread = lambda gr: np.median(gr.cell_edges.max(0) - gr.cell_edges.min(0))
    assert spread(sfc) < 16 and spread(rnd) > 10000


@pytest.mark.parametrize("k", [0, 1, 3, 5])
def test_bisection_curve_is_vertex_continuous(k):
    """Along the curve order every cell shares at least a vertex with the
    next one (root faces included), and most share an edge; the edges and
    vertices follow by first touch."""
    g = G.build_grid(k, order="curve")
    cv = g.cell_verts
    cnt = np.zeros(g.n_cells - 1, dtype=int)
    for a in range(3):
        for b in range(3):
            cnt += cv[a, :-1] == cv[b, 1:]
    assert cnt.min() >= 1
    assert (cnt >= 2).mean() > 0.6
    spread = np.median(g.cell_edges.max(0) - g.cell_edges.min(0))
    assert spread < 16

// nhgrid.cpp -- icosahedral triangular C-grid builder and renumbering.
//
// Host-only input generator: the grid (connectivity + geometry) is an input
// of the dynamical core, consumed unchanged by both the CPU oracle and the
// HIP library.  The construction, orientation and sign conventions are stated
// in include/nhgrid.h.  The dual grid of hexagons and 12 pentagons and the
// indirect neighbour indexing follow Sec. 3.2 of the paper; the grid sizes
// follow Table 2.

#include "nhgrid.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <random>
#include <stdexcept>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

struct V3 {
    double x, y, z;
};
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 scl(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 unit(V3 a) { return scl(a, 1.0 / norm(a)); }
// angle between two unit vectors, accurate for small angles
inline double angle(V3 a, V3 b) { return std::atan2(norm(cross(a, b)), dot(a, b)); }
// spherical excess of the triangle (p0,p1,p2) of unit vectors
inline double excess(V3 p0, V3 p1, V3 p2) {
    double num = std::fabs(dot(p0, cross(p1, p2)));
    double den = 1.0 + dot(p0, p1) + dot(p1, p2) + dot(p2, p0);
    return 2.0 * std::atan2(num, den);
}

// Small per-vertex adjacency table: up to 6 (neighbour, payload) pairs.
struct Adj6 {
    int32_t nb[6];
    int32_t val[6];
    int32_t n;
};

int32_t adj_find(const Adj6 &a, int32_t nb) {
    for (int i = 0; i < a.n; ++i)
        if (a.nb[i] == nb) return a.val[i];
    return -1;
}

bool adj_put(Adj6 &a, int32_t nb, int32_t val) {
    if (a.n >= 6) return false;
    a.nb[a.n] = nb;
    a.val[a.n] = val;
    ++a.n;
    return true;
}

}  // namespace

struct nhgrid {
    int k = 0;
    int order = NHGRID_ORDER_CANONICAL;
    int64_t nc = 0, ne = 0, nv = 0;
    double radius = 0;
    std::vector<int32_t> cell_edges, cell_verts, cell_cells;
    std::vector<int8_t> cell_sign;
    std::vector<int32_t> edge_cells, edge_verts;
    std::vector<int32_t> vert_edges, vert_cells, vert_valence;
    std::vector<int8_t> vert_sign;
    std::vector<double> cell_x, cell_area, edge_x, edge_normal, edge_tangent, edge_length,
        dual_length, dual_frac, vert_x, vert_area;
    std::vector<int32_t> canon_cell, canon_edge, canon_vert;
};

extern "C" void nhgrid_counts(int k, int64_t *n_cells, int64_t *n_edges, int64_t *n_verts) {
    int64_t p = int64_t(1) << (2 * (k + 1));  // 4^(k+1)
    if (n_cells) *n_cells = 20 * p;
    if (n_edges) *n_edges = 30 * p;
    if (n_verts) *n_verts = 10 * p + 2;
}

extern "C" const char *nhgrid_last_error(void) { return g_err.c_str(); }

namespace {

// Icosahedron: north pole, five upper-ring vertices (lat +atan(1/2), lon 72j),
// five lower-ring vertices (lat -atan(1/2), lon 36+72j), south pole.
void icosahedron(std::vector<V3> &pts, std::vector<int32_t> &tri) {
    const double pi = 3.14159265358979323846;
    const double lat = std::atan(0.5);
    pts.clear();
    pts.push_back({0.0, 0.0, 1.0});
    for (int j = 0; j < 5; ++j) {
        double lon = 2.0 * pi * j / 5.0;
        pts.push_back({std::cos(lat) * std::cos(lon), std::cos(lat) * std::sin(lon), std::sin(lat)});
    }
    for (int j = 0; j < 5; ++j) {
        double lon = 2.0 * pi * j / 5.0 + pi / 5.0;
        pts.push_back(
            {std::cos(lat) * std::cos(lon), std::cos(lat) * std::sin(lon), -std::sin(lat)});
    }
    pts.push_back({0.0, 0.0, -1.0});
    auto U = [](int j) { return 1 + (j % 5); };
    auto L = [](int j) { return 6 + (j % 5); };
    tri.clear();
    auto face = [&](int a, int b, int c) {
        // enforce counter-clockwise seen from outside
        V3 pa = pts[a], pb = pts[b], pc = pts[c];
        if (dot(cross(sub(pb, pa), sub(pc, pa)), add(add(pa, pb), pc)) < 0) std::swap(b, c);
        tri.push_back(a);
        tri.push_back(b);
        tri.push_back(c);
    };
    for (int j = 0; j < 5; ++j) face(0, U(j), U(j + 1));         // northern cap
    for (int j = 0; j < 5; ++j) face(U(j), L(j), U(j + 1));      // upper belt
    for (int j = 0; j < 5; ++j) face(L(j), L(j + 1), U(j + 1));  // lower belt
    for (int j = 0; j < 5; ++j) face(11, L(j + 1), L(j));        // southern cap
}

}  // namespace

extern "C" int nhgrid_build(int k, double radius, nhgrid **out) {
    if (!out) return fail(NHGRID_EINVAL, "nhgrid_build: out is NULL");
    *out = nullptr;
    if (k < 0 || k > 9) return fail(NHGRID_EINVAL, "nhgrid_build: k must be in [0, 9]");
    if (!(radius > 0) || !std::isfinite(radius))
        return fail(NHGRID_EINVAL, "nhgrid_build: radius must be positive and finite");
    nhgrid *g = new (std::nothrow) nhgrid;
    if (!g) return fail(NHGRID_ENOMEM, "nhgrid_build: out of memory");
    try {
        g->k = k;
        g->radius = radius;
        int64_t nc, ne, nv;
        nhgrid_counts(k, &nc, &ne, &nv);
        g->nc = nc;
        g->ne = ne;
        g->nv = nv;

        // ---- bisection, level by level (each triangle replaced in place by its
        // four children: the list order is then the depth-first path order) ----
        std::vector<V3> pts;
        std::vector<int32_t> tri;
        icosahedron(pts, tri);
        pts.reserve(nv);
        for (int lev = 0; lev < k + 1; ++lev) {
            int64_t nt = tri.size() / 3;
            std::vector<Adj6> mid(pts.size());
            for (auto &a : mid) a.n = 0;
            std::vector<int32_t> ntri;
            ntri.reserve(nt * 12);
            auto midpoint = [&](int32_t a, int32_t b) -> int32_t {
                int32_t m = adj_find(mid[a], b);
                if (m >= 0) return m;
                m = int32_t(pts.size());
                pts.push_back(unit(add(pts[a], pts[b])));  // (p+q)/|p+q|, symmetric in p,q
                if (!adj_put(mid[a], b, m) || !adj_put(mid[b], a, m))
                    throw std::runtime_error("valence overflow during bisection");
                mid.push_back(Adj6{{0}, {0}, 0});
                return m;
            };
            for (int64_t t = 0; t < nt; ++t) {
                int32_t p0 = tri[3 * t], p1 = tri[3 * t + 1], p2 = tri[3 * t + 2];
                int32_t m01 = midpoint(p0, p1), m12 = midpoint(p1, p2), m20 = midpoint(p2, p0);
                const int32_t ch[12] = {p0, m01, m20, m01, p1, m12, m20, m12, p2, m12, m20, m01};
                ntri.insert(ntri.end(), ch, ch + 12);
            }
            tri.swap(ntri);
        }
        if (int64_t(tri.size() / 3) != nc || int64_t(pts.size()) != nv)
            return delete g, fail(NHGRID_EINTERNAL, "nhgrid_build: entity counts disagree");

        // ---- canonical vertex ids: first appearance over cells, slots 0..2 ----
        std::vector<int32_t> vmap(nv, -1);
        std::vector<V3> vx(nv);
        int32_t nvid = 0;
        g->cell_verts.assign(3 * nc, -1);
        for (int64_t c = 0; c < nc; ++c)
            for (int j = 0; j < 3; ++j) {
                int32_t p = tri[3 * c + j];
                if (vmap[p] < 0) {
                    vmap[p] = nvid;
                    vx[nvid] = pts[p];
                    ++nvid;
                }
                g->cell_verts[j * nc + c] = vmap[p];
            }
        std::vector<int32_t>().swap(tri);
        std::vector<V3>().swap(pts);

        // ---- canonical edge ids: first appearance, edge slot j = (v_j, v_{j+1}) ----
        std::vector<Adj6> vadj(nv);
        for (auto &a : vadj) a.n = 0;
        g->cell_edges.assign(3 * nc, -1);
        g->edge_cells.assign(2 * ne, -1);
        int32_t neid = 0;
        std::vector<int32_t> eva(ne), evb(ne);
        for (int64_t c = 0; c < nc; ++c)
            for (int j = 0; j < 3; ++j) {
                int32_t a = g->cell_verts[j * nc + c], b = g->cell_verts[((j + 1) % 3) * nc + c];
                int32_t e = adj_find(vadj[a], b);
                if (e < 0) {
                    e = neid++;
                    if (e >= ne || !adj_put(vadj[a], b, e) || !adj_put(vadj[b], a, e))
                        return delete g, fail(NHGRID_EINTERNAL, "nhgrid_build: edge overflow");
                    eva[e] = a;
                    evb[e] = b;
                    g->edge_cells[e] = int32_t(c);  // first (lower-id) cell is c1
                } else {
                    if (g->edge_cells[ne + e] >= 0)
                        return delete g, fail(NHGRID_EINTERNAL, "nhgrid_build: edge with >2 cells");
                    g->edge_cells[ne + e] = int32_t(c);
                }
                g->cell_edges[j * nc + c] = e;
            }
        if (neid != ne) return delete g, fail(NHGRID_EINTERNAL, "nhgrid_build: edge count");

        // ---- neighbours and signs ----
        g->cell_cells.assign(3 * nc, -1);
        g->cell_sign.assign(3 * nc, 0);
        for (int64_t c = 0; c < nc; ++c)
            for (int j = 0; j < 3; ++j) {
                int32_t e = g->cell_edges[j * nc + c];
                int32_t c1 = g->edge_cells[e], c2 = g->edge_cells[ne + e];
                bool is1 = (c1 == c);
                g->cell_cells[j * nc + c] = is1 ? c2 : c1;
                g->cell_sign[j * nc + c] = is1 ? 1 : -1;
            }

        // ---- cell geometry ----
        const double a = radius;
        g->cell_x.assign(3 * nc, 0.0);
        g->cell_area.assign(nc, 0.0);
        std::vector<V3> cx(nc);
        for (int64_t c = 0; c < nc; ++c) {
            V3 p0 = vx[g->cell_verts[c]], p1 = vx[g->cell_verts[nc + c]],
               p2 = vx[g->cell_verts[2 * nc + c]];
            V3 cc = unit(cross(sub(p1, p0), sub(p2, p0)));
            cx[c] = cc;
            g->cell_x[c] = cc.x;
            g->cell_x[nc + c] = cc.y;
            g->cell_x[2 * nc + c] = cc.z;
            g->cell_area[c] = a * a * excess(p0, p1, p2);
        }

        // ---- edge geometry and orientation ----
        g->edge_x.assign(3 * ne, 0.0);
        g->edge_normal.assign(3 * ne, 0.0);
        g->edge_tangent.assign(3 * ne, 0.0);
        g->edge_length.assign(ne, 0.0);
        g->dual_length.assign(ne, 0.0);
        g->dual_frac.assign(ne, 0.0);
        g->edge_verts.assign(2 * ne, -1);
        for (int64_t e = 0; e < ne; ++e) {
            V3 va = vx[eva[e]], vb = vx[evb[e]];
            V3 xe = unit(add(va, vb));
            V3 c1 = cx[g->edge_cells[e]], c2 = cx[g->edge_cells[ne + e]];
            V3 d = sub(c2, c1);
            V3 n = unit(sub(d, scl(xe, dot(d, xe))));
            V3 t = cross(xe, n);
            int32_t v1 = eva[e], v2 = evb[e];
            if (dot(sub(vb, va), t) < 0) std::swap(v1, v2);
            g->edge_verts[e] = v1;
            g->edge_verts[ne + e] = v2;
            g->edge_x[e] = xe.x;
            g->edge_x[ne + e] = xe.y;
            g->edge_x[2 * ne + e] = xe.z;
            g->edge_normal[e] = n.x;
            g->edge_normal[ne + e] = n.y;
            g->edge_normal[2 * ne + e] = n.z;
            g->edge_tangent[e] = t.x;
            g->edge_tangent[ne + e] = t.y;
            g->edge_tangent[2 * ne + e] = t.z;
            g->edge_length[e] = a * angle(va, vb);
            g->dual_length[e] = a * angle(c1, c2);
            // the dual arc c1 -> c2 crosses the primal edge at its midpoint
            g->dual_frac[e] = angle(c1, xe) / angle(c1, c2);
        }

        // ---- vertex rings: counter-clockwise from the lowest-id incident edge ----
        g->vert_edges.assign(6 * nv, -1);
        g->vert_cells.assign(6 * nv, -1);
        g->vert_sign.assign(6 * nv, 0);
        g->vert_valence.assign(nv, 0);
        g->vert_x.assign(3 * nv, 0.0);
        g->vert_area.assign(nv, 0.0);
        for (int64_t v = 0; v < nv; ++v) {
            const Adj6 &ad = vadj[v];
            int m = ad.n;
            if (m != 5 && m != 6)
                return delete g, fail(NHGRID_EINTERNAL, "nhgrid_build: vertex valence not 5/6");
            V3 xv = vx[v];
            g->vert_x[v] = xv.x;
            g->vert_x[nv + v] = xv.y;
            g->vert_x[2 * nv + v] = xv.z;
            g->vert_valence[v] = m;
            // reference direction: the incident edge with the lowest id
            int i0 = 0;
            for (int i = 1; i < m; ++i)
                if (ad.val[i] < ad.val[i0]) i0 = i;
            auto tdir = [&](int i) {
                V3 q = vx[ad.nb[i]];
                return sub(q, scl(xv, dot(q, xv)));
            };
            V3 r = tdir(i0);
            const double twopi = 6.28318530717958647692;
            std::pair<double, int32_t> ring[6];
            for (int i = 0; i < m; ++i) {
                V3 d = tdir(i);
                double ang = std::atan2(dot(xv, cross(r, d)), dot(r, d));
                if (i == i0) ang = 0.0;
                else if (ang <= 0) ang += twopi;
                ring[i] = {ang, ad.val[i]};
            }
            std::sort(ring, ring + m);
            for (int j = 0; j < m; ++j) {
                int32_t e = ring[j].second;
                g->vert_edges[j * nv + v] = e;
                g->vert_sign[j * nv + v] = (g->edge_verts[ne + e] == v) ? 1 : -1;
            }
            // ring cell j: the cell holding both ring edges j and j+1
            double av = 0.0;
            for (int j = 0; j < m; ++j) {
                int32_t ej = ring[j].second, ek = ring[(j + 1) % m].second;
                int32_t cell = -1;
                for (int s = 0; s < 2; ++s) {
                    int32_t c = g->edge_cells[s * ne + ej];
                    for (int q = 0; q < 3; ++q)
                        if (g->cell_edges[q * nc + c] == ek) cell = c;
                }
                if (cell < 0)
                    return delete g, fail(NHGRID_EINTERNAL, "nhgrid_build: ring cell not found");
                g->vert_cells[j * nv + v] = cell;
            }
            for (int j = 0; j < m; ++j) {
                int32_t ca = g->vert_cells[j * nv + v], cb = g->vert_cells[((j + 1) % m) * nv + v];
                av += a * a * excess(xv, cx[ca], cx[cb]);
            }
            g->vert_area[v] = av;
        }

        g->canon_cell.resize(nc);
        g->canon_edge.resize(ne);
        g->canon_vert.resize(nv);
        std::iota(g->canon_cell.begin(), g->canon_cell.end(), 0);
        std::iota(g->canon_edge.begin(), g->canon_edge.end(), 0);
        std::iota(g->canon_vert.begin(), g->canon_vert.end(), 0);
    } catch (const std::bad_alloc &) {
        delete g;
        return fail(NHGRID_ENOMEM, "nhgrid_build: out of memory");
    } catch (const std::exception &ex) {
        delete g;
        return fail(NHGRID_EINTERNAL, std::string("nhgrid_build: ") + ex.what());
    }
    *out = g;
    g_err.clear();
    return NHGRID_OK;
}

namespace {

// 3-D Hilbert key of integer coordinates with `bits` bits each, following
// J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707 (2004):
// transform the axes to the transposed Hilbert index, then interleave bits.
uint64_t hilbert3(uint32_t x0, uint32_t x1, uint32_t x2, int bits) {
    uint32_t X[3] = {x0, x1, x2};
    const uint32_t M = 1u << (bits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t key = 0;
    for (int q = bits - 1; q >= 0; --q)
        for (int i = 0; i < 3; ++i) key = (key << 1) | ((X[i] >> q) & 1u);
    return key;
}

template <class T>
void permute_rows(std::vector<T> &arr, int64_t n, int rows, const std::vector<int32_t> &p) {
    // new[r*n + i] = old[r*n + p[i]]
    std::vector<T> out(arr.size());
    for (int r = 0; r < rows; ++r)
        for (int64_t i = 0; i < n; ++i) out[r * n + i] = arr[r * n + p[i]];
    arr.swap(out);
}

void remap_values(std::vector<int32_t> &arr, const std::vector<int32_t> &inv) {
    for (auto &v : arr)
        if (v >= 0) v = inv[v];
}

std::vector<int32_t> inverse(const std::vector<int32_t> &p) {
    std::vector<int32_t> inv(p.size());
    for (size_t i = 0; i < p.size(); ++i) inv[p[i]] = int32_t(i);
    return inv;
}

// Apply new->old permutations pc, pe, pv to every table of g.
void apply(nhgrid *g, const std::vector<int32_t> &pc, const std::vector<int32_t> &pe,
           const std::vector<int32_t> &pv) {
    const int64_t nc = g->nc, ne = g->ne, nv = g->nv;
    auto ic = inverse(pc), ie = inverse(pe), iv = inverse(pv);
    permute_rows(g->cell_edges, nc, 3, pc);
    permute_rows(g->cell_verts, nc, 3, pc);
    permute_rows(g->cell_cells, nc, 3, pc);
    permute_rows(g->cell_sign, nc, 3, pc);
    permute_rows(g->cell_x, nc, 3, pc);
    permute_rows(g->cell_area, nc, 1, pc);
    permute_rows(g->canon_cell, nc, 1, pc);
    permute_rows(g->edge_cells, ne, 2, pe);
    permute_rows(g->edge_verts, ne, 2, pe);
    permute_rows(g->edge_x, ne, 3, pe);
    permute_rows(g->edge_normal, ne, 3, pe);
    permute_rows(g->edge_tangent, ne, 3, pe);
    permute_rows(g->edge_length, ne, 1, pe);
    permute_rows(g->dual_length, ne, 1, pe);
    permute_rows(g->dual_frac, ne, 1, pe);
    permute_rows(g->canon_edge, ne, 1, pe);
    permute_rows(g->vert_edges, nv, 6, pv);
    permute_rows(g->vert_cells, nv, 6, pv);
    permute_rows(g->vert_sign, nv, 6, pv);
    permute_rows(g->vert_valence, nv, 1, pv);
    permute_rows(g->vert_x, nv, 3, pv);
    permute_rows(g->vert_area, nv, 1, pv);
    permute_rows(g->canon_vert, nv, 1, pv);
    remap_values(g->cell_edges, ie);
    remap_values(g->cell_verts, iv);
    remap_values(g->cell_cells, ic);
    remap_values(g->edge_cells, ic);
    remap_values(g->edge_verts, iv);
    remap_values(g->vert_edges, ie);
    remap_values(g->vert_cells, ic);
}

// Canonical cell ids in the order of a continuous curve over the bisection
// tree.  The canonical id of a cell is its root face followed by one base-4
// digit per bisection level (0..2: the child at the parent's vertex slot j,
// 3: the centre child).  A triangle entered at vertex slot a and left at slot
// b visits its children as: the child at a, the centre, the child at the
// third slot c, the child at b; consecutive children share a vertex, and every
// child is left at its own slot b (the child at a is entered at a, the centre
// and the child at b at c, the child at c at a).
void bisection_curve(int64_t base, int64_t quarter, int a, int b, std::vector<int32_t> &out) {
    if (quarter == 0) {
        out.push_back(int32_t(base));
        return;
    }
    const int c = 3 - a - b;
    const int64_t q = quarter / 4;
    bisection_curve(base + a * quarter, q, a, b, out);
    bisection_curve(base + 3 * quarter, q, c, b, out);
    bisection_curve(base + c * quarter, q, a, b, out);
    bisection_curve(base + b * quarter, q, c, b, out);
}

// An order of the root faces, each with entry and exit vertex slots, in which
// every face is entered at the vertex the previous one was left at (depth-
// first search over faces sharing that vertex; the first face is face 0).
bool chain_faces(const std::vector<std::array<int32_t, 3>> &corner, std::vector<int> &face,
                 std::vector<int> &entry, std::vector<int> &exit_, std::vector<char> &used,
                 int depth) {
    const int nf = int(corner.size());
    if (depth == nf) return true;
    const int prev = depth > 0 ? face[depth - 1] : -1;
    for (int f = 0; f < (prev < 0 ? 1 : nf); ++f) {
        if (used[f]) continue;
        for (int a = 0; a < 3; ++a) {
            if (prev >= 0 && corner[f][a] != corner[prev][exit_[depth - 1]]) continue;
            for (int b = 0; b < 3; ++b) {
                if (b == a) continue;
                used[f] = 1;
                face[depth] = f;
                entry[depth] = a;
                exit_[depth] = b;
                if (chain_faces(corner, face, entry, exit_, used, depth + 1)) return true;
                used[f] = 0;
            }
        }
    }
    return false;
}

}  // namespace

extern "C" int nhgrid_reorder(nhgrid *g, int order, uint64_t seed) {
    if (!g) return fail(NHGRID_EINVAL, "nhgrid_reorder: grid is NULL");
    const int64_t nc = g->nc, ne = g->ne, nv = g->nv;
    try {
        std::vector<int32_t> pc(nc), pe(ne), pv(nv);
        if (order == NHGRID_ORDER_CANONICAL) {
            // new id = canonical id
            for (int64_t i = 0; i < nc; ++i) pc[g->canon_cell[i]] = int32_t(i);
            for (int64_t i = 0; i < ne; ++i) pe[g->canon_edge[i]] = int32_t(i);
            for (int64_t i = 0; i < nv; ++i) pv[g->canon_vert[i]] = int32_t(i);
        } else if (order == NHGRID_ORDER_SFC) {
            const int bits = 21;
            const double scale = double((1u << bits) - 1);
            std::vector<std::pair<uint64_t, int32_t>> key(nc);
            for (int64_t c = 0; c < nc; ++c) {
                uint32_t q[3];
                for (int d = 0; d < 3; ++d) {
                    double u = 0.5 * (g->cell_x[d * nc + c] + 1.0);
                    u = std::min(std::max(u, 0.0), 1.0);
                    q[d] = uint32_t(u * scale);
                }
                key[c] = {hilbert3(q[0], q[1], q[2], bits), g->canon_cell[c]};
            }
            std::iota(pc.begin(), pc.end(), 0);
            std::sort(pc.begin(), pc.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
        } else if (order == NHGRID_ORDER_CURVE) {
            // current id of each canonical cell
            std::vector<int32_t> cur(nc);
            for (int64_t i = 0; i < nc; ++i) cur[g->canon_cell[i]] = int32_t(i);
            const int64_t per_face = nc / 20;  // 4^(bisection levels)
            // the root faces' corner vertices: the child at slot j on every
            // level carries the root's vertex j
            std::vector<std::array<int32_t, 3>> corner(20);
            for (int f = 0; f < 20; ++f)
                for (int j = 0; j < 3; ++j) {
                    const int64_t id = int64_t(f) * per_face + j * ((per_face - 1) / 3);
                    corner[f][j] = g->cell_verts[j * nc + cur[id]];
                }
            std::vector<int> face(20), entry(20), exit_(20);
            std::vector<char> used(20, 0);
            if (!chain_faces(corner, face, entry, exit_, used, 0))
                return fail(NHGRID_EINTERNAL, "nhgrid_reorder: no vertex chain over the root faces");
            std::vector<int32_t> canon_order;
            canon_order.reserve(nc);
            for (int i = 0; i < 20; ++i)
                bisection_curve(int64_t(face[i]) * per_face, per_face / 4, entry[i], exit_[i],
                                canon_order);
            if (int64_t(canon_order.size()) != nc)
                return fail(NHGRID_EINTERNAL, "nhgrid_reorder: curve length mismatch");
            for (int64_t i = 0; i < nc; ++i) pc[i] = cur[canon_order[i]];
        } else if (order == NHGRID_ORDER_RANDOM) {
            std::mt19937_64 rng(seed);
            auto shuffle = [&](std::vector<int32_t> &p) {
                std::iota(p.begin(), p.end(), 0);
                for (int64_t i = int64_t(p.size()) - 1; i > 0; --i) {
                    int64_t j = int64_t(rng() % uint64_t(i + 1));
                    std::swap(p[i], p[j]);
                }
            };
            shuffle(pc);
            shuffle(pe);
            shuffle(pv);
        } else {
            return fail(NHGRID_EINVAL, "nhgrid_reorder: unknown order");
        }
        if (order == NHGRID_ORDER_SFC || order == NHGRID_ORDER_CURVE) {
            // edges and vertices by first touch in the new cell order
            std::vector<char> seen_e(ne, 0), seen_v(nv, 0);
            int64_t ke = 0, kv = 0;
            for (int64_t i = 0; i < nc; ++i) {
                int32_t c = pc[i];
                for (int j = 0; j < 3; ++j) {
                    int32_t v = g->cell_verts[j * nc + c];
                    if (!seen_v[v]) seen_v[v] = 1, pv[kv++] = v;
                }
                for (int j = 0; j < 3; ++j) {
                    int32_t e = g->cell_edges[j * nc + c];
                    if (!seen_e[e]) seen_e[e] = 1, pe[ke++] = e;
                }
            }
            if (ke != ne || kv != nv)
                return fail(NHGRID_EINTERNAL, "nhgrid_reorder: first-touch count mismatch");
        }
        apply(g, pc, pe, pv);
        g->order = order;
    } catch (const std::bad_alloc &) {
        return fail(NHGRID_ENOMEM, "nhgrid_reorder: out of memory");
    }
    g_err.clear();
    return NHGRID_OK;
}

extern "C" int nhgrid_get_view(const nhgrid *g, nhgrid_view *v) {
    if (!g || !v) return fail(NHGRID_EINVAL, "nhgrid_get_view: NULL argument");
    v->k = g->k;
    v->order = g->order;
    v->n_cells = g->nc;
    v->n_edges = g->ne;
    v->n_verts = g->nv;
    v->radius = g->radius;
    v->cell_edges = g->cell_edges.data();
    v->cell_verts = g->cell_verts.data();
    v->cell_cells = g->cell_cells.data();
    v->cell_sign = g->cell_sign.data();
    v->edge_cells = g->edge_cells.data();
    v->edge_verts = g->edge_verts.data();
    v->vert_edges = g->vert_edges.data();
    v->vert_cells = g->vert_cells.data();
    v->vert_sign = g->vert_sign.data();
    v->vert_valence = g->vert_valence.data();
    v->cell_x = g->cell_x.data();
    v->cell_area = g->cell_area.data();
    v->edge_x = g->edge_x.data();
    v->edge_normal = g->edge_normal.data();
    v->edge_tangent = g->edge_tangent.data();
    v->edge_length = g->edge_length.data();
    v->dual_length = g->dual_length.data();
    v->dual_frac = g->dual_frac.data();
    v->vert_x = g->vert_x.data();
    v->vert_area = g->vert_area.data();
    v->canon_cell = g->canon_cell.data();
    v->canon_edge = g->canon_edge.data();
    v->canon_vert = g->canon_vert.data();
    return NHGRID_OK;
}

extern "C" void nhgrid_free(nhgrid *g) { delete g; }

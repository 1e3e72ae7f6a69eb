/*
 * nhgrid.h -- icosahedral triangular C-grid builder and renumbering (host only).
 *
 * The grid is the one the paper's atmosphere runs on (Sec. 2, "State of the
 * Art": nonhydrostatic formulation on an icosahedral-triangular C grid; Sec.
 * 3.2: a primal grid of triangles whose dual is made of hexagons and 12
 * pentagons, addressed through integer neighbour-index arrays).  Grid sizes
 * follow Table 2 (10 km = 0.05e8 cells, 1.25 km = 3.36e8 cells): R2Bk has
 * n_c = 20*4^(k+1) cells, n_e = 30*4^(k+1) edges, n_v = 10*4^(k+1)+2 vertices.
 *
 * Construction (canonical numbering):
 *   - icosahedron with vertices at the poles, five at latitude +atan(1/2)
 *     (longitudes 72*j deg) and five at -atan(1/2) (36+72*j deg); 20 faces CCW
 *     seen from outside;
 *   - k+1 bisections; the midpoint of (p,q) is (p+q)/|p+q|; the children of
 *     (p0,p1,p2) are (p0,m01,m20), (m01,p1,m12), (m20,m12,p2), (m12,m20,m01);
 *   - cells are numbered depth-first (face, then child path); vertices and
 *     edges by first appearance while scanning cells in that order, vertex
 *     slots first, then edge slots (edge slot j joins vertex slots j, j+1 mod 3).
 *
 * Geometry (radius a, metres): cell centre = circumcentre; A_c = a^2 E with the
 * spherical excess E from tan(E/2) = |p0.(p1 x p2)| / (1 + p0.p1 + p1.p2 + p2.p0);
 * x_e = unit(va+vb); l_e = a*angle(va,vb); d_e = a*angle(x_c1,x_c2).
 * Orientation: c1(e) is the adjacent cell with the lower canonical id; n_e is
 * the unit tangent-plane projection at x_e of x_c2 - x_c1; t_e = x_e x n_e;
 * (v1,v2) ordered so that (x_v2 - x_v1).t_e > 0.
 * Signs: s(c,e) = +1 if c == c1(e) else -1 (n_e points out of c);
 * sigma(v,e) = +1 if v == v2(e) else -1 (counter-clockwise circulation about v).
 * Vertex rings list edges (and cells) counter-clockwise seen from outside,
 * starting at the incident edge with the lowest canonical id; ring cell j lies
 * between ring edges j and j+1; pentagons carry a pad slot 5 of -1.
 * Dual area A_v = sum over consecutive ring cells of a^2 E(x_v, x_cj, x_cj+1).
 *
 * Array layout: every per-entity table is structure-of-arrays, slot-major:
 * c_e[j*n_c + c] is edge slot j of cell c.  Vectors are [3][n] (x, y, z rows).
 * Integer tables are int32, signs int8, geometry double.
 *
 * Renumbering (nhgrid_reorder) permutes cells, edges and vertices; every
 * entity keeps its slot order, orientation and signs (nothing is re-derived).
 *
 * Errors: every call returns 0 on success or a negative code; the message of
 * the last failure on the calling thread is returned by nhgrid_last_error().
 * Ownership: nhgrid_build allocates; nhgrid_free releases.  nhgrid_view hands
 * out pointers borrowed from the grid, valid until the next reorder or free.
 */
#ifndef NHGRID_H
#define NHGRID_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { NHGRID_OK = 0, NHGRID_EINVAL = -1, NHGRID_ENOMEM = -2, NHGRID_EINTERNAL = -3 };
enum { NHGRID_ORDER_CANONICAL = 0, NHGRID_ORDER_SFC = 1, NHGRID_ORDER_RANDOM = 2,
       NHGRID_ORDER_CURVE = 3 };

typedef struct nhgrid nhgrid;

typedef struct nhgrid_view {
    int32_t k;                 /* R2Bk */
    int32_t order;             /* NHGRID_ORDER_* of the current numbering */
    int64_t n_cells, n_edges, n_verts;
    double radius;             /* sphere radius a [m] */
    /* connectivity, slot-major */
    const int32_t *cell_edges;   /* [3][n_cells] edge slot j = (vertex j, vertex j+1) */
    const int32_t *cell_verts;   /* [3][n_cells] counter-clockwise */
    const int32_t *cell_cells;   /* [3][n_cells] neighbour across edge slot j */
    const int8_t  *cell_sign;    /* [3][n_cells] s(c, e_j) */
    const int32_t *edge_cells;   /* [2][n_edges] c1, c2 */
    const int32_t *edge_verts;   /* [2][n_edges] v1, v2 */
    const int32_t *vert_edges;   /* [6][n_verts] ring edges, -1 pad */
    const int32_t *vert_cells;   /* [6][n_verts] ring cells, -1 pad */
    const int8_t  *vert_sign;    /* [6][n_verts] sigma(v, e_j), 0 on pad */
    const int32_t *vert_valence; /* [n_verts] 5 or 6 */
    /* geometry */
    const double *cell_x;        /* [3][n_cells] unit circumcentre */
    const double *cell_area;     /* [n_cells] m^2 */
    const double *edge_x;        /* [3][n_edges] unit midpoint */
    const double *edge_normal;   /* [3][n_edges] n_e */
    const double *edge_tangent;  /* [3][n_edges] t_e */
    const double *edge_length;   /* [n_edges] primal length l_e [m] */
    const double *dual_length;   /* [n_edges] dual length d_e [m] */
    const double *dual_frac;     /* [n_edges] where the dual arc c1 -> c2 crosses the edge
                                    midpoint, as a fraction of d_e from c1 */
    const double *vert_x;        /* [3][n_verts] unit vectors */
    const double *vert_area;     /* [n_verts] dual area [m^2] */
    /* maps from the current numbering to canonical ids */
    const int32_t *canon_cell;   /* [n_cells] */
    const int32_t *canon_edge;   /* [n_edges] */
    const int32_t *canon_vert;   /* [n_verts] */
} nhgrid_view;

/* Entity counts of R2Bk from the closed forms (no construction). */
void nhgrid_counts(int k, int64_t *n_cells, int64_t *n_edges, int64_t *n_verts);

/* Build R2Bk (0 <= k <= 9) on a sphere of the given radius, canonical order. */
int nhgrid_build(int k, double radius, nhgrid **out);

/* Renumber in place.  order: NHGRID_ORDER_CANONICAL restores canonical ids;
 * NHGRID_ORDER_SFC sorts cells along a 3-D Hilbert curve through the cell
 * centres and numbers edges and vertices by first touch in that cell order;
 * NHGRID_ORDER_CURVE orders cells along a vertex-continuous curve over the
 * bisection tree (each triangle entered at one corner and left at another, its
 * children visited entry corner, centre, third corner, exit corner; the 20
 * root faces chained at shared vertices) and numbers edges and vertices by
 * first touch in that cell order;
 * NHGRID_ORDER_RANDOM applies independent seeded random permutations to cells,
 * edges and vertices (a locality worst case used for invariance tests). */
int nhgrid_reorder(nhgrid *g, int order, uint64_t seed);

/* Fill *view with borrowed pointers into g. */
int nhgrid_get_view(const nhgrid *g, nhgrid_view *view);

void nhgrid_free(nhgrid *g);

/* Message describing the last error on this thread ("" if none). */
const char *nhgrid_last_error(void);

#ifdef __cplusplus
}
#endif
#endif

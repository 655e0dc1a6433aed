/*
 * Mesh topology of the oracle (test infrastructure only).
 *
 * The sphere is meshed from a cube: each cube face is a spherical
 * quadrilateral that is subdivided recursively, every subdivision placing
 * great-circle midpoints on the edges and the great-circle intersection of
 * the two mid-lines at the centre (the geodesic-mesh construction of Section
 * II.a transposed from icosahedral triangles to the cube's quadrilaterals).
 * For 3 * 2^k zones per cube edge the face is first split 3 x 3 at the
 * thirds of its edges (by arc length).
 * The surface mesh is extruded radially into shells with geometrically
 * growing radii (self-similar, "logarithmically ratioed" zones, Section V.b).
 *
 * Everything here is generic and unstructured: zones are hexahedra given by
 * eight vertex ids, faces and edges are found by hashing sorted vertex ids.
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small open-addressing hash map on fixed-length int64 keys           */
typedef struct {
    int klen;
    size_t cap;
    int64_t *keys;
    int *vals;
} hmap;

static void hm_init(hmap *h, int klen, size_t n)
{
    size_t cap = 16;
    while (cap < 2 * n + 16) cap <<= 1;
    h->klen = klen;
    h->cap = cap;
    h->keys = malloc(sizeof(int64_t) * klen * cap);
    h->vals = malloc(sizeof(int) * cap);
    for (size_t i = 0; i < cap; i++) h->vals[i] = -1;
}

static void hm_free(hmap *h) { free(h->keys); free(h->vals); }

static size_t hm_hash(const int64_t *k, int klen)
{
    uint64_t x = 1469598103934665603ull;
    for (int i = 0; i < klen; i++) {
        x ^= (uint64_t)k[i];
        x *= 1099511628211ull;
        x ^= x >> 29;
    }
    return (size_t)x;
}

/* returns existing value, or inserts val and returns -1 */
static int hm_get_or_put(hmap *h, const int64_t *k, int val)
{
    size_t i = hm_hash(k, h->klen) & (h->cap - 1);
    for (;;) {
        if (h->vals[i] < 0) {
            memcpy(&h->keys[i * h->klen], k, sizeof(int64_t) * h->klen);
            h->vals[i] = val;
            return -1;
        }
        if (memcmp(&h->keys[i * h->klen], k, sizeof(int64_t) * h->klen) == 0) return h->vals[i];
        i = (i + 1) & (h->cap - 1);
    }
}

static int hm_get(const hmap *h, const int64_t *k)
{
    size_t i = hm_hash(k, h->klen) & (h->cap - 1);
    for (;;) {
        if (h->vals[i] < 0) return -1;
        if (memcmp(&h->keys[i * h->klen], k, sizeof(int64_t) * h->klen) == 0) return h->vals[i];
        i = (i + 1) & (h->cap - 1);
    }
}

static void sort_i64(int64_t *a, int n)
{
    for (int i = 1; i < n; i++) {
        int64_t t = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > t) { a[j + 1] = a[j]; j--; }
        a[j + 1] = t;
    }
}

/* ------------------------------------------------------------------ */
/* recursive spherical-quad subdivision                                */
static void normalize3(double *a)
{
    double n = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    a[0] /= n; a[1] /= n; a[2] /= n;
}

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void gc_mid(const double *a, const double *b, double *m)
{
    m[0] = a[0] + b[0]; m[1] = a[1] + b[1]; m[2] = a[2] + b[2];
    normalize3(m);
}

/* intersection of the great circle through p1,p2 with the one through q1,q2,
 * on the side of "hint" */
void rgo_gc_intersect(const double *p1, const double *p2, const double *q1, const double *q2,
                      const double *hint, double *out)
{
    double n1[3], n2[3];
    cross3(p1, p2, n1);
    cross3(q1, q2, n2);
    cross3(n1, n2, out);
    normalize3(out);
    if (out[0] * hint[0] + out[1] * hint[1] + out[2] * hint[2] < 0) {
        out[0] = -out[0]; out[1] = -out[1]; out[2] = -out[2];
    }
}

typedef struct {
    hmap vmap;
    int nv, nq, capv;
    double *vert;
    int *quad;
} subdiv_ctx;

static int vertex_id(subdiv_ctx *c, const double *p)
{
    int64_t k[3];
    memcpy(k, p, sizeof(double) * 3);
    int id = hm_get_or_put(&c->vmap, k, c->nv);
    if (id >= 0) return id;
    memcpy(&c->vert[3 * c->nv], p, sizeof(double) * 3);
    return c->nv++;
}

static void subdivide(subdiv_ctx *c, const double *a, const double *b, const double *cc,
                      const double *d, int depth)
{
    if (depth == 0) {
        int *q = &c->quad[4 * c->nq++];
        q[0] = vertex_id(c, a);
        q[1] = vertex_id(c, b);
        q[2] = vertex_id(c, cc);
        q[3] = vertex_id(c, d);
        return;
    }
    double mab[3], mbc[3], mcd[3], mda[3], ctr[3], hint[3];
    gc_mid(a, b, mab);
    gc_mid(b, cc, mbc);
    gc_mid(cc, d, mcd);
    gc_mid(d, a, mda);
    for (int i = 0; i < 3; i++) hint[i] = a[i] + b[i] + cc[i] + d[i];
    rgo_gc_intersect(mab, mcd, mbc, mda, hint, ctr);
    subdivide(c, a, mab, ctr, mda, depth - 1);
    subdivide(c, mab, b, mbc, ctr, depth - 1);
    subdivide(c, ctr, mbc, cc, mcd, depth - 1);
    subdivide(c, mda, ctr, mcd, d, depth - 1);
}

/* cube face frames (outward normal n, tangents u, v with u x v = n) */
static const double CUBE[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{-1, 0, 0}, {0, 0, 1}, {0, 1, 0}},
    {{0, 1, 0}, {0, 0, 1}, {1, 0, 0}},
    {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},
    {{0, 0, 1}, {1, 0, 0}, {0, 1, 0}},
    {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
};

/* the point k/3 (k = 1, 2) of the way along the great-circle arc from a to
 * b: a rotated about the arc's axis by k/3 of the arc's angle (Rodrigues).
 * Always computed from the lexicographically smaller endpoint, so that the
 * two cube faces sharing an edge produce the same bits for its points. */
static int lex_less(const double *a, const double *b)
{
    for (int i = 0; i < 3; i++)
        if (a[i] != b[i]) return a[i] < b[i];
    return 0;
}

static void arc_third(const double *a, const double *b, int k, double *out)
{
    if (!lex_less(a, b)) {
        const double *t = a;
        a = b;
        b = t;
        k = 3 - k;
    }
    double ax[3], w[3];
    cross3(a, b, ax);
    double s = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    double c = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double phi = atan2(s, c) * k / 3.0;
    for (int i = 0; i < 3; i++) ax[i] /= s;
    cross3(ax, a, w);   /* in-plane direction perpendicular to a, toward b */
    for (int i = 0; i < 3; i++) out[i] = cos(phi) * a[i] + sin(phi) * w[i];
    normalize3(out);
}

/* a cube face (corners a, b, cc, d counter-clockwise) split 3 x 3: its edges
 * at their thirds, the interior points where the great circles joining the
 * thirds of opposite edges meet; each part then subdivided depth times */
static void split3(subdiv_ctx *c, const double *a, const double *b, const double *cc, const double *d, int depth)
{
    double P[4][4][3];   /* P[j][i]: i along a -> b, j along a -> d */
    memcpy(P[0][0], a, 24);
    memcpy(P[0][3], b, 24);
    memcpy(P[3][3], cc, 24);
    memcpy(P[3][0], d, 24);
    for (int k = 1; k <= 2; k++) {
        arc_third(a, b, k, P[0][k]);
        arc_third(d, cc, k, P[3][k]);
        arc_third(a, d, k, P[k][0]);
        arc_third(b, cc, k, P[k][3]);
    }
    double hint[3];
    for (int i = 0; i < 3; i++) hint[i] = a[i] + b[i] + cc[i] + d[i];
    for (int j = 1; j <= 2; j++)
        for (int i = 1; i <= 2; i++) rgo_gc_intersect(P[0][i], P[3][i], P[j][0], P[j][3], hint, P[j][i]);
    for (int j = 0; j < 3; j++)
        for (int i = 0; i < 3; i++) subdivide(c, P[j][i], P[j][i + 1], P[j + 1][i + 1], P[j + 1][i], depth);
}

static int build_sphere(rgo_mesh *m)
{
    int N = m->n_ang, depth = 0;
    /* N = 2^depth, or 3 * 2^depth after a first split into 3 x 3 */
    const int three = (N % 3 == 0);
    const int base = three ? 3 : 1;
    while ((base << depth) < N) depth++;
    if ((base << depth) != N || N < 2) return -1;
    subdiv_ctx c;
    c.nv = 0;
    c.nq = 0;
    c.capv = 6 * N * N + 2;
    c.vert = malloc(sizeof(double) * 3 * c.capv);
    c.quad = malloc(sizeof(int) * 4 * 6 * N * N);
    hm_init(&c.vmap, 3, c.capv);
    const double s = 1.0 / sqrt(3.0);
    for (int f = 0; f < 6; f++) {
        double cr[4][3];
        const int ij[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
        for (int k = 0; k < 4; k++)
            for (int d = 0; d < 3; d++)
                cr[k][d] = s * (CUBE[f][0][d] + (2 * ij[k][0] - 1) * CUBE[f][1][d] +
                                (2 * ij[k][1] - 1) * CUBE[f][2][d]);
        if (three) split3(&c, cr[0], cr[1], cr[2], cr[3], depth);
        else subdivide(&c, cr[0], cr[1], cr[2], cr[3], depth);
    }
    hm_free(&c.vmap);
    if (c.nv != 6 * N * N + 2) return -1;
    m->nv = c.nv;
    m->nquad = c.nq;
    m->vert = c.vert;
    m->quad = c.quad;
    return 0;
}

/* ------------------------------------------------------------------ */
/* hexahedral extrusion                                                */

/* local face -> (quad corner, interface offset) of its 4 vertices */
static const int LF_VERT[6][4][2] = {
    {{0, 0}, {3, 0}, {3, 1}, {0, 1}},   /* xi-  */
    {{1, 0}, {2, 0}, {2, 1}, {1, 1}},   /* xi+  */
    {{0, 0}, {1, 0}, {1, 1}, {0, 1}},   /* eta- */
    {{3, 0}, {2, 0}, {2, 1}, {3, 1}},   /* eta+ */
    {{0, 0}, {1, 0}, {2, 0}, {3, 0}},   /* zeta- */
    {{0, 1}, {1, 1}, {2, 1}, {3, 1}},   /* zeta+ */
};

/* local edge -> first and second vertex (quad corner, interface offset);
 * the direction is the positive reference axis */
static const int LE_VERT[12][2][2] = {
    {{0, 0}, {1, 0}}, {{3, 0}, {2, 0}}, {{0, 1}, {1, 1}}, {{3, 1}, {2, 1}},
    {{0, 0}, {3, 0}}, {{1, 0}, {2, 0}}, {{0, 1}, {3, 1}}, {{1, 1}, {2, 1}},
    {{0, 0}, {0, 1}}, {{1, 0}, {1, 1}}, {{3, 0}, {3, 1}}, {{2, 0}, {2, 1}},
};

static int64_t hexv(const rgo_mesh *m, int vid, int kf) { return (int64_t)vid * (m->ktot + 1) + kf; }

int mesh_build_topology(rgo_mesh *m)
{
    if (build_sphere(m)) return -1;
    int K = m->ktot;
    m->radius = malloc(sizeof(double) * (K + 1));
    for (int kf = 0; kf <= K; kf++)
        m->radius[kf] = m->r_in * pow(m->r_out / m->r_in, (double)(kf - m->n_ghost) / m->n_rad);

    m->nz = m->nquad * K;
    int nz = m->nz;
    m->zone_quad = malloc(sizeof(int) * nz);
    m->zone_shell = malloc(sizeof(int) * nz);
    m->zone_face = malloc(sizeof(int) * nz * 6);
    m->zone_edge = malloc(sizeof(int) * nz * 12);
    m->zone_nbr = malloc(sizeof(int) * nz * 6);
    size_t fcap = (size_t)nz * 3 + 4 * m->nquad, ecap = (size_t)nz * 3 + 8 * m->nquad + 8 * m->nv;
    m->face_zone = malloc(sizeof(int) * fcap * 2);
    m->face_lf = malloc(sizeof(int) * fcap * 2);
    m->edge_hv = malloc(sizeof(int) * ecap * 2);
    m->edge_nz = calloc(ecap, sizeof(int));
    m->edge_zone = malloc(sizeof(int) * ecap * 4);
    m->edge_le = malloc(sizeof(int) * ecap * 4);
    m->edge_rev = malloc(sizeof(int) * ecap * 4);
    hmap fm, em;
    hm_init(&fm, 4, fcap);
    hm_init(&em, 2, ecap);
    int nf = 0, ne = 0;
    for (int qd = 0; qd < m->nquad; qd++)
        for (int k = 0; k < K; k++) {
            int z = qd * K + k;
            m->zone_quad[z] = qd;
            m->zone_shell[z] = k;
            const int *qv = &m->quad[4 * qd];
            for (int lf = 0; lf < 6; lf++) {
                int64_t key[4];
                for (int i = 0; i < 4; i++)
                    key[i] = hexv(m, qv[LF_VERT[lf][i][0]], k + LF_VERT[lf][i][1]);
                sort_i64(key, 4);
                int f = hm_get_or_put(&fm, key, nf);
                if (f < 0) {
                    f = nf++;
                    m->face_zone[2 * f] = z;
                    m->face_lf[2 * f] = lf;
                    m->face_zone[2 * f + 1] = -1;
                    m->face_lf[2 * f + 1] = -1;
                } else {
                    m->face_zone[2 * f + 1] = z;
                    m->face_lf[2 * f + 1] = lf;
                }
                m->zone_face[6 * z + lf] = f;
            }
            for (int le = 0; le < 12; le++) {
                int64_t a = hexv(m, qv[LE_VERT[le][0][0]], k + LE_VERT[le][0][1]);
                int64_t b = hexv(m, qv[LE_VERT[le][1][0]], k + LE_VERT[le][1][1]);
                int64_t key[2] = {a < b ? a : b, a < b ? b : a};
                int e = hm_get_or_put(&em, key, ne);
                if (e < 0) {
                    e = ne++;
                    m->edge_hv[2 * e] = (int)key[0];
                    m->edge_hv[2 * e + 1] = (int)key[1];
                }
                int s = m->edge_nz[e]++;
                if (s >= 4) return -1;
                m->edge_zone[4 * e + s] = z;
                m->edge_le[4 * e + s] = le;
                m->edge_rev[4 * e + s] = (a > b);
                m->zone_edge[12 * z + le] = e;
            }
        }
    hm_free(&fm);
    hm_free(&em);
    m->nf = nf;
    m->ne = ne;
    for (int z = 0; z < nz; z++)
        for (int lf = 0; lf < 6; lf++) {
            int f = m->zone_face[6 * z + lf];
            int o = m->face_zone[2 * f] == z ? m->face_zone[2 * f + 1] : m->face_zone[2 * f];
            m->zone_nbr[6 * z + lf] = o;
        }

    /* vertex -> zones, for the vertex-sharing stencil */
    int nhv = m->nv * (K + 1);
    int *cnt = calloc(nhv + 1, sizeof(int));
    for (int z = 0; z < nz; z++) {
        const int *qv = &m->quad[4 * m->zone_quad[z]];
        for (int c = 0; c < 4; c++)
            for (int dk = 0; dk < 2; dk++) cnt[hexv(m, qv[c], m->zone_shell[z] + dk) + 1]++;
    }
    for (int i = 0; i < nhv; i++) cnt[i + 1] += cnt[i];
    int *vz = malloc(sizeof(int) * cnt[nhv]);
    int *fill = calloc(nhv, sizeof(int));
    for (int z = 0; z < nz; z++) {
        const int *qv = &m->quad[4 * m->zone_quad[z]];
        for (int c = 0; c < 4; c++)
            for (int dk = 0; dk < 2; dk++) {
                int64_t h = hexv(m, qv[c], m->zone_shell[z] + dk);
                vz[cnt[h] + fill[h]++] = z;
            }
    }
    m->st_n = calloc(nz, sizeof(int));
    m->st_z = malloc(sizeof(int) * nz * RGO_MAXST);
    for (int z = 0; z < nz; z++) {
        int n = 0;
        int *st = &m->st_z[RGO_MAXST * z];
        const int *qv = &m->quad[4 * m->zone_quad[z]];
        for (int c = 0; c < 4; c++)
            for (int dk = 0; dk < 2; dk++) {
                int64_t h = hexv(m, qv[c], m->zone_shell[z] + dk);
                for (int i = cnt[h]; i < cnt[h + 1]; i++) {
                    int o = vz[i];
                    if (o == z) continue;
                    int dup = 0;
                    for (int j = 0; j < n; j++) dup |= (st[j] == o);
                    if (!dup) st[n++] = o;
                }
            }
        if (m->order == 4) {
            /* across each face neighbour's opposite face */
            for (int lf = 0; lf < 6; lf++) {
                int z1 = m->zone_nbr[6 * z + lf];
                if (z1 < 0) continue;
                int lf1 = -1;
                for (int j = 0; j < 6; j++)
                    if (m->zone_nbr[6 * z1 + j] == z && m->zone_face[6 * z1 + j] == m->zone_face[6 * z + lf]) lf1 = j;
                if (lf1 < 0) continue;
                int z2 = m->zone_nbr[6 * z1 + (lf1 ^ 1)];
                if (z2 < 0 || z2 == z) continue;
                int dup = 0;
                for (int j = 0; j < n; j++) dup |= (st[j] == z2);
                if (!dup) st[n++] = z2;
            }
        }
        m->st_n[z] = n;
    }
    free(cnt); free(vz); free(fill);
    return 0;
}

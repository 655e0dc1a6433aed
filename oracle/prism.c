/*
 * Triangular-prism element of the oracle (TEST INFRASTRUCTURE ONLY: only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; it shares no code with the GPU library).
 *
 * - The reference element is the equilateral prism with unit edges and its
 *   centroid at the origin (Appendices B-D): triangle vertices
 *   (-1/2, -1/(2 sqrt 3)), (1/2, -1/(2 sqrt 3)), (0, 1/sqrt 3), zeta in
 *   [-1/2, 1/2].  Nodes (Fig. 7): the six vertices; at third order the
 *   vertical-edge midpoints and the triangle-edge midpoints; at fourth order
 *   the vertical-edge thirds, the triangle-edge thirds and the two triangle
 *   centroids, numbered as in eqs. (C.2)-(C.16) and (D.2)-(D.27).
 *   Appendix B prints the second-order nodes with a vertex at the origin,
 *   but its bases (B.10)-(B.15) are those of the centred prism; the centred
 *   prism is used at every order.
 * - Monomials of eqs. (5.12)-(5.14); nodal Lagrange basis by eq. (5.3).
 * - Space-time Galerkin system of eqs. (5.24)-(5.29) integrated over the
 *   prism: a collapsed (Duffy) Gauss rule on the triangle times Gauss points
 *   in zeta, exact for the integrands' degrees.
 * - Geometry of a zone of the icosahedral geodesic mesh (Sections II.a-II.b):
 *   the zone's spherical triangle (vertices a, b, c on the unit sphere,
 *   counter-clockwise seen from outside) is interpolated by a triangle
 *   Lagrange map of degree order-1 through nodes on the sphere -- vertices,
 *   equidistant points along the great-circle edges and, for the cubic map,
 *   the spherical centroid (a + b + c)/|a + b + c|, where the three
 *   great-circle medians meet -- and the radial direction is linear:
 *   x = [(1/2 - zeta) r0 + (1/2 + zeta) r1] S(xi, eta).
 *   At the element nodes: position, Jacobian, and the flux metrics of
 *   eq. (5.11) in the conservative curl form (their discrete divergence
 *   vanishes, so a uniform state stays uniform).
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int rgo_predict_element(const rgo_refel *r, double gamma, double dt, const double *J, const double *met,
                        const double *Ua, double *Ulev, double *avgU, double *avgF);

static const double S3 = 1.7320508075688772935;

/* triangle vertices of the reference prism */
static void tri_vertex(int k, double *v)
{
    static const double vx[3] = {-0.5, 0.5, 0.0};
    v[0] = vx[k];
    v[1] = (k == 2) ? 1.0 / S3 : -0.5 / S3;
}

static int add_node(rgo_refel *r, int n, double x, double y, double z)
{
    r->node[n][0] = x;
    r->node[n][1] = y;
    r->node[n][2] = z;
    return n + 1;
}

/* point at fraction t along the triangle edge from vertex k to vertex k+1 */
static void tri_edge_point(int k, double t, double *p)
{
    double a[2], b[2];
    tri_vertex(k, a);
    tri_vertex((k + 1) % 3, b);
    p[0] = a[0] + t * (b[0] - a[0]);
    p[1] = a[1] + t * (b[1] - a[1]);
}

/* nodes of Fig. 7 in the numbering of Appendices B-D */
static int prism_nodes(rgo_refel *r, int order)
{
    int n = 0;
    double v[2], p[2];
    for (int s = 0; s < 2; s++)            /* vertices: top (zeta = 1/2), then bottom */
        for (int k = 0; k < 3; k++) { tri_vertex(k, v); n = add_node(r, n, v[0], v[1], s ? -0.5 : 0.5); }
    if (order == 3) {
        for (int k = 0; k < 3; k++) { tri_vertex(k, v); n = add_node(r, n, v[0], v[1], 0.0); }
        for (int s = 0; s < 2; s++)
            for (int k = 0; k < 3; k++) { tri_edge_point(k, 0.5, p); n = add_node(r, n, p[0], p[1], s ? -0.5 : 0.5); }
    } else if (order == 4) {
        for (int s = 0; s < 2; s++)
            for (int k = 0; k < 3; k++) { tri_vertex(k, v); n = add_node(r, n, v[0], v[1], s ? -1.0 / 6.0 : 1.0 / 6.0); }
        for (int s = 0; s < 2; s++)
            for (int k = 0; k < 3; k++)
                for (int t = 1; t <= 2; t++) {
                    tri_edge_point(k, t / 3.0, p);
                    n = add_node(r, n, p[0], p[1], s ? -0.5 : 0.5);
                }
        n = add_node(r, n, 0.0, 0.0, 0.5);
        n = add_node(r, n, 0.0, 0.0, -0.5);
    }
    return n;
}

/* monomial exponents (a, b, c) of xi^a eta^b zeta^c, eqs. (5.12)-(5.14) */
static const int MONO2[6][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {0, 1, 1}};
static const int MONO3[15][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0},
                                 {1, 0, 1}, {0, 1, 1}, {1, 1, 1}, {2, 0, 1}, {0, 2, 1}, {1, 0, 2}, {0, 1, 2}};
static const int MONO4[26][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2},
                                 {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {3, 0, 0}, {0, 3, 0}, {0, 0, 3}, {2, 1, 0},
                                 {2, 0, 1}, {1, 2, 0}, {0, 2, 1}, {1, 0, 2}, {0, 1, 2}, {1, 1, 1}, {1, 0, 3},
                                 {0, 1, 3}, {3, 0, 1}, {0, 3, 1}, {2, 1, 1}, {1, 2, 1}};

/* nodes, monomials and the nodal basis only */
static int prism_basis_init(rgo_refel *r, int order)
{
    memset(r, 0, sizeof(*r));
    if (order < 2 || order > 4) return -1;
    r->order = order;
    r->N = prism_nodes(r, order);
    const int(*mono)[3] = order == 2 ? MONO2 : order == 3 ? MONO3 : MONO4;
    for (int k = 0; k < r->N; k++) memcpy(r->exps[k], mono[k], sizeof(int) * 3);
    return lagrange3(r->N, &r->node[0][0], &r->exps[0][0], r->coef);
}

int prism_refel_init(rgo_refel *r, int order)
{
    if (prism_basis_init(r, order)) return -1;

    /* prism quadrature: on the triangle x = V1 + s (V2 - V1) + t (V3 - V1),
     * t = (1 - s) w, dA = 2 |T| (1 - s) ds dw with |T| = sqrt(3)/4; six
     * Gauss points in s, w and zeta integrate degree 11, above the degree 9
     * of psi_i dpsi_l psi_j */
    const int ng = 6;
    double gx[8], gw[8], v1[2], v2[2], v3[2];
    gauss01(ng, gx, gw);
    tri_vertex(0, v1);
    tri_vertex(1, v2);
    tri_vertex(2, v3);
    const int nq = ng * ng * ng;
    double *xq = malloc(sizeof(double) * 3 * nq), *wq = malloc(sizeof(double) * nq);
    int n = 0;
    for (int i = 0; i < ng; i++)
        for (int j = 0; j < ng; j++)
            for (int k = 0; k < ng; k++) {
                double s = gx[i], t = (1.0 - s) * gx[j];
                xq[3 * n] = v1[0] + s * (v2[0] - v1[0]) + t * (v3[0] - v1[0]);
                xq[3 * n + 1] = v1[1] + s * (v2[1] - v1[1]) + t * (v3[1] - v1[1]);
                xq[3 * n + 2] = gx[k] - 0.5;
                wq[n++] = 2.0 * (S3 / 4.0) * (1.0 - s) * gw[i] * gw[j] * gw[k];
            }
    int rc = refel_spacetime(r, order, nq, xq, wq);
    free(xq);
    free(wq);
    return rc;
}

/* ---------------------------------------------------------------- geometry */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void unit3(double *a)
{
    double n = sqrt(dot3(a, a));
    for (int i = 0; i < 3; i++) a[i] /= n;
}

/* point at fraction t of the central angle along the great circle from a to b */
static void great_circle_point(const double *a, const double *b, double t, double *p)
{
    double om = acos(fmax(-1.0, fmin(1.0, dot3(a, b)))), s = sin(om);
    double wa = sin((1.0 - t) * om) / s, wb = sin(t * om) / s;
    for (int i = 0; i < 3; i++) p[i] = wa * a[i] + wb * b[i];
}

typedef struct {
    int mo, nm;
    double node[10][3];     /* reference-triangle lattice nodes (zeta = 0) */
    int exps[10][3];
    double coef[100];
    double sph[10][3];      /* the matching points on the unit sphere */
} tri_map;

/* lattice nodes (i, j, k)/mo in barycentric coordinates and their points on
 * the sphere for the spherical triangle (a, b, c) */
static int tri_map_init(tri_map *t, int mo, const double *a, const double *b, const double *c)
{
    const double *P[3] = {a, b, c};
    double V[3][2];
    for (int k = 0; k < 3; k++) tri_vertex(k, V[k]);
    t->mo = mo;
    int n = 0;
    for (int i = mo; i >= 0; i--)
        for (int j = mo - i; j >= 0; j--) {
            int k = mo - i - j;
            double l[3] = {(double)i / mo, (double)j / mo, (double)k / mo};
            t->node[n][0] = l[0] * V[0][0] + l[1] * V[1][0] + l[2] * V[2][0];
            t->node[n][1] = l[0] * V[0][1] + l[1] * V[1][1] + l[2] * V[2][1];
            t->node[n][2] = 0.0;
            int nzero = (i == 0) + (j == 0) + (k == 0);
            if (nzero == 2) {
                const double *v = i ? a : j ? b : c;
                memcpy(t->sph[n], v, sizeof(double) * 3);
            } else if (nzero == 1) {
                /* on the edge between the two vertices with nonzero weight */
                int p = i == 0 ? 1 : 0, q = k == 0 ? 1 : 2;
                great_circle_point(P[p], P[q], l[q] / (l[p] + l[q]), t->sph[n]);
            } else {
                for (int d = 0; d < 3; d++) t->sph[n][d] = a[d] + b[d] + c[d];
                unit3(t->sph[n]);
            }
            n++;
        }
    t->nm = n;
    n = 0;
    for (int e = 0; e <= mo; e++)
        for (int f = 0; e + f <= mo; f++) {
            t->exps[n][0] = e;
            t->exps[n][1] = f;
            t->exps[n][2] = 0;
            n++;
        }
    return lagrange3(t->nm, &t->node[0][0], &t->exps[0][0], t->coef);
}

/* x(xi) and jac[i][j] = d x_i / d xi_j */
static void prism_map(const tri_map *t, double r0, double r1, const double *xi, double *x, double *jac)
{
    double S[3] = {0, 0, 0}, Sx[3] = {0, 0, 0}, Sy[3] = {0, 0, 0};
    for (int l = 0; l < t->nm; l++) {
        double p = 0.0, px = 0.0, py = 0.0;
        for (int k = 0; k < t->nm; k++) {
            double ck = t->coef[k * t->nm + l];
            p += ck * mono3(t->exps[k], xi);
            px += ck * dmono3(t->exps[k], 0, xi);
            py += ck * dmono3(t->exps[k], 1, xi);
        }
        for (int d = 0; d < 3; d++) {
            S[d] += p * t->sph[l][d];
            Sx[d] += px * t->sph[l][d];
            Sy[d] += py * t->sph[l][d];
        }
    }
    double R = (0.5 - xi[2]) * r0 + (0.5 + xi[2]) * r1, dR = r1 - r0;
    for (int d = 0; d < 3; d++) {
        x[d] = R * S[d];
        jac[d * 3 + 0] = R * Sx[d];
        jac[d * 3 + 1] = R * Sy[d];
        jac[d * 3 + 2] = dR * S[d];
    }
}

static double det3(const double *j)
{
    return j[0] * (j[4] * j[8] - j[5] * j[7]) - j[1] * (j[3] * j[8] - j[5] * j[6]) + j[2] * (j[3] * j[7] - j[4] * j[6]);
}

/* node positions x[N][3], Jacobians J[N] and curl-form metrics
 * met[N][d][n] = J d xi_d / d x_n of one zone */
static int zone_geometry(const rgo_refel *r, const double *a, const double *b, const double *c, double r0,
                         double r1, double *x, double *J, double *met)
{
    tri_map t;
    if (tri_map_init(&t, r->order - 1, a, b, c)) return -1;
    const int N = r->N;
    double *jac = malloc(sizeof(double) * N * 9), cen[3] = {0, 0, 0};
    for (int i = 0; i < N; i++) {
        prism_map(&t, r0, r1, r->node[i], &x[3 * i], &jac[9 * i]);
        J[i] = det3(&jac[9 * i]);
        for (int d = 0; d < 3; d++) cen[d] += x[3 * i + d] / N;
    }
    /* V[i][n][j] = (x_l - c_l) d x_m / d xi_j with (n, m, l) cyclic;
     * (J a^d)_n = -(curl_xi of the interpolated V_n)_d */
    double *V = malloc(sizeof(double) * N * 9);
    for (int i = 0; i < N; i++)
        for (int nn = 0; nn < 3; nn++) {
            int mm = (nn + 1) % 3, ll = (nn + 2) % 3;
            for (int j = 0; j < 3; j++) V[i * 9 + nn * 3 + j] = (x[3 * i + ll] - cen[ll]) * jac[9 * i + mm * 3 + j];
        }
    for (int i = 0; i < N; i++)
        for (int nn = 0; nn < 3; nn++) {
            double dV[3][3] = {{0}};
            for (int l = 0; l < N; l++)
                for (int d = 0; d < 3; d++) {
                    double dp = refel_dpsi(r, l, d, r->node[i]);
                    for (int j = 0; j < 3; j++) dV[j][d] += V[l * 9 + nn * 3 + j] * dp;
                }
            met[i * 9 + 0 * 3 + nn] = -(dV[2][1] - dV[1][2]);
            met[i * 9 + 1 * 3 + nn] = -(dV[0][2] - dV[2][0]);
            met[i * 9 + 2 * 3 + nn] = -(dV[1][0] - dV[0][1]);
        }
    free(V);
    free(jac);
    return 0;
}

/* geometry of nz zones: abc[z] = the triangle's vertices a, b, c (9
 * doubles), r01[z] = inner and outer radius; x[z][N][3], J[z][N],
 * met[z][N][9] */
int rgo_prism_geometry(int order, int nz, const double *abc, const double *r01, double *x, double *J, double *met)
{
    rgo_refel r;
    if (prism_basis_init(&r, order)) return -1;
    const int N = r.N;
    int rc = 0;
    for (int z = 0; z < nz && !rc; z++)
        rc = zone_geometry(&r, &abc[9 * z], &abc[9 * z + 3], &abc[9 * z + 6], r01[2 * z], r01[2 * z + 1],
                           &x[(size_t)z * N * 3], &J[(size_t)z * N], &met[(size_t)z * N * 9]);
    return rc;
}

/* reference-element matrices (as rgo_refel_query, for the prism) */
int rgo_prism_refel_query(int order, int *NM, double *tau, double *wt, double *nodes, int *exps, double *coef,
                          double *D, double *Kd, double *Kd0, double *Kt0)
{
    rgo_refel r;
    if (prism_refel_init(&r, order)) return -1;
    int N = r.N, M = r.M, E = (M - 1) * N;
    NM[0] = N;
    NM[1] = M;
    if (tau) memcpy(tau, r.tau, sizeof(double) * M);
    if (wt) memcpy(wt, r.wt, sizeof(double) * M);
    if (nodes) memcpy(nodes, r.node, sizeof(double) * 3 * N);
    if (exps) memcpy(exps, r.exps, sizeof(int) * 3 * N);
    if (coef)
        for (int k = 0; k < N; k++)
            for (int l = 0; l < N; l++) coef[k * N + l] = r.coef[k * N + l];
    if (D)
        for (int d = 0; d < 3; d++)
            for (int i = 0; i < N; i++)
                for (int l = 0; l < N; l++) D[(d * N + i) * N + l] = refel_dpsi(&r, l, d, r.node[i]);
    for (int d = 0; d < 3; d++) {
        if (Kd) memcpy(&Kd[(size_t)d * E * E], r.Kd[d], sizeof(double) * E * E);
        if (Kd0) memcpy(&Kd0[(size_t)d * E * N], r.Kd0[d], sizeof(double) * E * N);
    }
    if (Kt0) memcpy(Kt0, r.Kt0, sizeof(double) * E * N);
    refel_free(&r);
    return 0;
}

/* the ADER-CG predictor (Section V.d) of nz prism zones, one after another:
 * J[z][N], met[z][N][9], Ua[z][N][8] node-major as in rgo_predict_element;
 * Ulev[z][M][N][8] (J times the state at every time level; may be NULL),
 * avgU[z][N][8], avgF[z][N][3][8] */
int rgo_prism_predict(int order, int nz, double gamma, double dt, const double *J, const double *met,
                      const double *Ua, double *Ulev, double *avgU, double *avgF)
{
    rgo_refel r;
    if (prism_refel_init(&r, order)) return -1;
    const int N = r.N;
    int rc = 0;
    for (int z = 0; z < nz && !rc; z++)
        rc = rgo_predict_element(&r, gamma, dt, &J[(size_t)z * N], &met[(size_t)z * N * 9],
                                 &Ua[(size_t)z * N * NVAR], Ulev ? &Ulev[(size_t)z * r.M * N * NVAR] : NULL,
                                 &avgU[(size_t)z * N * NVAR],
                                 &avgF[(size_t)z * N * 3 * NVAR]);
    refel_free(&r);
    return rc;
}

/* ---------------------------------------------------------------- face traces
 * Face quadrature of Appendix A.  The rules are printed for the triangle
 * with vertices (0, 0), (1, 0), (1/2, sqrt 3 / 2) and the unit square; the
 * triangle points are moved to the centred reference triangle.  Triangle
 * faces: (A.1), (A.3), (A.5) at orders 2, 3, 4; the three quadrilateral side
 * faces: (A.2), (A.4), (A.6), with x along the triangle edge from vertex k to
 * vertex k+1 and y along zeta from -1/2 to 1/2.  Points are listed face by
 * face: zeta = +1/2, zeta = -1/2, then side faces k = 0, 1, 2.  Weights are
 * fractions of the face's reference area (they sum to one per face). */
static int tri_rule(int order, double (*p)[2], double *w)
{
    const double r3 = S3;
    if (order == 2) {
        const double P[3][3] = {{0.25, 0.25 / r3, 1.0 / 3}, {0.75, 0.25 / r3, 1.0 / 3}, {0.5, 1.0 / r3, 1.0 / 3}};
        for (int i = 0; i < 3; i++) { p[i][0] = P[i][0]; p[i][1] = P[i][1]; w[i] = P[i][2]; }
        return 3;
    }
    if (order == 3) {
        const double P[6][3] = {{0.125, 0.125 / r3, 0.125}, {0.875, 0.125 / r3, 0.125}, {0.5, 1.25 / r3, 0.125},
                                {0.375, r3 / 8, 5.0 / 24}, {0.625, r3 / 8, 5.0 / 24}, {0.5, r3 / 4, 5.0 / 24}};
        for (int i = 0; i < 6; i++) { p[i][0] = P[i][0]; p[i][1] = P[i][1]; w[i] = P[i][2]; }
        return 6;
    }
    const double a = 32.0 / 405, b = 14.0 / 135, c = 19.0 / 135;
    const double P[10][3] = {{0.125, r3 / 24, a},       {0.875, r3 / 24, a},       {0.5, 5 * r3 / 12, a},
                             {0.375, r3 / 24, b},       {0.625, r3 / 24, b},       {0.75, r3 / 6, b},
                             {0.625, 7 * r3 / 24, b},   {0.375, 7 * r3 / 24, b},   {0.25, r3 / 6, b},
                             {0.5, r3 / 6, c}};
    for (int i = 0; i < 10; i++) { p[i][0] = P[i][0]; p[i][1] = P[i][1]; w[i] = P[i][2]; }
    return 10;
}

static int square_rule(int order, double (*p)[2], double *w)
{
    const double g = 0.5 / S3, h = 0.5 * sqrt(3.0 / 5.0);
    if (order == 2) {
        const double P[3][3] = {{0.5 - g, 0.5 + g, 0.25}, {0.5 + g, 0.5 + g, 0.25}, {0.5, 0.5 - g, 0.5}};
        for (int i = 0; i < 3; i++) { p[i][0] = P[i][0]; p[i][1] = P[i][1]; w[i] = P[i][2]; }
        return 3;
    }
    if (order == 3) {
        const double P[4][3] = {{0.5 - g, 0.5 - g, 0.25}, {0.5 + g, 0.5 - g, 0.25}, {0.5 - g, 0.5 + g, 0.25},
                                {0.5 + g, 0.5 + g, 0.25}};
        for (int i = 0; i < 4; i++) { p[i][0] = P[i][0]; p[i][1] = P[i][1]; w[i] = P[i][2]; }
        return 4;
    }
    const double P[6][3] = {{0.5 - g, 0.5 - h, 5.0 / 36}, {0.5 + g, 0.5 - h, 5.0 / 36}, {0.5 - g, 0.5 + h, 5.0 / 36},
                            {0.5 + g, 0.5 + h, 5.0 / 36}, {0.5 - g, 0.5, 2.0 / 9},      {0.5 + g, 0.5, 2.0 / 9}};
    for (int i = 0; i < 6; i++) { p[i][0] = P[i][0]; p[i][1] = P[i][1]; w[i] = P[i][2]; }
    return 6;
}

/* reference points xi[q][3] and weights w[q] of all five faces; returns the
 * number of points (nt per triangle face in *nt, ns per side face in *ns) */
int rgo_prism_face_points(int order, double *xi, double *w, int *nt, int *ns)
{
    if (order < 2 || order > 4) return -1;
    double tp[10][2], tw[10], sp[6][2], sw[6], V[3][2];
    const int t = tri_rule(order, tp, tw), s = square_rule(order, sp, sw);
    for (int k = 0; k < 3; k++) tri_vertex(k, V[k]);
    /* the printed triangle has its first vertex at the origin: shift by the
     * centred triangle's first vertex */
    int q = 0;
    for (int f = 0; f < 2; f++)
        for (int i = 0; i < t; i++, q++) {
            xi[3 * q] = tp[i][0] + V[0][0];
            xi[3 * q + 1] = tp[i][1] + V[0][1];
            xi[3 * q + 2] = f == 0 ? 0.5 : -0.5;
            w[q] = tw[i];
        }
    for (int k = 0; k < 3; k++)
        for (int i = 0; i < s; i++, q++) {
            const double *a = V[k], *b = V[(k + 1) % 3];
            xi[3 * q] = a[0] + sp[i][0] * (b[0] - a[0]);
            xi[3 * q + 1] = a[1] + sp[i][0] * (b[1] - a[1]);
            xi[3 * q + 2] = sp[i][1] - 0.5;
            w[q] = sw[i];
        }
    *nt = t;
    *ns = s;
    return q;
}

/* traces of the time-averaged state and flux at the face points:
 * tr[z][q][0..8) = sum_l psi_l(xi_q) avgU[z][l], tr[z][q][8 + 8 d + v] the
 * same of avgF[z][l][d][v] */
int rgo_prism_traces(int order, int nz, const double *avgU, const double *avgF, double *tr)
{
    rgo_refel r;
    if (prism_basis_init(&r, order)) return -1;
    double xi[38 * 3], w[38];
    int nt, ns;
    const int Q = rgo_prism_face_points(order, xi, w, &nt, &ns), N = r.N;
    double *psi = malloc(sizeof(double) * Q * N);
    for (int q = 0; q < Q; q++)
        for (int l = 0; l < N; l++) psi[q * N + l] = refel_psi(&r, l, &xi[3 * q]);
    for (int z = 0; z < nz; z++)
        for (int q = 0; q < Q; q++) {
            double *o = &tr[((size_t)z * Q + q) * 32];
            for (int k = 0; k < 32; k++) o[k] = 0.0;
            for (int l = 0; l < N; l++) {
                const double p = psi[q * N + l];
                const double *u = &avgU[((size_t)z * N + l) * 8], *f = &avgF[((size_t)z * N + l) * 24];
                for (int v = 0; v < 8; v++) o[v] += p * u[v];
                for (int k = 0; k < 24; k++) o[8 + k] += p * f[k];
            }
        }
    free(psi);
    return 0;
}

/* ---------------------------------------------------------------- face fluxes
 * Geometry of the face points of nz zones: positions xq[z][Q][3] and the
 * outward area vectors dAw[z][Q][3], each the rule's weight times the face's
 * reference area (sqrt 3 / 4 for the triangles, 1 for the side faces) times
 * the cross product of the map's tangents: d x / d xi x d x / d eta on the
 * triangle faces (sign + on zeta = 1/2, - on zeta = -1/2), and on side face k
 * (d x / d s) x (d x / d zeta) with s along the edge from vertex k to k + 1,
 * which points out of a counter-clockwise triangle. */
int rgo_prism_face_geometry(int order, int nz, const double *abc, const double *r01, double *xq, double *dAw)
{
    rgo_refel r;
    if (prism_basis_init(&r, order)) return -1;
    double xi[38 * 3], w[38], V[3][2];
    int nt, ns;
    const int Q = rgo_prism_face_points(order, xi, w, &nt, &ns);
    for (int k = 0; k < 3; k++) tri_vertex(k, V[k]);
    for (int z = 0; z < nz; z++) {
        tri_map t;
        if (tri_map_init(&t, order - 1, &abc[9 * z], &abc[9 * z + 3], &abc[9 * z + 6])) return -1;
        for (int q = 0; q < Q; q++) {
            double jac[9], a[3], b[3], c[3];
            prism_map(&t, r01[2 * z], r01[2 * z + 1], &xi[3 * q], &xq[((size_t)z * Q + q) * 3], jac);
            double scale;
            if (q < 2 * nt) {
                for (int i = 0; i < 3; i++) { a[i] = jac[3 * i]; b[i] = jac[3 * i + 1]; }
                scale = (q < nt ? 1.0 : -1.0) * (S3 / 4.0) * w[q];
            } else {
                const int k = (q - 2 * nt) / ns;
                const double ex = V[(k + 1) % 3][0] - V[k][0], ey = V[(k + 1) % 3][1] - V[k][1];
                for (int i = 0; i < 3; i++) { a[i] = jac[3 * i] * ex + jac[3 * i + 1] * ey; b[i] = jac[3 * i + 2]; }
                scale = w[q];
            }
            c[0] = a[1] * b[2] - a[2] * b[1];
            c[1] = a[2] * b[0] - a[0] * b[2];
            c[2] = a[0] * b[1] - a[1] * b[0];
            for (int i = 0; i < 3; i++) dAw[((size_t)z * Q + q) * 3 + i] = scale * c[i];
        }
    }
    return 0;
}

/* HLL (Section II.c, as for the hexahedra) at np points: left and right
 * states U[np][8] and Cartesian fluxes F[np][3][8] (the traces of the
 * time averages), unit normals n[np][3] from left to right; Fs[np][8] */
void rgo_prism_hll(int np, const double *UL, const double *UR, const double *FL, const double *FR, const double *n,
                   double gamma, double *Fs)
{
    for (int p = 0; p < np; p++) {
        double FnL[NVAR], FnR[NVAR];
        const double *nn = &n[3 * p];
        for (int v = 0; v < NVAR; v++) {
            FnL[v] = nn[0] * FL[p * 24 + v] + nn[1] * FL[p * 24 + 8 + v] + nn[2] * FL[p * 24 + 16 + v];
            FnR[v] = nn[0] * FR[p * 24 + v] + nn[1] * FR[p * 24 + 8 + v] + nn[2] * FR[p * 24 + 16 + v];
        }
        hll_flux(&UL[p * NVAR], &UR[p * NVAR], FnL, FnR, nn, gamma, &Fs[p * NVAR]);
    }
}

/* zone volumes by a collapsed Gauss rule on the triangle times Gauss points
 * in zeta (six each way), exact for the maps' Jacobians */
int rgo_prism_volumes(int order, int nz, const double *abc, const double *r01, double *vol)
{
    const int ng = 6;
    double gx[8], gw[8], v1[2], v2[2], v3[2];
    gauss01(ng, gx, gw);
    tri_vertex(0, v1);
    tri_vertex(1, v2);
    tri_vertex(2, v3);
    for (int z = 0; z < nz; z++) {
        tri_map t;
        if (tri_map_init(&t, order - 1, &abc[9 * z], &abc[9 * z + 3], &abc[9 * z + 6])) return -1;
        double V = 0.0;
        for (int i = 0; i < ng; i++)
            for (int j = 0; j < ng; j++)
                for (int k = 0; k < ng; k++) {
                    double s = gx[i], tt = (1.0 - s) * gx[j], xi[3], x[3], jac[9];
                    xi[0] = v1[0] + s * (v2[0] - v1[0]) + tt * (v3[0] - v1[0]);
                    xi[1] = v1[1] + s * (v2[1] - v1[1]) + tt * (v3[1] - v1[1]);
                    xi[2] = gx[k] - 0.5;
                    prism_map(&t, r01[2 * z], r01[2 * z + 1], xi, x, jac);
                    V += 2.0 * (S3 / 4.0) * (1.0 - s) * gw[i] * gw[j] * gw[k] * det3(jac);
                }
        vol[z] = V;
    }
    return 0;
}

/* ---------------------------------------------------------------- divergence-free B
 * Section IV.b on the prism (five faces).  Per zone, in the zone's Taylor
 * frame X = (x - centroid) / l0, l0 = V^(1/3): each component carries the
 * monomials of degree <= p-1 and the degree-p monomials containing its own
 * coordinate (eqs. 4.1, 4.4, 4.7 generalised), each non-constant one minus its
 * zone mean.  Least squares: the coefficients of degree <= p-1 towards the
 * WENO-AO ones (the extras towards zero) (eqs. 4.3, 4.6, 4.9), and the normal
 * component at every face point towards the face's nodal normal B
 * (eq. 4.15).  Constraints: the divergence identities of eq. (4.10) without
 * its first member (the multi-indices 1 <= |mu| <= p-1) and the five face
 * averages (eq. 4.14) by each face's rule.  Inputs per zone, NIN values:
 * for each component its zone mean and its Taylor coefficients of degree
 * 1..p-1 (degree by degree, x exponent descending, then y descending), then
 * the normal B at the Q face points along the zone's outward normal (in the
 * order of rgo_prism_face_points), then the five outward face averages (faces
 * zeta = +1/2, -1/2, sides 0, 1, 2).  Outputs, 3N + 3 values: B at the N
 * element nodes (x components, then y, then z), then the three zone means of
 * the reconstruction. */
static int taylor_multi(int deg, int e[][3])
{
    int n = 0;
    for (int d = 1; d <= deg; d++)
        for (int a = d; a >= 0; a--)
            for (int b = d - a; b >= 0; b--) { e[n][0] = a; e[n][1] = b; e[n][2] = d - a - b; n++; }
    return n;
}

int rgo_prism_divfree(int order, int nz, const double *abc, const double *r01, const double *Bin, double *Bout)
{
    rgo_refel r;
    if (prism_basis_init(&r, order)) return -1;
    const int p = order, N = r.N;
    int te[40][3];
    const int nc = taylor_multi(p - 1, te);
    /* B basis of each component: constant, Taylor multi-indices, degree-p extras */
    int be[3][64][3], nb = 0;
    for (int c = 0; c < 3; c++) {
        int k = 0;
        be[c][k][0] = be[c][k][1] = be[c][k][2] = 0; k++;
        for (int a = 0; a < nc; a++) { memcpy(be[c][k], te[a], sizeof(int) * 3); k++; }
        for (int a = p; a >= 0; a--)
            for (int b = p - a; b >= 0; b--) {
                int e[3] = {a, b, p - a - b};
                if (e[c] >= 1) { memcpy(be[c][k], e, sizeof(int) * 3); k++; }
            }
        nb = k;
    }
    double xi[38 * 3], wr[38];
    int nt, ns;
    const int Q = rgo_prism_face_points(order, xi, wr, &nt, &ns);
    const int nu = 3 * nb, ndiv = nc, ncon = ndiv + 5, nrow = nu + Q, NIN = 3 * (nc + 1) + Q + 5, NOUT = 3 * N + 3;
    const int ng = 6;
    double gx[8], gw[8], v1[2], v2[2], v3[2];
    gauss01(ng, gx, gw);
    tri_vertex(0, v1);
    tri_vertex(1, v2);
    tri_vertex(2, v3);
    double *A = malloc(sizeof(double) * nrow * nu), *C = malloc(sizeof(double) * ncon * nu);
    double *K = malloc(sizeof(double) * (nu + ncon) * (nu + ncon)), *rhs = malloc(sizeof(double) * (nu + ncon));
    double *sol = malloc(sizeof(double) * (nu + ncon)), *b = malloc(sizeof(double) * nrow), *d = malloc(sizeof(double) * ncon);
    int rc = 0;
    for (int z = 0; z < nz && !rc; z++) {
        tri_map t;
        if (tri_map_init(&t, order - 1, &abc[9 * z], &abc[9 * z + 3], &abc[9 * z + 6])) { rc = -1; break; }
        const double r0 = r01[2 * z], r1 = r01[2 * z + 1];
        /* cubature: volume, centroid, moments of the Taylor frame */
        double V = 0.0, cen[3] = {0, 0, 0};
        double *px = malloc(sizeof(double) * ng * ng * ng * 4);
        int np = 0;
        for (int i = 0; i < ng; i++)
            for (int j = 0; j < ng; j++)
                for (int k = 0; k < ng; k++) {
                    double s = gx[i], tt = (1.0 - s) * gx[j], q3[3], x[3], jac[9];
                    q3[0] = v1[0] + s * (v2[0] - v1[0]) + tt * (v3[0] - v1[0]);
                    q3[1] = v1[1] + s * (v2[1] - v1[1]) + tt * (v3[1] - v1[1]);
                    q3[2] = gx[k] - 0.5;
                    prism_map(&t, r0, r1, q3, x, jac);
                    double wJ = 2.0 * (S3 / 4.0) * (1.0 - s) * gw[i] * gw[j] * gw[k] * det3(jac);
                    V += wJ;
                    for (int c = 0; c < 3; c++) cen[c] += wJ * x[c];
                    memcpy(&px[4 * np], x, 24);
                    px[4 * np + 3] = wJ;
                    np++;
                }
        for (int c = 0; c < 3; c++) cen[c] /= V;
        const double l0 = cbrt(V);
        double mom[6][6][6];
        memset(mom, 0, sizeof(mom));
        for (int q = 0; q < np; q++) {
            double X[3];
            for (int c = 0; c < 3; c++) X[c] = (px[4 * q + c] - cen[c]) / l0;
            for (int a = 0; a <= p; a++)
                for (int bb = 0; a + bb <= p; bb++)
                    for (int cc = 0; a + bb + cc <= p; cc++) {
                        int e[3] = {a, bb, cc};
                        mom[a][bb][cc] += px[4 * q + 3] * mono3(e, X) / V;
                    }
        }
        free(px);
#define TB(e, X) (((e)[0] + (e)[1] + (e)[2]) == 0 ? 1.0 : mono3((e), (X)) - mom[(e)[0]][(e)[1]][(e)[2]])
        const double *in = &Bin[(size_t)z * NIN];
        memset(A, 0, sizeof(double) * nrow * nu);
        memset(C, 0, sizeof(double) * ncon * nu);
        memset(b, 0, sizeof(double) * nrow);
        memset(d, 0, sizeof(double) * ncon);
        /* closeness to the WENO-AO coefficients */
        for (int c = 0; c < 3; c++)
            for (int k = 0; k < nb; k++) {
                A[(size_t)(c * nb + k) * nu + c * nb + k] = 1.0;
                b[c * nb + k] = k <= nc ? in[c * (nc + 1) + k] : 0.0;
            }
        /* face points: positions, outward normals, weights within each face */
        double area[5] = {0, 0, 0, 0, 0};
        double fx[38][3], fn[38][3], fa[38];
        for (int q = 0; q < Q; q++) {
            double jac[9], a3[3], b3[3], c3[3], sc;
            prism_map(&t, r0, r1, &xi[3 * q], fx[q], jac);
            if (q < 2 * nt) {
                for (int i = 0; i < 3; i++) { a3[i] = jac[3 * i]; b3[i] = jac[3 * i + 1]; }
                sc = (q < nt ? 1.0 : -1.0) * (S3 / 4.0) * wr[q];
            } else {
                const int k = (q - 2 * nt) / ns;
                double V0[2], V1[2];
                tri_vertex(k, V0);
                tri_vertex((k + 1) % 3, V1);
                for (int i = 0; i < 3; i++) { a3[i] = jac[3 * i] * (V1[0] - V0[0]) + jac[3 * i + 1] * (V1[1] - V0[1]); b3[i] = jac[3 * i + 2]; }
                sc = wr[q];
            }
            c3[0] = a3[1] * b3[2] - a3[2] * b3[1];
            c3[1] = a3[2] * b3[0] - a3[0] * b3[2];
            c3[2] = a3[0] * b3[1] - a3[1] * b3[0];
            const double m = sqrt(dot3(c3, c3));
            for (int i = 0; i < 3; i++) fn[q][i] = (sc > 0 ? 1.0 : -1.0) * c3[i] / m;
            fa[q] = fabs(sc) * m;
            const int f = q < nt ? 0 : q < 2 * nt ? 1 : 2 + (q - 2 * nt) / ns;
            area[f] += fa[q];
        }
        for (int q = 0; q < Q; q++) {
            const int f = q < nt ? 0 : q < 2 * nt ? 1 : 2 + (q - 2 * nt) / ns;
            double X[3];
            for (int c = 0; c < 3; c++) X[c] = (fx[q][c] - cen[c]) / l0;
            for (int c = 0; c < 3; c++)
                for (int k = 0; k < nb; k++) {
                    const double val = fn[q][c] * TB(be[c][k], X);
                    A[(size_t)(nu + q) * nu + c * nb + k] = val;
                    C[(size_t)(ndiv + f) * nu + c * nb + k] += fa[q] / area[f] * val;
                }
            b[nu + q] = in[3 * (nc + 1) + q];
        }
        for (int f = 0; f < 5; f++) d[ndiv + f] = in[3 * (nc + 1) + Q + f];
        /* divergence identities: coefficient of X^mu in div B vanishes, 1 <= |mu| <= p-1 */
        for (int i = 0; i < ndiv; i++)
            for (int c = 0; c < 3; c++) {
                int tmu[3] = {te[i][0], te[i][1], te[i][2]};
                tmu[c] += 1;
                for (int k = 0; k < nb; k++)
                    if (be[c][k][0] == tmu[0] && be[c][k][1] == tmu[1] && be[c][k][2] == tmu[2])
                        C[(size_t)i * nu + c * nb + k] += (double)tmu[c];
            }
        /* KKT [2 A^T A, C^T; C, 0] */
        const int n = nu + ncon;
        for (int i = 0; i < nu; i++) {
            for (int j = 0; j < nu; j++) {
                double s = 0.0;
                for (int k = 0; k < nrow; k++) s += A[(size_t)k * nu + i] * A[(size_t)k * nu + j];
                K[(size_t)i * n + j] = 2.0 * s;
            }
            double s = 0.0;
            for (int k = 0; k < nrow; k++) s += A[(size_t)k * nu + i] * b[k];
            rhs[i] = 2.0 * s;
        }
        for (int i = 0; i < ncon; i++) {
            for (int j = 0; j < nu; j++) {
                K[(size_t)(nu + i) * n + j] = C[(size_t)i * nu + j];
                K[(size_t)j * n + nu + i] = C[(size_t)i * nu + j];
            }
            for (int j = 0; j < ncon; j++) K[(size_t)(nu + i) * n + nu + j] = 0.0;
            rhs[nu + i] = d[i];
        }
        if (la_lu_solve(n, K, rhs, sol)) { rc = -2; break; }
        /* B at the element nodes and the zone means */
        double *out = &Bout[(size_t)z * NOUT];
        for (int i = 0; i < N; i++) {
            double x[3], jac[9], X[3];
            prism_map(&t, r0, r1, r.node[i], x, jac);
            for (int c = 0; c < 3; c++) X[c] = (x[c] - cen[c]) / l0;
            for (int c = 0; c < 3; c++) {
                double s = 0.0;
                for (int k = 0; k < nb; k++) s += sol[c * nb + k] * TB(be[c][k], X);
                out[c * N + i] = s;
            }
        }
        for (int c = 0; c < 3; c++) out[3 * N + c] = sol[c * nb];
#undef TB
    }
    free(A); free(C); free(K); free(rhs); free(sol); free(b); free(d);
    return rc;
}

/* sizes of the divergence-free map's input and output vectors */
void rgo_prism_divfree_sizes(int order, int *nin, int *nout)
{
    int te[40][3];
    const int nc = taylor_multi(order - 1, te);
    const int Q = order == 2 ? 15 : order == 3 ? 24 : 38, N = order == 2 ? 6 : order == 3 ? 15 : 26;
    *nin = 3 * (nc + 1) + Q + 5;
    *nout = 3 * N + 3;
}

/* zone centroid cen[z][3] and Taylor length l0[z] = V^(1/3) by the cubature
 * of rgo_prism_volumes */
int rgo_prism_frames(int order, int nz, const double *abc, const double *r01, double *cen, double *l0)
{
    const int ng = 6;
    double gx[8], gw[8], v1[2], v2[2], v3[2];
    gauss01(ng, gx, gw);
    tri_vertex(0, v1);
    tri_vertex(1, v2);
    tri_vertex(2, v3);
    for (int z = 0; z < nz; z++) {
        tri_map t;
        if (tri_map_init(&t, order - 1, &abc[9 * z], &abc[9 * z + 3], &abc[9 * z + 6])) return -1;
        double V = 0.0, c[3] = {0, 0, 0};
        for (int i = 0; i < ng; i++)
            for (int j = 0; j < ng; j++)
                for (int k = 0; k < ng; k++) {
                    double s = gx[i], tt = (1.0 - s) * gx[j], xi[3], x[3], jac[9];
                    xi[0] = v1[0] + s * (v2[0] - v1[0]) + tt * (v3[0] - v1[0]);
                    xi[1] = v1[1] + s * (v2[1] - v1[1]) + tt * (v3[1] - v1[1]);
                    xi[2] = gx[k] - 0.5;
                    prism_map(&t, r01[2 * z], r01[2 * z + 1], xi, x, jac);
                    const double wJ = 2.0 * (S3 / 4.0) * (1.0 - s) * gw[i] * gw[j] * gw[k] * det3(jac);
                    V += wJ;
                    for (int d = 0; d < 3; d++) c[d] += wJ * x[d];
                }
        for (int d = 0; d < 3; d++) cen[3 * z + d] = c[d] / V;
        l0[z] = cbrt(V);
    }
    return 0;
}

/*
 * Zone geometry of the oracle (test infrastructure only), computed zone by
 * zone from each zone's own isoparametric map.
 *
 * Map (eq. 5.2): the angular surface is a tensor Lagrange interpolant of order
 * map_order (2 = quadratic, 3 = cubic) through nodes on the unit sphere --
 * corners, equidistant great-circle (slerp) points on the edges, and
 * great-circle intersections inside -- and the radial direction is linear
 * (Section II.b):  x(xi,eta,zeta) = [(1/2-zeta) r_k + (1/2+zeta) r_{k+1}] S(xi,eta)
 * on the reference cube [-1/2,1/2]^3.
 *
 * From it: Gauss cubature (volume, centroid, moments of eq. 3.2-3.3), face
 * quadrature with area vectors (eqs. 5.6-5.8), Simpson points on edges
 * (Section II.c), and at the ADER nodes the Jacobian J and the flux metrics
 * (h_eta x h_zeta, h_zeta x h_xi, h_xi x h_eta) of eq. (5.11) in the
 * conservative curl form, so that their discrete divergence vanishes.
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

void rgo_gc_intersect(const double *p1, const double *p2, const double *q1, const double *q2,
                      const double *hint, double *out);

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void slerp(const double *a, const double *b, double t, double *out)
{
    double c[3];
    cross3(a, b, c);
    double th = atan2(sqrt(dot3(c, c)), dot3(a, b));
    double wa = sin((1.0 - t) * th) / sin(th), wb = sin(t * th) / sin(th);
    for (int i = 0; i < 3; i++) out[i] = wa * a[i] + wb * b[i];
}

/* equidistant 1-D Lagrange basis on t_a = -1/2 + a/mo */
static double lag_eq(int mo, int a, double x)
{
    double v = 1.0, ta = -0.5 + (double)a / mo;
    for (int b = 0; b <= mo; b++)
        if (b != a) v *= (x - (-0.5 + (double)b / mo)) / (ta - (-0.5 + (double)b / mo));
    return v;
}

static double dlag_eq(int mo, int a, double x)
{
    double s = 0.0, ta = -0.5 + (double)a / mo;
    for (int b = 0; b <= mo; b++) {
        if (b == a) continue;
        double v = 1.0 / (ta - (-0.5 + (double)b / mo));
        for (int c = 0; c <= mo; c++)
            if (c != a && c != b) v *= (x - (-0.5 + (double)c / mo)) / (ta - (-0.5 + (double)c / mo));
        s += v;
    }
    return s;
}

static void surface_nodes(const rgo_mesh *m, int z, double *sn)
{
    const int mo = m->map_order, n1 = mo + 1;
    const int *qv = &m->quad[4 * m->zone_quad[z]];
    const double *v0 = &m->vert[3 * qv[0]], *v1 = &m->vert[3 * qv[1]];
    const double *v2 = &m->vert[3 * qv[2]], *v3 = &m->vert[3 * qv[3]];
    double bot[4][3], top[4][3], lef[4][3], rig[4][3], hint[3];
    for (int a = 0; a <= mo; a++) {
        double t = (double)a / mo;
        if (a == 0) {
            memcpy(bot[a], v0, 24); memcpy(top[a], v3, 24); memcpy(lef[a], v0, 24); memcpy(rig[a], v1, 24);
        } else if (a == mo) {
            memcpy(bot[a], v1, 24); memcpy(top[a], v2, 24); memcpy(lef[a], v3, 24); memcpy(rig[a], v2, 24);
        } else {
            slerp(v0, v1, t, bot[a]);
            slerp(v3, v2, t, top[a]);
            slerp(v0, v3, t, lef[a]);
            slerp(v1, v2, t, rig[a]);
        }
    }
    for (int i = 0; i < 3; i++) hint[i] = v0[i] + v1[i] + v2[i] + v3[i];
    for (int b = 0; b <= mo; b++)
        for (int a = 0; a <= mo; a++) {
            double *p = &sn[3 * (a + n1 * b)];
            if (b == 0) memcpy(p, bot[a], 24);
            else if (b == mo) memcpy(p, top[a], 24);
            else if (a == 0) memcpy(p, lef[b], 24);
            else if (a == mo) memcpy(p, rig[b], 24);
            else rgo_gc_intersect(bot[a], top[a], lef[b], rig[b], hint, p);
        }
}

/* x(xi) and jac[n*3+d] = dx_n / dxi_d */
void zone_map(const rgo_mesh *m, int z, const double *xi, double *x, double *jac)
{
    const int mo = m->map_order, n1 = mo + 1;
    const double *sn = &m->snode[z * 48];
    double La[4], Lb[4], dLa[4], dLb[4];
    for (int a = 0; a <= mo; a++) {
        La[a] = lag_eq(mo, a, xi[0]);
        Lb[a] = lag_eq(mo, a, xi[1]);
        dLa[a] = dlag_eq(mo, a, xi[0]);
        dLb[a] = dlag_eq(mo, a, xi[1]);
    }
    double S[3] = {0, 0, 0}, Sa[3] = {0, 0, 0}, Sb[3] = {0, 0, 0};
    for (int b = 0; b <= mo; b++)
        for (int a = 0; a <= mo; a++) {
            const double *p = &sn[3 * (a + n1 * b)];
            for (int i = 0; i < 3; i++) {
                S[i] += La[a] * Lb[b] * p[i];
                Sa[i] += dLa[a] * Lb[b] * p[i];
                Sb[i] += La[a] * dLb[b] * p[i];
            }
        }
    int k = m->zone_shell[z];
    double rlo = m->radius[k], rhi = m->radius[k + 1];
    double R = (0.5 - xi[2]) * rlo + (0.5 + xi[2]) * rhi, dR = rhi - rlo;
    for (int i = 0; i < 3; i++) {
        x[i] = R * S[i];
        if (jac) {
            jac[i * 3 + 0] = R * Sa[i];
            jac[i * 3 + 1] = R * Sb[i];
            jac[i * 3 + 2] = dR * S[i];
        }
    }
}

static double det3(const double *j)
{
    return j[0] * (j[4] * j[8] - j[5] * j[7]) - j[1] * (j[3] * j[8] - j[5] * j[6]) +
           j[2] * (j[3] * j[7] - j[4] * j[6]);
}

/* reference coordinates of face-quadrature point q of local face lf */
void face_ref_point(const rgo_mesh *m, int lf, int q, double *xi)
{
    double gx[4], gw[4];
    int nq = m->nq_face;
    gauss01(nq, gx, gw);
    double u = gx[q % nq] - 0.5, v = gx[q / nq] - 0.5;
    double fix = (lf & 1) ? 0.5 : -0.5;
    int axis = lf / 2;
    if (axis == 0) { xi[0] = fix; xi[1] = u; xi[2] = v; }
    else if (axis == 1) { xi[0] = u; xi[1] = fix; xi[2] = v; }
    else { xi[0] = u; xi[1] = v; xi[2] = fix; }
}

/* reference coordinates at parameter s in [0,1] along local edge le */
void edge_ref_point(int le, double s, double *xi)
{
    int axis = le / 4, c = le % 4;
    int a1 = (axis == 0) ? 1 : 0, a2 = (axis == 2) ? 1 : 2;
    xi[axis] = s - 0.5;
    xi[a1] = (c & 1) ? 0.5 : -0.5;
    xi[a2] = (c & 2) ? 0.5 : -0.5;
}

static const int LF_EDGES[6][4] = {
    {4, 6, 8, 10}, {5, 7, 9, 11}, {0, 2, 8, 9}, {1, 3, 10, 11}, {0, 1, 4, 5}, {2, 3, 6, 7},
};

int mesh_build_geometry(rgo_mesh *m)
{
    const int nz = m->nz, N = m->ref.N, Q = m->nq_face * m->nq_face;
    m->snode = malloc(sizeof(double) * nz * 48);
    for (int z = 0; z < nz; z++) surface_nodes(m, z, &m->snode[z * 48]);

    /* cubature */
    int na = m->ncub_ang, nr = m->ncub_rad;
    double ax[16], aw[16], rx[16], rw[16];
    gauss01(na, ax, aw);
    gauss01(nr, rx, rw);
    m->ncub = na * na * nr;
    m->cub = malloc(sizeof(cub_pt) * (size_t)nz * m->ncub);
    m->vol = malloc(sizeof(double) * nz);
    m->cen = malloc(sizeof(double) * nz * 3);
    m->len = malloc(sizeof(double) * nz);
    m->mom = calloc((size_t)nz * 125, sizeof(double));
    m->nodex = malloc(sizeof(double) * nz * N * 3);
    m->nodeJ = malloc(sizeof(double) * nz * N);
    m->nodeMet = malloc(sizeof(double) * nz * N * 9);

    double *dpsi = malloc(sizeof(double) * N * N * 3);  /* d psi_l / d xi_d at node i */
    for (int i = 0; i < N; i++)
        for (int l = 0; l < N; l++)
            for (int d = 0; d < 3; d++) dpsi[(i * N + l) * 3 + d] = refel_dpsi(&m->ref, l, d, m->ref.node[i]);

#pragma omp parallel for schedule(dynamic, 16)
    for (int z = 0; z < nz; z++) {
        cub_pt *cp = &m->cub[(size_t)z * m->ncub];
        int n = 0;
        double vol = 0.0, c[3] = {0, 0, 0};
        for (int k = 0; k < nr; k++)
            for (int j = 0; j < na; j++)
                for (int i = 0; i < na; i++) {
                    double xi[3] = {ax[i] - 0.5, ax[j] - 0.5, rx[k] - 0.5}, jac[9];
                    zone_map(m, z, xi, cp[n].x, jac);
                    cp[n].wJ = aw[i] * aw[j] * rw[k] * det3(jac);
                    vol += cp[n].wJ;
                    for (int d = 0; d < 3; d++) c[d] += cp[n].wJ * cp[n].x[d];
                    n++;
                }
        for (int d = 0; d < 3; d++) c[d] /= vol;
        m->vol[z] = vol;
        memcpy(&m->cen[3 * z], c, 24);
        double l0 = cbrt(vol);
        m->len[z] = l0;
        double *mo = &m->mom[(size_t)z * 125];
        for (int p = 0; p < n; p++) {
            double X = (cp[p].x[0] - c[0]) / l0, Y = (cp[p].x[1] - c[1]) / l0, Z = (cp[p].x[2] - c[2]) / l0;
            double px[5], py[5], pz[5];
            px[0] = py[0] = pz[0] = 1.0;
            for (int e = 1; e < 5; e++) { px[e] = px[e - 1] * X; py[e] = py[e - 1] * Y; pz[e] = pz[e - 1] * Z; }
            for (int a = 0; a < 5; a++)
                for (int b = 0; a + b < 5; b++)
                    for (int cc = 0; a + b + cc < 5; cc++) mo[a * 25 + b * 5 + cc] += cp[p].wJ * px[a] * py[b] * pz[cc];
        }
        for (int i = 0; i < 125; i++) mo[i] /= vol;

        /* ADER nodes: position, Jacobian and curl-form metrics */
        double *nx = &m->nodex[(size_t)z * N * 3], *nJ = &m->nodeJ[(size_t)z * N];
        double *nM = &m->nodeMet[(size_t)z * N * 9];
        double *V = malloc(sizeof(double) * N * 9);   /* V[i][n][j] = (x_l - c_l) d x_m / d xi_j */
        for (int i = 0; i < N; i++) {
            double jac[9];
            zone_map(m, z, m->ref.node[i], &nx[3 * i], jac);
            nJ[i] = det3(jac);
            for (int nn = 0; nn < 3; nn++) {
                int mm = (nn + 1) % 3, ll = (nn + 2) % 3;
                for (int j = 0; j < 3; j++)
                    V[i * 9 + nn * 3 + j] = (nx[3 * i + ll] - c[ll]) * jac[mm * 3 + j];
            }
        }
        for (int i = 0; i < N; i++)
            for (int nn = 0; nn < 3; nn++) {
                double dV[3][3] = {{0}};   /* dV[j][d] = d/dxi_d of interpolated V_j at node i */
                for (int l = 0; l < N; l++)
                    for (int j = 0; j < 3; j++)
                        for (int d = 0; d < 3; d++) dV[j][d] += V[l * 9 + nn * 3 + j] * dpsi[(i * N + l) * 3 + d];
                /* (J a^d)_n = - (curl_xi V)_d */
                nM[i * 9 + 0 * 3 + nn] = -(dV[2][1] - dV[1][2]);
                nM[i * 9 + 1 * 3 + nn] = -(dV[0][2] - dV[2][0]);
                nM[i * 9 + 2 * 3 + nn] = -(dV[1][0] - dV[0][1]);
            }
        free(V);
    }
    free(dpsi);

    /* faces, from the owner's map */
    const int nf = m->nf;
    m->fx = malloc(sizeof(double) * nf * RGO_MAXQ * 3);
    m->fn = malloc(sizeof(double) * nf * RGO_MAXQ * 3);
    m->fdA = malloc(sizeof(double) * nf * RGO_MAXQ);
    m->farea = malloc(sizeof(double) * nf);
    m->fcen = malloc(sizeof(double) * nf * 3);
    m->face_perm = malloc(sizeof(int) * nf * RGO_MAXQ);
    double gx[4], gw[4];
    gauss01(m->nq_face, gx, gw);
#pragma omp parallel for schedule(static)
    for (int f = 0; f < nf; f++) {
        int z = m->face_zone[2 * f], lf = m->face_lf[2 * f];
        int axis = lf / 2, u = (axis == 0) ? 1 : 0, v = (axis == 2) ? 1 : 2;
        double sgn = (lf & 1) ? 1.0 : -1.0, area = 0.0, fc[3] = {0, 0, 0};
        for (int q = 0; q < Q; q++) {
            double xi[3], jac[9], hu[3], hv[3], dA[3];
            face_ref_point(m, lf, q, xi);
            zone_map(m, z, xi, &m->fx[(f * RGO_MAXQ + q) * 3], jac);
            for (int i = 0; i < 3; i++) { hu[i] = jac[i * 3 + u]; hv[i] = jac[i * 3 + v]; }
            cross3(hu, hv, dA);
            /* (u,v) = (eta,zeta), (xi,zeta), (xi,eta): outward is +, -, + for the upper face */
            double o = sgn * ((axis == 1) ? -1.0 : 1.0) * gw[q % m->nq_face] * gw[q / m->nq_face];
            double a = sqrt(dot3(dA, dA));
            for (int i = 0; i < 3; i++) m->fn[(f * RGO_MAXQ + q) * 3 + i] = (o > 0 ? 1.0 : -1.0) * dA[i] / a;
            m->fdA[f * RGO_MAXQ + q] = fabs(o) * a;
            area += fabs(o) * a;
            for (int i = 0; i < 3; i++) fc[i] += fabs(o) * a * m->fx[(f * RGO_MAXQ + q) * 3 + i];
        }
        m->farea[f] = area;
        for (int i = 0; i < 3; i++) m->fcen[3 * f + i] = fc[i] / area;
        /* matching point order on the other side */
        int z2 = m->face_zone[2 * f + 1], lf2 = m->face_lf[2 * f + 1];
        for (int q = 0; q < Q; q++) m->face_perm[f * RGO_MAXQ + q] = q;
        if (z2 >= 0) {
            for (int q2 = 0; q2 < Q; q2++) {
                double xi[3], x2[3];
                face_ref_point(m, lf2, q2, xi);
                zone_map(m, z2, xi, x2, NULL);
                int best = 0;
                double bd = 1e300;
                for (int q = 0; q < Q; q++) {
                    const double *p = &m->fx[(f * RGO_MAXQ + q) * 3];
                    double d = (p[0] - x2[0]) * (p[0] - x2[0]) + (p[1] - x2[1]) * (p[1] - x2[1]) +
                               (p[2] - x2[2]) * (p[2] - x2[2]);
                    if (d < bd) { bd = d; best = q; }
                }
                m->face_perm[f * RGO_MAXQ + best] = q2;
            }
        }
    }

    /* edges: Simpson points along the canonical direction, from the first zone */
    const int ne = m->ne;
    m->ex = malloc(sizeof(double) * ne * 9);
    m->et = malloc(sizeof(double) * ne * 9);
    m->edl = malloc(sizeof(double) * ne * 3);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < ne; e++) {
        int z = m->edge_zone[4 * e], le = m->edge_le[4 * e], rev = m->edge_rev[4 * e];
        for (int p = 0; p < 3; p++) {
            double s = 0.5 * p, xi[3], jac[9], t[3];
            edge_ref_point(le, rev ? 1.0 - s : s, xi);
            zone_map(m, z, xi, &m->ex[e * 9 + p * 3], jac);
            for (int i = 0; i < 3; i++) t[i] = (rev ? -1.0 : 1.0) * jac[i * 3 + le / 4];
            double a = sqrt(dot3(t, t));
            for (int i = 0; i < 3; i++) m->et[e * 9 + p * 3 + i] = t[i] / a;
            m->edl[e * 3 + p] = a;
        }
        /* zones around the edge, counter-clockwise about its direction */
        int nze = m->edge_nz[e];
        const double *xm = &m->ex[e * 9 + 3], *tm = &m->et[e * 9 + 3];
        double ea[3], eb[3], ang[4];
        const double *c0 = &m->cen[3 * m->edge_zone[4 * e]];
        for (int i = 0; i < 3; i++) ea[i] = c0[i] - xm[i];
        double pr = dot3(ea, tm);
        for (int i = 0; i < 3; i++) ea[i] -= pr * tm[i];
        double na_ = sqrt(dot3(ea, ea));
        for (int i = 0; i < 3; i++) ea[i] /= na_;
        cross3(tm, ea, eb);
        for (int s = 0; s < nze; s++) {
            const double *cz = &m->cen[3 * m->edge_zone[4 * e + s]];
            double d[3] = {cz[0] - xm[0], cz[1] - xm[1], cz[2] - xm[2]};
            ang[s] = atan2(dot3(d, eb), dot3(d, ea));
        }
        for (int i = 1; i < nze; i++)
            for (int j = i; j > 0 && ang[j - 1] > ang[j]; j--) {
                double ta = ang[j]; ang[j] = ang[j - 1]; ang[j - 1] = ta;
                int t1 = m->edge_zone[4 * e + j]; m->edge_zone[4 * e + j] = m->edge_zone[4 * e + j - 1]; m->edge_zone[4 * e + j - 1] = t1;
                t1 = m->edge_le[4 * e + j]; m->edge_le[4 * e + j] = m->edge_le[4 * e + j - 1]; m->edge_le[4 * e + j - 1] = t1;
                t1 = m->edge_rev[4 * e + j]; m->edge_rev[4 * e + j] = m->edge_rev[4 * e + j - 1]; m->edge_rev[4 * e + j - 1] = t1;
            }
    }

    /* face boundary edges with circulation signs about the face normal */
    m->face_edges = malloc(sizeof(int) * nf * 4);
    m->face_esign = malloc(sizeof(int) * nf * 4);
#pragma omp parallel for schedule(static)
    for (int f = 0; f < nf; f++) {
        int z = m->face_zone[2 * f], lf = m->face_lf[2 * f];
        double nbar[3] = {0, 0, 0};
        for (int q = 0; q < Q; q++)
            for (int i = 0; i < 3; i++) nbar[i] += m->fdA[f * RGO_MAXQ + q] * m->fn[(f * RGO_MAXQ + q) * 3 + i];
        for (int k = 0; k < 4; k++) {
            /* right-hand rule about the face normal: the edge runs
             * counter-clockwise when n x (its midpoint - an interior point)
             * points along it.  The midpoint of the opposite edge (local
             * edges pair up as k, k^1) serves as the interior point; the
             * face centroid does not, since on a thin curved face it can sag
             * below an edge. */
            int e = m->zone_edge[12 * z + LF_EDGES[lf][k]];
            int eo = m->zone_edge[12 * z + LF_EDGES[lf][k ^ 1]];
            const double *xm = &m->ex[e * 9 + 3], *tm = &m->et[e * 9 + 3], *xo = &m->ex[eo * 9 + 3];
            double r[3] = {xm[0] - xo[0], xm[1] - xo[1], xm[2] - xo[2]}, ccw[3];
            cross3(nbar, r, ccw);
            m->face_edges[4 * f + k] = e;
            m->face_esign[4 * f + k] = dot3(ccw, tm) > 0 ? 1 : -1;
        }
    }
    return 0;
}

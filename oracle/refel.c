/*
 * Reference element of the oracle (test infrastructure only).
 *
 * - Gauss-Legendre rules on [0, 1].
 * - A generic nodal Lagrange basis from any set of nodes and monomials: the
 *   construction of eq. (5.3), used with the prism node sets of Appendices B-D
 *   for checking and with hexahedral serendipity node sets for the scheme.
 * - The hexahedral serendipity element on [-1/2, 1/2]^3: vertices plus
 *   equidistant edge nodes (Section V.b), monomials of superlinear degree
 *   <= p-1 (20 functions at p = 3, 32 at p = 4).
 * - Time nodes tau = 0 plus Gauss points (eqs. 5.15-5.17).
 * - The full space-time Galerkin system of eqs. (5.24)-(5.27) built by
 *   quadrature over the space-time reference element, split into the
 *   non-evolving (level tau = 0) and evolving blocks, and reduced to the
 *   matrices of eq. (5.29).
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

void gauss01(int n, double *x, double *w)
{
    for (int i = 0; i < n; i++) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double pp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; j++) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-16) break;
        }
        /* z descends with i, so 0.5 (1 - z) ascends on [0, 1] */
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * pp * pp);
    }
}

double mono3(const int *e, const double *x)
{
    double v = 1.0;
    for (int d = 0; d < 3; d++)
        for (int k = 0; k < e[d]; k++) v *= x[d];
    return v;
}

double dmono3(const int *e, int dir, const double *x)
{
    if (e[dir] == 0) return 0.0;
    double v = (double)e[dir];
    for (int d = 0; d < 3; d++) {
        int p = e[d] - (d == dir ? 1 : 0);
        for (int k = 0; k < p; k++) v *= x[d];
    }
    return v;
}

/* psi_l(x) = sum_k coef[k*n + l] * x^{exps_k}  with psi_l(node_i) = delta_il */
int lagrange3(int n, const double *nodes, const int *exps, double *coef)
{
    double *V = malloc(sizeof(double) * n * n);
    if (!V) return -1;
    for (int i = 0; i < n; i++)
        for (int k = 0; k < n; k++) V[i * n + k] = mono3(&exps[3 * k], &nodes[3 * i]);
    int rc = la_inverse(n, V, coef);
    free(V);
    return rc;
}

static double basis_eval(int n, const int *exps, const double *coef, int l, const double *x)
{
    double s = 0.0;
    for (int k = 0; k < n; k++) s += coef[k * n + l] * mono3(&exps[3 * k], x);
    return s;
}

static double basis_deriv(int n, const int *exps, const double *coef, int l, int d,
                          const double *x)
{
    double s = 0.0;
    for (int k = 0; k < n; k++) s += coef[k * n + l] * dmono3(&exps[3 * k], d, x);
    return s;
}

double refel_psi(const rgo_refel *r, int l, const double *xi)
{
    return basis_eval(r->N, &r->exps[0][0], r->coef, l, xi);
}

double refel_dpsi(const rgo_refel *r, int l, int d, const double *xi)
{
    return basis_deriv(r->N, &r->exps[0][0], r->coef, l, d, xi);
}

/* hexahedral serendipity nodes on [-1/2,1/2]^3: 8 vertices, then p-1 nodes per
 * edge at equidistant positions; monomials of superlinear degree <= p-1 */
static int serendipity_nodes(int order, double node[][3], int exps[][3])
{
    int n = 0;
    for (int v = 0; v < 8; v++) {
        node[n][0] = (v & 1) ? 0.5 : -0.5;
        node[n][1] = (v & 2) ? 0.5 : -0.5;
        node[n][2] = (v & 4) ? 0.5 : -0.5;
        n++;
    }
    int per_edge = order - 2;
    for (int axis = 0; axis < 3; axis++) {
        int a1 = (axis + 1) % 3, a2 = (axis + 2) % 3;
        for (int c = 0; c < 4; c++) {
            for (int k = 1; k <= per_edge; k++) {
                double t = -0.5 + (double)k / (order - 1);
                node[n][axis] = t;
                node[n][a1] = (c & 1) ? 0.5 : -0.5;
                node[n][a2] = (c & 2) ? 0.5 : -0.5;
                n++;
            }
        }
    }
    int m = 0;
    int r = order - 1;
    for (int deg = 0; deg <= 3 * 3; deg++)
        for (int a = deg; a >= 0; a--)
            for (int b = deg - a; b >= 0; b--) {
                int c = deg - a - b;
                int lin = (a == 1) + (b == 1) + (c == 1);
                if (deg - lin <= r) {
                    if (m >= RGO_MAXN) return -1;
                    exps[m][0] = a; exps[m][1] = b; exps[m][2] = c;
                    m++;
                }
            }
    return (m == n) ? n : -1;
}

/* 1-D Lagrange basis on nodes t[0..M-1] */
static double lag1(int M, const double *t, int j, double x)
{
    double v = 1.0;
    for (int k = 0; k < M; k++)
        if (k != j) v *= (x - t[k]) / (t[j] - t[k]);
    return v;
}

static double dlag1(int M, const double *t, int j, double x)
{
    double s = 0.0;
    for (int k = 0; k < M; k++) {
        if (k == j) continue;
        double v = 1.0 / (t[j] - t[k]);
        for (int m = 0; m < M; m++)
            if (m != j && m != k) v *= (x - t[m]) / (t[j] - t[m]);
        s += v;
    }
    return s;
}

/* Time levels tau = 0 plus the M-1 Gauss points (eqs. 5.15-5.17) and the
 * full space-time Galerkin system of eqs. (5.24)-(5.27) for the element's
 * nodal basis, integrated with the given spatial quadrature (points xq,
 * weights wq) times M+1 Gauss points in time, split into the non-evolving and
 * evolving blocks and reduced to the matrices of eq. (5.29).  The spatial
 * rule must integrate the products psi_i dpsi_l exactly. */
int refel_spacetime(rgo_refel *r, int M, int nq, const double *xq, const double *wq)
{
    double gx[4], gw[4];
    gauss01(M - 1, gx, gw);
    r->M = M;
    r->tau[0] = 0.0;
    r->wt[0] = 0.0;
    for (int j = 1; j < M; j++) { r->tau[j] = gx[j - 1]; r->wt[j] = gw[j - 1]; }

    int N = r->N, L = N * M, E = L - N;
    r->L = L;
    const int nt = M + 1;
    double tx[8], tw[8];
    gauss01(nt, tx, tw);
    double *Kt = calloc((size_t)L * L, sizeof(double));
    double *Kx[3];
    for (int d = 0; d < 3; d++) Kx[d] = calloc((size_t)L * L, sizeof(double));
    double *psi = malloc(sizeof(double) * N), *dpsi = malloc(sizeof(double) * N * 3);
    double phi[4], dphi[4];
    for (int p = 0; p < nq; p++) {
        const double *xi = &xq[3 * p];
        double ws = wq[p];
        for (int i = 0; i < N; i++) {
            psi[i] = refel_psi(r, i, xi);
            for (int d = 0; d < 3; d++) dpsi[i * 3 + d] = refel_dpsi(r, i, d, xi);
        }
        for (int t = 0; t < nt; t++) {
            for (int j = 0; j < M; j++) {
                phi[j] = lag1(M, r->tau, j, tx[t]);
                dphi[j] = dlag1(M, r->tau, j, tx[t]);
            }
            double w = ws * tw[t];
            /* theta_{i + j N} = psi_i phi_j   (eq. 5.19) */
            for (int jj = 0; jj < L; jj++) {
                double th = psi[jj % N] * phi[jj / N];
                for (int ll = 0; ll < L; ll++) {
                    int i = ll % N, j = ll / N;
                    Kt[jj * L + ll] += w * th * psi[i] * dphi[j];
                    for (int d = 0; d < 3; d++)
                        Kx[d][jj * L + ll] += w * th * dpsi[i * 3 + d] * phi[j];
                }
            }
        }
    }
    /* split into blocks (eq. 5.27) and form eq. (5.29) */
    double *K11 = malloc(sizeof(double) * E * E), *K11i = malloc(sizeof(double) * E * E);
    for (int i = 0; i < E; i++)
        for (int j = 0; j < E; j++) K11[i * E + j] = Kt[(N + i) * L + N + j];
    if (la_inverse(E, K11, K11i)) return -1;
    r->Kt0 = calloc((size_t)E * N, sizeof(double));
    for (int d = 0; d < 3; d++) {
        r->Kd0[d] = calloc((size_t)E * N, sizeof(double));
        r->Kd[d] = calloc((size_t)E * E, sizeof(double));
    }
    for (int i = 0; i < E; i++) {
        for (int j = 0; j < N; j++) {
            double s = 0.0;
            for (int k = 0; k < E; k++) s += K11i[i * E + k] * Kt[(N + k) * L + j];
            r->Kt0[i * N + j] = -s;
            for (int d = 0; d < 3; d++) {
                double sd = 0.0;
                for (int k = 0; k < E; k++) sd += K11i[i * E + k] * Kx[d][(N + k) * L + j];
                r->Kd0[d][i * N + j] = sd;
            }
        }
        for (int j = 0; j < E; j++)
            for (int d = 0; d < 3; d++) {
                double sd = 0.0;
                for (int k = 0; k < E; k++) sd += K11i[i * E + k] * Kx[d][(N + k) * L + N + j];
                r->Kd[d][i * E + j] = sd;
            }
    }
    free(Kt);
    for (int d = 0; d < 3; d++) free(Kx[d]);
    free(psi); free(dpsi); free(K11); free(K11i);
    return 0;
}

int refel_init(rgo_refel *r, int order)
{
    memset(r, 0, sizeof(*r));
    if (order < 3 || order > 4) return -1;
    r->order = order;
    r->N = serendipity_nodes(order, r->node, r->exps);
    if (r->N <= 0) return -1;
    if (lagrange3(r->N, &r->node[0][0], &r->exps[0][0], r->coef)) return -1;

    /* spatial quadrature: 4^3 Gauss points on the cube, exact for the
     * products in eq. (5.26) */
    const int ns = 4;
    double sx[8], sw[8], xq[64 * 3], wq[64];
    gauss01(ns, sx, sw);
    int n = 0;
    for (int a = 0; a < ns; a++)
        for (int b = 0; b < ns; b++)
            for (int c = 0; c < ns; c++) {
                xq[3 * n] = sx[a] - 0.5;
                xq[3 * n + 1] = sx[b] - 0.5;
                xq[3 * n + 2] = sx[c] - 0.5;
                wq[n++] = sw[a] * sw[b] * sw[c];
            }
    return refel_spacetime(r, order, n, xq, wq);
}

void refel_free(rgo_refel *r)
{
    free(r->Kt0);
    for (int d = 0; d < 3; d++) { free(r->Kd0[d]); free(r->Kd[d]); }
    memset(r, 0, sizeof(*r));
}

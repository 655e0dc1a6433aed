/*
 * Initial states for the oracle (test infrastructure only): zone averages of
 * pointwise fields by the zone cubature, and face-averaged normal B from the
 * circulation of a vector potential around each face (Stokes), so that the
 * discrete divergence of B vanishes to round-off from the start.
 *
 * Field definitions (inputs, not part of the method):
 *  - harmonic: f(x) = sum_k a_k x^e_k / |x|^{|e_k|} for rho, v and A
 *    (35 monomials of degree <= 4 in a fixed order), p uniform;
 *  - alfven: circularly polarised Alfven wave along axis a with transverse
 *    frame (e1, e2): B = B0 a + dB (cos phi e1 + sin phi e2),
 *    v = -(dB / sqrt(rho)) (cos phi e1 + sin phi e2), phi = k (x.a - v_A t),
 *    A = (B0/2) a x r - (dB / k) (cos phi e1 + sin phi e2).
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int MONO[35][3];
static int mono_ready = 0;

static void init_monomials(void)
{
    if (mono_ready) return;
    int n = 0;
    for (int d = 0; d <= 4; d++)
        for (int a = d; a >= 0; a--)
            for (int b = d - a; b >= 0; b--) { MONO[n][0] = a; MONO[n][1] = b; MONO[n][2] = d - a - b; n++; }
    mono_ready = 1;
}

static double field_eval(const double *coef, const double *x, double *grad)
{
    double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2], r = sqrt(r2);
    double val = 0.0;
    if (grad) grad[0] = grad[1] = grad[2] = 0.0;
    for (int k = 0; k < 35; k++) {
        if (coef[k] == 0.0) continue;
        int d = MONO[k][0] + MONO[k][1] + MONO[k][2];
        double m = mono3(MONO[k], x), rd = pow(r, d);
        val += coef[k] * m / rd;
        if (grad)
            for (int i = 0; i < 3; i++)
                grad[i] += coef[k] * (dmono3(MONO[k], i, x) / rd - d * m * x[i] / (rd * r2));
    }
    return val;
}

typedef struct {
    int kind;
    double gamma;
    /* harmonic */
    const double *rho, *v, *A;
    double p;
    /* alfven */
    double frame[9], rho0, p0, B0, dB, kw, t;
} field_ctx;

static void fields(const field_ctx *c, const double *x, double *rho, double *v, double *p, double *B, double *A)
{
    if (c->kind == 0) {
        *rho = field_eval(c->rho, x, NULL);
        for (int i = 0; i < 3; i++) v[i] = field_eval(&c->v[35 * i], x, NULL);
        *p = c->p;
        double g[3][3];
        for (int i = 0; i < 3; i++) A[i] = field_eval(&c->A[35 * i], x, g[i]);
        B[0] = g[2][1] - g[1][2];
        B[1] = g[0][2] - g[2][0];
        B[2] = g[1][0] - g[0][1];
    } else {
        const double *e1 = &c->frame[0], *e2 = &c->frame[3], *a = &c->frame[6];
        double vA = c->B0 / sqrt(c->rho0);
        double ph = c->kw * (x[0] * a[0] + x[1] * a[1] + x[2] * a[2] - vA * c->t);
        double cs = cos(ph), sn = sin(ph);
        *rho = c->rho0;
        *p = c->p0;
        double ax[3] = {a[1] * x[2] - a[2] * x[1], a[2] * x[0] - a[0] * x[2], a[0] * x[1] - a[1] * x[0]};
        for (int i = 0; i < 3; i++) {
            double tr = cs * e1[i] + sn * e2[i];
            B[i] = c->B0 * a[i] + c->dB * tr;
            v[i] = -c->dB / sqrt(c->rho0) * tr;
            A[i] = 0.5 * c->B0 * ax[i] - c->dB / c->kw * tr;
        }
    }
}

static void init_state(const rgo_mesh *m, const field_ctx *c, double *U, double *Bf)
{
    init_monomials();
    const int nz = m->nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++) {
        double acc[NVAR] = {0};
        const cub_pt *cp = &m->cub[(size_t)z * m->ncub];
        for (int q = 0; q < m->ncub; q++) {
            double rho, v[3], p, B[3], A[3];
            fields(c, cp[q].x, &rho, v, &p, B, A);
            double u[NVAR];
            u[IRHO] = rho;
            for (int i = 0; i < 3; i++) { u[IMX + i] = rho * v[i]; u[IBX + i] = B[i]; }
            u[IEN] = p / (c->gamma - 1.0) + 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) +
                     0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
            for (int k = 0; k < NVAR; k++) acc[k] += cp[q].wJ * u[k];
        }
        for (int k = 0; k < NVAR; k++) U[(size_t)k * nz + z] = acc[k] / m->vol[z];
    }
    /* edge circulations of A with 5-point Gauss along each mapped edge */
    double gx[8], gw[8];
    gauss01(5, gx, gw);
    double *Gam = malloc(sizeof(double) * m->ne);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->ne; e++) {
        int z = m->edge_zone[4 * e], le = m->edge_le[4 * e], rev = m->edge_rev[4 * e];
        double s = 0.0;
        for (int q = 0; q < 5; q++) {
            double xi[3], x[3], jac[9], rho, v[3], p, B[3], A[3];
            edge_ref_point(le, rev ? 1.0 - gx[q] : gx[q], xi);
            zone_map(m, z, xi, x, jac);
            fields(c, x, &rho, v, &p, B, A);
            double sg = rev ? -1.0 : 1.0;
            for (int i = 0; i < 3; i++) s += gw[q] * A[i] * sg * jac[i * 3 + le / 4];
        }
        Gam[e] = s;
    }
    for (int f = 0; f < m->nf; f++) {
        double s = 0.0;
        for (int k = 0; k < 4; k++) s += m->face_esign[4 * f + k] * Gam[m->face_edges[4 * f + k]];
        Bf[f] = s / m->farea[f];
    }
    free(Gam);
}

void rgo_run_init_harmonic(const rgo_mesh *m, const double *rho, const double *v, const double *A, double p,
                           double gamma, double *U, double *Bf)
{
    field_ctx c;
    memset(&c, 0, sizeof(c));
    c.kind = 0;
    c.rho = rho;
    c.v = v;
    c.A = A;
    c.p = p;
    c.gamma = gamma;
    init_state(m, &c, U, Bf);
}

void rgo_run_init_alfven(const rgo_mesh *m, const double *frame, double rho, double p, double B0, double dB,
                         double wavelength, double gamma, double t, double *U, double *Bf)
{
    field_ctx c;
    memset(&c, 0, sizeof(c));
    c.kind = 1;
    memcpy(c.frame, frame, sizeof(double) * 9);
    c.rho0 = rho;
    c.p0 = p;
    c.B0 = B0;
    c.dB = dB;
    c.kw = 2.0 * M_PI / wavelength;
    c.t = t;
    c.gamma = gamma;
    init_state(m, &c, U, Bf);
}

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
 *    A = (B0/2) a x r - (dB / k) (cos phi e1 + sin phi e2);
 *  - spherical shock tube (Section VIII.c), pole on the z axis: primitive
 *    states (rho, p, v_r, v_theta, v_phi) on either side of r = r_m (no
 *    taper), a radial field B_r = B_r0 sin(theta) (r0 / r)^2 and a toroidal
 *    field B_phi = (sin(theta) / 2) T(r) from the radial vector potential
 *    A_r = (r cos(theta) / 2) T(r), T(r) = B_phiL (1 - tanh((r - r_m)/delta))
 *    + B_phiR (1 + tanh((r - r_m)/delta)).  The radial field has the same
 *    outward flux through every sphere and so no vector potential on the
 *    shell: its face fluxes are the solid-angle integrals of
 *    B_r0 r0^2 sin(theta) over each radial face (the same number for every
 *    radial face of a column, zero through the radially ruled angular faces),
 *    which keeps the discrete divergence at round-off.
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
    /* spherical shock tube: states (rho, p, v_r, v_theta, v_phi, B_theta, B_phi) */
    double sL[7], sR[7], Br0, r0, rm, delta;
    /* blast: p_in inside the ball |x - centre| < radius, uniform B along frame[6..8] */
    double centre[3], radius, p_in;
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
    } else if (c->kind == 3) {
        const double *a = &c->frame[6];
        double d2 = 0.0;
        for (int i = 0; i < 3; i++) d2 += (x[i] - c->centre[i]) * (x[i] - c->centre[i]);
        *rho = c->rho0;
        *p = d2 < c->radius * c->radius ? c->p_in : c->p0;
        double ax[3] = {a[1] * x[2] - a[2] * x[1], a[2] * x[0] - a[0] * x[2], a[0] * x[1] - a[1] * x[0]};
        for (int i = 0; i < 3; i++) {
            v[i] = 0.0;
            B[i] = c->B0 * a[i];
            A[i] = 0.5 * c->B0 * ax[i];
        }
    } else if (c->kind == 2) {
        double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]), s = sqrt(x[0] * x[0] + x[1] * x[1]);
        double st = s / r, ct = x[2] / r;
        double rh[3] = {x[0] / r, x[1] / r, x[2] / r}, th[3] = {0, 0, -st}, ph[3] = {0, 0, 0};
        if (s > 0) {
            th[0] = ct * x[0] / s;
            th[1] = ct * x[1] / s;
            ph[0] = -x[1] / s;
            ph[1] = x[0] / s;
        }
        const double *S = r <= c->rm ? c->sL : c->sR;
        double th_ = tanh((r - c->rm) / c->delta);
        double T = c->sL[6] * (1.0 - th_) + c->sR[6] * (1.0 + th_);
        double Br = c->Br0 * st * (c->r0 / r) * (c->r0 / r), Bp = 0.5 * st * T;
        *rho = S[0];
        *p = S[1];
        for (int i = 0; i < 3; i++) {
            v[i] = S[2] * rh[i] + S[3] * th[i] + S[4] * ph[i];
            B[i] = Br * rh[i] + Bp * ph[i];
            A[i] = 0.5 * x[2] * T * rh[i];
        }
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

/* Outward flux of B_r0 r0^2 sin(theta) r_hat / r^2 through each radial face,
 * added to its face average: the integral over the solid angle the face
 * subtends, sin(theta) (x . dA) / |x|^3, by a 6 x 6 Gauss rule on the owner's
 * map at its mid radius (the map is R(zeta) S(xi, eta), so every radial face
 * of a column subtends the same solid angle and gets the same number up to
 * rounding). */
static void radial_monopole_flux(const rgo_mesh *m, const field_ctx *c, double *Bf)
{
    double gx[8], gw[8];
    gauss01(6, gx, gw);
#pragma omp parallel for schedule(static)
    for (int f = 0; f < m->nf; f++) {
        int z = m->face_zone[2 * f], lf = m->face_lf[2 * f];
        if (lf < 4) continue;
        double flux = 0.0;
        for (int j = 0; j < 6; j++)
            for (int i = 0; i < 6; i++) {
                double xi[3] = {gx[i] - 0.5, gx[j] - 0.5, 0.0}, x[3], jac[9];
                zone_map(m, z, xi, x, jac);
                double R = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                double n[3] = {jac[3] * jac[7] - jac[6] * jac[4], jac[6] * jac[1] - jac[0] * jac[7],
                               jac[0] * jac[4] - jac[3] * jac[1]};   /* dx/dxi x dx/deta */
                double xn = fabs(x[0] * n[0] + x[1] * n[1] + x[2] * n[2]);
                double st = sqrt(x[0] * x[0] + x[1] * x[1]) / R;
                flux += gw[i] * gw[j] * c->Br0 * c->r0 * c->r0 * st * xn / (R * R * R);
            }
        /* the face's canonical normal is the owner's outward one: +r for the
         * upper face of the owner, -r for its lower face */
        Bf[f] += (lf == 5 ? flux : -flux) / m->farea[f];
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
    /* edge circulations of A with 5-point Gauss along each mapped edge (on
     * nsub equal pieces of it for the shock tube, whose taper is narrow) */
    double gx[8], gw[8];
    gauss01(5, gx, gw);
    const int nsub = c->kind == 2 ? 4 : 1;
    double *Gam = malloc(sizeof(double) * m->ne);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->ne; e++) {
        int z = m->edge_zone[4 * e], le = m->edge_le[4 * e], rev = m->edge_rev[4 * e];
        double s = 0.0;
        for (int j = 0; j < nsub; j++)
            for (int q = 0; q < 5; q++) {
                double xi[3], x[3], jac[9], rho, v[3], p, B[3], A[3], sp = (j + gx[q]) / nsub;
                edge_ref_point(le, rev ? 1.0 - sp : sp, xi);
                zone_map(m, z, xi, x, jac);
                fields(c, x, &rho, v, &p, B, A);
                double sg = rev ? -1.0 : 1.0;
                for (int i = 0; i < 3; i++) s += gw[q] / nsub * A[i] * sg * jac[i * 3 + le / 4];
            }
        Gam[e] = s;
    }
    for (int f = 0; f < m->nf; f++) {
        double s = 0.0;
        for (int k = 0; k < 4; k++) s += m->face_esign[4 * f + k] * Gam[m->face_edges[4 * f + k]];
        Bf[f] = s / m->farea[f];
    }
    free(Gam);
    if (c->kind == 2) radial_monopole_flux(m, c, Bf);
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

void rgo_run_init_tube(const rgo_mesh *m, const double *left, const double *right, double Br0, double r0,
                       double rm, double delta, double gamma, double *U, double *Bf)
{
    field_ctx c;
    memset(&c, 0, sizeof(c));
    c.kind = 2;
    memcpy(c.sL, left, sizeof(double) * 7);
    memcpy(c.sR, right, sizeof(double) * 7);
    c.Br0 = Br0;
    c.r0 = r0;
    c.rm = rm;
    c.delta = delta;
    c.gamma = gamma;
    init_state(m, &c, U, Bf);
}

/* magnetised blast (Section VIII.b): rho, v = 0, pressure p_in inside the
 * ball |x - centre| < radius and p outside (zone averages by the zone
 * cubature of this step function), uniform B = B0 a (A = (B0/2) a x r) */
void rgo_run_init_blast(const rgo_mesh *m, const double *axis, const double *centre, double radius, double rho,
                        double p_in, double p, double B0, double gamma, double *U, double *Bf)
{
    field_ctx c;
    memset(&c, 0, sizeof(c));
    c.kind = 3;
    memcpy(&c.frame[6], axis, sizeof(double) * 3);
    memcpy(c.centre, centre, sizeof(double) * 3);
    c.radius = radius;
    c.rho0 = rho;
    c.p_in = p_in;
    c.p0 = p;
    c.B0 = B0;
    c.gamma = gamma;
    init_state(m, &c, U, Bf);
}

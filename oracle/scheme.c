/*
 * One ADER-WENO-AO divergence-free MHD timestep, oracle version (test
 * infrastructure only; plain FP64, zone by zone, every matrix rebuilt and
 * solved directly).  Follows the pointwise description of Section VI:
 *
 *   1. geometry (built once, geom.c)
 *   2. WENO-AO reconstruction of all eight zone averages in the Taylor basis
 *      (Section III, eqs. 3.1-3.4)
 *   3. divergence-free reconstruction of B from the face averages with the
 *      zone B overwritten (Section IV, eqs. 4.1-4.15, steps 1-10 of IV.b)
 *   4. ADER-CG predictor on the serendipity element (Section V, eqs.
 *      5.20-5.29, steps 5-10 of V.d)
 *   5. corrector: 1-D Riemann solver at face quadrature points for the eight
 *      conserved variables, multidimensional Riemann solver at edge Simpson
 *      points for the electric field, finite-volume update and Yee-type
 *      constrained transport of the face-averaged normal B (eqs. 2.5-2.6).
 *
 * Units are rationalised (magnetic pressure B^2/2), i.e. eq. (2.2) with 4 pi
 * absorbed into B.
 *
 * Every function here is pinned by a CPU test against closed forms, values
 * worked out by hand, exactness on polynomial data or invariances (the
 * fast speed, the HLL branches, the four-state and three-zone edge solvers,
 * the WENO-AO indicators, weights and blend: tests/test_oracle_pins_solvers.py).
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "sreal.h"

#ifdef RGO_COMPLEX
/* the complex build's own names for the functions other files call */
#define phys_flux phys_flux_cx
#define fast_speed fast_speed_cx
#define hll_flux hll_flux_cx
#define rgo_predict_element rgo_predict_element_cx
#define rgo_emf4 rgo_emf4_cx
#define rgo_emf3 rgo_emf3_cx
#define rgo_run_step rgo_run_step_cx
#endif

#define WENO_GAMMA_HI 0.85
#define FLAG_LINEAR_WEIGHTS 1
#define FLAG_FALLBACK 2
#define FALLBACK_ROUNDS 4

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static sreal dot3s(const sreal *a, const sreal *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static sreal dot3m(const sreal *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void cross3m(const double *a, const sreal *b, sreal *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* ---------------- ideal MHD (eq. 2.2, rationalised units) ---------------- */
static sreal pressure(const sreal *U, double gamma)
{
    sreal rho = U[IRHO];
    sreal m2 = U[IMX] * U[IMX] + U[IMY] * U[IMY] + U[IMZ] * U[IMZ];
    sreal B2 = U[IBX] * U[IBX] + U[IBY] * U[IBY] + U[IBZ] * U[IBZ];
    return (gamma - 1.0) * (U[IEN] - 0.5 * m2 / rho - 0.5 * B2);
}

void phys_flux(const sreal *U, double gamma, sreal F[3][NVAR])
{
    sreal rho = U[IRHO];
    sreal v[3] = {U[IMX] / rho, U[IMY] / rho, U[IMZ] / rho};
    const sreal *B = &U[IBX];
    sreal p = pressure(U, gamma);
    sreal pt = p + 0.5 * dot3s(B, B), vB = dot3s(v, B);
    for (int d = 0; d < 3; d++) {
        F[d][IRHO] = U[IMX + d];
        for (int i = 0; i < 3; i++)
            F[d][IMX + i] = U[IMX + d] * v[i] + (d == i ? pt : 0.0) - B[d] * B[i];
        F[d][IEN] = (U[IEN] + pt) * v[d] - B[d] * vB;
        for (int i = 0; i < 3; i++) F[d][IBX + i] = v[d] * B[i] - B[d] * v[i];
    }
}

sreal fast_speed(const sreal *U, double gamma, const double *n)
{
    sreal rho = U[IRHO];
    const sreal *B = &U[IBX];
    sreal a2 = gamma * pressure(U, gamma) / rho;
    sreal b2 = dot3s(B, B) / rho;
    sreal bn = dot3m(B, n);
    sreal bn2 = bn * bn / rho;
    sreal s = a2 + b2;
    sreal disc = s * s - 4.0 * a2 * bn2;
    if (SRE(disc) < 0.0) disc = 0.0;
    return s_sqrt(0.5 * (s + s_sqrt(disc)));
}

/* HLL flux along unit normal n (pointing from L to R) with Davis speeds */
void hll_flux(const sreal *UL, const sreal *UR, const sreal *FnL, const sreal *FnR,
              const double *n, double gamma, sreal *Fs)
{
    sreal vL = dot3m(&UL[IMX], n) / UL[IRHO], vR = dot3m(&UR[IMX], n) / UR[IRHO];
    sreal cL = fast_speed(UL, gamma, n), cR = fast_speed(UR, gamma, n);
    sreal SL = s_min(vL - cL, vR - cR), SR = s_max(vL + cL, vR + cR);
    if (SRE(SL) >= 0.0) {
        for (int v = 0; v < NVAR; v++) Fs[v] = FnL[v];
    } else if (SRE(SR) <= 0.0) {
        for (int v = 0; v < NVAR; v++) Fs[v] = FnR[v];
    } else {
        for (int v = 0; v < NVAR; v++)
            Fs[v] = (SR * FnL[v] - SL * FnR[v] + SL * SR * (UR[v] - UL[v])) / (SR - SL);
    }
}

/* ---------------- Taylor basis (eq. 3.1) ---------------- */
static int taylor_list(int deg, int e[][3])
{
    int n = 0;
    for (int d = 1; d <= deg; d++)
        for (int a = d; a >= 0; a--)
            for (int b = d - a; b >= 0; b--) { e[n][0] = a; e[n][1] = b; e[n][2] = d - a - b; n++; }
    return n;
}

static double mom_of(const rgo_mesh *m, int z, const int *e)
{
    return m->mom[(size_t)z * 125 + e[0] * 25 + e[1] * 5 + e[2]];
}

static void to_X(const rgo_mesh *m, int z, const double *x, double *X)
{
    for (int i = 0; i < 3; i++) X[i] = (x[i] - m->cen[3 * z + i]) / m->len[z];
}

static double falling(int a, int b)
{
    double v = 1.0;
    for (int i = 0; i < b; i++) v *= (a - i);
    return v;
}

/* d^beta X^alpha */
static double dmono_multi(const int *alpha, const int *beta, const double *X)
{
    double v = 1.0;
    for (int i = 0; i < 3; i++) {
        if (beta[i] > alpha[i]) return 0.0;
        v *= falling(alpha[i], beta[i]);
        for (int k = 0; k < alpha[i] - beta[i]; k++) v *= X[i];
    }
    return v;
}

/* ---------------- per-step workspace ---------------- */
typedef struct {
    const rgo_mesh *m;
    double gamma, dt;
    int flags;
    double weno_eps;        /* epsilon of the WENO-AO weights */
    int deg, nc, nbx;       /* reconstruction degree p-1, # Taylor coeffs, # B coeffs per component */
    int te[40][3];          /* Taylor multi-indices 1..deg */
    int be[3][40][3];       /* divergence-free basis per component */
    sreal *U;               /* state after the boundary fill, [8][nz] */
    sreal *Bf;              /* [nf] */
    char *recon;            /* zone is reconstructed */
    sreal *wc;              /* nz * 8 * nc  WENO coefficients */
    sreal *bface;           /* nf * Q  limited nodal normal B (eqs. 4.11-4.12), owner order */
    sreal *bc;              /* nz * 3 * nbx divergence-free coefficients */
    sreal *avgU, *avgF;     /* nz * N * 8, nz * N * 24 */
    sreal *Phi;             /* nf * 8 */
    sreal *Gam;             /* ne */
    int first_order;        /* traces are the zones' states at t^n (the fallback's re-solve) */
    double *whi;            /* nz, or NULL: the smallest over the variables of w_hi / gamma_hi */
    double flat_kappa;      /* flattener threshold (0: off) */
    sreal *eta;             /* nz flattener values, or NULL */
    int dbg_z;              /* zone whose WENO-AO internals are recorded (test access), or -1 */
    double *dbg;            /* per variable: beta_hi, beta_s[7], weights[8], then the nc coefficients */
} step_ws;

static int zone_of(const rgo_mesh *m, int qd, int k) { return qd * m->ktot + k; }

/* copy the normal-B average of local face lfs of zone zs to local face lft of
 * zone zt, both measured along the respective zone's outward normal */
static void copy_face_value(step_ws *w, int zt, int lft, int zs, int lfs)
{
    const rgo_mesh *m = w->m;
    int ft = m->zone_face[6 * zt + lft], fs = m->zone_face[6 * zs + lfs];
    double st = (m->face_zone[2 * ft] == zt) ? 1.0 : -1.0, ss = (m->face_zone[2 * fs] == zs) ? 1.0 : -1.0;
    w->Bf[ft] = st * ss * w->Bf[fs];
}

/* ---- boundary fill (continuative copy of the nearest interior shell) ---- */
static void boundary_fill(step_ws *w)
{
    const rgo_mesh *m = w->m;
    int g = m->n_ghost, K = m->ktot, Nr = m->n_rad;
    for (int qd = 0; qd < m->nquad; qd++)
        for (int k = 0; k < K; k++) {
            int src = (k < g) ? g : (k >= g + Nr ? g + Nr - 1 : -1);
            if (src < 0) continue;
            int z = zone_of(m, qd, k), zs = zone_of(m, qd, src);
            for (int v = 0; v < NVAR; v++) w->U[(size_t)v * m->nz + z] = w->U[(size_t)v * m->nz + zs];
            for (int lf = 0; lf < 4; lf++) copy_face_value(w, z, lf, zs, lf);
        }
    for (int qd = 0; qd < m->nquad; qd++) {
        int zin = zone_of(m, qd, g), zout = zone_of(m, qd, g + Nr - 1);
        for (int kf = 0; kf < g; kf++) copy_face_value(w, zone_of(m, qd, kf), 4, zin, 4);
        for (int kf = g + Nr + 1; kf <= K; kf++) copy_face_value(w, zone_of(m, qd, kf - 1), 5, zout, 5);
    }
}

/* ---- WENO-AO reconstruction of one zone (Section III) ---- */
static sreal minmod(sreal a, sreal b)
{
    if (!(SRE(a) * SRE(b) > 0.0)) return 0.0;
    return (SRE(a) > 0 ? 1.0 : -1.0) * s_min(s_abs(a), s_abs(b));
}

/* ---- flattener (Section VII.a applies one to its coarse meshes and
 * defers its definition to other work).  The reading here: a zone is
 * flattened where the flow compresses faster than a fraction kappa of the
 * slowest signal speed around it.  With the discrete divergence of the zone
 * averages' velocity over the zone,
 *   D = (1/V) sum_faces s_f (sum_q dA_q n_q) . (v_zone + v_neighbour) / 2
 * (s_f = +1 on outward faces), the length l0 = V^(1/3) and c the smallest
 * fast speed sqrt(gamma p / rho + B^2 / rho) over the zone and its six face
 * neighbours, eta = min(1, max(0, -(l0 D + kappa c) / (kappa c))): zero
 * unless l0 D < -kappa c, one where l0 D <= -2 kappa c.  Every
 * reconstruction coefficient of the zone (all eight variables) is then
 * scaled by 1 - eta, so a fully flattened zone is first order. */
static sreal zone_fast_max(const step_ws *w, int z)
{
    sreal u[NVAR];
    for (int v = 0; v < NVAR; v++) u[v] = w->U[(size_t)v * w->m->nz + z];
    sreal a2 = w->gamma * pressure(u, w->gamma) / u[IRHO], b2 = dot3s(&u[IBX], &u[IBX]) / u[IRHO];
    return s_sqrt(s_max(a2, 0.0) + b2);
}

static sreal flattener_eta(const step_ws *w, int z)
{
    const rgo_mesh *m = w->m;
    const int nz = m->nz, Q = m->nq_face * m->nq_face;
    sreal vz[3], div = 0.0, c = zone_fast_max(w, z);
    for (int i = 0; i < 3; i++) vz[i] = w->U[(size_t)(IMX + i) * nz + z] / w->U[(size_t)IRHO * nz + z];
    for (int lf = 0; lf < 6; lf++) {
        int f = m->zone_face[6 * z + lf], zn = m->zone_nbr[6 * z + lf];
        double sg = (m->face_zone[2 * f] == z) ? 1.0 : -1.0, va[3] = {0, 0, 0};
        sreal vn[3] = {0, 0, 0};
        for (int q = 0; q < Q; q++)
            for (int i = 0; i < 3; i++) va[i] += m->fdA[f * RGO_MAXQ + q] * m->fn[(f * RGO_MAXQ + q) * 3 + i];
        for (int i = 0; i < 3; i++) vn[i] = w->U[(size_t)(IMX + i) * nz + zn] / w->U[(size_t)IRHO * nz + zn];
        for (int i = 0; i < 3; i++) div += sg * va[i] * 0.5 * (vz[i] + vn[i]);
        c = s_min(c, zone_fast_max(w, zn));
    }
    div /= m->vol[z];
    const sreal kc = w->flat_kappa * c;
    return s_min(1.0, s_max(0.0, -(m->len[z] * div + kc) / kc));
}

/* least squares and LU solves with a real matrix and a state right-hand
 * side: the complex build solves the real and imaginary parts in turn */
static int s_lsq_qr(int m, int n, const double *A, const sreal *b, sreal *x)
{
#ifdef RGO_COMPLEX
    double br[RGO_MAXST], bi[RGO_MAXST], xr[RGO_MAXST], xi[RGO_MAXST];
    for (int i = 0; i < m; i++) { br[i] = creal(b[i]); bi[i] = cimag(b[i]); }
    int rc = la_lsq_qr(m, n, A, br, xr) | la_lsq_qr(m, n, A, bi, xi);
    for (int i = 0; i < n; i++) x[i] = xr[i] + I * xi[i];
    return rc;
#else
    return la_lsq_qr(m, n, A, b, x);
#endif
}

static int s_lu_solve(int n, const double *A, const sreal *b, sreal *x)
{
#ifdef RGO_COMPLEX
    double *br = malloc(sizeof(double) * 4 * n), *bi = br + n, *xr = br + 2 * n, *xi = br + 3 * n;
    for (int i = 0; i < n; i++) { br[i] = creal(b[i]); bi[i] = cimag(b[i]); }
    int rc = la_lu_solve(n, A, br, xr) | la_lu_solve(n, A, bi, xi);
    for (int i = 0; i < n; i++) x[i] = xr[i] + I * xi[i];
    free(br);
    return rc;
#else
    return la_lu_solve(n, A, b, x);
#endif
}

/* large-stencil rows of zone z: volume average over each member zone j of
 * zone z's Taylor basis (eq. 3.4); A is ns x nc, row-major */
static void weno_rows(const step_ws *w, int z, double *A)
{
    const rgo_mesh *m = w->m;
    const int nc = w->nc, ns = m->st_n[z];
    const int *st = &m->st_z[RGO_MAXST * z];
    for (int j = 0; j < ns; j++) {
        int zj = st[j];
        const cub_pt *cp = &m->cub[(size_t)zj * m->ncub];
        for (int a = 0; a < nc; a++) A[j * nc + a] = 0.0;
        for (int p = 0; p < m->ncub; p++) {
            double X[3];
            to_X(m, z, cp[p].x, X);
            for (int a = 0; a < nc; a++) A[j * nc + a] += cp[p].wJ * mono3(w->te[a], X);
        }
        for (int a = 0; a < nc; a++) A[j * nc + a] = A[j * nc + a] / m->vol[zj] - mom_of(m, z, w->te[a]);
    }
}

static void weno_zone(step_ws *w, int z)
{
    const rgo_mesh *m = w->m;
    const int nc = w->nc, nz = m->nz;
    const int ns = m->st_n[z];
    const int *st = &m->st_z[RGO_MAXST * z];
    double *A = malloc(sizeof(double) * ns * nc);
    weno_rows(w, z, A);
    /* small stencils: central (all face neighbours) and one-sided (drop the
     * neighbour opposite direction d) with linear polynomials */
    int fnb[6];
    for (int lf = 0; lf < 6; lf++) fnb[lf] = m->zone_nbr[6 * z + lf];
    double Xn[6][3];
    for (int lf = 0; lf < 6; lf++) to_X(m, z, &m->cen[3 * fnb[lf]], Xn[lf]);

    const int nsm = 7;
    const double gs = (1.0 - WENO_GAMMA_HI) / nsm;
    sreal *coef = &w->wc[(size_t)z * NVAR * nc];
    sreal *rhs = malloc(sizeof(sreal) * ns);
    sreal chi[40], cs[7][3];
    const cub_pt *c0 = &m->cub[(size_t)z * m->ncub];
    /* derivative multi-indices for the smoothness indicator */
    int de[40][3];
    int nde = taylor_list(w->deg, de);
    for (int v = 0; v < NVAR; v++) {
        sreal u0 = w->U[(size_t)v * nz + z];
        for (int j = 0; j < ns; j++) rhs[j] = w->U[(size_t)v * nz + st[j]] - u0;
        s_lsq_qr(ns, nc, A, rhs, chi);
        for (int s = 0; s < nsm; s++) {
            double As[6 * 3];
            sreal bs[6];
            int n = 0;
            for (int lf = 0; lf < 6; lf++) {
                if (s > 0 && lf == ((s - 1) ^ 1)) continue;
                for (int i = 0; i < 3; i++) As[n * 3 + i] = Xn[lf][i];
                bs[n] = w->U[(size_t)v * nz + fnb[lf]] - u0;
                n++;
            }
            s_lsq_qr(n, 3, As, bs, cs[s]);
        }
        sreal wgt[8], beta[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (w->flags & FLAG_LINEAR_WEIGHTS) {
            wgt[0] = WENO_GAMMA_HI;
            for (int s = 0; s < nsm; s++) wgt[1 + s] = gs;
        } else {
            /* smoothness: volume average over zone 0 of all squared derivatives */
            sreal bhi = 0.0;
            for (int p = 0; p < m->ncub; p++) {
                double X[3];
                sreal acc = 0.0;
                to_X(m, z, c0[p].x, X);
                for (int b = 0; b < nde; b++) {
                    sreal dv = 0.0;
                    for (int a = 0; a < nc; a++) dv += chi[a] * dmono_multi(w->te[a], de[b], X);
                    acc += dv * dv;
                }
                bhi += c0[p].wJ * acc;
            }
            bhi /= m->vol[z];
            beta[0] = bhi;
            sreal tot = 0.0;
            const double eps = w->weno_eps;
            wgt[0] = WENO_GAMMA_HI / ((bhi + eps) * (bhi + eps));
            tot += wgt[0];
            for (int s = 0; s < nsm; s++) {
                sreal b = cs[s][0] * cs[s][0] + cs[s][1] * cs[s][1] + cs[s][2] * cs[s][2];
                beta[1 + s] = b;
                wgt[1 + s] = gs / ((b + eps) * (b + eps));
                tot += wgt[1 + s];
            }
            for (int s = 0; s <= nsm; s++) wgt[s] /= tot;
        }
        if (w->whi && (v == 0 || SRE(wgt[0]) / WENO_GAMMA_HI < w->whi[z])) w->whi[z] = SRE(wgt[0]) / WENO_GAMMA_HI;
        /* adaptive-order blend: (w_hi/g_hi)(P_hi - sum g_s P_s) + sum w_s P_s */
        for (int a = 0; a < nc; a++) {
            sreal lin = 0.0, nl = 0.0;
            if (a < 3)
                for (int s = 0; s < nsm; s++) { lin += gs * cs[s][a]; nl += wgt[1 + s] * cs[s][a]; }
            coef[v * nc + a] = wgt[0] / WENO_GAMMA_HI * (chi[a] - lin) + nl;
        }
        if (w->eta)   /* the flattener (above) */
            for (int a = 0; a < nc; a++) coef[v * nc + a] *= 1.0 - w->eta[z];
        if (w->dbg && z == w->dbg_z) {
            double *d = w->dbg + (size_t)v * (16 + nc);
            for (int s = 0; s < 8; s++) { d[s] = SRE(beta[s]); d[8 + s] = SRE(wgt[s]); }
            for (int a = 0; a < nc; a++) d[16 + a] = SRE(coef[v * nc + a]);
        }
    }
    free(A);
    free(rhs);
}

/* WENO polynomial of zone z, variable v, at physical point x */
static sreal weno_eval(const step_ws *w, int z, int v, const double *x)
{
    const rgo_mesh *m = w->m;
    double X[3];
    to_X(m, z, x, X);
    sreal s = w->U[(size_t)v * m->nz + z];
    const sreal *c = &w->wc[((size_t)z * NVAR + v) * w->nc];
    for (int a = 0; a < w->nc; a++) s += c[a] * (mono3(w->te[a], X) - mom_of(m, z, w->te[a]));
    return s;
}

/* ---- face nodal normal B, eqs. (4.11)-(4.12) ---- */
static void face_nodal_b(step_ws *w, int f)
{
    const rgo_mesh *m = w->m;
    const int Q = m->nq_face * m->nq_face;
    int zs[2] = {m->face_zone[2 * f], m->face_zone[2 * f + 1]};
    sreal mean = w->Bf[f];
    sreal *bn = &w->bface[(size_t)f * RGO_MAXQ];
    for (int q = 0; q < Q; q++) {
        const double *x = &m->fx[(f * RGO_MAXQ + q) * 3], *n = &m->fn[(f * RGO_MAXQ + q) * 3];
        sreal d[2];
        int have[2];
        for (int s = 0; s < 2; s++) {
            have[s] = (zs[s] >= 0 && w->recon[zs[s]]);
            if (!have[s]) { d[s] = 0.0; continue; }
            sreal B[3];
            for (int c = 0; c < 3; c++) B[c] = weno_eval(w, zs[s], IBX + c, x);
            d[s] = dot3m(B, n) - mean;
        }
        /* a face with only one reconstructed neighbour takes that side's value */
        if (!have[0]) d[0] = d[1];
        if (!have[1]) d[1] = d[0];
        bn[q] = mean + minmod(d[0], d[1]);
    }
    sreal s = 0.0;
    for (int q = 0; q < Q; q++) s += m->fdA[f * RGO_MAXQ + q] / m->farea[f] * bn[q];
    for (int q = 0; q < Q; q++) bn[q] += mean - s;
}

static double bbasis(const step_ws *w, int z, const int *e, const double *X)
{
    if (e[0] + e[1] + e[2] == 0) return 1.0;
    return mono3(e, X) - mom_of(w->m, z, e);
}

/* ---- divergence-free reconstruction of one zone, Section IV.b ---- */
static int divfree_zone(step_ws *w, int z)
{
    const rgo_mesh *m = w->m;
    const int nb = w->nbx, nu = 3 * nb, Q = m->nq_face * m->nq_face, deg = w->deg;
    int ndiv = w->nc;                     /* multi-indices 1 <= |mu| <= p-1 */
    int ncon = ndiv + 6;
    int nrow = nu + 6 * Q;
    double *A = calloc((size_t)nrow * nu, sizeof(double));
    sreal *b = calloc(nrow, sizeof(sreal));
    double *C = calloc((size_t)ncon * nu, sizeof(double));
    sreal *dcon = calloc(ncon, sizeof(sreal));
    /* closeness to the WENO-AO coefficients (eqs. 4.3, 4.6, 4.9) */
    for (int c = 0; c < 3; c++)
        for (int k = 0; k < nb; k++) {
            int r = c * nb + k;
            A[(size_t)r * nu + r] = 1.0;
            const int *e = w->be[c][k];
            int d = e[0] + e[1] + e[2];
            if (d == 0) b[r] = w->U[(size_t)(IBX + c) * m->nz + z];
            else if (d <= deg) {
                int a;
                for (a = 0; a < w->nc; a++)
                    if (w->te[a][0] == e[0] && w->te[a][1] == e[1] && w->te[a][2] == e[2]) break;
                b[r] = w->wc[((size_t)z * NVAR + IBX + c) * w->nc + a];
            } else b[r] = 0.0;
        }
    /* face nodal values (eq. 4.15) and face-flux constraints (eq. 4.14) */
    for (int lf = 0; lf < 6; lf++) {
        int f = m->zone_face[6 * z + lf];
        double sg = (m->face_zone[2 * f] == z) ? 1.0 : -1.0;
        for (int q = 0; q < Q; q++) {
            const double *x = &m->fx[(f * RGO_MAXQ + q) * 3], *n = &m->fn[(f * RGO_MAXQ + q) * 3];
            double X[3], wq = m->fdA[f * RGO_MAXQ + q] / m->farea[f];
            to_X(m, z, x, X);
            int r = nu + lf * Q + q;
            for (int c = 0; c < 3; c++)
                for (int k = 0; k < nb; k++) {
                    double val = sg * n[c] * bbasis(w, z, w->be[c][k], X);
                    A[(size_t)r * nu + c * nb + k] = val;
                    C[(size_t)(ndiv + lf) * nu + c * nb + k] += wq * val;
                }
            b[r] = sg * w->bface[(size_t)f * RGO_MAXQ + q];
        }
        dcon[ndiv + lf] = sg * w->Bf[f];
    }
    /* divergence identities (eq. 4.10 without its first member) */
    int mu[40][3];
    taylor_list(deg, mu);
    for (int i = 0; i < ndiv; i++)
        for (int c = 0; c < 3; c++) {
            int t[3] = {mu[i][0], mu[i][1], mu[i][2]};
            t[c] += 1;
            for (int k = 0; k < nb; k++)
                if (w->be[c][k][0] == t[0] && w->be[c][k][1] == t[1] && w->be[c][k][2] == t[2])
                    C[(size_t)i * nu + c * nb + k] += (double)t[c];
        }
    /* KKT system [2 A^T A, C^T; C, 0] */
    int n = nu + ncon;
    double *K = calloc((size_t)n * n, sizeof(double));
    sreal *rhs = calloc(n, sizeof(sreal)), *sol = malloc(sizeof(sreal) * n);
    for (int i = 0; i < nu; i++) {
        for (int j = 0; j < nu; j++) {
            double s = 0.0;
            for (int r = 0; r < nrow; r++) s += A[(size_t)r * nu + i] * A[(size_t)r * nu + j];
            K[(size_t)i * n + j] = 2.0 * s;
        }
        sreal s = 0.0;
        for (int r = 0; r < nrow; r++) s += A[(size_t)r * nu + i] * b[r];
        rhs[i] = 2.0 * s;
    }
    for (int i = 0; i < ncon; i++) {
        for (int j = 0; j < nu; j++) {
            K[(size_t)(nu + i) * n + j] = C[(size_t)i * nu + j];
            K[(size_t)j * n + nu + i] = C[(size_t)i * nu + j];
        }
        rhs[nu + i] = dcon[i];
    }
    int rc = s_lu_solve(n, K, rhs, sol);
    memcpy(&w->bc[(size_t)z * nu], sol, sizeof(sreal) * nu);
    free(A); free(b); free(C); free(dcon); free(K); free(rhs); free(sol);
    return rc;
}

static void divfree_eval(const step_ws *w, int z, const double *x, sreal *B)
{
    double X[3];
    to_X(w->m, z, x, X);
    const sreal *c = &w->bc[(size_t)z * 3 * w->nbx];
    for (int i = 0; i < 3; i++) {
        sreal s = 0.0;
        for (int k = 0; k < w->nbx; k++) s += c[i * w->nbx + k] * bbasis(w, z, w->be[i][k], X);
        B[i] = s;
    }
}

/* ---- ADER-CG predictor on one element, eqs. (5.22)-(5.29) ---- */
int rgo_predict_element(const rgo_refel *r, double gamma, double dt, const double *J, const double *met,
                        const sreal *Ua, sreal *Ulev, sreal *avgU, sreal *avgF)
{
    const int N = r->N, M = r->M, E = (M - 1) * N;
    sreal *U0 = malloc(sizeof(sreal) * N * NVAR), *U1 = malloc(sizeof(sreal) * E * NVAR);
    sreal *F0 = malloc(sizeof(sreal) * 3 * N * NVAR), *F1 = malloc(sizeof(sreal) * 3 * E * NVAR);
    sreal *Un = malloc(sizeof(sreal) * E * NVAR);
    sreal Fp[3][NVAR], u[NVAR];
    for (int i = 0; i < N; i++)
        for (int v = 0; v < NVAR; v++) U0[i * NVAR + v] = J[i] * Ua[i * NVAR + v];
    /* nodal fluxes in mapped form, eq. (5.23) with the zone's own metrics */
#define NODAL_FLUX(Uhat, i, Fout, stride)                                                     \
    do {                                                                                      \
        int ii = (i) % N;                                                                     \
        for (int v = 0; v < NVAR; v++) u[v] = (Uhat)[(i) * NVAR + v] / J[ii];                 \
        phys_flux(u, gamma, Fp);                                                              \
        for (int d = 0; d < 3; d++)                                                           \
            for (int v = 0; v < NVAR; v++) {                                                  \
                sreal s = 0.0;                                                                \
                for (int nn = 0; nn < 3; nn++) s += met[ii * 9 + d * 3 + nn] * Fp[nn][v];     \
                (Fout)[((size_t)d * (stride) + (i)) * NVAR + v] = dt * s;                     \
            }                                                                                 \
    } while (0)
    for (int i = 0; i < N; i++) NODAL_FLUX(U0, i, F0, N);
    /* initial iterate: every evolving level equals the tau = 0 level */
    for (int i = 0; i < E; i++)
        for (int v = 0; v < NVAR; v++) U1[i * NVAR + v] = U0[(i % N) * NVAR + v];
    for (int it = 0; it < r->order; it++) {
        for (int i = 0; i < E; i++) NODAL_FLUX(U1, i, F1, E);
        for (int i = 0; i < E; i++)
            for (int v = 0; v < NVAR; v++) {
                sreal s = 0.0;
                for (int j = 0; j < N; j++) {
                    s += r->Kt0[i * N + j] * U0[j * NVAR + v];
                    for (int d = 0; d < 3; d++) s -= r->Kd0[d][i * N + j] * F0[((size_t)d * N + j) * NVAR + v];
                }
                for (int j = 0; j < E; j++)
                    for (int d = 0; d < 3; d++) s -= r->Kd[d][i * E + j] * F1[((size_t)d * E + j) * NVAR + v];
                Un[i * NVAR + v] = s;
            }
        memcpy(U1, Un, sizeof(sreal) * E * NVAR);
    }
    if (Ulev) {
        memcpy(Ulev, U0, sizeof(sreal) * N * NVAR);
        memcpy(Ulev + N * NVAR, U1, sizeof(sreal) * E * NVAR);
    }
    /* time averages over the Gauss levels (step 10 of Section V.d) */
    for (int i = 0; i < N; i++) {
        for (int v = 0; v < NVAR; v++) avgU[i * NVAR + v] = 0.0;
        for (int k = 0; k < 3 * NVAR; k++) avgF[i * 3 * NVAR + k] = 0.0;
        for (int t = 1; t < M; t++) {
            for (int v = 0; v < NVAR; v++) u[v] = U1[((t - 1) * N + i) * NVAR + v] / J[i];
            phys_flux(u, gamma, Fp);
            for (int v = 0; v < NVAR; v++) avgU[i * NVAR + v] += r->wt[t] * u[v];
            for (int d = 0; d < 3; d++)
                for (int v = 0; v < NVAR; v++) avgF[i * 3 * NVAR + d * NVAR + v] += r->wt[t] * Fp[d][v];
        }
    }
#undef NODAL_FLUX
    free(U0); free(U1); free(F0); free(F1); free(Un);
    return 0;
}

static void predictor_zone(step_ws *w, int z)
{
    const rgo_mesh *m = w->m;
    const int N = m->ref.N;
    sreal *Ua = malloc(sizeof(sreal) * N * NVAR);
    for (int i = 0; i < N; i++) {
        const double *x = &m->nodex[((size_t)z * N + i) * 3];
        for (int v = 0; v < IBX; v++) Ua[i * NVAR + v] = weno_eval(w, z, v, x);
        divfree_eval(w, z, x, &Ua[i * NVAR + IBX]);
    }
    rgo_predict_element(&m->ref, w->gamma, w->dt, &m->nodeJ[(size_t)z * N], &m->nodeMet[(size_t)z * N * 9], Ua,
                        NULL, &w->avgU[(size_t)z * N * NVAR], &w->avgF[(size_t)z * N * 3 * NVAR]);
    free(Ua);
}

/* Conserved state of zone z at t^n: its eight averages after the boundary
 * fill (zone B as carried, consistent with the total energy) */
static void zone_state(const step_ws *w, int z, sreal *U)
{
    const int nz = w->m->nz;
    for (int v = 0; v < NVAR; v++) U[v] = w->U[(size_t)v * nz + z];
}

/* time-averaged state and flux of zone z at reference point xi; in the
 * re-solve of the first-order fallback, the zone's conserved state at t^n
 * and the physical flux of that state instead */
static void trace(const step_ws *w, int z, const double *xi, sreal *U, sreal F[3][NVAR])
{
    const rgo_mesh *m = w->m;
    const int N = m->ref.N;
    if (w->first_order) {
        zone_state(w, z, U);
        phys_flux(U, w->gamma, F);
        return;
    }
    for (int v = 0; v < NVAR; v++) { U[v] = 0.0; F[0][v] = F[1][v] = F[2][v] = 0.0; }
    for (int l = 0; l < N; l++) {
        double p = refel_psi(&m->ref, l, xi);
        if (p == 0.0) continue;
        const sreal *au = &w->avgU[((size_t)z * N + l) * NVAR], *af = &w->avgF[((size_t)z * N + l) * 3 * NVAR];
        for (int v = 0; v < NVAR; v++) U[v] += p * au[v];
        for (int d = 0; d < 3; d++)
            for (int v = 0; v < NVAR; v++) F[d][v] += p * af[d * NVAR + v];
    }
}

/* ---- face flux integral ---- */
static void face_flux(step_ws *w, int f)
{
    const rgo_mesh *m = w->m;
    const int Q = m->nq_face * m->nq_face;
    int zL = m->face_zone[2 * f], zR = m->face_zone[2 * f + 1];
    int lL = m->face_lf[2 * f], lR = m->face_lf[2 * f + 1];
    sreal *Phi = &w->Phi[(size_t)f * NVAR];
    for (int v = 0; v < NVAR; v++) Phi[v] = 0.0;
    for (int q = 0; q < Q; q++) {
        const double *n = &m->fn[(f * RGO_MAXQ + q) * 3];
        double xi[3];
        sreal UL[NVAR], UR[NVAR], FL[3][NVAR], FR[3][NVAR], FnL[NVAR], FnR[NVAR], Fs[NVAR];
        face_ref_point(m, lL, q, xi);
        trace(w, zL, xi, UL, FL);
        face_ref_point(m, lR, m->face_perm[f * RGO_MAXQ + q], xi);
        trace(w, zR, xi, UR, FR);
        for (int v = 0; v < NVAR; v++) {
            FnL[v] = n[0] * FL[0][v] + n[1] * FL[1][v] + n[2] * FL[2][v];
            FnR[v] = n[0] * FR[0][v] + n[1] * FR[1][v] + n[2] * FR[2][v];
        }
        hll_flux(UL, UR, FnL, FnR, n, w->gamma, Fs);
        for (int v = 0; v < NVAR; v++) Phi[v] += m->fdA[f * RGO_MAXQ + q] * Fs[v];
    }
}

/* ---- multidimensional HLL electric field at one edge point ---- */
/* states in counter-clockwise order about t (SW, SE, NE, NW); E[s] = time-averaged E vector */
sreal rgo_emf4(const sreal U[4][NVAR], const sreal E[4][3], const double cen[4][3], const double *t,
               double gamma)
{
    /* frame: directions from the zone centroids, orthonormalised symmetrically */
    double u[3], v[3];
    for (int i = 0; i < 3; i++) {
        u[i] = cen[1][i] + cen[2][i] - cen[0][i] - cen[3][i];
        v[i] = cen[2][i] + cen[3][i] - cen[0][i] - cen[1][i];
    }
    double pu = dot3(u, t), pv = dot3(v, t);
    for (int i = 0; i < 3; i++) { u[i] -= pu * t[i]; v[i] -= pv * t[i]; }
    double nu = sqrt(dot3(u, u)), nv = sqrt(dot3(v, v));
    double b[3], bp[3], e1[3], e2[3];
    for (int i = 0; i < 3; i++) b[i] = u[i] / nu + v[i] / nv;
    double nb = sqrt(dot3(b, b));
    for (int i = 0; i < 3; i++) b[i] /= nb;
    cross3(t, b, bp);
    const double h = sqrt(0.5);
    for (int i = 0; i < 3; i++) { e1[i] = h * (b[i] - bp[i]); e2[i] = h * (b[i] + bp[i]); }
    sreal ap1 = 0.0, am1 = 0.0, ap2 = 0.0, am2 = 0.0, Et[4], B1[4], B2[4];
    for (int s = 0; s < 4; s++) {
        sreal v1 = dot3m(&U[s][IMX], e1) / U[s][IRHO], v2 = dot3m(&U[s][IMX], e2) / U[s][IRHO];
        sreal c1 = fast_speed(U[s], gamma, e1), c2 = fast_speed(U[s], gamma, e2);
        ap1 = s_max(ap1, v1 + c1); am1 = s_max(am1, -(v1 - c1));
        ap2 = s_max(ap2, v2 + c2); am2 = s_max(am2, -(v2 - c2));
        Et[s] = dot3m(E[s], t);
        B1[s] = dot3m(&U[s][IBX], e1);
        B2[s] = dot3m(&U[s][IBX], e2);
    }
    /* SW=0, SE=1, NE=2, NW=3 */
    sreal den = (ap1 + am1) * (ap2 + am2);
    sreal Es = (ap1 * ap2 * Et[0] + ap1 * am2 * Et[3] + am1 * ap2 * Et[1] + am1 * am2 * Et[2]) / den;
    Es += ap1 * am1 * (0.5 * (B2[1] + B2[2]) - 0.5 * (B2[0] + B2[3])) / (ap1 + am1);
    Es -= ap2 * am2 * (0.5 * (B1[2] + B1[3]) - 0.5 * (B1[0] + B1[1])) / (ap2 + am2);
    return Es;
}

/* three zones about an edge: mean of the 1-D HLL induction fluxes of the three faces */
sreal rgo_emf3(const sreal U[3][NVAR], const sreal E[3][3], const double n[3][3], const double *t,
               double gamma)
{
    sreal acc = 0.0;
    for (int s = 0; s < 3; s++) {
        int s2 = (s + 1) % 3;
        const double *nn = n[s];
        sreal FL[NVAR] = {0}, FR[NVAR] = {0}, Fs[NVAR];
        double tn[3];
        /* induction flux n x E for B, zero for the fluid rows (they do not enter) */
        cross3m(nn, E[s], &FL[IBX]);
        cross3m(nn, E[s2], &FR[IBX]);
        hll_flux(U[s], U[s2], FL, FR, nn, gamma, Fs);
        cross3(t, nn, tn);
        acc += -(Fs[IBX] * tn[0] + Fs[IBY] * tn[1] + Fs[IBZ] * tn[2]);
    }
    return acc / 3.0;
}

static void edge_emf(step_ws *w, int e)
{
    const rgo_mesh *m = w->m;
    const double simpson[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    int nze = m->edge_nz[e];
    sreal G = 0.0;
    for (int p = 0; p < 3; p++) {
        double s = 0.5 * p, cen[4][3];
        sreal U[4][NVAR], E[4][3], F[3][NVAR];
        const double *t = &m->et[e * 9 + p * 3];
        for (int k = 0; k < nze; k++) {
            int z = m->edge_zone[4 * e + k], le = m->edge_le[4 * e + k], rev = m->edge_rev[4 * e + k];
            double xi[3];
            edge_ref_point(le, rev ? 1.0 - s : s, xi);
            trace(w, z, xi, U[k], F);
            /* E_x = H[B_y], E_y = F[B_z], E_z = G[B_x]  (eq. 2.3) */
            E[k][0] = F[2][IBY];
            E[k][1] = F[0][IBZ];
            E[k][2] = F[1][IBX];
            memcpy(cen[k], &m->cen[3 * z], 24);
        }
        sreal Es;
        if (nze == 4) {
            Es = rgo_emf4(U, E, cen, t, w->gamma);
        } else {
            /* normals of the faces between consecutive zones, from zone k toward zone k+1 */
            double nrm[3][3];
            for (int k = 0; k < 3; k++) {
                int z = m->edge_zone[4 * e + k], z2 = m->edge_zone[4 * e + (k + 1) % 3];
                int le = m->edge_le[4 * e + k], rev = m->edge_rev[4 * e + k];
                int lfs = -1;
                for (int lf = 0; lf < 6; lf++)
                    if (m->zone_nbr[6 * z + lf] == z2) lfs = lf;
                double xi[3], x[3], jac[9], hu[3], hv[3];
                edge_ref_point(le, rev ? 1.0 - s : s, xi);
                zone_map(m, z, xi, x, jac);
                int axis = lfs / 2, ua = (axis == 0) ? 1 : 0, va = (axis == 2) ? 1 : 2;
                for (int i = 0; i < 3; i++) { hu[i] = jac[i * 3 + ua]; hv[i] = jac[i * 3 + va]; }
                cross3(hu, hv, nrm[k]);
                double d[3];
                for (int i = 0; i < 3; i++) d[i] = m->cen[3 * z2 + i] - m->cen[3 * z + i];
                double sg = dot3(nrm[k], d) > 0 ? 1.0 : -1.0, nn = sqrt(dot3(nrm[k], nrm[k]));
                for (int i = 0; i < 3; i++) nrm[k][i] *= sg / nn;
            }
            Es = rgo_emf3((const sreal(*)[NVAR])U, (const sreal(*)[3])E, (const double(*)[3])nrm, t, w->gamma);
        }
        G += simpson[p] * Es * m->edl[e * 3 + p];
    }
    w->Gam[e] = G;
}

/* zone averages of zone z after the finite-volume update with the current
 * face fluxes; zone B starts from the divergence-free reconstruction's mean
 * (step 10 of Section IV.b), or, for a zone of the first-order fallback
 * (own != 0), from its own conserved B, so that its update is the
 * first-order finite-volume scheme on its eight averages */
static void update_zone(const step_ws *w, int z, int own, sreal *u)
{
    const rgo_mesh *m = w->m;
    const int nz = m->nz;
    sreal acc[NVAR] = {0};
    for (int lf = 0; lf < 6; lf++) {
        int f = m->zone_face[6 * z + lf];
        double sg = (m->face_zone[2 * f] == z) ? 1.0 : -1.0;
        for (int v = 0; v < NVAR; v++) acc[v] += sg * w->Phi[(size_t)f * NVAR + v];
    }
    const sreal *bcz = &w->bc[(size_t)z * 3 * w->nbx];
    for (int v = 0; v < NVAR; v++) {
        sreal base = (v >= IBX && !own) ? bcz[(v - IBX) * w->nbx] : w->U[(size_t)v * nz + z];
        u[v] = base - w->dt / m->vol[z] * acc[v];
    }
}

/* ---------------- the step ---------------- */
static void setup_bases(step_ws *w)
{
    int p = w->m->order;
    w->deg = p - 1;
    w->nc = taylor_list(w->deg, w->te);
    /* component c: every monomial of degree <= p-1, plus degree-p monomials containing x_c */
    for (int c = 0; c < 3; c++) {
        int n = 0;
        w->be[c][n][0] = w->be[c][n][1] = w->be[c][n][2] = 0;
        n++;
        for (int a = 0; a < w->nc; a++) { memcpy(w->be[c][n], w->te[a], sizeof(int) * 3); n++; }
        for (int a = p; a >= 0; a--)
            for (int b = p - a; b >= 0; b--) {
                int e[3] = {a, b, p - a - b};
                if (e[c] >= 1) { memcpy(w->be[c][n], e, sizeof(int) * 3); n++; }
            }
        w->nbx = n;
    }
}

int rgo_run_step(const rgo_mesh *m, double gamma, double dt, int bc_kind, int flags, double weno_eps,
                 double flat_kappa, const sreal *U, const sreal *Bf, sreal *Uout, sreal *Bfout, sreal *dbgPhi,
                 sreal *dbgGam, unsigned char *fallback_zones, double *eta_out)
{
    step_ws w;
    memset(&w, 0, sizeof(w));
    w.m = m;
    w.gamma = gamma;
    w.dt = dt;
    w.flags = flags;
    w.weno_eps = weno_eps;
    setup_bases(&w);
    const int nz = m->nz, nf = m->nf, ne = m->ne, N = m->ref.N, g = m->n_ghost, Nr = m->n_rad;
    w.U = malloc(sizeof(sreal) * NVAR * nz);
    w.Bf = malloc(sizeof(sreal) * nf);
    memcpy(w.U, U, sizeof(sreal) * NVAR * nz);
    memcpy(w.Bf, Bf, sizeof(sreal) * nf);
    if (bc_kind == 0) boundary_fill(&w);

    w.recon = calloc(nz, 1);
    for (int z = 0; z < nz; z++) {
        int k = m->zone_shell[z];
        w.recon[z] = (k >= g - 1 && k <= g + Nr);
    }
    if (flat_kappa > 0.0) {
        w.flat_kappa = flat_kappa;
        w.eta = calloc(nz, sizeof(sreal));
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            if (w.recon[z]) w.eta[z] = flattener_eta(&w, z);
        if (eta_out)
            for (int z = 0; z < nz; z++) eta_out[z] = SRE(w.eta[z]);
    }
    w.wc = calloc((size_t)nz * NVAR * w.nc, sizeof(sreal));
    w.bface = calloc((size_t)nf * RGO_MAXQ, sizeof(sreal));
    w.bc = calloc((size_t)nz * 3 * w.nbx, sizeof(sreal));
    w.avgU = calloc((size_t)nz * N * NVAR, sizeof(sreal));
    w.avgF = calloc((size_t)nz * N * 3 * NVAR, sizeof(sreal));
    w.Phi = calloc((size_t)nf * NVAR, sizeof(sreal));
    w.Gam = calloc(ne, sizeof(sreal));

#pragma omp parallel for schedule(dynamic, 8)
    for (int z = 0; z < nz; z++)
        if (w.recon[z]) weno_zone(&w, z);

    char *fneed = calloc(nf, 1);
    for (int z = 0; z < nz; z++)
        if (w.recon[z])
            for (int lf = 0; lf < 6; lf++) fneed[m->zone_face[6 * z + lf]] = 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int f = 0; f < nf; f++)
        if (fneed[f]) face_nodal_b(&w, f);

    int fail = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : fail)
    for (int z = 0; z < nz; z++)
        if (w.recon[z]) {
            fail |= divfree_zone(&w, z);
            predictor_zone(&w, z);
        }

    /* corrector on the faces and edges of the interior zones */
    char *upd = calloc(nz, 1), *fupd = calloc(nf, 1), *eupd = calloc(ne, 1);
    for (int z = 0; z < nz; z++) {
        int k = m->zone_shell[z];
        upd[z] = (k >= g && k < g + Nr);
        if (upd[z])
            for (int lf = 0; lf < 6; lf++) fupd[m->zone_face[6 * z + lf]] = 1;
    }
    for (int f = 0; f < nf; f++)
        if (fupd[f])
            for (int k = 0; k < 4; k++) eupd[m->face_edges[4 * f + k]] = 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int f = 0; f < nf; f++)
        if (fupd[f]) face_flux(&w, f);
#pragma omp parallel for schedule(dynamic, 64)
    for (int e = 0; e < ne; e++)
        if (eupd[e]) edge_emf(&w, e);

    /* first-order fallback (flag FLAG_FALLBACK).  The paper leaves positivity
     * to the ruggedised-WENO literature (Section I); this oracle follows the
     * step's own definition: an interior zone is flagged when the update with
     * the current fluxes would leave its density or pressure not positive
     * (or not finite), and every face and edge of a flagged zone is solved
     * again with the same Riemann solvers on the zones' conserved states at
     * t^n, and a flagged zone's B average is advanced from its own value
     * (not the reconstruction's mean), so its update is the first-order
     * finite-volume scheme.  A re-solved face can in turn drive a neighbour
     * negative, so the check is repeated with the new fluxes, for at most
     * FALLBACK_ROUNDS rounds and until a round flags no new zone; the update
     * below then takes the final fluxes and electric fields */
    char *bad = calloc(nz, 1);
    if (flags & FLAG_FALLBACK) {
        char *fbad = calloc(nf, 1), *ebad = calloc(ne, 1);
        for (int round = 0; round < FALLBACK_ROUNDS; round++) {
            int added = 0;
            for (int z = 0; z < nz; z++) {
                if (!upd[z] || bad[z]) continue;
                sreal u[NVAR];
                update_zone(&w, z, 0, u);
                if (SRE(u[IRHO]) > 0.0 && SRE(pressure(u, gamma)) > 0.0) continue;
                bad[z] = (char)(round + 1);   /* the round that flagged it, 1-based */
                added = 1;
                for (int lf = 0; lf < 6; lf++) {
                    int f = m->zone_face[6 * z + lf];
                    fbad[f] = 1;
                    for (int k = 0; k < 4; k++) ebad[m->face_edges[4 * f + k]] = 1;
                }
            }
            if (!added) break;
            w.first_order = 1;
#pragma omp parallel for schedule(dynamic, 64)
            for (int f = 0; f < nf; f++)
                if (fbad[f]) face_flux(&w, f);
#pragma omp parallel for schedule(dynamic, 64)
            for (int e = 0; e < ne; e++)
                if (ebad[e]) edge_emf(&w, e);
            w.first_order = 0;
        }
        free(fbad); free(ebad);
    }
    if (fallback_zones) memcpy(fallback_zones, bad, nz);

    /* finite-volume update of the eight zone averages, zone B taken from the
     * divergence-free reconstruction (step 10 of Section IV.b) */
    memcpy(Uout, w.U, sizeof(sreal) * NVAR * nz);
    for (int z = 0; z < nz; z++) {
        if (!upd[z]) continue;
        sreal u[NVAR];
        update_zone(&w, z, bad[z], u);
        for (int v = 0; v < NVAR; v++) Uout[(size_t)v * nz + z] = u[v];
    }
    free(bad);
    /* constrained transport: Faraday's law on each face (eqs. 2.5-2.6) */
    memcpy(Bfout, w.Bf, sizeof(sreal) * nf);
    for (int f = 0; f < nf; f++) {
        if (!fupd[f]) continue;
        sreal s = 0.0;
        for (int k = 0; k < 4; k++) s += m->face_esign[4 * f + k] * w.Gam[m->face_edges[4 * f + k]];
        Bfout[f] = w.Bf[f] - dt / m->farea[f] * s;
    }
    if (dbgPhi) memcpy(dbgPhi, w.Phi, sizeof(sreal) * nf * NVAR);
    if (dbgGam) memcpy(dbgGam, w.Gam, sizeof(sreal) * ne);

    free(w.U); free(w.Bf); free(w.recon); free(w.wc); free(w.bface); free(w.bc);
    free(w.avgU); free(w.avgF); free(w.Phi); free(w.Gam); free(w.eta);
    free(fneed); free(upd); free(fupd); free(eupd);
    return fail ? -1 : 0;
}

#ifndef RGO_COMPLEX
/* test access to single parts of the step (the real oracle only) */

/* reconstructed fields of one zone at arbitrary points (test access) */
int rgo_run_recon(const rgo_mesh *m, int flags, double weno_eps, const double *U, const double *Bf, int z,
                  int npts, const double *pts, double *weno_vals, double *divB_vals)
{
    step_ws w;
    memset(&w, 0, sizeof(w));
    w.m = m;
    w.flags = flags;
    w.weno_eps = weno_eps;
    w.gamma = 5.0 / 3.0;
    setup_bases(&w);
    const int nz = m->nz, nf = m->nf;
    w.U = malloc(sizeof(double) * NVAR * nz);
    w.Bf = malloc(sizeof(double) * nf);
    memcpy(w.U, U, sizeof(double) * NVAR * nz);
    memcpy(w.Bf, Bf, sizeof(double) * nf);
    w.recon = calloc(nz, 1);
    w.wc = calloc((size_t)nz * NVAR * w.nc, sizeof(double));
    w.bface = calloc((size_t)nf * RGO_MAXQ, sizeof(double));
    w.bc = calloc((size_t)nz * 3 * w.nbx, sizeof(double));
    /* the zone and its face neighbours (each must have a full stencil) */
    int list[7];
    list[0] = z;
    for (int lf = 0; lf < 6; lf++) list[1 + lf] = m->zone_nbr[6 * z + lf];
    int edge = 0;
    for (int i = 0; i < 7 && !edge; i++) {
        edge = list[i] < 0;
        for (int lf = 0; lf < 6 && !edge; lf++) edge = m->zone_nbr[6 * list[i] + lf] < 0;
    }
    if (edge) {
        free(w.U); free(w.Bf); free(w.recon); free(w.wc); free(w.bface); free(w.bc);
        return -1;
    }
    for (int i = 0; i < 7; i++) {
        w.recon[list[i]] = 1;
        weno_zone(&w, list[i]);
    }
    for (int lf = 0; lf < 6; lf++) face_nodal_b(&w, m->zone_face[6 * z + lf]);
    int rc = divfree_zone(&w, z);
    for (int p = 0; p < npts; p++) {
        if (weno_vals)
            for (int v = 0; v < NVAR; v++) weno_vals[p * NVAR + v] = weno_eval(&w, z, v, &pts[3 * p]);
        if (divB_vals) divfree_eval(&w, z, &pts[3 * p], &divB_vals[3 * p]);
    }
    free(w.U); free(w.Bf); free(w.recon); free(w.wc); free(w.bface); free(w.bc);
    return rc;
}

/* divergence-identity residual of the B coefficients and nodal face values (test access) */
int rgo_run_divfree_coeffs(const rgo_mesh *m, int flags, double weno_eps, const double *U, const double *Bf, int z,
                           double *coeffs, int *exps, double *face_nodal)
{
    step_ws w;
    memset(&w, 0, sizeof(w));
    w.m = m;
    w.flags = flags;
    w.weno_eps = weno_eps;
    setup_bases(&w);
    const int nz = m->nz, nf = m->nf, Q = m->nq_face * m->nq_face;
    w.U = malloc(sizeof(double) * NVAR * nz);
    w.Bf = malloc(sizeof(double) * nf);
    memcpy(w.U, U, sizeof(double) * NVAR * nz);
    memcpy(w.Bf, Bf, sizeof(double) * nf);
    w.recon = calloc(nz, 1);
    w.wc = calloc((size_t)nz * NVAR * w.nc, sizeof(double));
    w.bface = calloc((size_t)nf * RGO_MAXQ, sizeof(double));
    w.bc = calloc((size_t)nz * 3 * w.nbx, sizeof(double));
    int list[7];
    list[0] = z;
    for (int lf = 0; lf < 6; lf++) list[1 + lf] = m->zone_nbr[6 * z + lf];
    for (int i = 0; i < 7; i++)
        if (list[i] < 0) { free(w.U); free(w.Bf); free(w.recon); free(w.wc); free(w.bface); free(w.bc); return -1; }
    for (int i = 0; i < 7; i++)
        for (int lf = 0; lf < 6; lf++)
            if (m->zone_nbr[6 * list[i] + lf] < 0) {
                free(w.U); free(w.Bf); free(w.recon); free(w.wc); free(w.bface); free(w.bc);
                return -1;
            }
    for (int i = 0; i < 7; i++) {
        w.recon[list[i]] = 1;
        weno_zone(&w, list[i]);
    }
    for (int lf = 0; lf < 6; lf++) face_nodal_b(&w, m->zone_face[6 * z + lf]);
    int rc = divfree_zone(&w, z);
    if (coeffs) memcpy(coeffs, w.bc + (size_t)z * 3 * w.nbx, sizeof(double) * 3 * w.nbx);
    if (exps)
        for (int c = 0; c < 3; c++)
            for (int k = 0; k < w.nbx; k++)
                for (int i = 0; i < 3; i++) exps[(c * w.nbx + k) * 3 + i] = w.be[c][k][i];
    if (face_nodal)
        for (int lf = 0; lf < 6; lf++) {
            int f = m->zone_face[6 * z + lf];
            for (int q = 0; q < Q; q++) face_nodal[lf * Q + q] = w.bface[(size_t)f * RGO_MAXQ + q];
        }
    int nbx = w.nbx;
    free(w.U); free(w.Bf); free(w.recon); free(w.wc); free(w.bface); free(w.bc);
    return rc < 0 ? rc : nbx;
}

/* WENO-AO order indicator (test access): for every reconstructed zone the
 * smallest over the eight variables of the large stencil's nonlinear weight
 * over its linear weight (Section III); other zones get 0 */
int rgo_run_weno_order(const rgo_mesh *m, int bc_kind, int flags, double weno_eps, const double *U, const double *Bf,
                       double *whi)
{
    step_ws w;
    memset(&w, 0, sizeof(w));
    w.m = m;
    w.flags = flags;
    w.weno_eps = weno_eps;
    setup_bases(&w);
    const int nz = m->nz, nf = m->nf, g = m->n_ghost, Nr = m->n_rad;
    w.U = malloc(sizeof(double) * NVAR * nz);
    w.Bf = malloc(sizeof(double) * nf);
    memcpy(w.U, U, sizeof(double) * NVAR * nz);
    memcpy(w.Bf, Bf, sizeof(double) * nf);
    if (bc_kind == 0) boundary_fill(&w);
    w.wc = calloc((size_t)nz * NVAR * w.nc, sizeof(double));
    w.whi = whi;
    for (int z = 0; z < nz; z++) whi[z] = 0.0;
#pragma omp parallel for schedule(dynamic, 8)
    for (int z = 0; z < nz; z++) {
        int k = m->zone_shell[z];
        if (k >= g - 1 && k <= g + Nr) weno_zone(&w, z);
    }
    free(w.U); free(w.Bf); free(w.wc);
    return 0;
}

/* WENO-AO internals of one zone (test access): for each of the eight
 * variables, out[v * (16 + nc) + ...] holds the smoothness indicator of the
 * large stencil and of the seven small stencils, the eight normalised
 * nonlinear weights (large stencil first) and the nc blended Taylor
 * coefficients (Section III).  No boundary fill: U holds every zone's
 * average.  Returns nc. */
int rgo_run_weno_detail(const rgo_mesh *m, int flags, double weno_eps, const double *U, int z, double *out)
{
    step_ws w;
    memset(&w, 0, sizeof(w));
    w.m = m;
    w.flags = flags;
    w.weno_eps = weno_eps;
    setup_bases(&w);
    const int nz = m->nz;
    w.U = malloc(sizeof(double) * NVAR * nz);
    memcpy(w.U, U, sizeof(double) * NVAR * nz);
    w.wc = calloc((size_t)nz * NVAR * w.nc, sizeof(double));
    w.dbg_z = z;
    w.dbg = out;
    weno_zone(&w, z);
    int nc = w.nc;
    free(w.U); free(w.wc);
    return nc;
}

/* the large-stencil least-squares matrix of zone z (test access): A[ns][nc]
 * row-major in the stencil's member order; returns ns */
int rgo_run_weno_rows(const rgo_mesh *m, int z, double *A)
{
    step_ws w;
    memset(&w, 0, sizeof(w));
    w.m = m;
    setup_bases(&w);
    weno_rows(&w, z, A);
    return m->st_n[z];
}

double rgo_run_cfl(const rgo_mesh *m, double gamma, double cfl, const double *U)
{
    int g = m->n_ghost, Nr = m->n_rad;
    double dtmin = 1e300;
    for (int z = 0; z < m->nz; z++) {
        int k = m->zone_shell[z];
        if (k < g || k >= g + Nr) continue;
        /* in-sphere diameter: twice the least distance from the centroid to a face plane */
        double dmin = 1e300;
        for (int lf = 0; lf < 6; lf++) {
            int f = m->zone_face[6 * z + lf];
            double nb[3] = {0, 0, 0};
            for (int q = 0; q < m->nq_face * m->nq_face; q++)
                for (int i = 0; i < 3; i++) nb[i] += m->fdA[f * RGO_MAXQ + q] * m->fn[(f * RGO_MAXQ + q) * 3 + i];
            double nn = sqrt(dot3(nb, nb)), d[3];
            for (int i = 0; i < 3; i++) d[i] = m->fcen[3 * f + i] - m->cen[3 * z + i];
            dmin = fmin(dmin, fabs(dot3(d, nb)) / nn);
        }
        double u[NVAR];
        for (int v = 0; v < NVAR; v++) u[v] = U[(size_t)v * m->nz + z];
        double rho = u[IRHO], vv = sqrt(dot3(&u[IMX], &u[IMX])) / rho;
        double a2 = gamma * pressure(u, gamma) / rho, b2 = dot3(&u[IBX], &u[IBX]) / rho;
        double cf = sqrt(a2 + b2);
        dtmin = fmin(dtmin, cfl * 2.0 * dmin / (vv + cf));
    }
    return dtmin;
}

#endif /* RGO_COMPLEX */

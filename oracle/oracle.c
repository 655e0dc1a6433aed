/*
 * Public entry points of the oracle (test infrastructure only).  Loaded by the
 * test-suite through ctypes; never by the GPU library.
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int rgo_run_step(const rgo_mesh *m, double gamma, double dt, int bc_kind, int flags, double weno_eps,
                 double flat_kappa, const double *U, const double *Bf, double *Uout, double *Bfout, double *dbgPhi,
                 double *dbgGam, unsigned char *fallback_zones, double *eta_out);
/* the same step with complex state (scheme_cx.c): state arrays are
 * interleaved (real, imaginary) pairs, i.e. C99 double complex */
int rgo_run_step_cx(const rgo_mesh *m, double gamma, double dt, int bc_kind, int flags, double weno_eps,
                    double flat_kappa, const double _Complex *U, const double _Complex *Bf, double _Complex *Uout,
                    double _Complex *Bfout, double _Complex *dbgPhi, double _Complex *dbgGam,
                    unsigned char *fallback_zones, double *eta_out);
int rgo_run_weno_order(const rgo_mesh *m, int bc_kind, int flags, double weno_eps, const double *U, const double *Bf,
                       double *whi);
int rgo_run_recon(const rgo_mesh *m, int flags, double weno_eps, const double *U, const double *Bf, int z,
                  int npts, const double *pts, double *weno_vals, double *divB_vals);
int rgo_run_divfree_coeffs(const rgo_mesh *m, int flags, double weno_eps, const double *U, const double *Bf, int z,
                           double *coeffs, int *exps, double *face_nodal);
double rgo_run_cfl(const rgo_mesh *m, double gamma, double cfl, const double *U);
void rgo_run_init_blast(const rgo_mesh *m, const double *axis, const double *centre, double radius, double rho,
                        double p_in, double p, double B0, double gamma, double *U, double *Bf);
int rgo_run_weno_rows(const rgo_mesh *m, int z, double *A);
int rgo_run_weno_detail(const rgo_mesh *m, int flags, double weno_eps, const double *U, int z, double *out);
double rgo_emf3(const double U[3][NVAR], const double E[3][3], const double n[3][3], const double *t, double gamma);
void rgo_run_init_harmonic(const rgo_mesh *m, const double *rho, const double *v, const double *A, double p,
                           double gamma, double *U, double *Bf);
void rgo_run_init_tube(const rgo_mesh *m, const double *left, const double *right, double Br0, double r0,
                       double rm, double delta, double gamma, double *U, double *Bf);
void rgo_run_init_alfven(const rgo_mesh *m, const double *frame, double rho, double p, double B0, double dB,
                         double wavelength, double gamma, double t, double *U, double *Bf);
int rgo_predict_element(const rgo_refel *r, double gamma, double dt, const double *J, const double *met,
                        const double *Ua, double *Ulev, double *avgU, double *avgF);
double rgo_emf4(const double U[4][NVAR], const double E[4][3], const double cen[4][3], const double *t,
                double gamma);

rgo_mesh *rgo_create(int n_ang, int n_rad, double r_in, double r_out, int n_ghost, int map_order, int order)
{
    if (order < 3 || order > 4 || map_order < 2 || map_order > 3 || n_rad < 1) return NULL;
    if (n_ghost < order - 1) return NULL;
    rgo_mesh *m = calloc(1, sizeof(rgo_mesh));
    m->n_ang = n_ang;
    m->n_rad = n_rad;
    m->n_ghost = n_ghost;
    m->ktot = n_rad + 2 * n_ghost;
    m->map_order = map_order;
    m->order = order;
    m->r_in = r_in;
    m->r_out = r_out;
    m->nq_face = order - 1;
    m->ncub_ang = (order == 3) ? 8 : 10;
    m->ncub_rad = 6;
    if (refel_init(&m->ref, order)) { free(m); return NULL; }
    if (mesh_build_topology(m)) { free(m); return NULL; }
    if (mesh_build_geometry(m)) { free(m); return NULL; }
    return m;
}

void rgo_destroy(rgo_mesh *m)
{
    if (!m) return;
    void *p[] = {m->radius, m->vert, m->quad, m->zone_quad, m->zone_shell, m->zone_face, m->zone_edge,
                 m->zone_nbr, m->face_zone, m->face_lf, m->face_perm, m->edge_hv, m->edge_nz, m->edge_zone,
                 m->edge_le, m->edge_rev, m->face_edges, m->face_esign, m->st_n, m->st_z, m->snode, m->vol,
                 m->cen, m->len, m->mom, m->cub, m->nodex, m->nodeJ, m->nodeMet, m->fx, m->fn, m->fdA,
                 m->farea, m->fcen, m->ex, m->et, m->edl};
    for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); i++) free(p[i]);
    refel_free(&m->ref);
    free(m);
}

/* nz, nf, ne, ktot, n_ghost, nquad, nv, N(ADER nodes) */
void rgo_sizes(const rgo_mesh *m, int64_t *out)
{
    out[0] = m->nz; out[1] = m->nf; out[2] = m->ne; out[3] = m->ktot;
    out[4] = m->n_ghost; out[5] = m->nquad; out[6] = m->nv; out[7] = m->ref.N;
}

void rgo_zone_data(const rgo_mesh *m, double *cen, double *vol, int *shell, int *stencil_n)
{
    if (cen) memcpy(cen, m->cen, sizeof(double) * 3 * m->nz);
    if (vol) memcpy(vol, m->vol, sizeof(double) * m->nz);
    if (shell) memcpy(shell, m->zone_shell, sizeof(int) * m->nz);
    if (stencil_n) memcpy(stencil_n, m->st_n, sizeof(int) * m->nz);
}

void rgo_zone_faces(const rgo_mesh *m, int *faces, int *nbrs)
{
    if (faces) memcpy(faces, m->zone_face, sizeof(int) * 6 * m->nz);
    if (nbrs) memcpy(nbrs, m->zone_nbr, sizeof(int) * 6 * m->nz);
}

/* face centre, averaged unit normal (canonical orientation), area, owner/other zones */
void rgo_face_data(const rgo_mesh *m, double *cen, double *nrm, double *area, int *zones)
{
    const int Q = m->nq_face * m->nq_face;
    for (int f = 0; f < m->nf; f++) {
        if (cen) memcpy(&cen[3 * f], &m->fcen[3 * f], 24);
        if (nrm) {
            double nb[3] = {0, 0, 0};
            for (int q = 0; q < Q; q++)
                for (int i = 0; i < 3; i++) nb[i] += m->fdA[f * RGO_MAXQ + q] * m->fn[(f * RGO_MAXQ + q) * 3 + i];
            double n = sqrt(nb[0] * nb[0] + nb[1] * nb[1] + nb[2] * nb[2]);
            for (int i = 0; i < 3; i++) nrm[3 * f + i] = nb[i] / n;
        }
        if (area) area[f] = m->farea[f];
        if (zones) { zones[2 * f] = m->face_zone[2 * f]; zones[2 * f + 1] = m->face_zone[2 * f + 1]; }
    }
}

/* face quadrature points, unit normals and |dA| (owner order) */
void rgo_face_quad(const rgo_mesh *m, double *x, double *n, double *dA)
{
    const int Q = m->nq_face * m->nq_face;
    for (int f = 0; f < m->nf; f++)
        for (int q = 0; q < Q; q++) {
            if (x) memcpy(&x[(f * Q + q) * 3], &m->fx[(f * RGO_MAXQ + q) * 3], 24);
            if (n) memcpy(&n[(f * Q + q) * 3], &m->fn[(f * RGO_MAXQ + q) * 3], 24);
            if (dA) dA[f * Q + q] = m->fdA[f * RGO_MAXQ + q];
        }
}

void rgo_edge_data(const rgo_mesh *m, double *mid, double *tan, int *nzones)
{
    for (int e = 0; e < m->ne; e++) {
        if (mid) memcpy(&mid[3 * e], &m->ex[e * 9 + 3], 24);
        if (tan) memcpy(&tan[3 * e], &m->et[e * 9 + 3], 24);
        if (nzones) nzones[e] = m->edge_nz[e];
    }
}

void rgo_face_edges(const rgo_mesh *m, int *edges, int *signs)
{
    memcpy(edges, m->face_edges, sizeof(int) * 4 * m->nf);
    memcpy(signs, m->face_esign, sizeof(int) * 4 * m->nf);
}

void rgo_cubature(const rgo_mesh *m, int z, double *x, double *wJ)
{
    for (int q = 0; q < m->ncub; q++) {
        memcpy(&x[3 * q], m->cub[(size_t)z * m->ncub + q].x, 24);
        wJ[q] = m->cub[(size_t)z * m->ncub + q].wJ;
    }
}

int rgo_ncub(const rgo_mesh *m) { return m->ncub; }

void rgo_node_data(const rgo_mesh *m, int z, double *x, double *J, double *met)
{
    const int N = m->ref.N;
    if (x) memcpy(x, &m->nodex[(size_t)z * N * 3], sizeof(double) * N * 3);
    if (J) memcpy(J, &m->nodeJ[(size_t)z * N], sizeof(double) * N);
    if (met) memcpy(met, &m->nodeMet[(size_t)z * N * 9], sizeof(double) * N * 9);
}

/* largest deviation of the mapped surface |S(xi,eta)| from the unit sphere */
double rgo_sphericity(const rgo_mesh *m, int samples)
{
    double worst = 0.0;
    for (int z = 0; z < m->nz; z += m->ktot) {
        int k = m->zone_shell[z];
        for (int i = 0; i <= samples; i++)
            for (int j = 0; j <= samples; j++) {
                double xi[3] = {-0.5 + (double)i / samples, -0.5 + (double)j / samples, -0.5}, x[3];
                zone_map(m, z, xi, x, NULL);
                double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) / m->radius[k];
                worst = fmax(worst, fabs(r - 1.0));
            }
    }
    return worst;
}

/* flags: 1 linear WENO weights (checks), 2 first-order fallback; fallback_zones
 * (may be NULL) receives 1 for every zone the fallback took */
int rgo_step(const rgo_mesh *m, double gamma, double dt, int bc_kind, int flags, double weno_eps, double flat_kappa,
             const double *U, const double *Bf, double *Uout, double *Bfout, double *dbgPhi, double *dbgGam,
             unsigned char *fallback_zones, double *eta)
{
    return rgo_run_step(m, gamma, dt, bc_kind, flags, weno_eps, flat_kappa, U, Bf, Uout, Bfout, dbgPhi, dbgGam,
                        fallback_zones, eta);
}

int rgo_recon(const rgo_mesh *m, int flags, double weno_eps, const double *U, const double *Bf, int z, int npts,
              const double *pts, double *weno, double *divB)
{
    return rgo_run_recon(m, flags, weno_eps, U, Bf, z, npts, pts, weno, divB);
}

int rgo_divfree(const rgo_mesh *m, int flags, double weno_eps, const double *U, const double *Bf, int z,
                double *coeffs, int *exps, double *face_nodal)
{
    return rgo_run_divfree_coeffs(m, flags, weno_eps, U, Bf, z, coeffs, exps, face_nodal);
}

int rgo_weno_order(const rgo_mesh *m, int bc_kind, int flags, double weno_eps, const double *U, const double *Bf,
                   double *whi)
{
    return rgo_run_weno_order(m, bc_kind, flags, weno_eps, U, Bf, whi);
}

double rgo_cfl_dt(const rgo_mesh *m, double gamma, double cfl, const double *U)
{
    return rgo_run_cfl(m, gamma, cfl, U);
}

void rgo_init_harmonic(const rgo_mesh *m, const double *rho, const double *v, const double *A, double p,
                       double gamma, double *U, double *Bf)
{
    rgo_run_init_harmonic(m, rho, v, A, p, gamma, U, Bf);
}

void rgo_init_alfven(const rgo_mesh *m, const double *frame, double rho, double p, double B0, double dB,
                     double wavelength, double gamma, double t, double *U, double *Bf)
{
    rgo_run_init_alfven(m, frame, rho, p, B0, dB, wavelength, gamma, t, U, Bf);
}

/* spherical shock tube (Section VIII.c): states (rho, p, v_r, v_theta, v_phi,
 * B_theta, B_phi) inside and outside r = rm, B_r = Br0 sin(theta) (r0/r)^2 */
void rgo_init_tube(const rgo_mesh *m, const double *left, const double *right, double Br0, double r0, double rm,
                   double delta, double gamma, double *U, double *Bf)
{
    rgo_run_init_tube(m, left, right, Br0, r0, rm, delta, gamma, U, Bf);
}

/* reference-element matrices for checks: time nodes and weights, nodes,
 * nodal derivative matrices D[d][i][l] = d psi_l / d xi_d at node i, and the
 * full-Galerkin reduced matrices of eq. (5.29) */
int rgo_refel_query(int order, int *NM, double *tau, double *wt, double *nodes, double *D, double *Kd,
                    double *Kd0, double *Kt0)
{
    rgo_refel r;
    if (refel_init(&r, order)) return -1;
    int N = r.N, M = r.M, E = (M - 1) * N;
    NM[0] = N; NM[1] = M;
    if (tau) memcpy(tau, r.tau, sizeof(double) * M);
    if (wt) memcpy(wt, r.wt, sizeof(double) * M);
    if (nodes) memcpy(nodes, r.node, sizeof(double) * 3 * N);
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

int rgo_refel_eval(int order, int npts, const double *xi, double *psi)
{
    rgo_refel r;
    if (refel_init(&r, order)) return -1;
    for (int p = 0; p < npts; p++)
        for (int l = 0; l < r.N; l++) psi[p * r.N + l] = refel_psi(&r, l, &xi[3 * p]);
    refel_free(&r);
    return 0;
}

int rgo_lagrange(int n, const double *nodes, const int *exps, double *coef)
{
    return lagrange3(n, nodes, exps, coef);
}

void rgo_gauss01(int n, double *x, double *w) { gauss01(n, x, w); }

int rgo_predict(int order, double gamma, double dt, const double *J, const double *met, const double *Ua,
                double *Ulev, double *avgU, double *avgF)
{
    rgo_refel r;
    if (refel_init(&r, order)) return -1;
    int rc = rgo_predict_element(&r, gamma, dt, J, met, Ua, Ulev, avgU, avgF);
    refel_free(&r);
    return rc;
}

void rgo_hll(const double *UL, const double *UR, const double *n, double gamma, double *Fs)
{
    double FL[3][NVAR], FR[3][NVAR], FnL[NVAR], FnR[NVAR];
    phys_flux(UL, gamma, FL);
    phys_flux(UR, gamma, FR);
    for (int v = 0; v < NVAR; v++) {
        FnL[v] = n[0] * FL[0][v] + n[1] * FL[1][v] + n[2] * FL[2][v];
        FnR[v] = n[0] * FR[0][v] + n[1] * FR[1][v] + n[2] * FR[2][v];
    }
    hll_flux(UL, UR, FnL, FnR, n, gamma, Fs);
}

void rgo_flux(const double *U, double gamma, double *F)
{
    double Fp[3][NVAR];
    phys_flux(U, gamma, Fp);
    memcpy(F, Fp, sizeof(Fp));
}

double rgo_emf(const double *U4, const double *E4, const double *cen4, const double *t, double gamma)
{
    return rgo_emf4((const double(*)[NVAR])U4, (const double(*)[3])E4, (const double(*)[3])cen4, t, gamma);
}

/* test access to single pieces of the method */
double rgo_fast(const double *U, double gamma, const double *n) { return fast_speed(U, gamma, n); }

double rgo_emf3x(const double *U3, const double *E3, const double *n3, const double *t, double gamma)
{
    return rgo_emf3((const double(*)[NVAR])U3, (const double(*)[3])E3, (const double(*)[3])n3, t, gamma);
}

int rgo_weno_detail(const rgo_mesh *m, int flags, double weno_eps, const double *U, int z, double *out)
{
    return rgo_run_weno_detail(m, flags, weno_eps, U, z, out);
}

int rgo_weno_rows(const rgo_mesh *m, int z, double *A) { return rgo_run_weno_rows(m, z, A); }

void rgo_init_blast(const rgo_mesh *m, const double *axis, const double *centre, double radius, double rho,
                    double p_in, double p, double B0, double gamma, double *U, double *Bf)
{
    rgo_run_init_blast(m, axis, centre, radius, rho, p_in, p, B0, gamma, U, Bf);
}

/* one step with complex state (complex-step derivatives; see sreal.h) */
int rgo_step_cx(const rgo_mesh *m, double gamma, double dt, int bc_kind, int flags, double weno_eps,
                double flat_kappa, const double _Complex *U, const double _Complex *Bf, double _Complex *Uout,
                double _Complex *Bfout)
{
    return rgo_run_step_cx(m, gamma, dt, bc_kind, flags, weno_eps, flat_kappa, U, Bf, Uout, Bfout, NULL, NULL, NULL,
                           NULL);
}

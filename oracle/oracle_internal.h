/*
 * Internal declarations of the reference oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, FP64 CPU
 * implementation of one ADER-WENO-AO divergence-free MHD timestep
 * (Balsara et al., "Efficient, divergence-free, high order MHD on 3D
 * spherical meshes with optimal geodesic meshing", Sections II-VI and
 * Appendices A-D).  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code with the GPU library.
 */
#ifndef RGO_INTERNAL_H
#define RGO_INTERNAL_H

#include <stdint.h>
#include <stddef.h>

#define NVAR 8
enum { IRHO = 0, IMX = 1, IMY = 2, IMZ = 3, IEN = 4, IBX = 5, IBY = 6, IBZ = 7 };

/* ---------------- dense linear algebra (row-major) ---------------- */
int la_inverse(int n, const double *A, double *Ainv);
int la_lu_solve(int n, const double *A, const double *b, double *x);
int la_lsq_qr(int m, int n, const double *A, const double *b, double *x);

/* ---------------- reference element ---------------- */
void gauss01(int n, double *x, double *w);
int lagrange3(int n, const double *nodes, const int *exps, double *coef);
double mono3(const int *e, const double *x);
double dmono3(const int *e, int dir, const double *x);

#define RGO_MAXN 32
typedef struct {
    int order, N, M, L;
    double node[RGO_MAXN][3];
    int exps[RGO_MAXN][3];
    double coef[RGO_MAXN * RGO_MAXN];
    double tau[4];
    double wt[4];
    double *Kt0;     /* (L-N) x N        : -(K_tau^11)^-1 K_tau^10          */
    double *Kd0[3];  /* (L-N) x N        :  (K_tau^11)^-1 K_d^10            */
    double *Kd[3];   /* (L-N) x (L-N)    :  (K_tau^11)^-1 K_d^11            */
} rgo_refel;

int refel_init(rgo_refel *r, int order);
int refel_spacetime(rgo_refel *r, int M, int nq, const double *xq, const double *wq);
void refel_free(rgo_refel *r);
double refel_psi(const rgo_refel *r, int l, const double *xi);
double refel_dpsi(const rgo_refel *r, int l, int d, const double *xi);

/* ---------------- mesh + geometry ---------------- */
#define RGO_MAXQ 9       /* face quadrature points (3x3) */
#define RGO_MAXST 40     /* large-stencil capacity       */

typedef struct {
    double x[3];
    double wJ;
} cub_pt;

typedef struct {
    int n_ang, n_rad, n_ghost, ktot, map_order, order;
    int nq_face;           /* quadrature points per face direction (2 or 3) */
    int ncub_ang, ncub_rad;
    double r_in, r_out;
    double *radius;        /* ktot+1 interface radii (extended index) */

    int nv, nquad;
    double *vert;          /* nv*3 unit vectors */
    int *quad;             /* nquad*4 vertex ids, counter-clockwise seen from outside */

    int nz, nf, ne;
    int *zone_quad, *zone_shell;
    int *zone_face;        /* nz*6  */
    int *zone_edge;        /* nz*12 */
    int *zone_nbr;         /* nz*6, -1 if none */

    int *face_zone;        /* nf*2 owner, other (-1) */
    int *face_lf;          /* nf*2 */
    int *face_perm;        /* nf*RGO_MAXQ : other's local point matching owner point q */
    int *edge_hv;          /* ne*2 hex-vertex ids, low then high */
    int *edge_nz;          /* ne */
    int *edge_zone;        /* ne*4, counter-clockwise around the edge direction */
    int *edge_le;          /* ne*4 local edge in that zone */
    int *edge_rev;         /* ne*4 */
    int *face_edges;       /* nf*4 */
    int *face_esign;       /* nf*4 */

    int *st_n, *st_z;      /* large stencil */

    /* per-zone geometry */
    double *snode;         /* nz*16*3 surface map nodes (unit sphere) */
    double *vol, *cen, *len;
    double *mom;           /* nz*125: C[a][b][c] = avg (X^a Y^b Z^c), a,b,c<5 */
    int ncub;
    cub_pt *cub;           /* nz*ncub */
    double *nodex, *nodeJ, *nodeMet;   /* nz*N*3, nz*N, nz*N*9 */

    /* per-face geometry (from the owner's map) */
    double *fx, *fn, *fdA; /* nf*Q*3, nf*Q*3, nf*Q  */
    double *farea, *fcen;  /* nf, nf*3 */
    /* per-edge geometry */
    double *ex, *et, *edl; /* ne*3*3, ne*3*3, ne*3 */

    rgo_refel ref;
} rgo_mesh;

/* geometry helpers */
void zone_map(const rgo_mesh *m, int z, const double *xi, double *x, double *jac);
void face_ref_point(const rgo_mesh *m, int lf, int q, double *xi);
void edge_ref_point(int le, double s, double *xi);

int mesh_build_topology(rgo_mesh *m);
int mesh_build_geometry(rgo_mesh *m);

/* physics */
void phys_flux(const double *U, double gamma, double F[3][NVAR]);
double fast_speed(const double *U, double gamma, const double *n);
void hll_flux(const double *UL, const double *UR, const double *FnL, const double *FnR,
              const double *n, double gamma, double *Fs);

#endif
